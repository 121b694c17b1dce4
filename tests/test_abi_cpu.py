"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vest.h")
HEADERS = [os.path.join(ROOT, "include", h) for h in ("vest.h", "vest_serve.h")]
LIB = os.path.join(ROOT, "paper_1904_02603_amd", "libvest.so")


def declared():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vest_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1904_02603_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ["vest_workspace_bytes", "vest_init", "vest_sweep_factor", "vest_sweep_core",
              "vest_responsibility", "vest_prune", "vest_loss", "vest_destroy", "vest_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_1904_02603_amd import vest
    assert sorted(vest.EXPORTS) == declared()


def test_strerror_is_host_only(lib):
    lib.vest_strerror.restype = ctypes.c_char_p
    assert lib.vest_strerror(0) == b"ok"
    assert b"workspace" in lib.vest_strerror(-2)
    assert lib.vest_strerror(-99) == b"unknown error"


def test_error_codes_match_header():
    from paper_1904_02603_amd import vest
    src = open(HEADER).read()
    for name, val in [("VEST_OK", vest.OK), ("VEST_EINVAL", vest.EINVAL), ("VEST_ENOSPC", vest.ENOSPC),
                      ("VEST_EDEVICE", vest.EDEVICE), ("VEST_ESTATE", vest.ESTATE),
                      ("VEST_EUNSUPPORTED", vest.EUNSUPPORTED)]:
        assert re.search(r"%s\s*=\s*%d" % (name, val), src), name


def test_descriptor_layout_matches_header():
    from paper_1904_02603_amd import vest
    # int32 x4, double, int64, int64[10], int32[10]
    assert ctypes.sizeof(vest.Desc) == 4 * 4 + 8 + 8 + 80 + 40
