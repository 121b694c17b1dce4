"""vest_model_error_noalloc (the allocation-free entry point) against
vest_test_error, through the C ABI.

The two compute the same loss terms (Eq. 4 on a held-out entry set) with
different contraction orders, so the FP64 bar is 1e-10 relative.  Each test
makes two calls in a row, the second with a smaller entry set, so that the
second call reads partials the first one left in the shared static scratch
only where it wrote them itself.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_1904_02603_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def V():
    from paper_1904_02603_amd import vest
    return vest


def heldout(dims, n, seed):
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, d, n) for d in dims], 1).astype(np.int32)
    val = rng.normal(size=n)
    return idx, val


def noalloc(model_f, model_c, idx, val):
    v = V()
    i = torch.as_tensor(idx, device="cuda")
    x = torch.as_tensor(val, device="cuda")
    out = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
    v.model_error_noalloc(model_f, model_c, i, x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def close(a, b):
    return abs(a - b) <= RTOL * abs(b)


@pytest.mark.parametrize("shape", [((60, 50, 40), (5, 5, 5), 5000), ((30, 25, 20, 24), (8, 8, 8, 8), 4000),
                                   ((200, 150, 100), (10, 10, 10), 20_000)],
                         ids=["N3J5", "N4J8", "N3J10"])
def test_noalloc_matches_test_error_two_calls(shape):
    v = V()
    dims, ranks, nnz = shape
    p = synth.make_problem(dims, nnz, ranks, 41, noise_var=0.01)
    g = v.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=v.REG_LF, lam=0.05)
    g.iteration()
    for n_test in (3000, 700):   # second call smaller than the first
        idx, val = heldout(dims, n_test, n_test)
        ref = g.test_error(idx, val)
        got = noalloc(g.factors, g.core, idx, val)
        print("n", n_test, "sse", got[0], ref["sse"], flush=True)
        assert got[3] == 0.0
        assert close(got[0], ref["sse"]), (got[0], ref["sse"])
        assert close(got[1], ref["xnorm2"]), (got[1], ref["xnorm2"])
        assert close(got[2], ref["re"]), (got[2], ref["re"])
    g.close()


def test_noalloc_unequal_ranks_match_oracle():
    # per-mode ranks (Table 1: J_n per mode): the oracle's loss on the held-out
    # entries with the same model
    dims, ranks = (40, 30, 20, 10), (3, 5, 2, 4)
    rng = np.random.default_rng(7)
    fac = [rng.random((d, r)) for d, r in zip(dims, ranks)]
    core = rng.random(ranks)
    for n_test in (5000, 1200):
        idx, val = heldout(dims, n_test, 100 + n_test)
        _, keep = np.unique(idx, axis=0, return_index=True)
        idx, val = idx[np.sort(keep)], val[np.sort(keep)]
        o = Oracle(idx, val, fac, core, reg=0, lam=0.01)
        ol = o.loss()
        got = noalloc([torch.as_tensor(f, device="cuda") for f in fac], torch.as_tensor(core, device="cuda"),
                      idx, val)
        assert close(got[0], ol["sse"]), (got[0], ol["sse"])
        assert close(got[1], ol["xnorm2"]), (got[1], ol["xnorm2"])
        assert close(got[2], ol["re"]), (got[2], ol["re"])


def test_noalloc_edge_cases():
    v = V()
    dims, ranks = (20, 20, 20), (3, 3, 3)
    rng = np.random.default_rng(8)
    fac = [torch.as_tensor(rng.random((d, r)), device="cuda") for d, r in zip(dims, ranks)]
    core = torch.as_tensor(rng.random(ranks), device="cuda")
    # empty set: zeros
    got = noalloc(fac, core, np.zeros((0, 3), np.int32), np.zeros(0))
    assert list(got) == [0.0, 0.0, 0.0, 0.0]
    # an index out of range is counted; the sums are NaN
    idx, val = heldout(dims, 2000, 9)
    idx[1500, 2] = 20
    got = noalloc(fac, core, idx, val)
    assert got[3] == 1.0 and np.isnan(got[0]) and np.isnan(got[2])
    # beyond the static scratch bound: rejected on the host, nothing enqueued
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    i = torch.zeros((1, 3), dtype=torch.int32, device="cuda")
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    lib = v.load_library()
    d = v.make_desc(dims, ranks, 1)
    import ctypes as C
    rc = lib.vest_model_error_noalloc(C.byref(d), None, v._ptr_array(fac), v._ptr(core), v._ptr(i), v._ptr(x),
                                      v.NOALLOC_MAX_ENTRIES + 1, v._ptr(out))
    assert rc == v.EINVAL
    assert b"VEST_NOALLOC_MAX_ENTRIES" in lib.vest_last_error()
