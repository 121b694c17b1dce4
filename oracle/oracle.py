"""ctypes front end of the FP64 CPU oracle (``vest_oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline may import this module; the product path never does.  It shares no
code with the GPU library.

Paper: Park, Jang, Sael, "VeST: Very Sparse Tucker Factorization of
Large-Scale Tensors" (arXiv:1904.02603).  Every method here names the
equation or algorithm of the paper that the C function follows.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vest_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
MAX_ORDER = 10

REG_LF = 0
REG_L1 = 1


def build(force=False, omp=False):
    """Compile the oracle with gcc (no FMA contraction, no fast-math).
    omp=True builds the optional OpenMP variant (liboracle_omp.so), which
    splits only independent sums and returns the same bits."""
    lib = _LIB_OMP if omp else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math"]
                              + (["-fopenmp"] if omp else []) + ["-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


class _State(C.Structure):
    _fields_ = [
        ("order", C.c_int32),
        ("reg", C.c_int32),
        ("lam", C.c_double),
        ("nnz", C.c_int64),
        ("dims", C.c_int64 * MAX_ORDER),
        ("ranks", C.c_int32 * MAX_ORDER),
        ("idx", C.c_void_p),
        ("val", C.c_void_p),
        ("factors", C.c_void_p * MAX_ORDER),
        ("core", C.c_void_p),
        ("fmask", C.c_void_p * MAX_ORDER),
        ("cmask", C.c_void_p),
        ("row_ptr", C.c_void_p * MAX_ORDER),
        ("row_ent", C.c_void_p * MAX_ORDER),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(build(omp=os.environ.get("VEST_ORACLE_OMP") == "1"))
        P = C.POINTER(_State)
        vp = C.c_void_p
        lib.or_build_rows.argtypes = [P]
        lib.or_build_rows.restype = C.c_int
        lib.or_free_rows.argtypes = [P]
        lib.or_delta.argtypes = [P, C.c_int32, C.c_int64, vp]
        lib.or_recon.argtypes = [P, C.c_int64]
        lib.or_recon.restype = C.c_double
        lib.or_residual.argtypes = [P, vp]
        lib.or_update_row.argtypes = [P, C.c_int32, C.c_int64]
        lib.or_update_factor_elem.argtypes = [P, C.c_int32, C.c_int64, C.c_int32]
        lib.or_sweep_factor.argtypes = [P, C.c_int32]
        lib.or_update_core_elem.argtypes = [P, C.c_int64]
        lib.or_sweep_core.argtypes = [P]
        lib.or_loss.argtypes = [P, vp]
        lib.or_responsibility.argtypes = [P, vp, vp]
        lib.or_prune.argtypes = [P, vp, vp, C.c_int64, vp]
        lib.or_prune.restype = C.c_int
        lib.or_normalize.argtypes = [P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """VeST state (factors, core, marking table) plus the observed tensor.

    Arrays are owned by this object as numpy arrays and updated in place by
    the C routines.  ``idx`` is [nnz, N] int32, 0-based; ``val`` is [nnz]
    float64; factors are [I_n, J_n] float64; ``core`` has shape (J_1..J_N).
    Masks are bool arrays of the same shapes (True = pruned, Sec. 3.3).
    """

    def __init__(self, idx, val, factors, core, reg=REG_LF, lam=0.01,
                 fmask=None, cmask=None):
        self.lib = _load()
        self.idx = np.ascontiguousarray(idx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.N = self.idx.shape[1]
        assert 1 <= self.N <= MAX_ORDER and self.idx.shape[0] == self.val.shape[0]
        self.factors = [np.array(f, dtype=np.float64, order="C", copy=True) for f in factors]
        self.core = np.array(core, dtype=np.float64, order="C", copy=True)
        self.dims = [f.shape[0] for f in self.factors]
        self.ranks = [f.shape[1] for f in self.factors]
        assert tuple(self.core.shape) == tuple(self.ranks)
        self.fmask = [np.zeros(f.shape, np.uint8) if fmask is None else
                      np.ascontiguousarray(fmask[n], dtype=np.uint8) for n, f in enumerate(self.factors)]
        self.cmask = (np.zeros(self.core.shape, np.uint8) if cmask is None else
                      np.ascontiguousarray(cmask, dtype=np.uint8))
        self.reg = int(reg)
        self.lam = float(lam)
        st = _State()
        st.order = self.N
        st.reg = self.reg
        st.lam = self.lam
        st.nnz = self.idx.shape[0]
        for n in range(self.N):
            st.dims[n] = self.dims[n]
            st.ranks[n] = self.ranks[n]
            st.factors[n] = self.factors[n].ctypes.data
            st.fmask[n] = self.fmask[n].ctypes.data
        st.idx = self.idx.ctypes.data
        st.val = self.val.ctypes.data
        st.core = self.core.ctypes.data
        st.cmask = self.cmask.ctypes.data
        self.st = st
        rc = self.lib.or_build_rows(C.byref(st))
        if rc != 0:
            raise ValueError("oracle: bad index (rc=%d)" % rc)

    def __del__(self):
        try:
            self.lib.or_free_rows(C.byref(self.st))
        except Exception:
            pass

    # ---- Eq. 11, Eq. 7
    def delta(self, n, e):
        out = np.zeros(self.ranks[n])
        self.lib.or_delta(C.byref(self.st), n, e, _ptr(out))
        return out

    def recon(self, e):
        return self.lib.or_recon(C.byref(self.st), e)

    def residual(self):
        out = np.zeros(self.idx.shape[0])
        self.lib.or_residual(C.byref(self.st), _ptr(out))
        return out

    # ---- Alg. 4, Eq. 9 / 13
    def update_row(self, n, i):
        self.lib.or_update_row(C.byref(self.st), n, i)

    def update_factor_elem(self, n, i, j):
        self.lib.or_update_factor_elem(C.byref(self.st), n, i, j)

    def sweep_factor(self, n):
        self.lib.or_sweep_factor(C.byref(self.st), n)

    # ---- Eq. 12 / 14
    def update_core_elem(self, flat):
        self.lib.or_update_core_elem(C.byref(self.st), flat)

    def sweep_core(self):
        self.lib.or_sweep_core(C.byref(self.st))

    # ---- Eq. 1 / 2 / 4
    def loss(self):
        out = np.zeros(5)
        self.lib.or_loss(C.byref(self.st), _ptr(out))
        return {"sse": out[0], "xnorm2": out[1], "reg": out[2], "loss": out[3], "re": out[4]}

    # ---- Eq. 5 / 6
    def responsibility(self):
        ck = np.zeros(self.core.shape)
        fk = [np.zeros(f.shape) for f in self.factors]
        arr = (C.c_void_p * self.N)(*[f.ctypes.data for f in fk])
        self.lib.or_responsibility(C.byref(self.st), _ptr(ck), arr)
        return ck, fk

    # ---- Sec. 3.3, Alg. 3
    def prune(self, core_key, factor_keys, core_k, factor_k):
        ck = np.ascontiguousarray(core_key, dtype=np.float64)
        fk = [np.ascontiguousarray(k, dtype=np.float64) for k in factor_keys]
        arr = (C.c_void_p * self.N)(*[k.ctypes.data for k in fk])
        kk = np.ascontiguousarray(factor_k, dtype=np.int64)
        rc = self.lib.or_prune(C.byref(self.st), _ptr(ck), arr, int(core_k), _ptr(kk))
        if rc != 0:
            raise ValueError("oracle: prune count exceeds unmarked elements")

    # ---- final normalisation of Alg. 2
    def normalize(self):
        self.lib.or_normalize(C.byref(self.st))

    # ---- Alg. 2 body without pruning
    def iteration(self):
        for n in range(self.N):
            self.sweep_factor(n)
        self.sweep_core()
