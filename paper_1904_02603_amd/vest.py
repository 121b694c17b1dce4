"""ctypes binding of the libvest C ABI (include/vest.h).

Argument marshalling only: every step runs in the HIP kernels of libvest.so.
Device memory and streams come from PyTorch.  The library must be built
(``python -m paper_1904_02603_amd.build``); importing this module on a
machine where it is missing raises immediately -- there is no fallback.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvest.so")
MAX_ORDER = 10

OK, EINVAL, ENOSPC, EDEVICE, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
REG_LF, REG_L1 = 0, 1
FP64, FP32, BF16 = 0, 1, 2
KERNEL_AUTO, KERNEL_DENSE, KERNEL_GATHER = 0, 1, 2

EXPORTS = ["vest_workspace_bytes", "vest_init", "vest_sweep_factor", "vest_sweep_core",
           "vest_responsibility", "vest_prune", "vest_loss", "vest_normalize", "vest_count_nonzeros",
           "vest_export", "vest_test_error", "vest_value_keys", "vest_compact", "vest_set_kernel",
           "vest_layout_stats", "vest_slab_timing", "vest_slab_time", "vest_destroy", "vest_strerror",
           "vest_last_error", "vest_model_error_noalloc", "vest_iterate_many",
           "vest_server_create", "vest_server_submit", "vest_server_progress", "vest_server_status",
           "vest_server_fetch", "vest_server_stats", "vest_server_destroy"]
JOB_QUEUED, JOB_ACTIVE, JOB_DONE, JOB_FAILED = 0, 1, 2, 3


class VestError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


class Desc(C.Structure):
    _fields_ = [
        ("order", C.c_int32),
        ("reg", C.c_int32),
        ("precision", C.c_int32),
        ("reserved", C.c_int32),
        ("lam", C.c_double),
        ("nnz", C.c_int64),
        ("dims", C.c_int64 * MAX_ORDER),
        ("ranks", C.c_int32 * MAX_ORDER),
    ]


_lib = None


def load_library(path=LIB_PATH):
    """Load libvest.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libvest.so is not built (%s); run python -m paper_1904_02603_amd.build" % path)
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    PD = C.POINTER(Desc)
    lib.vest_workspace_bytes.argtypes = [PD, C.POINTER(C.c_size_t)]
    lib.vest_init.argtypes = [PD, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, C.POINTER(vp)]
    lib.vest_sweep_factor.argtypes = [vp, i32]
    lib.vest_sweep_core.argtypes = [vp]
    lib.vest_responsibility.argtypes = [vp, vp, vp]
    lib.vest_prune.argtypes = [vp, i64, vp]
    lib.vest_loss.argtypes = [vp, vp]
    lib.vest_set_kernel.argtypes = [vp, i32]
    lib.vest_compact.argtypes = [vp, C.POINTER(i64)]
    lib.vest_normalize.argtypes = [vp]
    lib.vest_count_nonzeros.argtypes = [vp, vp]
    lib.vest_export.argtypes = [vp, vp, vp, vp, vp]
    lib.vest_test_error.argtypes = [vp, vp, vp, i64, vp]
    lib.vest_model_error_noalloc.argtypes = [PD, vp, vp, vp, vp, vp, i64, vp]
    lib.vest_iterate_many.argtypes = [vp, i32, vp, vp, vp, C.c_size_t]
    lib.vest_value_keys.argtypes = [vp, vp, vp]
    lib.vest_layout_stats.argtypes = [vp, i32, vp]
    lib.vest_slab_timing.argtypes = [vp, i32]
    lib.vest_slab_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64)]
    lib.vest_destroy.argtypes = [vp]
    lib.vest_strerror.argtypes = [C.c_int]
    lib.vest_strerror.restype = C.c_char_p
    lib.vest_last_error.argtypes = []
    lib.vest_last_error.restype = C.c_char_p
    lib.vest_server_create.argtypes = [C.c_size_t, i32, C.POINTER(vp)]
    lib.vest_server_submit.argtypes = [vp, C.POINTER(Job), C.POINTER(i64)]
    lib.vest_server_progress.argtypes = [vp, C.POINTER(i32)]
    lib.vest_server_status.argtypes = [vp, i64, C.POINTER(i32), C.POINTER(i32), vp]
    lib.vest_server_fetch.argtypes = [vp, i64, vp, vp, vp]
    lib.vest_server_stats.argtypes = [vp, vp]
    lib.vest_server_destroy.argtypes = [vp]
    for name in ["vest_server_create", "vest_server_submit", "vest_server_progress", "vest_server_status",
                 "vest_server_fetch", "vest_server_stats", "vest_server_destroy"]:
        getattr(lib, name).restype = C.c_int
    for name in ["vest_workspace_bytes", "vest_init", "vest_sweep_factor", "vest_sweep_core",
                 "vest_responsibility", "vest_prune", "vest_loss", "vest_normalize", "vest_count_nonzeros",
                 "vest_export", "vest_test_error", "vest_value_keys", "vest_compact", "vest_set_kernel",
                 "vest_layout_stats", "vest_destroy", "vest_model_error_noalloc", "vest_iterate_many"]:
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc, where):
    if rc != OK:
        msg = _lib.vest_last_error().decode(errors="replace")
        raise VestError(rc, where, msg)


def make_desc(dims, ranks, nnz, reg=REG_LF, lam=0.01, precision=FP64):
    d = Desc()
    d.order = len(dims)
    d.reg = reg
    d.precision = precision
    d.reserved = 0
    d.lam = lam
    d.nnz = nnz
    for n in range(len(dims)):
        d.dims[n] = int(dims[n])
        d.ranks[n] = int(ranks[n])
    return d


def workspace_bytes(dims, ranks, nnz, reg=REG_LF, lam=0.01, precision=FP64):
    lib = load_library()
    d = make_desc(dims, ranks, nnz, reg, lam, precision)
    out = C.c_size_t(0)
    _check(lib.vest_workspace_bytes(C.byref(d), C.byref(out)), "vest_workspace_bytes")
    return int(out.value)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _ptr_array(ts):
    return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def masks_to_bool(fmask, J):
    """int32 bit masks [I] -> bool [I, J]."""
    bits = torch.arange(J, device=fmask.device, dtype=torch.int32)
    return ((fmask.unsqueeze(1) >> bits) & 1).bool()


def bool_to_masks(mask_bool):
    """bool [I, J] -> int32 bit masks [I] (J <= 31)."""
    J = mask_bool.shape[1]
    w = (torch.ones(J, dtype=torch.int64, device=mask_bool.device) << torch.arange(J, device=mask_bool.device))
    return (mask_bool.to(torch.int64) * w).sum(dim=1).to(torch.int32)


class VestContext:
    """One factorisation job: device-resident state plus its libvest context.

    factors / core / masks are torch CUDA tensors owned by this object and
    updated in place by the library (factors float64 [I_n, J], core float64
    with shape (J,)*N, factor masks int32 [I_n] bit masks, core mask uint8).
    """

    def __init__(self, idx, val, factors, core, reg=REG_LF, lam=0.01, precision=FP64,
                 fmask=None, cmask=None, stream=None, device="cuda"):
        self.lib = load_library()
        dev = torch.device(device)
        self.idx = torch.as_tensor(idx, dtype=torch.int32, device=dev).contiguous()
        self.val = torch.as_tensor(val, dtype=torch.float64, device=dev).contiguous()
        self.N = self.idx.shape[1]
        self.factors = [torch.as_tensor(f, dtype=torch.float64, device=dev).clone().contiguous() for f in factors]
        self.core = torch.as_tensor(core, dtype=torch.float64, device=dev).clone().contiguous()
        self.dims = [int(f.shape[0]) for f in self.factors]
        self.ranks = [int(f.shape[1]) for f in self.factors]
        self.J = self.ranks[0]
        self.fmask = ([torch.zeros(I, dtype=torch.int32, device=dev) for I in self.dims] if fmask is None
                      else [torch.as_tensor(m, dtype=torch.int32, device=dev).clone().contiguous() for m in fmask])
        self.cmask = (torch.zeros(self.core.shape, dtype=torch.uint8, device=dev) if cmask is None
                      else torch.as_tensor(cmask, dtype=torch.uint8, device=dev).clone().contiguous())
        self.reg, self.lam, self.precision = reg, lam, precision
        self.nnz = int(self.idx.shape[0])
        self.desc = make_desc(self.dims, self.ranks, self.nnz, reg, lam, precision)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        nb = C.c_size_t(0)
        _check(self.lib.vest_workspace_bytes(C.byref(self.desc), C.byref(nb)), "vest_workspace_bytes")
        self.ws_bytes = int(nb.value)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.ctx = C.c_void_p()
        with torch.cuda.stream(self.stream):
            rc = self.lib.vest_init(C.byref(self.desc), C.c_void_p(self.stream.cuda_stream),
                                    _ptr(self.idx), _ptr(self.val), _ptr_array(self.factors),
                                    _ptr(self.core), _ptr_array(self.fmask), _ptr(self.cmask),
                                    C.c_void_p(self._ws_ptr), C.c_size_t(self.ws_bytes), C.byref(self.ctx))
        _check(rc, "vest_init")
        self.core_key = torch.empty(self.core.shape, dtype=torch.float64, device=dev)
        self.factor_keys = [torch.empty_like(f) for f in self.factors]

    # -- Alg. 4
    def sweep_factor(self, mode):
        _check(self.lib.vest_sweep_factor(self.ctx, int(mode)), "vest_sweep_factor")

    # -- Eq. 12 / 14
    def sweep_core(self):
        _check(self.lib.vest_sweep_core(self.ctx), "vest_sweep_core")

    # -- Eq. 5 / 6
    def responsibility(self):
        _check(self.lib.vest_responsibility(self.ctx, _ptr(self.core_key), _ptr_array(self.factor_keys)),
               "vest_responsibility")
        return self.core_key, self.factor_keys

    # -- Sec. 3.3
    def prune(self, core_k, factor_k):
        arr = (C.c_int64 * self.N)(*[int(k) for k in factor_k])
        _check(self.lib.vest_prune(self.ctx, int(core_k), arr), "vest_prune")

    # -- Eq. 1 / 2 / 4
    def loss(self):
        out = (C.c_double * 5)()
        _check(self.lib.vest_loss(self.ctx, out), "vest_loss")
        return {"sse": out[0], "xnorm2": out[1], "reg": out[2], "loss": out[3], "re": out[4]}

    def iteration(self):
        for n in range(self.N):
            self.sweep_factor(n)
        self.sweep_core()

    def normalize(self):
        """Final column normalisation of Alg. 2 (reconstruction unchanged)."""
        _check(self.lib.vest_normalize(self.ctx), "vest_normalize")

    def count_nonzeros(self):
        out = (C.c_int64 * (self.N + 1))()
        _check(self.lib.vest_count_nonzeros(self.ctx, out), "vest_count_nonzeros")
        return list(out)

    def export(self):
        """Sparse model: [(flat_idx, values) per factor], (flat_idx, values) of the core."""
        cnt = self.count_nonzeros()
        fi = [torch.empty(max(c, 1), dtype=torch.int64, device=self.core.device) for c in cnt[:-1]]
        fv = [torch.empty(max(c, 1), dtype=torch.float64, device=self.core.device) for c in cnt[:-1]]
        ci = torch.empty(max(cnt[-1], 1), dtype=torch.int64, device=self.core.device)
        cv = torch.empty(max(cnt[-1], 1), dtype=torch.float64, device=self.core.device)
        _check(self.lib.vest_export(self.ctx, _ptr_array(fi), _ptr_array(fv), _ptr(ci), _ptr(cv)), "vest_export")
        torch.cuda.synchronize()
        return [(a[:c], b[:c]) for a, b, c in zip(fi, fv, cnt)], (ci[:cnt[-1]], cv[:cnt[-1]])

    def test_error(self, idx, val):
        """(sum (X-B)^2, sum X^2, RE) of the current model on held-out entries."""
        i = torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32), device=self.core.device)
        v = torch.as_tensor(np.ascontiguousarray(val, dtype=np.float64), device=self.core.device)
        out = (C.c_double * 3)()
        _check(self.lib.vest_test_error(self.ctx, _ptr(i), _ptr(v), int(i.shape[0]), out), "vest_test_error")
        return {"sse": out[0], "xnorm2": out[1], "re": out[2]}

    def value_keys(self):
        """Magnitude keys (value-pruning comparator); the next prune uses them."""
        self.core_key = torch.empty_like(self.core)
        self.factor_keys = [torch.empty_like(f) for f in self.factors]
        _check(self.lib.vest_value_keys(self.ctx, _ptr(self.core_key), _ptr_array(self.factor_keys)),
               "vest_value_keys")
        return self.core_key, self.factor_keys

    def compact(self):
        """Drop entries with a fully marked row in some mode; returns the kept count."""
        live = C.c_int64(0)
        _check(self.lib.vest_compact(self.ctx, C.byref(live)), "vest_compact")
        return live.value

    def set_kernel(self, kernel):
        """Contraction kernel policy: KERNEL_AUTO, KERNEL_DENSE or KERNEL_GATHER."""
        _check(self.lib.vest_set_kernel(self.ctx, int(kernel)), "vest_set_kernel")

    def slab_timing(self, enable=True):
        """Record the duration of every slab pass of the core sweep (instrumentation)."""
        _check(self.lib.vest_slab_timing(self.ctx, 1 if enable else 0), "vest_slab_timing")

    def slab_time(self):
        """(summed milliseconds, launches) of the slab passes recorded since the last call."""
        ms, n = C.c_double(0.0), C.c_int64(0)
        _check(self.lib.vest_slab_time(self.ctx, C.byref(ms), C.byref(n)), "vest_slab_time")
        return ms.value, n.value

    def layout_stats(self, mode):
        out = (C.c_int64 * 8)()
        _check(self.lib.vest_layout_stats(self.ctx, int(mode), out), "vest_layout_stats")
        keys = ["slots", "pad", "waves", "long_rows", "long_chunks", "max_row", "rows", "nnz"]
        return dict(zip(keys, list(out)))

    def factor_masks_bool(self):
        return [masks_to_bool(m, J) for m, J in zip(self.fmask, self.ranks)]

    def marked_counts(self):
        return [int(masks_to_bool(m, J).sum()) for m, J in zip(self.fmask, self.ranks)], int(self.cmask.sum())

    def close(self):
        if self.ctx is not None and self.ctx.value:
            self.lib.vest_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """vest_iterate_many: one Alg. 2 iteration of several contexts of one
    shape in one sequence of launches.  Owns a device table buffer and a
    pinned host staging buffer of `table_bytes`."""

    def __init__(self, table_bytes=4 << 20, device="cuda"):
        self.lib = load_library()
        self.bytes = int(table_bytes)
        self.dev = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        self.host = torch.empty(self.bytes, dtype=torch.uint8, pin_memory=True)

    def iterate(self, ctxs, stream=None, wait=True):
        """Returns VEST_OK, or EUNSUPPORTED when the batched path does not
        take these contexts (nothing was enqueued then).  The staging buffer
        is reused, so by default the stream is drained first (wait=False when
        the previous upload from this Batch is known to be complete)."""
        st = stream if stream is not None else torch.cuda.current_stream()
        arr = (C.c_void_p * len(ctxs))(*[c.ctx.value for c in ctxs])
        if wait:
            st.synchronize()
        rc = self.lib.vest_iterate_many(arr, len(ctxs), C.c_void_p(st.cuda_stream), _ptr(self.dev), _ptr(self.host),
                                        C.c_size_t(self.bytes))
        if rc not in (OK, EUNSUPPORTED):
            _check(rc, "vest_iterate_many")
        return rc


NOALLOC_MAX_ENTRIES = 1 << 24


def model_error_noalloc(factors, core, idx, val, out, stream=None):
    """vest_model_error_noalloc: held-out loss terms of a model given as device
    tensors (factors: list of float64 [I_n, J_n], core float64), entries idx
    int32 [n, N] and val float64 [n] on the device; out is a float64 device
    tensor of 4 values, written on `stream` (no synchronisation)."""
    lib = load_library()
    dims = [int(f.shape[0]) for f in factors]
    ranks = [int(f.shape[1]) for f in factors]
    desc = make_desc(dims, ranks, max(1, int(idx.shape[0])))
    st = stream if stream is not None else torch.cuda.current_stream(out.device)
    _check(lib.vest_model_error_noalloc(C.byref(desc), C.c_void_p(st.cuda_stream), _ptr_array(factors), _ptr(core),
                                        _ptr(idx), _ptr(val), int(idx.shape[0]), _ptr(out)),
           "vest_model_error_noalloc")


def job_footprint(dims, ranks, nnz, reg=REG_LF, lam=0.01, precision=FP32, prune_target=0.0):
    """Device bytes a server reserves to admit a job (see vest_serve.h)."""
    def a(x):
        return (int(x) + 255) // 256 * 256
    N = len(dims)
    G = int(np.prod(ranks))
    ws = workspace_bytes(dims, ranks, nnz, reg, lam, precision)
    fac = sum(I * J for I, J in zip(dims, ranks))
    keys = a((G + fac) * 8) if prune_target > 0 else 0
    return (a(ws) + a(fac * 8) + a(G * 8) + a(sum(dims) * 4) + a(G) + a(nnz * N * 4) + a(nnz * 8) + keys)


class Job(C.Structure):
    """vest_job of vest_serve.h."""
    _fields_ = [("desc", Desc), ("idx", C.c_void_p), ("val", C.c_void_p), ("factors", C.c_void_p),
                ("core", C.c_void_p), ("iterations", C.c_int32), ("reserved", C.c_int32),
                ("prune_target", C.c_double)]


class VestServer:
    """Request loop of vest_serve.h: jobs share one device arena of
    `device_bytes` and `slots` streams; see the header for the policy."""

    def __init__(self, device_bytes, slots):
        self.lib = load_library()
        self.srv = C.c_void_p()
        _check(self.lib.vest_server_create(int(device_bytes), int(slots), C.byref(self.srv)), "vest_server_create")
        self._keep = {}
        self._shape = {}

    def submit(self, idx, val, factors, core, reg=REG_LF, lam=0.01, precision=FP32, iterations=10,
               prune_target=0.0):
        """Queue a job (numpy host arrays); returns its id.  prune_target > 0
        runs VeST^man toward that sparsity (see vest_job in vest_serve.h)."""
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        factors = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
        core = np.ascontiguousarray(core, dtype=np.float64)
        dims = [f.shape[0] for f in factors]
        ranks = [f.shape[1] for f in factors]
        fp = (C.c_void_p * len(factors))(*[f.ctypes.data for f in factors])
        j = Job()
        j.desc = make_desc(dims, ranks, idx.shape[0], reg, lam, precision)
        j.idx, j.val, j.factors, j.core = idx.ctypes.data, val.ctypes.data, C.cast(fp, C.c_void_p), core.ctypes.data
        j.iterations = int(iterations)
        j.reserved = 0
        j.prune_target = float(prune_target)
        jid = C.c_int64(0)
        _check(self.lib.vest_server_submit(self.srv, C.byref(j), C.byref(jid)), "vest_server_submit")
        self._keep[jid.value] = (idx, val, factors, core, fp, j)
        self._shape[jid.value] = (dims, ranks)
        return jid.value

    def progress(self):
        """One scheduling pass; returns the number of jobs retired by it."""
        done = C.c_int32(0)
        _check(self.lib.vest_server_progress(self.srv, C.byref(done)), "vest_server_progress")
        return done.value

    def status(self, jid):
        st, err = C.c_int32(0), C.c_int32(0)
        t = (C.c_double * 3)()
        _check(self.lib.vest_server_status(self.srv, int(jid), C.byref(st), C.byref(err), t), "vest_server_status")
        if st.value != JOB_QUEUED:
            self._keep.pop(jid, None)  # inputs were read at admission
        return {"state": st.value, "error": err.value, "arrive": t[0], "admit": t[1], "done": t[2]}

    def fetch(self, jid):
        """Factors (list of numpy [I_n, J]), core and loss dict of a finished job."""
        dims, ranks = self._shape[jid]
        fac = [np.empty((I, J)) for I, J in zip(dims, ranks)]
        core = np.empty(tuple(ranks))
        loss = (C.c_double * 5)()
        fp = (C.c_void_p * len(fac))(*[f.ctypes.data for f in fac])
        _check(self.lib.vest_server_fetch(self.srv, int(jid), fp, core.ctypes.data, loss), "vest_server_fetch")
        return fac, core, dict(zip(["sse", "xnorm2", "reg", "loss", "re"], list(loss)))

    def stats(self):
        out = (C.c_int64 * 8)()
        _check(self.lib.vest_server_stats(self.srv, out), "vest_server_stats")
        return dict(zip(["queued", "active", "finished", "bytes_used", "bytes_total", "largest_free", "batches",
                         "batched_job_iterations"], list(out)))

    def close(self):
        if self.srv is not None and self.srv.value:
            self.lib.vest_server_destroy(self.srv)
            self.srv = C.c_void_p()
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
