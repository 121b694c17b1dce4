"""GPU parity of every C-ABI call against the FP64 CPU oracle.

Each test feeds the same seeded state to libvest (through the ctypes binding)
and to the oracle, runs the same step on both and compares element by element.

Bar (FP64 path), per tensor (each factor matrix, the core, every key array):
    |gpu - oracle| <= RTOL * max(|oracle|, FLOOR * max|oracle|)
element by element, RTOL = 1e-10 and FLOOR = 1e-4: every element whose
magnitude is at least 1e-4 of the tensor's largest is within 1e-10 of its
own value; smaller ones (near-cancelled updates, whose rounding error scales
with the magnitude of the summed terms rather than with the result) are held
to 1e-14 of the tensor's largest.  Loss terms within 1e-10 relative (1e-12
where stated).  Prune masks identical.  The GPU sums in a different order
than the oracle's compensated sums, so bit equality of values is not
expected; masks are integer decisions and must match exactly.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle, REG_LF, REG_L1
from paper_1904_02603_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-10
FLOOR = 1e-4


def V():
    from paper_1904_02603_amd import vest
    return vest


def make(dims, ranks, nnz, seed, zipf=None):
    return synth.make_problem(dims, nnz, ranks, seed, zipf=zipf, noise_var=0.01)


def pair(p, reg, lam, precision=0, fmask=None, cmask=None):
    v = V()
    fac = [f.copy() for f in p["factors"]]
    core = p["core"].copy()
    if fmask is not None:
        fac = [f * (1 - m) for f, m in zip(fac, fmask)]
    if cmask is not None:
        core = core * (1 - cmask)
    gm = None if fmask is None else [v.bool_to_masks(torch.from_numpy(m.astype(bool))) for m in fmask]
    g = v.VestContext(p["idx"], p["val"], fac, core, reg=reg, lam=lam, precision=precision,
                      fmask=gm, cmask=None if cmask is None else torch.from_numpy(cmask.astype(np.uint8)))
    o = Oracle(p["idx"], p["val"], fac, core, reg=reg, lam=lam,
               fmask=None if fmask is None else [m.astype(np.uint8) for m in fmask],
               cmask=None if cmask is None else cmask.astype(np.uint8))
    return g, o


def _np(x):
    return x.detach().cpu().numpy() if torch.is_tensor(x) else np.asarray(x)


def rel_err(gpu, ref, floor=FLOOR):
    """max over elements of |gpu - ref| / max(|ref|, floor * max|ref|)
    (finite reference elements only)."""
    a, b = _np(gpu), _np(ref)
    fin = np.isfinite(b)
    a, b = a[fin], b[fin]
    if b.size == 0:
        return 0.0
    scale = max(float(np.abs(b).max()), 1e-300)
    return float((np.abs(a - b) / np.maximum(np.abs(b), floor * scale)).max())


def rms_err(gpu, ref):
    """Relative RMSE: ||gpu - ref||_2 / ||ref||_2."""
    a, b = _np(gpu), _np(ref)
    return float(np.sqrt(((a - b) ** 2).sum()) / max(np.sqrt((b * b).sum()), 1e-300))


def assert_state(g, o, rtol=RTOL, what=""):
    torch.cuda.synchronize()
    for n in range(o.N):
        e = rel_err(g.factors[n], o.factors[n])
        assert e <= rtol, "%s factor %d: rel err %.3e" % (what, n, e)
    e = rel_err(g.core, o.core)
    assert e <= rtol, "%s core: rel err %.3e" % (what, e)


def say(*a):
    print(*a, flush=True)


SHAPES = [
    # dims, ranks, nnz, zipf
    ((40, 50, 30), (3, 3, 3), 2000, None),
    ((100, 100, 100), (5, 5, 5), 10_000, None),
    ((200, 150, 100), (10, 10, 10), 20_000, None),
    ((12, 10, 8, 9), (2, 2, 2, 2), 3000, None),
    ((30, 25, 20, 24), (8, 8, 8, 8), 5000, None),
    ((60, 70), (3, 3), 1500, None),
    ((2000, 300, 50), (4, 4, 4), 30_000, (1.1, 1.0, None)),
    ((25, 20, 30, 16), (5, 5, 5, 5), 4000, None),
]
IDS = ["N3J3", "N3J5", "N3J10", "N4J2", "N4J8", "N2J3", "zipfN3J4", "N4J5"]


@pytest.mark.parametrize("reg", [REG_LF, REG_L1], ids=["LF", "L1"])
@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_factor_sweeps_match_oracle(shape, reg):
    dims, ranks, nnz, zipf = shape
    say("case", dims, ranks, nnz, reg)
    p = make(dims, ranks, nnz, 11, zipf)
    g, o = pair(p, reg, 0.05 if reg == REG_LF else 0.5)
    for n in range(len(dims)):
        g.sweep_factor(n)
        o.sweep_factor(n)
        assert_state(g, o, what="after mode %d" % n)


@pytest.mark.parametrize("reg", [REG_LF, REG_L1], ids=["LF", "L1"])
@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_core_sweep_matches_oracle(shape, reg):
    dims, ranks, nnz, zipf = shape
    say("case", dims, ranks, nnz, reg)
    p = make(dims, ranks, nnz, 12, zipf)
    g, o = pair(p, reg, 0.05 if reg == REG_LF else 0.5)
    g.sweep_core()
    o.sweep_core()
    assert_state(g, o, what="core sweep")
    gl, ol = g.loss(), o.loss()
    for k in ["sse", "xnorm2", "reg", "loss", "re"]:
        assert abs(gl[k] - ol[k]) <= RTOL * abs(ol[k]) + 1e-300, (k, gl[k], ol[k])


@pytest.mark.parametrize("shape", SHAPES[:5], ids=IDS[:5])
def test_loss_matches_oracle(shape):
    dims, ranks, nnz, zipf = shape
    p = make(dims, ranks, nnz, 13, zipf)
    for reg in (REG_LF, REG_L1):
        g, o = pair(p, reg, 0.3)
        gl, ol = g.loss(), o.loss()
        for k in ["sse", "xnorm2", "reg", "loss", "re"]:
            assert abs(gl[k] - ol[k]) <= 1e-12 * abs(ol[k]), (reg, k, gl[k], ol[k])


def keys_close(gk, ok, what):
    a = gk.detach().cpu().numpy()
    b = np.asarray(ok)
    assert np.array_equal(np.isinf(a), np.isinf(b)), what + ": +inf pattern"
    err = rel_err(a, b)
    assert err <= RTOL, "%s: element-wise rel err %.3e" % (what, err)


@pytest.mark.parametrize("reg", [REG_LF, REG_L1], ids=["LF", "L1"])
@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_responsibility_and_prune_match_oracle(shape, reg):
    dims, ranks, nnz, zipf = shape
    say("case", dims, ranks, nnz, reg)
    p = make(dims, ranks, nnz, 14, zipf)
    rng = np.random.default_rng(5)
    fmask = [(rng.random((d, r)) < 0.05).astype(np.uint8) for d, r in zip(dims, ranks)]
    cmask = (rng.random(ranks) < 0.1).astype(np.uint8)
    g, o = pair(p, reg, 0.05, fmask=fmask, cmask=cmask)
    g.iteration()
    o.iteration()
    assert_state(g, o, what="iteration")
    gck, gfk = g.responsibility()
    ock, ofk = o.responsibility()
    keys_close(gck, ock, "core keys")
    for n in range(len(dims)):
        keys_close(gfk[n], ofk[n], "factor keys %d" % n)
    ck = max(1, int(0.2 * (cmask == 0).sum()))
    fk = [max(1, int(0.1 * (m == 0).sum())) for m in fmask]
    g.prune(ck, fk)
    o.prune(ock, ofk, ck, fk)
    torch.cuda.synchronize()
    assert np.array_equal(g.cmask.cpu().numpy().astype(bool), o.cmask.astype(bool)), "core mask"
    for n, m in enumerate(g.factor_masks_bool()):
        assert np.array_equal(m.cpu().numpy(), o.fmask[n].astype(bool)), "factor mask %d" % n
    assert_state(g, o, what="after prune")
    g.iteration()
    o.iteration()
    assert_state(g, o, what="iteration after prune")


def test_planted_workload_ten_iterations_then_prune_to_half_core():
    # 100^3, 1e4 entries, core 5^3, L_F 0.01: 10 sweeps, responsibility,
    # ceil(0.5 * 125) = 63 core elements pruned, loss.
    p = synth.workload("planted-100^3-nnz1e4-r5")
    g, o = pair(p, p["reg"], p["lam"])
    for it in range(10):
        g.iteration()
        o.iteration()
    assert_state(g, o, what="10 iterations")
    gck, gfk = g.responsibility()
    ock, ofk = o.responsibility()
    keys_close(gck, ock, "core keys")
    g.prune(63, [0, 0, 0])
    o.prune(ock, ofk, 63, [0, 0, 0])
    torch.cuda.synchronize()
    assert np.array_equal(g.cmask.cpu().numpy().astype(bool), o.cmask.astype(bool))
    assert int(g.cmask.sum()) == 63
    gl, ol = g.loss(), o.loss()
    assert abs(gl["re"] - ol["re"]) <= RTOL * ol["re"]
    assert_state(g, o, what="final")


def test_long_rows_and_empty_rows():
    # mode-0 rows of ~4000 entries (> one 2048-entry chunk), many empty mode-1 rows
    p = make((3, 5000, 4), (3, 3, 3), 12_000, 15)
    g, o = pair(p, REG_LF, 0.02)
    st = [g.layout_stats(n) for n in range(3)]
    assert st[0]["long_rows"] == 3 and st[0]["long_chunks"] >= 6
    assert st[2]["long_rows"] == 4
    g.iteration()
    o.iteration()
    assert_state(g, o, what="iteration")
    gck, gfk = g.responsibility()
    ock, ofk = o.responsibility()
    keys_close(gck, ock, "core keys")
    for n in range(3):
        keys_close(gfk[n], ofk[n], "factor keys %d" % n)


def test_single_entry_and_tiny_dims():
    idx = np.array([[1, 0, 2]], np.int32)
    p = {"idx": idx, "val": np.array([0.7]), "factors": [np.full((2, 2), 0.5), np.full((1, 2), 0.3),
                                                         np.full((3, 2), 0.2)], "core": np.ones((2, 2, 2))}
    g, o = pair(p, REG_LF, 0.1)
    g.iteration()
    o.iteration()
    assert_state(g, o, what="single entry")


def test_results_are_deterministic():
    p = make((300, 200, 100), (10, 10, 10), 30_000, 16, (1.1, None, None))
    outs = []
    for _ in range(2):
        g, _o = pair(p, REG_LF, 0.05)
        g.iteration()
        g.responsibility()
        torch.cuda.synchronize()
        outs.append([f.cpu().numpy().copy() for f in g.factors] + [g.core.cpu().numpy().copy(),
                                                                    g.core_key.cpu().numpy().copy()])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_invalid_inputs_are_rejected_without_touching_state():
    v = V()
    p = make((20, 20, 20), (3, 3, 3), 500, 17)
    for what in ["dup", "range", "nan"]:
        idx, val = p["idx"].copy(), p["val"].copy()
        if what == "dup":
            idx[7] = idx[3]
        elif what == "range":
            idx[5, 1] = 20
        else:
            val[9] = np.nan
        fac = [torch.from_numpy(f.copy()).cuda() for f in p["factors"]]
        with pytest.raises(v.VestError) as ei:
            v.VestContext(idx, val, fac, p["core"])
        assert ei.value.code == v.EINVAL
    with pytest.raises(v.VestError) as ei:
        v.VestContext(p["idx"], p["val"], p["factors"], p["core"], lam=0.0)
    assert ei.value.code == v.EINVAL


def test_call_order_and_count_errors():
    v = V()
    p = make((20, 20, 20), (3, 3, 3), 500, 18)
    g, _ = pair(p, REG_LF, 0.1)
    with pytest.raises(v.VestError) as ei:
        g.prune(1, [0, 0, 0])
    assert ei.value.code == v.ESTATE
    g.responsibility()
    with pytest.raises(v.VestError) as ei:
        g.prune(28, [0, 0, 0])
    assert ei.value.code == v.EINVAL
    with pytest.raises(v.VestError) as ei:
        g.sweep_factor(3)
    assert ei.value.code == v.EINVAL


def test_fp32_form_rmse_within_1e4_of_oracle():
    p = synth.workload("planted-100^3-nnz1e4-r5")
    g, o = pair(p, p["reg"], p["lam"], precision=V().FP32)
    for _ in range(5):
        g.iteration()
        o.iteration()
    gl, ol = g.loss(), o.loss()
    gap = abs(gl["re"] - ol["re"]) / ol["re"]
    say("fp32 relative RMSE gap", gap, "factor rel err", rel_err(g.factors[0], o.factors[0]))
    assert gap <= 1e-4


@pytest.mark.parametrize("shape", [SHAPES[1], SHAPES[2], SHAPES[4]], ids=["N3J5", "N3J10", "N4J8"])
def test_keys_without_a_preceding_core_sweep(shape):
    # keys straight after init and after a factor sweep: the core keys cannot
    # reuse the Gram diagonals of a core sweep and take the full statistics path
    dims, ranks, nnz, zipf = shape
    p = make(dims, ranks, nnz, 19, zipf)
    g, o = pair(p, REG_LF, 0.05)
    for step in range(2):
        gck, gfk = g.responsibility()
        ock, ofk = o.responsibility()
        keys_close(gck, ock, "core keys, step %d" % step)
        for n in range(len(dims)):
            keys_close(gfk[n], ofk[n], "factor keys %d, step %d" % (n, step))
        g.sweep_factor(0)
        o.sweep_factor(0)
