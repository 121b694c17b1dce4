"""GPU parity for the rank range 2..10 at orders 3 and 4 and for unequal
per-mode ranks J_n (Table 1 gives every mode its own rank; the MovieLens
model of the paper's Table 2 is 6 x 6 x 2 x 2).

A context with unequal ranks runs the kernels of its largest rank on a
padded copy of the model in which every element outside the caller's
J_1 x .. x J_N model is marked (zero, never updated), and copies the caller's
part back after every call; the oracle runs the unequal-rank model directly.
Same FP64 bar as test_gpu_parity: element-wise 1e-10 relative above a floor
of 1e-4 of each tensor's largest magnitude, keys too, masks identical.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import REG_L1, REG_LF, Oracle
from test_gpu_parity import RTOL, V, assert_state, keys_close, make, pair, rel_err, say

pytestmark = pytest.mark.gpu

CASES = [
    # dims, ranks, nnz
    ((120, 100, 80), (7, 7, 7), 12_000),
    ((150, 120, 100), (9, 9, 9), 15_000),
    ((40, 30, 20, 24), (7, 7, 7, 7), 6000),
    ((30, 25, 20, 24), (9, 9, 9, 9), 5000),
    ((25, 20, 16, 24), (10, 10, 10, 10), 4000),
    ((100, 80, 60), (3, 5, 4), 8000),
    ((60, 50, 20, 24), (6, 6, 2, 2), 8000),
    ((80, 60, 40, 24), (4, 7, 5, 3), 8000),
    ((90, 70, 50), (10, 4, 7), 9000),
]
IDS = ["N3J7", "N3J9", "N4J7", "N4J9", "N4J10", "N3J354", "N4J6622", "N4J4753", "N3J1047"]


def masks_equal(g, o, what):
    torch.cuda.synchronize()
    assert np.array_equal(g.cmask.cpu().numpy().astype(bool), o.cmask.astype(bool)), what + ": core mask"
    for n, m in enumerate(g.factor_masks_bool()):
        assert np.array_equal(m.cpu().numpy(), o.fmask[n].astype(bool)), what + ": factor mask %d" % n


@pytest.mark.parametrize("reg", [REG_LF, REG_L1], ids=["LF", "L1"])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_ranks_iteration_keys_prune(case, reg):
    """Where the core has at least as many elements as there are entries
    (order 4 at ranks 9 and 10 here) the core sweep solves an underdetermined
    system and amplifies rounding-order differences from one step to the next
    (as at order 10, test_gpu_orders); there every step starts from the
    oracle's state, so the element-wise bar applies to each step."""
    from test_gpu_orders import resync
    dims, ranks, nnz = case
    stepwise = int(np.prod(ranks)) >= nnz
    say("case", dims, ranks, nnz, reg, "stepwise" if stepwise else "")
    p = make(dims, ranks, nnz, 101)
    rng = np.random.default_rng(102)
    fmask = [(rng.random((d, r)) < 0.05).astype(np.uint8) for d, r in zip(dims, ranks)]
    cmask = (rng.random(ranks) < 0.1).astype(np.uint8)
    lam = 0.05 if reg == REG_LF else 0.3
    g, o = pair(p, reg, lam, fmask=fmask, cmask=cmask)
    for it in range(2):
        if stepwise and it > 0:
            g = resync(o, reg, lam, p)
        g.iteration()
        o.iteration()
        assert_state(g, o, what="iteration %d" % it)
    gl, ol = g.loss(), o.loss()
    for k in ["sse", "xnorm2", "reg", "loss", "re"]:
        assert abs(gl[k] - ol[k]) <= RTOL * abs(ol[k]) + 1e-300, (k, gl[k], ol[k])
    gck, gfk = g.responsibility()
    ock, ofk = o.responsibility()
    keys_close(gck, ock, "core keys")
    for n in range(len(dims)):
        keys_close(gfk[n], ofk[n], "factor keys %d" % n)
    ck = max(1, int(0.2 * (o.cmask == 0).sum()))
    fk = [max(1, int(0.1 * (m == 0).sum())) for m in o.fmask]
    g.prune(ck, fk)
    o.prune(ock, ofk, ck, fk)
    masks_equal(g, o, "after prune")
    assert_state(g, o, what="after prune")
    if stepwise:
        g = resync(o, reg, lam, p)
    g.iteration()
    o.iteration()
    assert_state(g, o, what="iteration after prune")


@pytest.mark.parametrize("kernel", ["DENSE", "GATHER"])
def test_unequal_ranks_both_contraction_forms(kernel):
    v = V()
    dims, ranks = (70, 60, 30, 24), (6, 6, 2, 2)
    p = make(dims, ranks, 7000, 103)
    g, o = pair(p, REG_LF, 0.05)
    g.set_kernel(getattr(v, "KERNEL_" + kernel))
    for it in range(2):
        g.iteration()
        o.iteration()
        assert_state(g, o, what="%s iteration %d" % (kernel, it))


def test_unequal_ranks_output_side():
    """Normalisation, sparse export (caller's flat order), nonzero counts,
    held-out error and value pruning of an unequal-rank context."""
    v = V()
    dims, ranks = (80, 60, 50), (5, 3, 4)
    p = make(dims, ranks, 8000, 104)
    rng = np.random.default_rng(105)
    test = rng.random(p["idx"].shape[0]) < 0.1
    tr = dict(p, idx=p["idx"][~test], val=p["val"][~test])
    g, o = pair(tr, REG_LF, 0.05)
    g.iteration()
    o.iteration()
    ge = g.test_error(p["idx"][test], p["val"][test])
    ot = Oracle(p["idx"][test], p["val"][test], o.factors, o.core, reg=REG_LF, lam=0.05).loss()
    assert abs(ge["sse"] - ot["sse"]) <= RTOL * ot["sse"]
    ck, fk = g.value_keys()
    g.prune(6, [40, 20, 30])
    o.prune(np.abs(o.core), [np.abs(f) for f in o.factors], 6, [40, 20, 30])
    masks_equal(g, o, "value pruning")
    g.normalize()
    o.normalize()
    assert_state(g, o, what="normalised")
    cnt = g.count_nonzeros()
    assert cnt == [int((f != 0).sum()) for f in o.factors] + [int((o.core != 0).sum())]
    (fac, (ci, cv)) = g.export()
    for n in range(3):
        fi, fv = fac[n]
        flat = o.factors[n].ravel()
        nz = np.flatnonzero(flat)
        assert np.array_equal(fi.cpu().numpy(), nz)
        assert rel_err(fv, flat[nz]) <= RTOL
    nz = np.flatnonzero(o.core.ravel())
    assert np.array_equal(ci.cpu().numpy(), nz)
    assert rel_err(cv, o.core.ravel()[nz]) <= RTOL


def test_unequal_ranks_fp32_form():
    v = V()
    dims, ranks = (100, 80, 60), (6, 4, 5)
    p = make(dims, ranks, 10_000, 106)
    g, o = pair(p, REG_LF, 0.01, precision=v.FP32)
    for _ in range(5):
        g.iteration()
        o.iteration()
    gl, ol = g.loss(), o.loss()
    gap = abs(gl["re"] - ol["re"]) / ol["re"]
    say("unequal-rank FP32 RE gap %.2e" % gap)
    assert gap <= 1e-4
