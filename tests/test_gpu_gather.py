"""GPU parity of the pruned-phase gather contraction against the FP64 oracle.

The gather form (vest_set_kernel(VEST_KERNEL_GATHER)) evaluates Eq. 11 over
the nonzero factor values and nonzero core columns only; it must reproduce the
oracle's full sums to the FP64 bar (1e-10 element-wise relative above a floor, keys too, masks
identical) at any sparsity, including none.  Random marking tables of 0, 60
and 95 % are planted on core and factors (marked elements are zero, Sec. 3.3).
"""
import numpy as np
import pytest
import torch

from oracle.oracle import REG_L1, REG_LF
from test_gpu_parity import IDS, SHAPES, V, assert_state, keys_close, make, pair, rel_err, say

pytestmark = pytest.mark.gpu


def planted_masks(p, frac, seed):
    rng = np.random.default_rng(seed)
    fmask = [rng.random(f.shape) < frac for f in p["factors"]]
    cmask = rng.random(p["core"].shape) < frac
    return fmask, cmask


@pytest.mark.parametrize("frac", [0.0, 0.6, 0.95], ids=["dense", "p60", "p95"])
@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_gather_iteration_and_keys_match_oracle(shape, frac):
    dims, ranks, nnz, zipf = shape
    say("case", dims, ranks, nnz, frac)
    p = make(dims, ranks, nnz, 41, zipf)
    fmask, cmask = planted_masks(p, frac, 42)
    g, o = pair(p, REG_LF, 0.05, fmask=fmask, cmask=cmask)
    g.set_kernel(V().KERNEL_GATHER)
    for it in range(2):
        g.iteration()
        o.iteration()
        assert_state(g, o, what="iteration %d" % it)
    gck, gfk = g.responsibility()
    ock, ofk = o.responsibility()
    keys_close(gck, ock, "core keys")
    for n in range(len(dims)):
        keys_close(gfk[n], ofk[n], "factor keys %d" % n)


@pytest.mark.parametrize("shape", [SHAPES[2], SHAPES[4], SHAPES[6]], ids=[IDS[2], IDS[4], IDS[6]])
def test_gather_l1_and_auto_policy_match_oracle(shape):
    dims, ranks, nnz, zipf = shape
    p = make(dims, ranks, nnz, 43, zipf)
    fmask, cmask = planted_masks(p, 0.9, 44)
    for policy in ["KERNEL_GATHER", "KERNEL_AUTO"]:
        g, o = pair(p, REG_L1, 0.5, fmask=fmask, cmask=cmask)
        g.set_kernel(getattr(V(), policy))
        g.iteration()
        o.iteration()
        assert_state(g, o, what=policy)


@pytest.mark.parametrize("prec", ["FP32", "BF16"])
def test_gather_low_precision_forms_track_oracle(prec):
    # pruned phase of the low-precision forms: FP32 gather contraction
    p = make((200, 150, 100), (10, 10, 10), 20_000, 45)
    fmask, cmask = planted_masks(p, 0.95, 46)
    g, o = pair(p, REG_LF, 0.05, precision=getattr(V(), prec), fmask=fmask, cmask=cmask)
    g.set_kernel(V().KERNEL_GATHER)
    for n in range(3):
        g.sweep_factor(n)
        o.sweep_factor(n)
    gl, ol = g.loss(), o.loss()
    gap = abs(gl["loss"] - ol["loss"]) / ol["loss"]
    say("%s gather loss gap %.3e" % (prec, gap))
    assert gap <= 1e-7


def test_bad_kernel_policy_is_rejected():
    v = V()
    p = make((20, 20, 20), (3, 3, 3), 500, 47)
    g, _ = pair(p, REG_LF, 0.1)
    with pytest.raises(v.VestError) as ei:
        g.set_kernel(7)
    assert ei.value.code == v.EINVAL
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape", [SHAPES[1], SHAPES[2], SHAPES[4], SHAPES[6]], ids=[IDS[1], IDS[2], IDS[4], IDS[6]])
def test_compaction_keeps_every_result(shape):
    # entries with a fully marked row are dropped; the loss right after, and
    # the following iteration, keys and prune, equal the oracle's on the full set
    dims, ranks, nnz, zipf = shape
    p = make(dims, ranks, nnz, 48, zipf)
    fmask, cmask = planted_masks(p, 0.85, 49)
    g, o = pair(p, REG_LF, 0.05, fmask=fmask, cmask=cmask)
    before = g.loss()
    live = g.compact()
    after = g.loss()
    say("kept", live, "of", nnz)
    assert 0 < live < nnz
    assert g.layout_stats(0)["nnz"] == live
    assert abs(after["loss"] - before["loss"]) <= 1e-12 * before["loss"]
    ol = o.loss()
    assert abs(after["sse"] - ol["sse"]) <= 1e-10 * ol["sse"]
    for it in range(2):
        g.iteration()
        o.iteration()
        assert_state(g, o, what="compacted iteration %d" % it)
    gck, gfk = g.responsibility()
    ock, ofk = o.responsibility()
    keys_close(gck, ock, "core keys")
    for n in range(len(dims)):
        keys_close(gfk[n], ofk[n], "factor keys %d" % n)
    kc = int(0.05 * p["core"].size)
    kf = [int(0.05 * f.size) for f in p["factors"]]
    g.prune(kc, kf)
    o.prune(ock, ofk, kc, kf)
    live2 = g.compact()
    assert live2 <= live
    g.iteration()
    o.iteration()
    assert_state(g, o, what="after second compaction")
    gl, ol = g.loss(), o.loss()
    assert abs(gl["re"] - ol["re"]) <= 1e-10 * ol["re"]


def test_compaction_in_the_fp32_form():
    p = make((200, 150, 100), (10, 10, 10), 20_000, 50)
    fmask, cmask = planted_masks(p, 0.9, 51)
    g, o = pair(p, REG_LF, 0.05, precision=V().FP32, fmask=fmask, cmask=cmask)
    g.compact()
    g.iteration()
    o.iteration()
    gl, ol = g.loss(), o.loss()
    assert abs(gl["loss"] - ol["loss"]) / ol["loss"] <= 1e-6


def test_schedule_loop_with_and_without_compaction_agree():
    from paper_1904_02603_amd.schedule import PruneSchedule, run
    v = V()
    p = make((200, 150, 100), (5, 5, 5), 20_000, 52)
    hist = []
    ctxs = []
    for every in (0, 2):
        g = v.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=REG_LF, lam=0.05)
        sched = PruneSchedule(mode="manual", target=0.9, init_pr=0.1, max_pr=0.3)
        hist.append(run(g, 10, sched, compact_every=every))
        ctxs.append(g)
    say("RE", hist[0][-1], hist[1][-1], "kept", ctxs[1].layout_stats(0)["nnz"])
    assert ctxs[1].layout_stats(0)["nnz"] < p["idx"].shape[0]
    for a, b in zip(*hist):
        assert abs(a - b) <= 1e-10 * abs(a)
    for n in range(3):
        assert rel_err(ctxs[1].factors[n], ctxs[0].factors[n]) <= 1e-10
