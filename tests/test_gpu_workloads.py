"""GPU parity at the shapes of the benchmark workloads.

* Full size, 10^7 entries over (10^5)^3, ranks 10 (the configuration the
  benchmark times), launched exactly as the benchmark launches it: one sweep
  of mode 0 from the seeded initial state; the oracle recomputes sampled rows
  one by one (Alg. 4 rows are independent given the other modes), FP64 rows
  element-wise within 1e-10 (above a floor of 1e-4 of the largest), FP32 and
  split-BF16 rows within 1e-4 relative RMSE.
* Rating-shaped Zipf tensor at its full dimensions (500k x 20k x 2k, values
  1..5, L_1 lambda 0.1, ranks 10) with 2e6 entries: the same sampled-row check
  of the first mode-0 sweep in the three forms, the Zipf head row included.
* The same tensor scaled down to 5000 x 2000 x 200, 2e5 entries: two full
  iterations FP64 against the oracle at the FP64 bar, FP32 and split-BF16
  within 1e-4 relative RE and factor RMSE.
* Order-4 Zipf tensor (the 50k x 50k x 1000 x 24 workload scaled down to
  300 x 300 x 40 x 24, 2e4 entries, ranks 8): iterations with responsibility
  and prune steps up to 85 % marked, FP64, masks identical after every prune.
* 1.2e6 entries over 300 x 200 x 2000 (Zipf last mode, rows up to ~6e4
  entries, ranks 5): large enough that the core keys run on the context's
  second stream beside the factor keys, long rows in every mode; keys,
  masks and the next iteration against the oracle.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import REG_L1, Oracle
from paper_1904_02603_amd import synth
from test_gpu_parity import V, assert_state, keys_close, make, pair, rel_err, rms_err, say

pytestmark = pytest.mark.gpu


def test_full_size_mode0_sweep_sampled_rows():
    v = V()
    p = synth.workload("planted-1e5^3-nnz1e7-r10")
    o = Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"])
    counts = np.bincount(p["idx"][:, 0], minlength=p["factors"][0].shape[0])
    rng = np.random.default_rng(3)
    rows = sorted(set(rng.choice(len(counts), 48, replace=False).tolist()
                      + [int(counts.argmax()), int(counts.argmin())]))
    for i in rows:
        o.update_row(0, i)
    ref = o.factors[0][rows]
    say("rows", len(rows), "lengths", int(counts[rows].min()), "..", int(counts[rows].max()))
    check_rows_three_forms(p, rows, ref)


def check_rows_three_forms(p, rows, ref):
    v = V()
    for prec in ("FP64", "FP32", "BF16"):
        g = v.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                          precision=getattr(v, prec))
        g.sweep_factor(0)
        torch.cuda.synchronize()
        got = g.factors[0].cpu().numpy()[rows]
        ew, rm = rel_err(got, ref), rms_err(got, ref)
        say(prec, "sampled rows: element-wise rel err %.3e, rel RMSE %.3e" % (ew, rm))
        if prec == "FP64":
            assert ew <= 1e-10, (prec, ew)
        else:
            assert rm <= 1e-4, (prec, rm)
        g.close()


def test_rating_shaped_zipf_full_dims_mode0_rows():
    p = synth.workload("rating-zipf-500k.20k.2k-nnz1e8-r10", nnz=2_000_000)
    o = Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"])
    counts = np.bincount(p["idx"][:, 0], minlength=p["factors"][0].shape[0])
    rng = np.random.default_rng(4)
    busy = np.flatnonzero((counts > 0) & (counts <= 4000))
    rows = sorted(set(rng.choice(busy, 48, replace=False).tolist() + [int(counts.argmax())]))
    for i in rows:
        o.update_row(0, i)
    say("rows", len(rows), "lengths", int(counts[rows].min()), "..", int(counts[rows].max()))
    check_rows_three_forms(p, rows, o.factors[0][rows])


def test_rating_shaped_zipf_tensor_l1_two_iterations():
    p = synth.make_problem((5000, 2000, 200), 200_000, (10, 10, 10), 71, zipf=(1.1, 1.0, None), rating=True)
    g, o = pair(p, REG_L1, 0.1)
    for it in range(2):
        g.iteration()
        o.iteration()
        assert_state(g, o, what="iteration %d" % it)
    gl, ol = g.loss(), o.loss()
    assert abs(gl["re"] - ol["re"]) <= 1e-10 * ol["re"]


@pytest.mark.parametrize("prec", ["FP32", "BF16"])
def test_rating_shaped_zipf_tensor_reduced_forms(prec):
    v = V()
    p = synth.make_problem((5000, 2000, 200), 200_000, (10, 10, 10), 71, zipf=(1.1, 1.0, None), rating=True)
    g, o = pair(p, REG_L1, 0.1, precision=getattr(v, prec))
    for it in range(2):
        g.iteration()
        o.iteration()
    gl, ol = g.loss(), o.loss()
    gap = abs(gl["re"] - ol["re"]) / ol["re"]
    torch.cuda.synchronize()
    fr = max(rms_err(f.cpu().numpy(), of) for f, of in zip(g.factors, o.factors))
    say(prec, "RE gap %.2e, factor rel RMSE %.2e" % (gap, fr))
    assert gap <= 1e-4 and fr <= 1e-4


def test_order4_zipf_tensor_pruned_to_85_percent():
    p = make((300, 300, 40, 24), (8, 8, 8, 8), 20_000, 72, (1.1, 1.0, None, None))
    g, o = pair(p, 0, 0.01)
    sizes = [f.size for f in p["factors"]]
    marked_c, marked_f = 0, [0] * 4
    for t, frac in enumerate([0.3, 0.6, 0.85]):
        g.iteration()
        o.iteration()
        assert_state(g, o, what="iteration %d" % t)
        gck, gfk = g.responsibility()
        ock, ofk = o.responsibility()
        keys_close(gck, ock, "core keys %d" % t)
        for n in range(4):
            keys_close(gfk[n], ofk[n], "factor keys %d/%d" % (n, t))
        kc = int(frac * 4096) - marked_c
        kf = [int(frac * s) - m for s, m in zip(sizes, marked_f)]
        g.prune(kc, kf)
        o.prune(ock, ofk, kc, kf)
        marked_c += kc
        marked_f = [m + k for m, k in zip(marked_f, kf)]
        torch.cuda.synchronize()
        assert np.array_equal(g.cmask.cpu().numpy().astype(bool), o.cmask.astype(bool))
        for n, m in enumerate(g.factor_masks_bool()):
            assert np.array_equal(m.cpu().numpy(), o.fmask[n].astype(bool)), (t, n)
    g.iteration()
    o.iteration()
    assert_state(g, o, what="after pruning")


def test_keys_on_two_streams_with_long_rows_match_oracle():
    p = synth.make_problem((300, 200, 2000), 1_200_000, (5, 5, 5), 93, zipf=(None, None, 1.1), noise_var=0.01)
    g, o = pair(p, REG_L1, 0.3)
    g.iteration()
    o.iteration()
    assert_state(g, o, what="iteration")
    gck, gfk = g.responsibility()
    ock, ofk = o.responsibility()
    keys_close(gck, ock, "core keys")
    for n in range(3):
        keys_close(gfk[n], ofk[n], "factor keys %d" % n)
    kc, kf = 40, [450, 300, 3000]
    g.prune(kc, kf)
    o.prune(ock, ofk, kc, kf)
    torch.cuda.synchronize()
    assert np.array_equal(g.cmask.cpu().numpy().astype(bool), o.cmask.astype(bool))
    for n, m in enumerate(g.factor_masks_bool()):
        assert np.array_equal(m.cpu().numpy(), o.fmask[n].astype(bool)), n
    g.iteration()
    o.iteration()
    assert_state(g, o, what="after pruning")
