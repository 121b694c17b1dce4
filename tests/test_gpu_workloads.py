"""GPU parity at the shapes of the benchmark workloads.

* Full size, 10^7 entries over (10^5)^3, ranks 10 (the configuration the
  benchmark times), launched exactly as the benchmark launches it: one sweep
  of mode 0 from the seeded initial state; the oracle recomputes sampled rows
  one by one (Alg. 4 rows are independent given the other modes), FP64 rows
  within 1e-10, FP32 and split-BF16 rows within 1e-4.
* Rating-shaped Zipf tensor (the 500k x 20k x 2k workload scaled down to
  5000 x 2000 x 200, 2e5 entries, values 1..5, L_1 lambda 0.1, ranks 10): two
  full iterations FP64 against the oracle.
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
from test_gpu_parity import V, assert_state, keys_close, make, pair, say

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
    for prec, bar in [("FP64", 1e-10), ("FP32", 1e-4), ("BF16", 1e-4)]:
        g = v.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                          precision=getattr(v, prec))
        g.sweep_factor(0)
        torch.cuda.synchronize()
        got = g.factors[0].cpu().numpy()[rows]
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
        say(prec, "sampled-row rel err %.3e" % err)
        assert err <= bar, (prec, err)
        g.close()


def test_rating_shaped_zipf_tensor_l1_two_iterations():
    p = synth.make_problem((5000, 2000, 200), 200_000, (10, 10, 10), 71, zipf=(1.1, 1.0, None), rating=True)
    g, o = pair(p, REG_L1, 0.1)
    for it in range(2):
        g.iteration()
        o.iteration()
        assert_state(g, o, what="iteration %d" % it)
    gl, ol = g.loss(), o.loss()
    assert abs(gl["re"] - ol["re"]) <= 1e-10 * ol["re"]


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
