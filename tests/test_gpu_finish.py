"""GPU checks of the output side: final normalisation (Alg. 2), sparse export,
held-out reconstruction error (a 90 / 10 split of Omega, Eq. 4 on the test
entries) and the value-pruning comparator, each against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle.oracle import REG_L1, REG_LF, Oracle
from test_gpu_parity import SHAPES, IDS, V, assert_state, make, pair, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [SHAPES[1], SHAPES[2], SHAPES[4], SHAPES[6]], ids=[IDS[1], IDS[2], IDS[4], IDS[6]])
def test_normalisation_matches_oracle_and_keeps_the_loss(shape):
    dims, ranks, nnz, zipf = shape
    p = make(dims, ranks, nnz, 81, zipf)
    g, o = pair(p, REG_L1, 0.3)
    for _ in range(2):
        g.iteration()
        o.iteration()
    before = g.loss()
    g.normalize()
    o.normalize()
    assert_state(g, o, what="normalised")
    after = g.loss()
    assert abs(after["sse"] - before["sse"]) <= 1e-10 * before["sse"]
    for f in g.factors:
        n = torch.linalg.vector_norm(f, dim=0).cpu().numpy()
        assert np.all((np.abs(n - 1.0) < 1e-12) | (n == 0.0))
    g.iteration()
    o.iteration()
    assert_state(g, o, what="iteration after normalisation")


def test_sparse_export_lists_the_nonzeros():
    p = make((200, 150, 100), (10, 10, 10), 20_000, 82)
    g, o = pair(p, REG_L1, 0.5)
    g.iteration()
    g.responsibility()
    g.prune(300, [400, 300, 200])
    torch.cuda.synchronize()
    cnt = g.count_nonzeros()
    fac, (ci, cv) = g.export()
    for n, f in enumerate(g.factors):
        d = f.cpu().numpy().ravel()
        nz = np.flatnonzero(d)
        assert cnt[n] == nz.size
        assert np.array_equal(fac[n][0].cpu().numpy(), nz)
        assert np.array_equal(fac[n][1].cpu().numpy(), d[nz])
    dc = g.core.cpu().numpy().ravel()
    nz = np.flatnonzero(dc)
    assert cnt[-1] == nz.size and np.array_equal(ci.cpu().numpy(), nz) and np.array_equal(cv.cpu().numpy(), dc[nz])


@pytest.mark.parametrize("prec", ["FP64", "FP32"])
def test_held_out_error_matches_oracle(prec):
    v = V()
    p = make((300, 200, 100), (5, 5, 5), 30_000, 83, (1.1, None, None))
    rng = np.random.default_rng(84)
    test = rng.random(p["idx"].shape[0]) < 0.1
    tr = dict(p, idx=p["idx"][~test], val=p["val"][~test])
    g, o = pair(tr, REG_LF, 0.05, precision=getattr(v, prec))
    for _ in range(3):
        g.iteration()
        o.iteration()
    ge = g.test_error(p["idx"][test], p["val"][test])
    ot = Oracle(p["idx"][test], p["val"][test], o.factors, o.core, reg=REG_LF, lam=0.05).loss()
    say(prec, "test RE gpu %.12f oracle %.12f" % (ge["re"], ot["re"]))
    bar = 1e-10 if prec == "FP64" else 1e-5
    assert abs(ge["sse"] - ot["sse"]) <= bar * ot["sse"]
    assert abs(ge["xnorm2"] - ot["xnorm2"]) <= 1e-12 * ot["xnorm2"]
    bad = p["idx"][test][:5].copy()
    bad[2, 1] = 10_000
    with pytest.raises(v.VestError) as ei:
        g.test_error(bad, p["val"][test][:5])
    assert ei.value.code == v.EINVAL


def test_value_pruning_comparator_prunes_smallest_magnitudes():
    p = make((100, 80, 60), (5, 5, 5), 5000, 85)
    g, o = pair(p, REG_LF, 0.05)
    ck, fk = g.value_keys()
    torch.cuda.synchronize()
    oc = np.abs(o.core)
    of = [np.abs(f) for f in o.factors]
    g.prune(40, [50, 40, 30])
    o.prune(oc, of, 40, [50, 40, 30])
    torch.cuda.synchronize()
    assert np.array_equal(g.cmask.cpu().numpy().astype(bool), o.cmask.astype(bool))
    for n, m in enumerate(g.factor_masks_bool()):
        assert np.array_equal(m.cpu().numpy(), o.fmask[n].astype(bool))
    g.iteration()
    o.iteration()
    assert_state(g, o, what="after value pruning")
