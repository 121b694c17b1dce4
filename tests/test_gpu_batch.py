"""GPU checks of vest_iterate_many: one Alg. 2 iteration of several contexts
of one shape in one sequence of launches (the batched path of the request
loop).

* Every context's result after batched iterations equals the same context
  run alone through vest_sweep_factor / vest_sweep_core (the batched kernels
  run the same per-context arithmetic), bit for bit, for the FP64, FP32 and
  split-BF16 forms at orders 3 and 4, with long rows and Zipf skew.
* FP64 batched iterations against the oracle at the FP64 bar of
  test_gpu_parity.
* Contexts that do not fit the batched path (different shapes, unequal
  ranks, marks that select the gather contraction) are refused with
  EUNSUPPORTED and nothing is enqueued.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_1904_02603_amd import synth
from test_gpu_parity import V, assert_state, say

pytestmark = pytest.mark.gpu

CASES = [
    # dims, rank, nnz, zipf, precision, reg
    ((100, 80, 60), 5, 5000, None, "FP64", 0),
    ((300, 200, 100), 10, 30_000, None, "BF16", 1),
    ((3, 5000, 4), 3, 12_000, None, "FP32", 0),           # rows longer than one chunk
    ((2000, 300, 50), 4, 30_000, (1.1, 1.0, None), "FP64", 1),
    ((30, 25, 20, 24), 8, 5000, None, "FP32", 0),
    ((40, 30, 20, 24), 7, 6000, None, "FP64", 1),
]
IDS = ["N3J5f64", "N3J10bf16", "longN3J3f32", "zipfN3J4f64", "N4J8f32", "N4J7f64"]


def contexts(case, k, seeds):
    v = V()
    dims, J, nnz, zipf, prec, reg = case
    lam = 0.05 if reg == 0 else 0.5
    out = []
    for s in seeds:
        p = synth.make_problem(dims, nnz, (J,) * len(dims), 200 + 10 * k + s, zipf=zipf, noise_var=0.01)
        out.append((p, v.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam,
                                     precision=getattr(v, prec))))
    return out, reg, lam


@pytest.mark.parametrize("k", range(len(CASES)), ids=IDS)
def test_batched_iterations_equal_contexts_alone(k):
    v = V()
    case = CASES[k]
    batch = v.Batch()
    seeds = [0, 1, 2]
    bat, reg, lam = contexts(case, k, seeds)
    solo, _, _ = contexts(case, k, seeds)
    for it in range(3):
        assert batch.iterate([c for _, c in bat]) == v.OK
        for _, c in solo:
            c.iteration()
    torch.cuda.synchronize()
    for (p, b), (_, a) in zip(bat, solo):
        for n in range(len(case[0])):
            assert torch.equal(b.factors[n], a.factors[n]), ("factor", n)
        assert torch.equal(b.core, a.core)
        lb, la = b.loss(), a.loss()
        assert lb["loss"] == la["loss"] and lb["re"] == la["re"]
    say("batched == alone for", len(seeds), "contexts")


def test_batched_fp64_matches_oracle():
    v = V()
    case = ((150, 120, 90), 6, 12_000, (1.1, None, None), "FP64", 0)
    bat, reg, lam = contexts(case, 9, [0, 1])
    orcs = [Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam) for p, _ in bat]
    batch = v.Batch()
    for it in range(2):
        assert batch.iterate([c for _, c in bat]) == v.OK
        for o in orcs:
            o.iteration()
    for (p, c), o in zip(bat, orcs):
        assert_state(c, o, what="batched iterations")


def test_batch_refuses_what_does_not_fit():
    v = V()
    batch = v.Batch()
    a, _, _ = contexts(CASES[0], 0, [0])
    b, _, _ = contexts(CASES[5], 5, [0])
    before = [f.clone() for f in a[0][1].factors]
    assert batch.iterate([a[0][1], b[0][1]]) == v.EUNSUPPORTED         # two shapes
    p = synth.make_problem((50, 40, 30), 3000, (4, 3, 5), 7, noise_var=0.01)
    pad = v.VestContext(p["idx"], p["val"], p["factors"], p["core"])
    assert batch.iterate([pad]) == v.EUNSUPPORTED                       # unequal ranks
    g = a[0][1]
    g.set_kernel(v.KERNEL_GATHER)
    assert batch.iterate([g]) == v.EUNSUPPORTED                         # gather contraction
    torch.cuda.synchronize()
    for f0, f in zip(before, g.factors):
        assert torch.equal(f0, f)                                       # nothing ran
