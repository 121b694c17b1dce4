"""Slab-pass timing instrumentation (vest_slab_timing / vest_slab_time).

Each core sweep runs J^(N-2) slab passes, the first of them inside the
residual pass when that pass has to run (the first core sweep after init or
after the factors changed); with timing enabled each separate slab pass is
bracketed by events, the query returns their count and a positive duration
and clears the record; disabled, nothing is recorded.  Results are unchanged
by the instrumentation.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import REG_LF
from test_gpu_parity import V, assert_state, make, pair, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [((60, 50, 40), (5, 5, 5)), ((20, 18, 16, 12), (4, 4, 4, 4))], ids=["N3J5", "N4J4"])
def test_slab_passes_are_timed_and_results_unchanged(shape):
    dims, ranks = shape
    p = make(dims, ranks, 3000, 61)
    g, o = pair(p, REG_LF, 0.05)
    nslab = ranks[0] ** (len(dims) - 2)
    g.slab_timing(True)
    for it in range(2):
        g.sweep_core()
        o.sweep_core()
    ms, n = g.slab_time()
    say("slab passes", n, "total ms %.4f" % ms)
    # first sweep: residual formed with the first slab's sums; second: residual current
    assert n == 2 * nslab - 1
    assert ms > 0.0
    assert g.slab_time() == (0.0, 0)
    assert_state(g, o, what="timed core sweeps")
    g.slab_timing(False)
    g.sweep_core()
    assert g.slab_time() == (0.0, 0)
    torch.cuda.synchronize()
