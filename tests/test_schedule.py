"""The product's host schedule against the oracle's and hand-computed values."""
import numpy as np
import pytest

from oracle import schedule as OS
from paper_1904_02603_amd.schedule import PruneSchedule


@pytest.mark.parametrize("t", [1, 2, 3, 7, 10, 11, 40])
def test_rate_matches(t):
    assert PruneSchedule().rate(t) == pytest.approx(OS.pruning_rate(t))


@pytest.mark.parametrize("size,target", [(125, 0.5), (4096, 0.95), (1000, 0.3), (7, 0.9)])
def test_counts_match_oracle_over_a_run(size, target):
    p = PruneSchedule(mode="manual", target=target)
    o = OS.ManualSchedule(target)
    mp = mo = 0
    for t in range(1, 40):
        kp = p.count(t, size, mp)
        ko = o.counts(t, [size], [mo])[0]
        assert kp == ko
        mp += kp
        mo += ko
    assert mp == int(np.ceil(target * size))


def test_elbow_decisions_match_oracle():
    rng = np.random.default_rng(3)
    for trial in range(50):
        re = list(np.cumsum(rng.random(12) * 0.02) + 0.1)
        if trial % 3 == 0:
            re[6:] = [r + 0.3 for r in re[6:]]
        p = PruneSchedule(mode="auto")
        o = OS.AutoSchedule()
        for t in range(1, len(re) + 1):
            assert p.should_prune(t, re[:t], 0.0) == o.should_prune(t, re[:t], 0.0)
