"""Pins of the oracle's pruning schedule (Alg. 2 pruning rate, Sec. 3.3)."""
import numpy as np
import pytest

from oracle import schedule as S


def test_rate_ramp_defaults():
    assert [S.pruning_rate(t) for t in (1, 2, 5, 10, 11, 50)] == pytest.approx(
        [0.01, 0.02, 0.05, 0.1, 0.1, 0.1])


def test_single_step_to_half_core_sparsity():
    # 5x5x5 core pruned to at least 50% in one step: ceil(0.5 * 125) = 63
    assert S.prune_count(0.5, 125, 0, target=0.5) == 63
    assert S.prune_count(0.5, 125, 63, target=0.5) == 0


def test_ramp_reaches_95_percent_in_14_steps():
    size, marked, steps = 4096, 0, 0
    sched = S.ManualSchedule(0.95)
    t = 0
    while marked < int(np.ceil(0.95 * size)):
        t += 1
        marked += sched.counts(t, [size], [marked])[0]
        steps += 1
    assert steps == 14


def test_manual_stop_uses_zero_count_sparsity():
    sched = S.ManualSchedule(0.5)
    a = np.array([0.0, 1.0, 0.0, 2.0])
    assert sched.should_prune(3, [], S.sparsity([a])) is False
    assert sched.should_prune(3, [], S.sparsity([a, np.ones(2)])) is True


def test_auto_elbow_fires_once_and_stays_off():
    sched = S.AutoSchedule()
    # flat RE, then a jump: second difference / pr at t=4 is (0.5+0.1-0.2)/0.04 = 10
    hist = [0.10, 0.10]
    assert sched.should_prune(2, hist, 0.0) is True          # needs 3 points
    hist.append(0.10)
    assert sched.should_prune(3, hist, 0.1) is True           # elbow 0
    hist.append(0.5)
    assert sched.should_prune(4, hist, 0.2) is False
    hist.append(0.5)
    assert sched.should_prune(5, hist, 0.2) is False          # stays stopped


def test_elbow_formula_value():
    assert S.elbow([0.2, 0.25, 0.4], 0.05) == pytest.approx((0.4 + 0.2 - 0.5) / 0.05)
    assert S.elbow([0.2, 0.25], 0.05) is None
    assert S.elbow([0.2, 0.25, 0.3], 0.0) is None


def test_elbow_ignores_the_convex_decrease_of_early_iterations():
    # from a random start the RE falls fast, then slowly: the second
    # difference is large and positive, but the curve is not rising, so this
    # is not the elbow where the RE shoots up (Sec. 3.1, 3.3)
    hist = [0.9, 0.6, 0.5]
    assert (hist[2] + hist[0] - 2 * hist[1]) / 0.03 > 0.05
    assert S.elbow(hist, 0.03) is None
    sched = S.AutoSchedule()
    assert sched.should_prune(3, hist, 0.0) is True
    # a rise that accelerates fires it
    assert S.elbow([0.30, 0.301, 0.33], 0.05) == pytest.approx((0.33 + 0.30 - 0.602) / 0.05)
    assert sched.should_prune(4, [0.9, 0.6, 0.5, 0.30, 0.301, 0.33], 0.1) is False
