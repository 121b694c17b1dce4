"""Pruning schedule of VeST written for the oracle (Sec. 3.1 Alg. 2, Sec. 3.3).

TEST INFRASTRUCTURE ONLY (see ``oracle.py``).

Readings taken here:
  * iterations are counted t = 1, 2, ... and the pruning rate of iteration t is
    pr_t = min(INIT_PR * t, MAX_PR) (pruning step of Alg. 2; defaults 0.01 / 0.1
    from Sec. 3.3);
  * a tensor T of |T| elements loses ceil(pr_t |T|) new elements per prune
    step, chosen among its unmarked ones; in the manual form the cumulative
    number of marks of T never exceeds ceil(s |T|) and pruning stops once the
    total sparsity reaches the target s (a lower bound on the final sparsity);
  * the automatic form stops pruning for good the first time the elbow
    estimate (RE_t + RE_{t-2} - 2 RE_{t-1}) / pr_t exceeds 0.05 while the RE
    curve is rising (RE_t > RE_{t-1}): the rule is meant to find the point
    where the RE starts to shoot up (Sec. 3.1 overview, Sec. 3.3), and the
    convex decrease of the first iterations from a random start would
    otherwise stop pruning at t = 3; it is only evaluated when RE_{t-2}
    exists and pr_t > 0;
  * sparsity = (number of zero values) / (|G| + sum_n |A^(n)|)  (Sec. 4.2
    prints the complementary ratio under that name).
"""
import math

INIT_PR = 0.01
MAX_PR = 0.1
ELBOW = 0.05


def pruning_rate(t, init_pr=INIT_PR, max_pr=MAX_PR):
    return min(init_pr * t, max_pr)


def prune_count(pr, size, marked, target=None):
    """Number of new elements to prune in one tensor of ``size`` elements."""
    k = int(math.ceil(pr * size - 1e-12))
    k = min(k, size - marked)
    if target is not None:
        k = min(k, max(0, int(math.ceil(target * size - 1e-12)) - marked))
    return max(k, 0)


def sparsity(arrays):
    zeros = sum(int((a == 0).sum()) for a in arrays)
    total = sum(int(a.size) for a in arrays)
    return zeros / total


def elbow(re_hist, pr_t):
    """Second-difference estimate of the RE curve at the latest iteration
    (None unless three points exist, pr_t > 0 and the curve is rising)."""
    if len(re_hist) < 3 or pr_t <= 0 or not re_hist[-1] > re_hist[-2]:
        return None
    return (re_hist[-1] + re_hist[-3] - 2.0 * re_hist[-2]) / pr_t


class ManualSchedule:
    """VeST^man: prune until total sparsity >= target s."""

    def __init__(self, target, init_pr=INIT_PR, max_pr=MAX_PR):
        self.target, self.init_pr, self.max_pr = target, init_pr, max_pr

    def should_prune(self, t, re_hist, current_sparsity):
        return current_sparsity < self.target

    def counts(self, t, sizes, marked):
        pr = pruning_rate(t, self.init_pr, self.max_pr)
        return [prune_count(pr, s, m, self.target) for s, m in zip(sizes, marked)]


class AutoSchedule:
    """VeST^auto: prune until the RE elbow is detected (or a sparsity cap)."""

    def __init__(self, cap=1.0, init_pr=INIT_PR, max_pr=MAX_PR, threshold=ELBOW):
        self.cap, self.init_pr, self.max_pr, self.threshold = cap, init_pr, max_pr, threshold
        self.stopped = False

    def should_prune(self, t, re_hist, current_sparsity):
        if self.stopped:
            return False
        est = elbow(re_hist, pruning_rate(t, self.init_pr, self.max_pr))
        if est is not None and est > self.threshold:
            self.stopped = True
            return False
        return current_sparsity < self.cap

    def counts(self, t, sizes, marked):
        pr = pruning_rate(t, self.init_pr, self.max_pr)
        return [prune_count(pr, s, m, self.cap) for s, m in zip(sizes, marked)]
