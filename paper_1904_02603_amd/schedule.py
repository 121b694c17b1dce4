"""Host-side pruning schedule and the outer loop of Alg. 2.

The per-iteration work runs in libvest; this module only decides how many
elements each tensor loses per prune step and when pruning stops:

  * pruning rate of iteration t (t = 1, 2, ...): pr_t = min(INIT_PR t, MAX_PR)
    with INIT_PR = 0.01, MAX_PR = 0.1 (the pruning step of Alg. 2, Sec. 3.3);
  * a tensor of |T| elements loses ceil(pr_t |T|) unmarked elements per step;
    with a target sparsity s (VeST^man) the marks of a tensor never exceed
    ceil(s |T|) and pruning stops once the total sparsity reaches s;
  * VeST^auto stops pruning for good when the elbow estimate
    (RE_t + RE_{t-2} - 2 RE_{t-1}) / pr_t exceeds 0.05 at a point where the RE
    is rising (RE_t > RE_{t-1}; the elbow the rule looks for is where the RE
    starts to shoot up, Sec. 3.1 and 3.3), optionally also at a sparsity cap;
  * sparsity = zero values / (|G| + sum_n |A^(n)|).
"""
import math
from dataclasses import dataclass, field

import torch


@dataclass
class PruneSchedule:
    mode: str = "manual"          # "manual" (VeST^man) | "auto" (VeST^auto) | "off"
    target: float = 0.0           # manual: target sparsity s; auto: sparsity cap (0 = none)
    init_pr: float = 0.01
    max_pr: float = 0.1
    elbow_threshold: float = 0.05
    stopped: bool = field(default=False, init=False)

    def rate(self, t):
        return min(self.init_pr * t, self.max_pr)

    def elbow(self, re_hist, t):
        pr = self.rate(t)
        if len(re_hist) < 3 or pr <= 0.0 or not re_hist[-1] > re_hist[-2]:
            return None
        return (re_hist[-1] - 2.0 * re_hist[-2] + re_hist[-3]) / pr

    def should_prune(self, t, re_hist, sparsity):
        if self.mode == "off" or self.stopped:
            return False
        if self.mode == "auto":
            est = self.elbow(re_hist, t)
            if est is not None and est > self.elbow_threshold:
                self.stopped = True
                return False
            return self.target <= 0.0 or sparsity < self.target
        return sparsity < self.target

    def count(self, t, size, marked):
        """New elements to prune in a tensor of `size` elements, `marked` already pruned."""
        want = math.ceil(self.rate(t) * size - 1e-12)
        room = size - marked
        if self.target > 0.0:
            room = min(room, math.ceil(self.target * size - 1e-12) - marked)
        return max(0, min(want, room))


def sparsity(ctx):
    zeros = int((ctx.core == 0).sum().item()) + sum(int((f == 0).sum().item()) for f in ctx.factors)
    total = ctx.core.numel() + sum(f.numel() for f in ctx.factors)
    return zeros / total


def run(ctx, iterations, schedule=None, tol=None, log=None, compact_every=5, normalize=True):
    """Alg. 2 on a VestContext: factor sweeps, core sweep, RE, maybe prune,
    and at the end the column normalisation (normalize=True).

    Entries with a fully marked row are dropped from the layouts (vest_compact)
    every `compact_every` prune steps and once pruning has stopped (0 = never);
    results do not change, later passes touch fewer entries.
    """
    schedule = schedule or PruneSchedule(mode="off")
    re_hist = []
    prunes, compacted_at = 0, 0
    for t in range(1, iterations + 1):
        ctx.iteration()
        L = ctx.loss()
        re_hist.append(L["re"])
        sp = sparsity(ctx)
        pruned = False
        if schedule.should_prune(t, re_hist, sp):
            ctx.responsibility()
            fmarked, cmarked = ctx.marked_counts()
            ck = schedule.count(t, ctx.core.numel(), cmarked)
            fk = [schedule.count(t, f.numel(), m) for f, m in zip(ctx.factors, fmarked)]
            ctx.prune(ck, fk)
            pruned = True
            prunes += 1
            if compact_every and prunes - compacted_at >= compact_every:
                ctx.compact()
                compacted_at = prunes
        elif compact_every and prunes > compacted_at:
            ctx.compact()
            compacted_at = prunes
        if log is not None:
            log({"iter": t, "re": L["re"], "loss": L["loss"], "sparsity": sp, "pruned": pruned})
        if tol is not None and len(re_hist) > 1 and abs(re_hist[-1] - re_hist[-2]) < tol and not pruned:
            break
    if normalize:
        ctx.normalize()
    torch.cuda.current_stream().synchronize()
    return re_hist
