"""Expected values of the full-size parity tests, written by the FP64 oracle.

    python tests/golden/make_golden.py config2-full    # ~10 min, one core
    python tests/golden/make_golden.py config2-1e6     # ~15 min
    python tests/golden/make_golden.py config4-auto    # ~1-2 h

Each case regenerates its seeded synthetic input (paper_1904_02603_amd.synth,
which only draws numbers), runs the oracle (oracle/, single-threaded FP64,
compensated sums) through the steps named below, and stores what the GPU test
compares in tests/golden/<case>.npz: loss terms, the whole core, and for every
factor matrix a seeded sample of rows (values and, where keys are taken,
their responsibility keys).  Prune decisions are stored as the sorted flat
indices of the newly marked elements when they are few, else as the SHA-256
of the boolean marking table with its count.  Nothing here reads a GPU result.

Cases (stand-ins for the paper's rating tensors, synthetic recipes of the
package's synth module):
  config2-full  the 10^7-entry planted workload over (10^5)^3, ranks 10^3,
                L_F 0.01: one Alg. 2 iteration (factor sweeps of modes 1..3,
                core sweep), loss; responsibility keys (Eq. 5, 6) and one
                prune step at pr_1 = 0.01 (Sec. 3.3); loss after the prune.
  config2-1e6   the same recipe at 10^6 entries over (10^4)^3 (about 100
                entries per row, as at full size): 20 iterations, loss after
                each.
  config4-auto  the order-4 Zipf workload 50k x 50k x 1000 x 24, ranks 8^4,
                L_F 0.01, at 10^6 entries: VeST^auto (elbow rule, sparsity cap
                0.95), up to 20 iterations, then the column normalisation;
                also the whole state (factors, core, marking tables) the
                last iteration starts from.
"""
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import schedule as OS  # noqa: E402
from oracle.oracle import Oracle  # noqa: E402
from paper_1904_02603_amd import synth  # noqa: E402

SAMPLE_ROWS = 128


def sample_rows(idx, dims, seed):
    """Seeded sample of rows per mode, plus the longest and the shortest."""
    rng = np.random.default_rng(seed)
    out = []
    for n, d in enumerate(dims):
        cnt = np.bincount(idx[:, n], minlength=d)
        rows = set(rng.choice(d, min(SAMPLE_ROWS, d), replace=False).tolist())
        rows |= {int(cnt.argmax()), int(cnt.argmin())}
        out.append(np.array(sorted(rows), dtype=np.int64))
    return out


def mask_digest(mask_bool):
    b = np.ascontiguousarray(np.asarray(mask_bool, dtype=np.uint8))
    return hashlib.sha256(b.tobytes()).hexdigest(), int(b.sum())


def problem(case):
    if case == "config2-full":
        return synth.workload("planted-1e5^3-nnz1e7-r10")
    if case == "config2-1e6":
        return synth.workload("planted-1e5^3-nnz1e7-r10", nnz=10 ** 6, dims=(10 ** 4,) * 3)
    if case == "config4-auto":
        return synth.workload("planted-zipf-50k.50k.1k.24-nnz5e7-r8", nnz=10 ** 6)
    raise SystemExit("unknown case " + case)


def log(*a):
    print(*a, flush=True)


def loss_vec(o):
    L = o.loss()
    return np.array([L["sse"], L["xnorm2"], L["reg"], L["loss"], L["re"]])


def config2_full(p, out):
    o = Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"])
    dims = [f.shape[0] for f in p["factors"]]
    rows = sample_rows(p["idx"], dims, 2)
    t0 = time.time()
    for n in range(len(dims)):
        o.sweep_factor(n)
        log("  factor sweep %d done, %.0f s" % (n, time.time() - t0))
    o.sweep_core()
    log("  core sweep done, %.0f s" % (time.time() - t0))
    out["loss_it1"] = loss_vec(o)
    out["core_it1"] = o.core.copy()
    for n in range(len(dims)):
        out["rows_m%d" % n] = rows[n]
        out["vals_m%d" % n] = o.factors[n][rows[n]].copy()
    ck, fk = o.responsibility()
    log("  keys done, %.0f s" % (time.time() - t0))
    out["core_key"] = np.asarray(ck).copy()
    for n in range(len(dims)):
        out["keys_m%d" % n] = np.asarray(fk[n])[rows[n]].copy()
    kc = OS.prune_count(OS.pruning_rate(1), o.core.size, 0)
    kf = [OS.prune_count(OS.pruning_rate(1), f.size, 0) for f in o.factors]
    cm0 = o.cmask.astype(bool).copy()
    fm0 = [m.astype(bool).copy() for m in o.fmask]
    o.prune(ck, fk, kc, kf)
    out["prune_counts"] = np.array([kc] + kf, dtype=np.int64)
    out["pruned_core"] = np.flatnonzero(o.cmask.astype(bool) & ~cm0).astype(np.int64)
    for n in range(len(dims)):
        out["pruned_m%d" % n] = np.flatnonzero(o.fmask[n].astype(bool) & ~fm0[n]).astype(np.int64)
    out["loss_after_prune"] = loss_vec(o)


def config2_1e6(p, out, iters=20):
    o = Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"])
    dims = [f.shape[0] for f in p["factors"]]
    rows = sample_rows(p["idx"], dims, 3)
    losses = []
    t0 = time.time()
    for it in range(iters):
        o.iteration()
        losses.append(loss_vec(o))
        log("  iteration %d RE %.12f, %.0f s" % (it + 1, losses[-1][4], time.time() - t0))
        if it + 1 == 1:
            out["core_it1"] = o.core.copy()
    out["loss_per_iteration"] = np.array(losses)
    out["core_final"] = o.core.copy()
    for n in range(len(dims)):
        out["rows_m%d" % n] = rows[n]
        out["vals_m%d" % n] = o.factors[n][rows[n]].copy()


def config4_auto(p, out, iters=20, cap=0.95):
    o = Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"])
    dims = [f.shape[0] for f in p["factors"]]
    rows = sample_rows(p["idx"], dims, 4)
    sched = OS.AutoSchedule(cap=cap)
    re_hist, steps = [], []
    t0 = time.time()
    for t in range(1, iters + 1):
        if t == iters:
            # the state the last iteration starts from: a GPU context loaded
            # with it runs that iteration from identical inputs
            for n in range(len(dims)):
                out["pre_factor_m%d" % n] = o.factors[n].copy()
                out["pre_fmask_m%d" % n] = np.packbits(o.fmask[n].astype(bool).ravel())
            out["pre_core"] = o.core.copy()
            out["pre_cmask"] = o.cmask.astype(np.uint8).copy()
        o.iteration()
        L = loss_vec(o)
        re_hist.append(L[4])
        sp = OS.sparsity([o.core] + list(o.factors))
        rec = [t, L[4], sp, 0, 0]
        if sched.should_prune(t, re_hist, sp):
            ck, fk = o.responsibility()
            marked = [int(o.cmask.sum())] + [int(m.sum()) for m in o.fmask]
            sizes = [o.core.size] + [f.size for f in o.factors]
            k = sched.counts(t, sizes, marked)
            o.prune(ck, fk, k[0], k[1:])
            rec[3], rec[4] = 1, sum(k)
        steps.append(rec)
        log("  t %d RE %.12f sparsity %.4f pruned %d (%d), %.0f s" % (t, L[4], sp, rec[3], rec[4], time.time() - t0))
    o.normalize()
    out["steps"] = np.array(steps, dtype=np.float64)   # t, RE, sparsity before the prune, pruned?, count
    out["loss_final"] = loss_vec(o)
    out["core_final"] = o.core.copy()
    out["core_mask"] = o.cmask.astype(np.uint8).copy()
    dig = []
    for n in range(len(dims)):
        out["rows_m%d" % n] = rows[n]
        out["vals_m%d" % n] = o.factors[n][rows[n]].copy()
        dig.append(mask_digest(o.fmask[n]))
    out["mask_digest"] = np.array([d for d, _ in dig])
    out["mask_count"] = np.array([c for _, c in dig], dtype=np.int64)


def main():
    case = sys.argv[1]
    t0 = time.time()
    p = problem(case)
    log("%s: dims %s, nnz %d, inputs in %.1f s" % (case, [f.shape[0] for f in p["factors"]], p["idx"].shape[0],
                                                   time.time() - t0))
    out = {}
    {"config2-full": config2_full, "config2-1e6": config2_1e6, "config4-auto": config4_auto}[case](p, out)
    path = os.path.join(HERE, case + ".npz")
    np.savez_compressed(path, **out)
    meta = {"case": case, "seconds": round(time.time() - t0, 1), "arrays": sorted(out),
            "writer": "tests/golden/make_golden.py (oracle only)"}
    with open(os.path.join(HERE, case + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    log("wrote", path, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
