#!/usr/bin/env python3
"""Benchmark of the VeST hot path on one MI355X.

One step = one iteration of Alg. 2 on the whole workload, every step of the
hot path included: the factor sweep of each mode (Alg. 4), the core sweep
(Eq. 12), the loss / RE (Eq. 1, 4, one device->host read), the
responsibility keys of every element (Eq. 5, 6) and a prune step (Sec. 3.3)
with the VeST^man ramp pr_t = min(0.01 t, 0.1) toward 95 % sparsity.
Inputs (indices, values, factors, core) are resident in HBM before timing.

value = N * |Omega| / (seconds per step): observed-entry coordinate-descent
updates per second, counting one update per entry and mode of the factor
sweeps (the core sweep, loss, keys and prune are inside the timed step but
not counted as updates).

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DEFAULT_WORKLOAD = "planted-1e5^3-nnz1e7-r10"
METRIC = "observed-entry CD updates/sec per sweep (FP64 vs FP32/BF16) + p99 job latency"
PEAK = {"f64": 78.6, "f32": 157.3}        # TFLOP/s, MI355X vector FP64 / FP32
HBM_PEAK = 8000.0                          # GB/s
SERVE_SEED = 20190407


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_flops_per_entry(N, J):
    # delta (factored contraction, Eq. 11): 2 * sum_{m=2..N} J^m
    # V (Eq. 10, symmetric): J (J + 1); numerator c (Eq. 9): 2 J
    return 2 * sum(J ** m for m in range(2, N + 1)) + J * (J + 1) + 2 * J


def slab_bytes_per_launch(N, J, nnz, dims, ts):
    """Algorithmic HBM bytes of one timed slab pass of the core sweep (passes 2
    to J^(N-2); the first slab's statistics come from the residual pass): per
    entry the residual read and written, the slot copy of the mode N-2 row (J
    values) and the N-2 leading indices; once per pass the per-row statistics
    of the last mode (J + J(J+1)/2 FP64 values), that mode's factor rows and
    the two leading-factor columns."""
    per_entry = 2 * ts + J * ts + 4 * (N - 2)
    rows = dims[N - 1]
    once = rows * (J + J * (J + 1) // 2) * 8 + rows * J * ts + sum(2 * d * ts for d in dims[:N - 2])
    return nnz * per_entry + once


def run_leg(p, precision, steps, warmup, target):
    import torch
    from paper_1904_02603_amd import vest
    from paper_1904_02603_amd.schedule import PruneSchedule

    N = p["idx"].shape[1]
    nnz = p["idx"].shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = vest.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                           precision=precision)
    torch.cuda.synchronize()
    log("  init (layout build) %.2f s, workspace %.2f GB" % (time.perf_counter() - t0, ctx.ws_bytes / 1e9))
    stream = torch.cuda.current_stream()
    sched = PruneSchedule(mode="manual", target=target)
    sizes = [f.numel() for f in ctx.factors]
    marked = {"core": 0, "fac": [0] * N}
    names = ["sweep_factor_%d" % n for n in range(N)] + ["sweep_core", "loss", "responsibility", "prune"]
    events = {k: [] for k in names}

    def timed(name, fn, rec):
        if rec:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            out = fn()
            b.record(stream)
            events[name].append((a, b))
            return out
        return fn()

    def step(t, rec):
        for n in range(N):
            timed("sweep_factor_%d" % n, lambda: ctx.sweep_factor(n), rec)
        timed("sweep_core", ctx.sweep_core, rec)
        L = timed("loss", ctx.loss, rec)
        timed("responsibility", ctx.responsibility, rec)
        ck = sched.count(t, ctx.core.numel(), marked["core"])
        fk = [sched.count(t, s, m) for s, m in zip(sizes, marked["fac"])]
        timed("prune", lambda: ctx.prune(ck, fk), rec)
        marked["core"] += ck
        marked["fac"] = [m + k for m, k in zip(marked["fac"], fk)]
        return L

    t = 0
    for _ in range(warmup):
        t += 1
        step(t, False)
    ctx.slab_timing(True)   # events around every slab pass of the timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    re = None
    for _ in range(steps):
        t += 1
        re = step(t, True)["re"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    slab_total, slab_n = ctx.slab_time()
    ctx.slab_timing(False)
    ms = {k: sum(a.elapsed_time(b) for a, b in v) / len(v) for k, v in events.items() if v}
    ms_step = elapsed * 1e3 / steps
    J = ctx.J
    fl = sweep_flops_per_entry(N, J) * nnz
    sweep_ms = sum(ms["sweep_factor_%d" % n] for n in range(N)) / N
    dims = [int(f.shape[0]) for f in ctx.factors]
    ts = 8 if precision == vest.FP64 else 4
    ctx.close()
    return {
        "slab_kernel_ms": slab_total / max(1, slab_n),
        "slab_launches": slab_n,
        "slab_bytes_per_launch": slab_bytes_per_launch(N, J, nnz, dims, ts),
        "ms_per_step": ms_step,
        "value": N * nnz / (ms_step / 1e3),
        "sweep_only_value": N * nnz / (sweep_ms * N / 1e3),
        "breakdown_ms": {k: round(v, 4) for k, v in ms.items()},
        "sweep_kernel_ms": sweep_ms,
        "sweep_flops_per_launch": fl,
        "final_re": re,
    }


def dense_accuracy(p, iters):
    """RE and factor error of the FP32 / BF16 forms against the FP64 path after
    `iters` full iterations without pruning (same start, same masks)."""
    import torch
    from paper_1904_02603_amd import vest
    out, ref = {}, None
    for name, prec in [("fp64", vest.FP64), ("fp32", vest.FP32), ("bf16", vest.BF16)]:
        ctx = vest.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                               precision=prec)
        for _ in range(iters):
            ctx.iteration()
        L = ctx.loss()
        fac = [f.double().cpu() for f in ctx.factors]
        ctx.close()
        if ref is None:
            ref = (L["re"], fac)
            out["fp64_re"] = L["re"]
            continue
        err = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(fac, ref[1]))
        out[name] = {"re": L["re"], "re_gap_vs_fp64": abs(L["re"] - ref[0]) / ref[0], "factor_rel_err": err}
    out["iterations"] = iters
    return out


def sparse_phase(p, frac, steps, precision):
    """Factor sweeps of the pruned phase: fraction `frac` of every factor
    matrix and of the core marked (zero) at random, sweeps timed with the
    dense and with the gather contraction.  Algorithmic bytes of one sweep:
    the streamed entries ((N-1) int32 indices + one value) plus every factor
    matrix once (own read and written, the others read)."""
    import numpy as np
    import torch
    from paper_1904_02603_amd import vest
    rng = np.random.default_rng(20190402)
    N, nnz = p["idx"].shape[1], p["idx"].shape[0]
    fm = [rng.random(f.shape) < frac for f in p["factors"]]
    cm = rng.random(p["core"].shape) < frac
    fac = [f * (1 - m) for f, m in zip(p["factors"], fm)]
    ctx = vest.VestContext(p["idx"], p["val"], fac, p["core"] * (1 - cm), reg=p["reg"], lam=p["lam"],
                           precision=precision,
                           fmask=[vest.bool_to_masks(torch.from_numpy(m)) for m in fm],
                           cmask=torch.from_numpy(cm.astype(np.uint8)))
    stream = torch.cuda.current_stream()
    vb = 8 if precision == vest.FP64 else 4
    alg = nnz * ((N - 1) * 4 + vb) + sum(f.shape[0] * f.shape[1] * 8 for f in p["factors"]) * (N + 1) / N
    out = {"marked_fraction": frac, "algorithmic_bytes_per_sweep": alg}
    for name, kern in [("dense", vest.KERNEL_DENSE), ("gather", vest.KERNEL_GATHER)]:
        ctx.set_kernel(kern)
        for n in range(N):
            ctx.sweep_factor(n)
        ev = []
        for _ in range(steps):
            for n in range(N):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                ctx.sweep_factor(n)
                b.record(stream)
                ev.append((a, b))
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
        out[name + "_ms_per_sweep"] = ms
        out[name + "_entry_updates_per_s"] = nnz / (ms / 1e3)
    gbs = alg / (out["gather_ms_per_sweep"] / 1e3) / 1e9
    out["gather_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK, "unit": "GB/s",
                              "frac": gbs / HBM_PEAK}
    # entries with a fully marked row dropped from the layouts (vest_compact)
    t0 = time.perf_counter()
    live = ctx.compact()
    out["compaction_s"] = time.perf_counter() - t0
    out["live_entries"] = live
    ctx.set_kernel(vest.KERNEL_AUTO)
    for n in range(N):
        ctx.sweep_factor(n)
    ev = []
    for _ in range(steps):
        for n in range(N):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.sweep_factor(n)
            b.record(stream)
            ev.append((a, b))
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
    out["compacted_ms_per_sweep"] = ms
    out["compacted_entry_updates_per_s"] = nnz / (ms / 1e3)
    alg_live = live * ((N - 1) * 4 + vb) + sum(f.shape[0] * f.shape[1] * 8 for f in p["factors"]) * (N + 1) / N
    gl = alg_live / (ms / 1e3) / 1e9
    out["compacted_roofline"] = {"bound": "hbm", "achieved": gl, "peak": HBM_PEAK, "unit": "GB/s",
                                 "frac": gl / HBM_PEAK, "algorithmic_bytes": alg_live}
    ctx.close()
    return out


def serving_bench(n_jobs, pool, arena_bytes, slots, calib):
    """Serving stream: a pool of observed tensors and n_jobs jobs over it
    (synth.serving_jobs); a serial pass of the first `calib` jobs (one slot,
    all submitted at once) gives the serial rate; then the jobs arrive as a
    Poisson stream at 0.8 x that rate and run through one server with `slots`
    slots and an arena of arena_bytes.  Latency = completion - arrival, both
    taken by the server."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    from paper_1904_02603_amd import synth, vest
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        tensors = list(ex.map(synth.serving_tensor, range(pool)))
    jobs = synth.serving_jobs(n_jobs, tensors)
    log("  pool of %d tensors (%.1f M entries) in %.1f s" % (
        pool, sum(t["idx"].shape[0] for t in tensors) / 1e6, time.perf_counter() - t0))

    def submit(srv, j):
        t = tensors[j["tensor"]]
        fac, core = synth.serving_init(j, t["dims"])
        return srv.submit(t["idx"], t["val"], fac, core, reg=j["reg"], lam=j["lam"],
                          precision=getattr(vest, j["form"]), iterations=j["iterations"])

    def run(srv, arrivals):
        start = time.perf_counter()
        ids, i, retired = [], 0, 0
        while retired < len(arrivals):
            now = time.perf_counter() - start
            while i < len(arrivals) and arrivals[i] <= now:
                ids.append(submit(srv, jobs[i]))
                i += 1
            got = srv.progress()
            retired += got
            if got == 0:
                time.sleep(0.0002)
        recs = []
        for jid in ids:
            st = srv.status(jid)
            if st["state"] != vest.JOB_DONE:
                raise RuntimeError("serving job %d failed: %s" % (jid, st))
            srv.fetch(jid)
            recs.append((st["arrive"], st["admit"], st["done"]))
        return np.array(recs)

    srv = vest.VestServer(arena_bytes, 1)
    r = run(srv, np.zeros(calib))
    srv.close()
    serial_rate = calib / (r[:, 2].max() - r[:, 0].min())
    rate = 0.8 * serial_rate
    arrivals = np.cumsum(np.random.default_rng(SERVE_SEED).exponential(1.0 / rate, n_jobs))
    srv = vest.VestServer(arena_bytes, slots)
    r = run(srv, arrivals)
    srv.close()
    # saturated: the whole stream queued at once (capacity of the server)
    srv = vest.VestServer(arena_bytes, slots)
    rs = run(srv, np.zeros(n_jobs))
    srv.close()
    sat_rate = n_jobs / (rs[:, 2].max() - rs[:, 0].min())
    lat = r[:, 2] - r[:, 0]
    wait = r[:, 1] - r[:, 0]
    span = r[:, 2].max() - r[:, 0].min()
    forms = {f: sum(1 for j in jobs if j["form"] == f) for f in ("FP32", "BF16")}
    return {"jobs": n_jobs, "jobs_per_s": n_jobs / span, "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)), "latency_mean_s": float(lat.mean()),
            "admission_wait_p99_s": float(np.percentile(wait, 99)),
            "saturated_jobs_per_s": sat_rate, "serial_jobs_per_s": serial_rate, "serial_calibration_jobs": calib, "arrival_rate_per_s": rate,
            "slots": slots, "arena_bytes": arena_bytes, "pool_tensors": pool,
            "pool_entries": int(sum(t["idx"].shape[0] for t in tensors)),
            "job_entries_total": int(sum(tensors[j["tensor"]]["idx"].shape[0] for j in jobs)),
            "forms": forms, "orders": {str(o): sum(1 for j in jobs if len(j["ranks"]) == o) for o in (3, 4)},
            "iterations_per_job": 10}


TRAFFIC = {   # committed counter summary and the sources of the kernel it measured
    "slab": ("traffic_k_slab_planted-1e5^3-nnz1e7-r10_fp64.md", ["core.hip", "device.h", "internal.h"]),
    "sweep": ("traffic_k_rowgroup_sweep_planted-1e5^3-nnz1e7-r10_fp64.md", ["rowgroup.hip", "device.h", "internal.h"]),
}


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1904_02603_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def scaling_study(iters=3, warmup=1):
    """Time per Alg. 2 iteration (all factor sweeps + core sweep + loss) on the
    synthetic tensors of the paper's scalability runs (Sec. 4, Fig. 4a-c),
    ranks 3, FP64: (a) order 3..10 at dimensionality and |Omega| 10^3,
    (b) dimensionality 10^3..10^8 at order 3
    with |Omega| equal to it, (c) |Omega| 10^3..10^7 at order 3, dimensionality
    10^3."""
    import torch
    from paper_1904_02603_amd import synth, vest
    runs = {"order": [(N, 10 ** 3, 10 ** 3) for N in range(3, 11)],
            "dimensionality": [(3, 10 ** e, 10 ** e) for e in range(3, 9)],
            "entries": [(3, 10 ** 3, 10 ** e) for e in range(3, 8)]}
    out = {}
    for name, cases in runs.items():
        out[name] = []
        for N, I, nnz in cases:
            t0 = time.perf_counter()
            p = synth.scaling_problem(N, I, nnz)
            gen = time.perf_counter() - t0
            ctx = vest.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"])
            del p
            for _ in range(warmup):
                ctx.iteration()
                ctx.loss()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(iters):
                ctx.iteration()
                ctx.loss()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / iters
            out[name].append({"order": N, "dim": I, "nnz": nnz, "ms_per_iteration": ms,
                              "entry_updates_per_s": N * nnz / (ms / 1e3)})
            log("  %s: N %d, I %d, nnz %d: %.3f ms per iteration (inputs %.1f s)" % (name, N, I, nnz, ms, gen))
            ctx.close()
            del ctx
            torch.cuda.empty_cache()
    return out


def measured_traffic(kernel):
    """Calibrated HBM bytes per launch of a kernel from its committed counter
    summary, or None if the kernel's sources changed since."""
    import re
    name, files = TRAFFIC[kernel]
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+)", txt)
    s = re.search(r"source-sha256: ([0-9a-f]+)", txt)
    if not m or not s or s.group(1) != source_hash(files):
        return None
    return float(m.group(1))


def cpu_baseline(p, seconds):
    """The FP64 oracle's Alg. 4 row update, timed on a bounded row sample."""
    import numpy as np
    from oracle.oracle import Oracle
    idx = p["idx"]
    N = idx.shape[1]
    t0 = time.perf_counter()
    o = Oracle(idx, p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"])
    log("  oracle set-up %.1f s" % (time.perf_counter() - t0))
    rng = np.random.default_rng(1)
    entries, rows, spent = 0, 0, 0.0
    for n in range(N):
        counts = np.bincount(idx[:, n], minlength=o.dims[n])
        order = rng.permutation(o.dims[n])
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < seconds / N and k < len(order):
            i = int(order[k])
            o.update_row(n, i)
            entries += int(counts[i])
            k += 1
        spent += time.perf_counter() - t0
        rows += k
    return {"value": entries / spent, "unit": "entry-updates/s", "cores": 1, "kind": "oracle",
            "sample": "single-threaded FP64 oracle, Alg. 4 row updates of %d randomly chosen rows "
                      "(%d observed entries, all modes) of the same workload, %.1f s" % (rows, entries, spent)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--nnz", type=int, default=None, help="smaller nnz for a quick run (not a bench line)")
    ap.add_argument("--target", type=float, default=0.95)
    ap.add_argument("--no-fp32", action="store_true", help="FP64 leg only (no FP32 / BF16 legs)")
    ap.add_argument("--accuracy-iters", type=int, default=5)
    ap.add_argument("--sparse-frac", type=float, default=0.95,
                    help="marked fraction of the pruned-phase sweep section (0 = skip it)")
    ap.add_argument("--serve-jobs", type=int, default=512, help="serving stream length (0 = skip)")
    ap.add_argument("--serve-pool", type=int, default=32)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-arena-gb", type=float, default=32.0)
    ap.add_argument("--serve-calib", type=int, default=32)
    ap.add_argument("--legs", default="fp64,fp32,bf16",
                    help="comma list of forms to time (the first must be fp64 for a bench line)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 512 MiB device copy first (reference for HBM counters)")
    ap.add_argument("--scaling", action="store_true",
                    help="run only the scalability study (order, dimensionality, entries) and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_02603_amd import synth, vest
    vest.load_library()
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.scaling:
        log("scalability study ...")
        print(json.dumps({"study": "scalability (Sec. 4, Fig. 4a-c)", "ranks": 3, "dtype": "f64", "data": "synthetic",
                          "timing": "wall clock per Alg. 2 iteration (factor sweeps + core sweep + loss), 3 after 1",
                          "results": scaling_study()}))
        return
    t0 = time.perf_counter()
    log("generating workload %s ..." % args.workload)
    p = synth.workload(args.workload, nnz=args.nnz)
    N, nnz = p["idx"].shape[1], p["idx"].shape[0]
    J = p["factors"][0].shape[1]
    log("  %.1f s: dims %s, nnz %d, ranks %d" % (time.perf_counter() - t0, [f.shape[0] for f in p["factors"]], nnz, J))

    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    if args.no_fp32:
        legs = ["fp64"]
    if "fp64" not in legs:
        # profiling runs of one low-precision form: time it, print nothing else
        for name in legs:
            r = run_leg(p, {"fp32": vest.FP32, "bf16": vest.BF16}[name], args.steps, args.warmup, args.target)
            log("%s: %.3f ms/step, sweep kernel %.3f ms" % (name, r["ms_per_step"], r["sweep_kernel_ms"]))
        return
    log("FP64 leg ...")
    f64 = run_leg(p, vest.FP64, args.steps, args.warmup, args.target)
    log("  %.3f ms/step, sweep kernel %.3f ms" % (f64["ms_per_step"], f64["sweep_kernel_ms"]))
    lowp = {}
    acc = None
    if len(legs) > 1:
        for name, prec in [(n, {"fp32": vest.FP32, "bf16": vest.BF16}[n]) for n in legs if n != "fp64"]:
            log("%s leg ..." % name.upper())
            lowp[name] = run_leg(p, prec, args.steps, args.warmup, args.target)
            log("  %.3f ms/step, sweep kernel %.3f ms" % (lowp[name]["ms_per_step"], lowp[name]["sweep_kernel_ms"]))
        if args.accuracy_iters > 0:
            log("dense-phase accuracy (%d iterations, no pruning) ..." % args.accuracy_iters)
            acc = dense_accuracy(p, args.accuracy_iters)
    sparse = {}
    if args.sparse_frac > 0:
        for name in legs:
            log("pruned-phase sweeps (%s, %.0f %% marked) ..." % (name, 100 * args.sparse_frac))
            sparse[name] = sparse_phase(p, args.sparse_frac, args.steps,
                                        {"fp64": vest.FP64, "fp32": vest.FP32, "bf16": vest.BF16}[name])
            log("  dense %.3f ms, gather %.3f ms per sweep; compacted to %d entries in %.2f s: %.3f ms" % (
                sparse[name]["dense_ms_per_sweep"], sparse[name]["gather_ms_per_sweep"],
                sparse[name]["live_entries"], sparse[name]["compaction_s"], sparse[name]["compacted_ms_per_sweep"]))
    serving = None
    if args.serve_jobs > 0:
        log("serving stream (%d jobs) ..." % args.serve_jobs)
        serving = serving_bench(args.serve_jobs, args.serve_pool, int(args.serve_arena_gb * (1 << 30)),
                                args.serve_slots, min(args.serve_calib, args.serve_jobs))
        log("  %.2f jobs/s, p50 %.3f s, p99 %.3f s (serial %.2f jobs/s)" % (
            serving["jobs_per_s"], serving["latency_p50_s"], serving["latency_p99_s"], serving["serial_jobs_per_s"]))
    cpu = None
    if args.cpu_seconds > 0:
        log("oracle CPU baseline ...")
        cpu = cpu_baseline(p, args.cpu_seconds)

    achieved = f64["sweep_flops_per_launch"] / (f64["sweep_kernel_ms"] / 1e3) / 1e12
    slab_gbs = f64["slab_bytes_per_launch"] / (f64["slab_kernel_ms"] / 1e3) / 1e9
    named = args.workload == DEFAULT_WORKLOAD and args.nnz is None
    out = {
        "metric": METRIC,
        "value": f64["value"],
        "unit": "entry-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dims": [int(f.shape[0]) for f in p["factors"]], "nnz": nnz,
                   "ranks": [J] * N, "reg": "L_F" if p["reg"] == 0 else "L_1", "lambda": p["lam"],
                   "step": "factor sweeps (all modes) + core sweep + loss + responsibility + prune",
                   "prune": "manual ramp min(0.01 t, 0.1) toward %.2f" % args.target},
        # the kernel with the largest share of the step: J^(N-2) slab passes per core sweep
        "roofline": {"kernel": "k_slab (slab pass of the core sweep)", "bound": "hbm",
                     "achieved": slab_gbs, "peak": HBM_PEAK, "unit": "GB/s", "frac": slab_gbs / HBM_PEAK,
                     "traffic": measured_traffic("slab") if named else None,
                     "bytes_per_launch": f64["slab_bytes_per_launch"],
                     "avg_launch_ms": f64["slab_kernel_ms"], "launches_timed": f64["slab_launches"]},
        "roofline_sweep": {"kernel": "k_rowgroup<OP_SWEEP> (factor sweep, one mode)", "bound": "alu",
                           "achieved": achieved, "peak": PEAK["f64"], "unit": "TFLOP/s",
                           "frac": achieved / PEAK["f64"],
                           "traffic": measured_traffic("sweep") if named else None,
                           "flops_per_launch": f64["sweep_flops_per_launch"],
                           "avg_launch_ms": f64["sweep_kernel_ms"]},
        "cpu_baseline": cpu,
        "breakdown_ms": f64["breakdown_ms"],
        "sweep_only_value": f64["sweep_only_value"],
        "final_re": f64["final_re"],
    }
    for name, r in lowp.items():
        out[name] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                     "sweep_only_value": r["sweep_only_value"], "breakdown_ms": r["breakdown_ms"],
                     "sweep_tflops": r["sweep_flops_per_launch"] / (r["sweep_kernel_ms"] / 1e3) / 1e12,
                     "slab_pass_ms": r["slab_kernel_ms"],
                     "slab_pass_gbs": r["slab_bytes_per_launch"] / (r["slab_kernel_ms"] / 1e3) / 1e9,
                     "final_re": r["final_re"],
                     "re_gap_vs_fp64_pruned": abs(r["final_re"] - f64["final_re"]) / f64["final_re"]}
    if acc is not None:
        out["accuracy_dense"] = acc
    if sparse:
        out["pruned_phase"] = sparse
    if serving is not None:
        out["serving"] = serving
    if args.nnz is not None:
        out["config"]["note"] = "reduced nnz: not the named workload"
    print(json.dumps(out))


if __name__ == "__main__":
    main()
