#!/usr/bin/env python3
"""Benchmark of the VeST hot path on one MI355X.

Headline: the dense-core workload of 10^7 observed entries over (10^5)^3,
ranks 10^3, L_F lambda 0.01, 20 sweeps, FP64 path against the FP32 and
split-BF16 forms, no pruning.  One step = one iteration of Alg. 2 without a
prune step: the factor sweep of each mode (Alg. 4, Eq. 9-11), the core sweep
(Eq. 12) and the loss / RE (Eq. 1, 4; one device->host read).  Inputs
(indices, values, factors, core) are resident in HBM before timing.

value = N * |Omega| / (seconds per step): observed-entry coordinate-descent
updates per second, one update per entry and mode of the factor sweeps (the
core sweep and the loss are inside the timed step but not counted).

Labelled sections beside the headline:
  * prune_step: the responsibility keys (Eq. 5, 6) and one prune step
    (Sec. 3.3) on the state the FP64 leg reached, timed per call;
  * prune_ramp: the three forms from the same start through the VeST^man
    ramp pr_t = min(0.01 t, 0.1) toward 95 % sparsity, in lockstep, with the
    prune masks of the FP32 / BF16 forms compared with the FP64 ones after
    every prune step (differing elements and their key gaps) and the RE gap;
  * pruned_phase: factor sweeps with 95 % of every tensor marked (dense and
    gather contraction, and after compaction);
  * serving: the request loop over a Poisson stream of jobs.

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


def slab_alg_bytes_per_launch(N, J, nnz, dims, ts):
    """Algorithmic HBM bytes of one slab pass of the core sweep, by the count
    of the method: per observed entry its N int32 indices and the residual
    read and written (4 N + 2 s_val bytes); once per pass the factor matrices
    the pass reads (the last two modes' rows, one column of each leading
    mode).  Gathered factor rows are counted once per matrix."""
    per_entry = 4 * N + 2 * ts
    once = (dims[N - 2] + dims[N - 1]) * J * 8 + sum(d * 8 for d in dims[:N - 2])
    return nnz * per_entry + once


def slab_design_bytes_per_launch(N, J, nnz, dims, ts):
    """Bytes one slab pass of this implementation streams by design (passes 2
    to J^(N-2); the first slab's statistics come from the residual pass): per
    entry the residual read and written, the slot copy of the mode N-2 row (J
    values) and the N-2 leading indices; once per pass the per-row statistics
    of the last mode (J + J(J+1)/2 FP64 values), that mode's factor rows and
    the leading-factor columns."""
    per_entry = 2 * ts + J * ts + 4 * (N - 2)
    rows = dims[N - 1]
    once = rows * (J + J * (J + 1) // 2) * 8 + rows * J * ts + sum(2 * d * ts for d in dims[:N - 2])
    return nnz * per_entry + once


def sweep_alg_bytes(N, nnz, dims, J, ts):
    """Algorithmic HBM bytes of one factor sweep (one mode): the streamed
    entries ((N-1) int32 indices + one value) plus every factor matrix once
    (the swept one read and written, the others read); averaged over modes."""
    return nnz * ((N - 1) * 4 + ts) + sum(d * J * 8 for d in dims) * (N + 1) / N


class EventLog:
    """HIP events around library calls on the context's stream."""

    def __init__(self, stream):
        self.stream = stream
        self.ev = {}

    def timed(self, name, fn, rec=True):
        import torch
        if not rec:
            return fn()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        out = fn()
        b.record(self.stream)
        self.ev.setdefault(name, []).append((a, b))
        return out

    def ms(self):
        return {k: sum(a.elapsed_time(b) for a, b in v) / len(v) for k, v in self.ev.items() if v}


def dense_leg(p, precision, steps, warmup):
    """The headline leg of one form: `warmup` untimed and `steps` timed
    iterations (factor sweeps of every mode, core sweep, loss), no pruning.
    Returns the timings and the context, left open at its final state."""
    import torch
    from paper_1904_02603_amd import vest

    N = p["idx"].shape[1]
    nnz = p["idx"].shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = vest.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                           precision=precision)
    torch.cuda.synchronize()
    log("  init (layout build) %.2f s, workspace %.2f GB" % (time.perf_counter() - t0, ctx.ws_bytes / 1e9))
    log_ = EventLog(torch.cuda.current_stream())

    def step(rec):
        for n in range(N):
            log_.timed("sweep_factor_%d" % n, lambda: ctx.sweep_factor(n), rec)
        log_.timed("sweep_core", ctx.sweep_core, rec)
        return log_.timed("loss", ctx.loss, rec)

    for _ in range(warmup):
        step(False)
    ctx.slab_timing(True)   # events around every slab pass of the timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = None
    for _ in range(steps):
        L = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    slab_total, slab_n = ctx.slab_time()
    ctx.slab_timing(False)
    ms = log_.ms()
    ms_step = elapsed * 1e3 / steps
    J = ctx.J
    sweep_ms = sum(ms["sweep_factor_%d" % n] for n in range(N)) / N
    dims = [int(f.shape[0]) for f in ctx.factors]
    ts = 8 if precision == vest.FP64 else 4
    return ctx, {
        "slab_kernel_ms": slab_total / max(1, slab_n),
        "slab_launches": slab_n,
        "slab_alg_bytes_per_launch": slab_alg_bytes_per_launch(N, J, nnz, dims, ts),
        "slab_design_bytes_per_launch": slab_design_bytes_per_launch(N, J, nnz, dims, ts),
        "ms_per_step": ms_step,
        "value": N * nnz / (ms_step / 1e3),
        "sweep_only_value": N * nnz / (sweep_ms * N / 1e3),
        "full_sweep_value": nnz / ((sweep_ms * N + ms["sweep_core"]) / 1e3),
        "core_value": nnz * ctx.core.numel() / (ms["sweep_core"] / 1e3),
        "breakdown_ms": {k: round(v, 4) for k, v in ms.items()},
        "sweep_kernel_ms": sweep_ms,
        "sweep_flops_per_launch": sweep_flops_per_entry(N, J) * nnz,
        "sweep_alg_bytes": sweep_alg_bytes(N, nnz, dims, J, ts),
        "final_re": L["re"],
        "final_loss": L["loss"],
    }


def compare_states(ctx, ref):
    """Relative RE gap and factor / core errors of a context against the FP64
    leg's final state (same start, same number of iterations)."""
    import torch
    L = ctx.loss()
    out = {"re": L["re"], "re_gap_vs_fp64": abs(L["re"] - ref["re"]) / ref["re"]}
    errs, rms = [], []
    for a, b in zip(list(ctx.factors) + [ctx.core], ref["tensors"]):
        d = (a - b).abs()
        errs.append(float(d.max() / b.abs().max()))
        rms.append(float(torch.sqrt((d * d).mean()) / torch.sqrt((b * b).mean())))
    out["factor_rel_err_max"] = max(errs[:-1])
    out["core_rel_err_max"] = errs[-1]
    out["rel_rmse_factors"] = max(rms[:-1])
    out["rel_rmse_core"] = rms[-1]
    return out


def prune_step_section(ctx, reps=1):
    """Responsibility keys (Eq. 5, 6) and one prune step (Sec. 3.3, first
    ramp step pr_1 = 0.01) on a context's current state, per-call times.  One
    untimed call first (the first call of a process also loads the key
    kernels and creates the second stream), then a core sweep, which leaves
    the state an Alg. 2 iteration leaves (the residual lagging its last slab,
    caught up by the timed call)."""
    import torch
    from paper_1904_02603_amd.schedule import PruneSchedule
    lg = EventLog(torch.cuda.current_stream())
    ctx.responsibility()
    ctx.sweep_core()
    for _ in range(reps):
        lg.timed("responsibility", ctx.responsibility)
    sched = PruneSchedule(mode="manual", target=0.95)
    ck = sched.count(1, ctx.core.numel(), 0)
    fk = [sched.count(1, f.numel(), 0) for f in ctx.factors]
    lg.timed("prune", lambda: ctx.prune(ck, fk))
    torch.cuda.synchronize()
    ms = lg.ms()
    return {"responsibility_ms": ms["responsibility"], "prune_ms": ms["prune"], "responsibility_calls": reps,
            "pruned": {"core": ck, "factors": fk}}


def mask_differences(ref_ctx, ref_keys, new_ref, ctx, new):
    """A23 report for one prune step: elements whose prune decision differs
    between a reduced-precision form and the FP64 path, and the gap of their
    FP64 keys to the FP64 selection threshold (largest selected key) relative
    to that threshold's magnitude."""
    import torch
    diff, gaps = 0, []
    for rk, rnew, nnew in zip(ref_keys, new_ref, new):
        d = rnew ^ nnew
        n = int(d.sum())
        diff += n
        if n and bool(rnew.any()):
            thr = rk[rnew].max()
            g = ((rk[d] - thr).abs() / thr.abs().clamp_min(1e-300))
            g = g[torch.isfinite(g)]
            if g.numel():
                gaps.append(float(g.max()))
    return diff, (max(gaps) if gaps else None)


def prune_ramp_section(p, iters, target):
    """The three forms from the same start through the VeST^man ramp, in
    lockstep: iteration, loss, responsibility, prune (counts from the shared
    schedule).  Reports time per step of every form, the RE gap of FP32 /
    BF16 against FP64 after the ramp, and per prune step the number of
    elements whose prune decision differs from FP64's and their key gaps."""
    import torch
    from paper_1904_02603_amd import vest
    from paper_1904_02603_amd.schedule import PruneSchedule
    forms = [("fp64", vest.FP64), ("fp32", vest.FP32), ("bf16", vest.BF16)]
    ctxs = {n: vest.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                                precision=f) for n, f in forms}
    N = p["idx"].shape[1]
    sched = PruneSchedule(mode="manual", target=target)
    sizes = [f.size for f in p["factors"]]
    csize = p["core"].size
    mc, mf = 0, [0] * N
    logs = {n: EventLog(torch.cuda.current_stream()) for n, _ in forms}
    steps = []
    for t in range(1, iters + 1):
        ck = sched.count(t, csize, mc)
        fk = [sched.count(t, s, m) for s, m in zip(sizes, mf)]
        rec = {"t": t, "pruned": ck + sum(fk)}
        before = {}
        for name, _ in forms:
            c = ctxs[name]
            before[name] = [m.clone() for m in c.factor_masks_bool()] + [c.cmask.bool().clone()]

            def one(c=c):
                c.iteration()
                L = c.loss()
                c.responsibility()
                c.prune(ck, fk)
                return L
            L = logs[name].timed("step", one)
            rec[name + "_re"] = L["re"]
        torch.cuda.synchronize()
        new = {}
        for name, _ in forms:
            c = ctxs[name]
            after = [m for m in c.factor_masks_bool()] + [c.cmask.bool()]
            new[name] = [a & ~b for a, b in zip(after, before[name])]
        refk = list(ctxs["fp64"].factor_keys) + [ctxs["fp64"].core_key]
        for name in ("fp32", "bf16"):
            d, g = mask_differences(ctxs["fp64"], refk, new["fp64"], ctxs[name], new[name])
            rec[name + "_mask_diff"] = d
            rec[name + "_max_key_gap"] = g
        mc += ck
        mf = [m + k for m, k in zip(mf, fk)]
        steps.append(rec)
    out = {"iterations": iters, "target": target, "steps": steps,
           "marked_fraction": (mc + sum(mf)) / (csize + sum(sizes))}
    L64 = ctxs["fp64"].loss()
    for name, _ in forms:
        out[name + "_ms_per_step"] = logs[name].ms()["step"]
        if name != "fp64":
            L = ctxs[name].loss()
            out[name + "_re_gap_vs_fp64"] = abs(L["re"] - L64["re"]) / L64["re"]
            out[name + "_first_divergent_step"] = next(
                (s["t"] for s in steps if s[name + "_mask_diff"]), None)
    out["fp64_final_re"] = L64["re"]
    for c in ctxs.values():
        c.close()
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
    (synth.serving_jobs, half of them pruning with VeST^man); a serial pass of the first `calib` jobs (one slot,
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
                          precision=getattr(vest, j["form"]), iterations=j["iterations"],
                          prune_target=j["prune_target"])

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
    st_p = srv.stats()
    srv.close()
    # saturated: the whole stream queued at once (capacity of the server)
    srv = vest.VestServer(arena_bytes, slots)
    rs = run(srv, np.zeros(n_jobs))
    st_s = srv.stats()
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
            "pruning_jobs": sum(1 for j in jobs if j["prune_target"] > 0),
            "iterations_per_job": 10,
            "batched_iterations": {"poisson": st_p["batches"], "saturated": st_s["batches"]},
            "jobs_per_batch": {"poisson": st_p["batched_job_iterations"] / max(1, st_p["batches"]),
                               "saturated": st_s["batched_job_iterations"] / max(1, st_s["batches"])}}


def gen_workload(name):
    """Seeded inputs of a named workload (run in a worker process)."""
    from paper_1904_02603_amd import synth
    synth.THREADS = 4      # leave host cores to the process that drives the GPU
    t0 = time.perf_counter()
    p = synth.workload(name)
    p.pop("planted", None)
    p["gen_s"] = time.perf_counter() - t0
    return p


def sampled_rows_vs_oracle(p, mode, got, rows):
    """The oracle's Alg. 4 update of sampled rows of `mode` from the initial
    state (rows are independent given the other modes), against the rows a
    GPU form produced in its first sweep of that mode.  Returns the oracle's
    rows and its time."""
    from oracle.oracle import Oracle
    o = Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"])
    t0 = time.perf_counter()
    for i in rows:
        o.update_row(mode, int(i))
    dt = time.perf_counter() - t0
    ref = o.factors[mode][rows].copy()
    del o
    return ref, dt


def pick_rows(idx, mode, dim, k, max_len, seed):
    import numpy as np
    cnt = np.bincount(idx[:, mode], minlength=dim)
    ok = np.flatnonzero((cnt > 0) & (cnt <= max_len))
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(ok, min(k, ok.size), replace=False))
    return rows, int(cnt[rows].sum())


def rel_errs(got, ref):
    import numpy as np
    d = np.abs(got - ref)
    s = np.abs(ref).max()
    return {"elementwise_floor_1e-4": float((d / np.maximum(np.abs(ref), 1e-4 * s)).max()),
            "rel_rmse": float(np.sqrt((d * d).sum() / max((ref * ref).sum(), 1e-300)))}


def rating_leg(p, steps, warmup):
    """Rating-shaped Zipf tensor, 10^8 entries: FP64, FP32 and split-BF16
    forms from the same start, `warmup` + `steps` iterations each (factor
    sweeps + core sweep + loss); the first mode-0 sweep's sampled rows against
    the oracle; FP32 / BF16 state against FP64 after the run."""
    import numpy as np
    import torch
    from paper_1904_02603_amd import vest
    N, nnz = p["idx"].shape[1], p["idx"].shape[0]
    dims = [f.shape[0] for f in p["factors"]]
    J = p["factors"][0].shape[1]
    rows, row_entries = pick_rows(p["idx"], 0, dims[0], 48, 4000, 7)
    out = {"workload": "rating-zipf-500k.20k.2k-nnz1e8-r10", "dims": dims, "nnz": nnz, "ranks": [J] * N,
           "reg": "L_1", "lambda": p["lam"], "iterations_timed": steps, "warmup": warmup,
           "input_generation_s": p.get("gen_s")}
    first_rows, final = {}, {}
    for name, prec in [("fp64", vest.FP64), ("fp32", vest.FP32), ("bf16", vest.BF16)]:
        ctx = vest.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                               precision=prec)
        lg = EventLog(torch.cuda.current_stream())
        ctx.sweep_factor(0)
        first_rows[name] = ctx.factors[0][torch.as_tensor(rows, device="cuda")].cpu().numpy()
        for n in range(1, N):
            ctx.sweep_factor(n)
        ctx.sweep_core()
        for _ in range(max(0, warmup - 1)):
            ctx.iteration()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for n in range(N):
                lg.timed("sweep_factor", lambda: ctx.sweep_factor(n))
            lg.timed("sweep_core", ctx.sweep_core)
            L = lg.timed("loss", ctx.loss)
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) * 1e3 / steps
        ms = lg.ms()
        ts = 8 if prec == vest.FP64 else 4
        alg = sweep_alg_bytes(N, nnz, dims, J, ts)
        r = {"ms_per_step": ms_step, "value": N * nnz / (ms_step / 1e3),
             "sweep_only_value": nnz / (ms["sweep_factor"] / 1e3), "breakdown_ms": ms, "final_re": L["re"],
             "sweep_roofline": {"bound": "hbm", "achieved": alg / (ms["sweep_factor"] / 1e3) / 1e9,
                                "peak": HBM_PEAK, "unit": "GB/s",
                                "frac": alg / (ms["sweep_factor"] / 1e3) / 1e9 / HBM_PEAK,
                                "algorithmic_bytes_per_launch": alg}}
        if name == "bf16":
            mf = 2 * J ** N * nnz   # first contraction stage on matrix cores, algorithmic
            r["sweep_mfma"] = {"achieved": mf / (ms["sweep_factor"] / 1e3) / 1e12, "peak": 2500.0,
                               "unit": "TFLOP/s", "algorithmic_flops_per_launch": mf,
                               "note": "split form issues three products per algorithmic one"}
        final[name] = ([f.clone() for f in ctx.factors] + [ctx.core.clone()], L["re"])
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        out[name] = r
        log("  %s: %.2f ms/step, factor sweep %.3f ms, core sweep %.3f ms" % (
            name, ms_step, ms["sweep_factor"], ms["sweep_core"]))
    ref_t, ref_re = final["fp64"]
    for name in ("fp32", "bf16"):
        t, re_ = final[name]
        out[name]["vs_fp64"] = {"re_gap": abs(re_ - ref_re) / ref_re,
                                "rel_rmse_factors": max(float(torch.sqrt(((a - b) ** 2).sum() / (b * b).sum()))
                                                        for a, b in zip(t[:-1], ref_t[:-1])),
                                "rel_rmse_core": float(torch.sqrt(((t[-1] - ref_t[-1]) ** 2).sum()
                                                                  / (ref_t[-1] ** 2).sum()))}
    del final, ref_t
    ref, dt = sampled_rows_vs_oracle(p, 0, None, rows)
    out["oracle_sample"] = {"rows": int(rows.size), "entries": row_entries, "oracle_s": dt,
                            "oracle_entry_updates_per_s": row_entries / dt,
                            "what": "first mode-0 sweep from the initial state, sampled rows of <= 4000 entries",
                            **{name: rel_errs(first_rows[name], ref) for name in first_rows}}
    return out


def order4_auto_leg(p, iters, target):
    """Order-4 Zipf tensor, 5e7 entries, ranks 8^4: VeST^auto (elbow rule,
    sparsity cap `target`) through the host schedule in FP32 and FP64 from the
    same start, time and RE of every iteration; dense-phase and final
    (pruned, compacted) factor-sweep rooflines of the FP32 form; sampled rows
    of the first mode-0 sweep against the oracle."""
    import numpy as np
    import torch
    from paper_1904_02603_amd import vest
    from paper_1904_02603_amd.schedule import PruneSchedule, run
    N, nnz = p["idx"].shape[1], p["idx"].shape[0]
    dims = [f.shape[0] for f in p["factors"]]
    J = p["factors"][0].shape[1]
    rows, row_entries = pick_rows(p["idx"], 0, dims[0], 48, 4000, 8)
    out = {"workload": "planted-zipf-50k.50k.1k.24-nnz5e7-r8", "dims": dims, "nnz": nnz, "ranks": [J] * N,
           "reg": "L_F", "lambda": p["lam"], "schedule": "VeST^auto, elbow 0.05, cap %.2f" % target,
           "max_iterations": iters, "input_generation_s": p.get("gen_s")}
    first_rows, finals = {}, {}
    for name, prec in [("fp32", vest.FP32), ("fp64", vest.FP64)]:
        ctx = vest.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                               precision=prec)
        lg = EventLog(torch.cuda.current_stream())
        # dense phase: the first iteration's factor sweeps, timed
        for n in range(N):
            lg.timed("dense_sweep", lambda: ctx.sweep_factor(n))
            if n == 0:
                first_rows[name] = ctx.factors[0][torch.as_tensor(rows, device="cuda")].cpu().numpy()
        torch.cuda.synchronize()
        ctx.close()
        ctx = vest.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=p["reg"], lam=p["lam"],
                               precision=prec)
        hist = []
        tl = [time.perf_counter()]

        def rec(d):
            tl.append(time.perf_counter())
            d = dict(d)
            d["ms"] = (tl[-1] - tl[-2]) * 1e3
            hist.append(d)
        run(ctx, iters, PruneSchedule(mode="auto", target=target), log=rec, compact_every=5, normalize=False)
        live = ctx.layout_stats(0)["nnz"]
        for _ in range(3):
            for n in range(N):
                lg.timed("final_sweep", lambda: ctx.sweep_factor(n))
        torch.cuda.synchronize()
        ms = lg.ms()
        fl = sweep_flops_per_entry(N, J) * nnz
        peak = PEAK["f32"] if prec == vest.FP32 else PEAK["f64"]
        ts = 4 if prec == vest.FP32 else 8
        alg_final = live * ((N - 1) * 4 + ts) + sum(d * J * 8 for d in dims) * (N + 1) / N
        r = {"iterations": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in h.items()} for h in hist],
             "final_re": hist[-1]["re"], "final_sparsity": hist[-1]["sparsity"],
             "prune_steps": sum(1 for h in hist if h["pruned"]),
             "dense_sweep_ms": ms["dense_sweep"],
             "dense_sweep_roofline": {"bound": "alu", "achieved": fl / (ms["dense_sweep"] / 1e3) / 1e12,
                                      "peak": peak, "unit": "TFLOP/s",
                                      "frac": fl / (ms["dense_sweep"] / 1e3) / 1e12 / peak,
                                      "flops_per_launch": fl},
             "dense_entry_updates_per_s": nnz / (ms["dense_sweep"] / 1e3),
             "final_sweep_ms": ms["final_sweep"], "live_entries_final": live,
             "final_entry_updates_per_s": nnz / (ms["final_sweep"] / 1e3),
             "final_sweep_roofline": {"bound": "hbm", "achieved": alg_final / (ms["final_sweep"] / 1e3) / 1e9,
                                      "peak": HBM_PEAK, "unit": "GB/s",
                                      "frac": alg_final / (ms["final_sweep"] / 1e3) / 1e9 / HBM_PEAK,
                                      "algorithmic_bytes_per_launch": alg_final}}
        finals[name] = ([m.clone() for m in ctx.factor_masks_bool()] + [ctx.cmask.bool().clone()], hist[-1]["re"])
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        out[name] = r
        log("  %s: %d iterations, %d prune steps, sparsity %.3f, RE %.6f; dense sweep %.2f ms, final sweep %.3f ms"
            % (name, len(hist), r["prune_steps"], r["final_sparsity"], r["final_re"], ms["dense_sweep"],
               ms["final_sweep"]))
    m32, re32 = finals["fp32"]
    m64, re64 = finals["fp64"]
    out["fp32"]["vs_fp64"] = {"re_gap": abs(re32 - re64) / re64,
                              "mask_elements_differing": int(sum(int((a ^ b).sum()) for a, b in zip(m32, m64)))}
    ref, dt = sampled_rows_vs_oracle(p, 0, None, rows)
    out["oracle_sample"] = {"rows": int(rows.size), "entries": row_entries, "oracle_s": dt,
                            "oracle_entry_updates_per_s": row_entries / dt,
                            "what": "first mode-0 sweep from the initial state, sampled rows of <= 4000 entries",
                            **{name: rel_errs(first_rows[name], ref) for name in first_rows}}
    return out


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
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": entries / spent, "unit": "entry-updates/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_nproc": os.cpu_count(), "host_affinity": len(os.sched_getaffinity(0)),
            "sample": "single-threaded FP64 oracle, Alg. 4 row updates of %d randomly chosen rows "
                      "(%d observed entries, all modes) of the same workload, %.1f s" % (rows, entries, spent)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--nnz", type=int, default=None, help="smaller nnz for a quick run (not a bench line)")
    ap.add_argument("--target", type=float, default=0.95)
    ap.add_argument("--legs", default="fp64,fp32,bf16",
                    help="comma list of forms to time (the first must be fp64 for a bench line)")
    ap.add_argument("--ramp-iters", type=int, default=16,
                    help="iterations of the prune-ramp section (0 = skip it)")
    ap.add_argument("--sparse-frac", type=float, default=0.95,
                    help="marked fraction of the pruned-phase sweep section (0 = skip it)")
    ap.add_argument("--serve-jobs", type=int, default=512, help="serving stream length (0 = skip)")
    ap.add_argument("--serve-pool", type=int, default=32)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-arena-gb", type=float, default=32.0)
    ap.add_argument("--serve-calib", type=int, default=32)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--config3", type=int, default=1, help="run the 1e8-entry rating-tensor leg (BF16, L_1)")
    ap.add_argument("--config4", type=int, default=1, help="run the order-4 5e7-entry VeST^auto leg (FP32)")
    ap.add_argument("--big-steps", type=int, default=10, help="timed iterations of the 1e8-entry leg")
    ap.add_argument("--auto-iters", type=int, default=20, help="iteration cap of the VeST^auto leg")
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
    pool, futs = None, {}
    if args.config3 or args.config4:
        # inputs of the large legs drawn in worker processes while the headline runs
        from concurrent.futures import ProcessPoolExecutor
        import multiprocessing as mp
        pool = ProcessPoolExecutor(max_workers=2, mp_context=mp.get_context("spawn"))
        if args.config3:
            futs["config3"] = pool.submit(gen_workload, "rating-zipf-500k.20k.2k-nnz1e8-r10")
        if args.config4:
            futs["config4"] = pool.submit(gen_workload, "planted-zipf-50k.50k.1k.24-nnz5e7-r8")
    t0 = time.perf_counter()
    log("generating workload %s ..." % args.workload)
    p = synth.workload(args.workload, nnz=args.nnz)
    N, nnz = p["idx"].shape[1], p["idx"].shape[0]
    J = p["factors"][0].shape[1]
    log("  %.1f s: dims %s, nnz %d, ranks %d" % (time.perf_counter() - t0, [f.shape[0] for f in p["factors"]], nnz, J))
    forms = {"fp64": vest.FP64, "fp32": vest.FP32, "bf16": vest.BF16}
    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    if legs[0] != "fp64":
        # profiling runs of one low-precision form: time it, print nothing else
        for name in legs:
            ctx, r = dense_leg(p, forms[name], args.steps, args.warmup)
            ctx.close()
            log("%s: %.3f ms/step, sweep kernel %.3f ms" % (name, r["ms_per_step"], r["sweep_kernel_ms"]))
        return

    log("FP64 leg (%d + %d dense iterations) ..." % (args.warmup, args.steps))
    ctx64, f64 = dense_leg(p, vest.FP64, args.steps, args.warmup)
    log("  %.3f ms/step, sweep kernel %.3f ms, slab pass %.3f ms" % (
        f64["ms_per_step"], f64["sweep_kernel_ms"], f64["slab_kernel_ms"]))
    ref = {"re": f64["final_re"], "tensors": [f.clone() for f in ctx64.factors] + [ctx64.core.clone()]}
    log("prune step section (responsibility + one prune step on the FP64 state) ...")
    prune_step = prune_step_section(ctx64)
    ctx64.close()
    del ctx64
    lowp = {}
    for name in legs[1:]:
        log("%s leg ..." % name.upper())
        ctx, r = dense_leg(p, forms[name], args.steps, args.warmup)
        r["vs_fp64"] = compare_states(ctx, ref)
        ctx.close()
        lowp[name] = r
        log("  %.3f ms/step, sweep kernel %.3f ms; RE gap vs FP64 %.2e" % (
            r["ms_per_step"], r["sweep_kernel_ms"], r["vs_fp64"]["re_gap_vs_fp64"]))
    del ref
    torch.cuda.empty_cache()
    ramp = None
    if args.ramp_iters > 0 and len(legs) == 3:
        log("prune ramp (%d iterations, three forms in lockstep) ..." % args.ramp_iters)
        ramp = prune_ramp_section(p, args.ramp_iters, args.target)
        log("  FP64 %.3f ms/step; RE gap FP32 %.2e, BF16 %.2e; first differing masks FP32 t=%s, BF16 t=%s" % (
            ramp["fp64_ms_per_step"], ramp["fp32_re_gap_vs_fp64"], ramp["bf16_re_gap_vs_fp64"],
            ramp["fp32_first_divergent_step"], ramp["bf16_first_divergent_step"]))
    sparse = {}
    if args.sparse_frac > 0:
        for name in legs:
            log("pruned-phase sweeps (%s, %.0f %% marked) ..." % (name, 100 * args.sparse_frac))
            sparse[name] = sparse_phase(p, args.sparse_frac, min(args.steps, 10), forms[name])
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
    for f in futs.values():   # the CPU baseline runs with no input generation beside it
        f.exception()
    if args.cpu_seconds > 0:
        log("oracle CPU baseline ...")
        cpu = cpu_baseline(p, args.cpu_seconds)
    dims0, reg0, lam0 = [int(f.shape[0]) for f in p["factors"]], p["reg"], p["lam"]
    del p
    legs_big = {}
    if "config3" in futs:
        log("rating-shaped Zipf tensor, 1e8 entries (waiting for its inputs) ...")
        p3 = futs["config3"].result()
        log("  inputs drawn in %.1f s" % p3["gen_s"])
        legs_big["rating_zipf_1e8"] = rating_leg(p3, args.big_steps, 1)
        del p3
    if "config4" in futs:
        log("order-4 Zipf tensor, 5e7 entries, VeST^auto (waiting for its inputs) ...")
        p4 = futs["config4"].result()
        log("  inputs drawn in %.1f s" % p4["gen_s"])
        legs_big["order4_zipf_auto"] = order4_auto_leg(p4, args.auto_iters, 0.95)
        del p4
    if pool is not None:
        pool.shutdown()

    named = args.workload == DEFAULT_WORKLOAD and args.nnz is None
    slab_gbs = f64["slab_alg_bytes_per_launch"] / (f64["slab_kernel_ms"] / 1e3) / 1e9
    sweep_tf = f64["sweep_flops_per_launch"] / (f64["sweep_kernel_ms"] / 1e3) / 1e12
    slab_share = f64["slab_kernel_ms"] * f64["slab_launches"] / args.steps / f64["ms_per_step"]
    sweep_share = f64["sweep_kernel_ms"] * N / f64["ms_per_step"]
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
        "config": {"workload": args.workload, "dims": dims0, "nnz": nnz,
                   "ranks": [J] * N, "reg": "L_F" if reg0 == 0 else "L_1", "lambda": lam0,
                   "core": "dense", "sweeps_timed": args.steps,
                   "step": "factor sweeps (all modes) + core sweep + loss; no pruning",
                   "forms": "FP64 (value) vs FP32 / split-BF16 (keys fp32, bf16)"},
        # the kernel with the largest share of the step: the slab passes of the core sweep
        "roofline": {"kernel": "k_slab (slab pass of the core sweep)", "bound": "hbm",
                     "achieved": slab_gbs, "peak": HBM_PEAK, "unit": "GB/s", "frac": slab_gbs / HBM_PEAK,
                     "traffic": measured_traffic("slab") if named else None,
                     "algorithmic_bytes_per_launch": f64["slab_alg_bytes_per_launch"],
                     "design_bytes_per_launch": f64["slab_design_bytes_per_launch"],
                     "avg_launch_ms": f64["slab_kernel_ms"], "launches_timed": f64["slab_launches"],
                     "share_of_step": slab_share},
        "roofline_sweep": {"kernel": "k_rowgroup<OP_SWEEP> dense contraction (factor sweep, one mode)",
                           "bound": "alu", "achieved": sweep_tf, "peak": PEAK["f64"], "unit": "TFLOP/s",
                           "frac": sweep_tf / PEAK["f64"],
                           "traffic": measured_traffic("sweep") if named else None,
                           "algorithmic_bytes_per_launch": f64["sweep_alg_bytes"],
                           "flops_per_launch": f64["sweep_flops_per_launch"],
                           "avg_launch_ms": f64["sweep_kernel_ms"], "share_of_step": sweep_share},
        "cpu_baseline": cpu,
        "breakdown_ms": f64["breakdown_ms"],
        "sweep_only_value": f64["sweep_only_value"],
        "full_sweep_value": f64["full_sweep_value"],
        "core_value": f64["core_value"],
        "final_re": f64["final_re"],
        "prune_step": prune_step,
    }
    out["prune_step"]["step_with_prune_ms"] = (f64["ms_per_step"] + prune_step["responsibility_ms"]
                                               + prune_step["prune_ms"])
    for name, r in lowp.items():
        out[name] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "speedup_vs_fp64": r["value"] / f64["value"],
                     "sweep_only_value": r["sweep_only_value"], "breakdown_ms": r["breakdown_ms"],
                     "sweep_tflops": r["sweep_flops_per_launch"] / (r["sweep_kernel_ms"] / 1e3) / 1e12,
                     "slab_pass_ms": r["slab_kernel_ms"],
                     "slab_pass_alg_gbs": r["slab_alg_bytes_per_launch"] / (r["slab_kernel_ms"] / 1e3) / 1e9,
                     "accuracy_vs_fp64": r["vs_fp64"]}
    if ramp is not None:
        out["prune_ramp"] = ramp
    if sparse:
        out["pruned_phase"] = sparse
    if serving is not None:
        out["serving"] = serving
    out.update(legs_big)
    if args.nnz is not None:
        out["config"]["note"] = "reduced nnz: not the named workload"
    print(json.dumps(out))


if __name__ == "__main__":
    main()
