"""GPU checks of the request loop (vest_serve.h).

Jobs of different order, rank, regulariser and precision run through one
server with fewer slots than jobs, so some wait and the admitted ones overlap
on the device, jobs of one shape in batched iterations (vest_iterate_many);
each result must equal bit for bit the same job run alone through the plain
context (every kernel sums in a fixed order and the batched kernels run the
same per-job arithmetic, so the mix cannot change a result).  Served results
are checked against the oracle (FP64 at the FP64 bar, FP32 / split-BF16
within 1e-4 relative RE and factor RMSE).  Jobs with a VeST^man prune target
(Sec. 3.3) end where the same schedule on a plain context ends, bit for bit,
and an FP64 one where the oracle ends.  The arena bound, the rejection of a
job larger than the arena and the failure of a job with invalid data are
checked as well.
"""
import time

import numpy as np
import pytest
import torch

from paper_1904_02603_amd import synth
from test_gpu_parity import V, say

pytestmark = pytest.mark.gpu

JOBS = [
    # dims, ranks, nnz, zipf, reg, lam, precision
    ((100, 80, 60), 5, 5000, None, 0, 0.05, "FP32"),
    ((300, 200, 100), 10, 30_000, None, 1, 0.5, "BF16"),
    ((30, 25, 20, 24), 8, 5000, None, 0, 0.05, "FP32"),
    ((2000, 300, 50), 4, 30_000, (1.1, 1.0, None), 1, 0.5, "FP64"),
    ((40, 50, 30), 3, 2000, None, 0, 0.05, "BF16"),
    ((12, 10, 8, 9), 3, 3000, None, 0, 0.1, "FP64"),
]


def job_inputs(k):
    dims, J, nnz, zipf, reg, lam, prec = JOBS[k]
    p = synth.make_problem(dims, nnz, (J,) * len(dims), 60 + k, zipf=zipf, noise_var=0.01)
    return p, reg, lam, getattr(V(), prec)


def drain(srv, ids, limit_s=120.0):
    t0 = time.time()
    peak = {"active": 0, "bytes": 0}
    while True:
        srv.progress()
        st = srv.stats()
        peak["active"] = max(peak["active"], st["active"])
        peak["bytes"] = max(peak["bytes"], st["bytes_used"])
        assert st["bytes_used"] <= st["bytes_total"]
        if all(srv.status(i)["state"] >= V().JOB_DONE for i in ids):
            return peak
        assert time.time() - t0 < limit_s, "server did not finish"
        time.sleep(0.0005)


def alone(p, reg, lam, prec, iters):
    ctx = V().VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec)
    for _ in range(iters):
        ctx.iteration()
    L = ctx.loss()
    torch.cuda.synchronize()
    out = ([f.cpu().numpy().copy() for f in ctx.factors], ctx.core.cpu().numpy().copy(), L)
    ctx.close()
    return out


def test_results_in_the_mix_equal_results_alone():
    v = V()
    iters = 3
    srv = v.VestServer(1 << 30, 3)
    ins = [job_inputs(k) for k in range(len(JOBS))]
    ids = [srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec,
                      iterations=iters) for p, reg, lam, prec in ins]
    peak = drain(srv, ids)
    st = srv.stats()
    say("peak active", peak["active"], "batches", st["batches"], "batched job-iterations",
        st["batched_job_iterations"])
    assert peak["active"] >= 2  # jobs overlapped
    assert st["batched_job_iterations"] == iters * len(JOBS)   # every iteration ran batched
    for k, (jid, (p, reg, lam, prec)) in enumerate(zip(ids, ins)):
        st = srv.status(jid)
        assert st["state"] == v.JOB_DONE, (k, st)
        assert st["arrive"] <= st["admit"] <= st["done"]
        fac, core, loss = srv.fetch(jid)
        afac, acore, aloss = alone(p, reg, lam, prec, iters)
        for n in range(len(fac)):
            assert np.array_equal(fac[n], afac[n]), (k, n)
        assert np.array_equal(core, acore), k
        assert loss["loss"] == aloss["loss"] and loss["re"] == aloss["re"], k
    srv.close()


def test_admission_keeps_the_arena_bound():
    v = V()
    p, reg, lam, prec = job_inputs(1)
    dims = [f.shape[0] for f in p["factors"]]
    fp = v.job_footprint(dims, [10] * 3, p["idx"].shape[0], reg, lam, prec)
    srv = v.VestServer(int(2.5 * fp), 8)   # room for two jobs at a time
    ids = [srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec,
                      iterations=2) for _ in range(5)]
    peak = drain(srv, ids)
    say("footprint", fp, "peak active", peak["active"], "peak bytes", peak["bytes"])
    assert peak["active"] <= 2
    res = [srv.fetch(i) for i in ids]
    for f, c, L in res[1:]:
        assert np.array_equal(c, res[0][1]) and L["loss"] == res[0][2]["loss"]
    srv.close()


def test_oversized_and_invalid_jobs():
    v = V()
    p, reg, lam, prec = job_inputs(4)
    dims = [f.shape[0] for f in p["factors"]]
    fp = v.job_footprint(dims, [3] * 3, p["idx"].shape[0], reg, lam, prec)
    srv = v.VestServer(fp // 2, 2)
    with pytest.raises(v.VestError) as ei:
        srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec)
    assert ei.value.code == v.ENOSPC
    srv.close()
    srv = v.VestServer(4 * fp, 2)
    bad = p["idx"].copy()
    bad[1] = bad[0]  # duplicate index tuple
    jb = srv.submit(bad, p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec, iterations=1)
    jg = srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec, iterations=1)
    drain(srv, [jb, jg])
    assert srv.status(jb)["state"] == v.JOB_FAILED and srv.status(jb)["error"] == v.EINVAL
    assert srv.status(jg)["state"] == v.JOB_DONE
    with pytest.raises(v.VestError) as ei:
        srv.fetch(jb)
    assert ei.value.code == v.ESTATE
    srv.fetch(jg)
    assert srv.stats()["bytes_used"] == 0
    srv.close()


def test_served_jobs_match_oracle():
    from oracle.oracle import Oracle
    from test_gpu_parity import rel_err, rms_err
    v = V()
    iters = 3
    picks = [0, 1, 2, 3, 0]   # FP32, BF16, FP32 order 4, FP64 Zipf; a second FP32 job of the first shape
    ins = [job_inputs(k) for k in picks]
    srv = v.VestServer(1 << 30, 8)
    ids = [srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec,
                      iterations=iters) for p, reg, lam, prec in ins]
    drain(srv, ids)
    for jid, (p, reg, lam, prec) in zip(ids, ins):
        fac, core, loss = srv.fetch(jid)
        o = Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam)
        for _ in range(iters):
            o.iteration()
        ol = o.loss()
        gap = abs(loss["re"] - ol["re"]) / ol["re"]
        fr = max(rms_err(f, of) for f, of in zip(fac, o.factors))
        say(prec, "served: RE gap %.2e, factor rel RMSE %.2e" % (gap, fr))
        if prec == v.FP64:
            for f, of in zip(fac, o.factors):
                assert rel_err(f, of) <= 1e-10
            assert rel_err(core, o.core) <= 1e-10
        else:
            assert gap <= 1e-4 and fr <= 1e-4
    srv.close()


PRUNE_JOBS = [
    # job index in JOBS, iterations, prune target (VeST^man)
    (0, 8, 0.6),     # FP32, order 3
    (2, 6, 0.5),     # FP32, order 4
    (1, 10, 0.9),    # split-BF16, rank 10, L_1
    (5, 6, 0.7),     # FP64, order 4
]


def pruned_alone(p, reg, lam, prec, iters, target):
    """The server's VeST^man on a plain context: iteration t, then (t below
    the last iteration, marked fraction below the target) keys and one prune
    step with the counts of the host schedule."""
    from paper_1904_02603_amd.schedule import PruneSchedule
    v = V()
    sched = PruneSchedule(mode="manual", target=target)
    ctx = v.VestContext(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec)
    total = ctx.core.numel() + sum(f.numel() for f in ctx.factors)
    steps = 0
    for t in range(1, iters + 1):
        ctx.iteration()
        if t < iters:
            fm, cm = ctx.marked_counts()
            if cm + sum(fm) < target * total:
                ctx.responsibility()
                ctx.prune(sched.count(t, ctx.core.numel(), cm),
                          [sched.count(t, f.numel(), m) for f, m in zip(ctx.factors, fm)])
                steps += 1
    L = ctx.loss()
    torch.cuda.synchronize()
    out = ([f.cpu().numpy().copy() for f in ctx.factors], ctx.core.cpu().numpy().copy(), L, steps)
    ctx.close()
    return out


def test_served_pruning_equals_plain_context():
    """Jobs with a VeST^man target, mixed with plain jobs in one server, end
    bit for bit where the same schedule run on a plain context ends."""
    v = V()
    srv = v.VestServer(1 << 30, 3)
    ins = [job_inputs(k) for k, _, _ in PRUNE_JOBS]
    ids = [srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec,
                      iterations=it, prune_target=tg)
           for (p, reg, lam, prec), (_, it, tg) in zip(ins, PRUNE_JOBS)]
    plain = [job_inputs(k) for k in (3, 4)]
    ids += [srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec, iterations=3)
            for p, reg, lam, prec in plain]
    drain(srv, ids)
    for jid, (p, reg, lam, prec), (k, it, tg) in zip(ids, ins, PRUNE_JOBS):
        assert srv.status(jid)["state"] == v.JOB_DONE, (k, srv.status(jid))
        fac, core, loss = srv.fetch(jid)
        afac, acore, aloss, steps = pruned_alone(p, reg, lam, prec, it, tg)
        zeros = (sum(int((f == 0).sum()) for f in fac) + int((core == 0).sum())) / (
            sum(f.size for f in fac) + core.size)
        say("job %d: %d prune steps, zeros %.3f, RE %.6f" % (k, steps, zeros, loss["re"]))
        assert steps >= 2
        for n in range(len(fac)):
            assert np.array_equal(fac[n], afac[n]), (k, n)
        assert np.array_equal(core, acore), k
        assert loss["loss"] == aloss["loss"] and loss["re"] == aloss["re"], k
    for jid in ids[len(PRUNE_JOBS):]:
        assert srv.status(jid)["state"] == v.JOB_DONE
    srv.close()


def test_served_fp64_pruning_matches_oracle():
    from oracle.oracle import Oracle
    from paper_1904_02603_amd.schedule import PruneSchedule
    from test_gpu_parity import rel_err
    v = V()
    p, reg, lam, prec = job_inputs(5)    # FP64, order 4
    iters, target = 6, 0.7
    srv = v.VestServer(1 << 30, 2)
    jid = srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec,
                     iterations=iters, prune_target=target)
    drain(srv, [jid])
    fac, core, loss = srv.fetch(jid)
    srv.close()
    o = Oracle(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam)
    sched = PruneSchedule(mode="manual", target=target)
    total = o.core.size + sum(f.size for f in o.factors)
    for t in range(1, iters + 1):
        o.iteration()
        marked = int(o.cmask.sum()) + sum(int(m.sum()) for m in o.fmask)
        if t < iters and marked < target * total:
            ck, fk = o.responsibility()
            o.prune(ck, fk, sched.count(t, o.core.size, int(o.cmask.sum())),
                    [sched.count(t, f.size, int(m.sum())) for f, m in zip(o.factors, o.fmask)])
    for f, of in zip(fac, o.factors):
        assert np.array_equal(f == 0, of == 0)
        assert rel_err(f, of) <= 1e-10
    assert np.array_equal(core == 0, o.core == 0)
    assert rel_err(core, o.core) <= 1e-10
    ol = o.loss()
    assert abs(loss["re"] - ol["re"]) <= 1e-10 * ol["re"]


def test_pruning_job_arguments():
    v = V()
    p, reg, lam, prec = job_inputs(0)
    srv = v.VestServer(1 << 28, 2)
    for bad in (-0.1, 1.0):
        with pytest.raises(v.VestError) as ei:
            srv.submit(p["idx"], p["val"], p["factors"], p["core"], reg=reg, lam=lam, precision=prec,
                       prune_target=bad)
        assert ei.value.code == v.EINVAL
    q = synth.make_problem((50, 40, 30), 3000, (4, 3, 5), 7, noise_var=0.01)
    with pytest.raises(v.VestError) as ei:   # unequal ranks
        srv.submit(q["idx"], q["val"], q["factors"], q["core"], prune_target=0.5)
    assert ei.value.code == v.EINVAL
    srv.close()
