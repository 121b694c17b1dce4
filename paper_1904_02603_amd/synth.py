"""Seeded synthetic inputs for VeST runs (shared by tests, smoke and bench).

This module only draws numbers: observed index sets, planted-model values and
initial factors.  It imports nothing else from this package and holds none of
the factorisation arithmetic (no delta, no update rule, no responsibility);
both the GPU path and the CPU oracle consume what it returns.

Workload recipe (stand-ins for the paper's rating tensors, Sec. 4.1 Table 2,
which are not available here):
  * observed indices: per mode uniform or bounded Zipf (P(r) ~ r^-s over ranks
    1..I, inverse-CDF sampling, ranks mapped to indices by a seeded
    permutation); duplicate tuples are rejected and redrawn, so Omega is a set;
  * values: a planted Tucker model with core and factors i.i.d. N(0, 1),
    evaluated at the observed entries, plus Gaussian noise of a stated variance
    or SNR; the rating-shaped workload clips 3 + 1.25 z / sqrt(|G|) to the
    integers 1..5;
  * initial state: factors and core i.i.d. U[0, 1) (initialisation of Alg. 2).
"""
import math

import numpy as np

SEED_BASE = 20190402
THREADS = None      # worker threads of planted_values (None: up to 16)


def _zipf_sampler(I, s, rng):
    w = np.arange(1, I + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm = rng.permutation(I)

    def draw(m):
        r = np.searchsorted(cdf, rng.random(m), side="right")
        return perm[np.minimum(r, I - 1)]
    return draw


def _uniform_sampler(I, rng):
    def draw(m):
        return rng.integers(0, I, size=m)
    return draw


def observed_indices(dims, nnz, rng, zipf=None):
    """nnz distinct index tuples, shape [nnz, N] int32, in draw order."""
    N = len(dims)
    total = 1
    for d in dims:
        total *= int(d)
    if nnz > total:
        raise ValueError("nnz exceeds the number of cells")
    zipf = zipf or [None] * N
    samplers = [(_zipf_sampler(dims[n], zipf[n], rng) if zipf[n] else _uniform_sampler(dims[n], rng))
                for n in range(N)]
    linear = total < 2 ** 62
    if linear:
        # rounds of draws; a round keeps its first occurrences that are not
        # already taken, in draw order (taken keys kept sorted for lookup)
        parts, taken, count = [], np.empty(0, dtype=np.int64), 0
        while count < nnz:
            need = nnz - count
            draw = int(need * 1.05) + 64
            cand = np.stack([samplers[n](draw) for n in range(N)], axis=1).astype(np.int64)
            key = np.zeros(draw, dtype=np.int64)
            for n in range(N):
                key = key * int(dims[n]) + cand[:, n]
            _, first = np.unique(key, return_index=True)
            first.sort()
            kc = key[first]
            pos = np.searchsorted(taken, kc)
            seen = (pos < taken.shape[0]) & (taken[np.minimum(pos, max(taken.shape[0] - 1, 0))] == kc) \
                if taken.shape[0] else np.zeros(kc.shape[0], dtype=bool)
            new = first[~seen][:need]
            parts.append(cand[new])
            count += new.shape[0]
            tk = np.sort(key[new])
            taken = np.insert(taken, np.searchsorted(taken, tk), tk)
        got = np.concatenate(parts, axis=0)
    else:
        got = np.empty((0, N), dtype=np.int64)
        while got.shape[0] < nnz:
            need = nnz - got.shape[0]
            draw = int(need * 1.05) + 64
            cand = np.stack([samplers[n](draw) for n in range(N)], axis=1).astype(np.int64)
            allt = np.concatenate([got, cand], axis=0)
            _, first = np.unique(allt, axis=0, return_index=True)
            first.sort()
            got = allt[first][:nnz]
    return np.ascontiguousarray(got, dtype=np.int32)


def planted_values(idx, core, factors, chunk=1 << 17, threads=None):
    """Planted model value at every observed entry (Tucker model, Sec. 2.2).

    Evaluated by contracting the core with one factor row per mode, last mode
    first, with numpy tensordot on chunks of entries.  Chunks are independent
    and computed the same way whichever thread takes them, so the values do
    not depend on the thread count.
    """
    import os
    from concurrent.futures import ThreadPoolExecutor
    N = idx.shape[1]
    out = np.empty(idx.shape[0], dtype=np.float64)

    def one(s):
        sl = idx[s:s + chunk]
        m = sl.shape[0]
        t = np.broadcast_to(core, (m,) + core.shape)
        for n in range(N - 1, -1, -1):
            rows = factors[n][sl[:, n]]                     # [m, J_n]
            t = np.einsum("m...j,mj->m...", t, rows)
        out[s:s + chunk] = t

    starts = range(0, idx.shape[0], chunk)
    nt = threads or THREADS or min(16, os.cpu_count() or 1)
    if nt > 1 and len(starts) > 1:
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(one, starts))
    else:
        for s in starts:
            one(s)
    return out


def planted_model(ranks, dims, rng):
    core = rng.standard_normal(tuple(ranks))
    factors = [rng.standard_normal((dims[n], ranks[n])) for n in range(len(dims))]
    return core, factors


def initial_state(dims, ranks, rng):
    """Factors and core i.i.d. U[0, 1) (initialisation of Alg. 2)."""
    factors = [rng.random((dims[n], ranks[n])) for n in range(len(dims))]
    core = rng.random(tuple(ranks))
    return factors, core


def make_problem(dims, nnz, ranks, seed, zipf=None, planted_ranks=None,
                 noise_var=None, snr_db=None, rating=False):
    """Observed tensor plus an initial state.

    Returns dict(idx, val, factors, core, planted=(core, factors)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = observed_indices(dims, nnz, rng, zipf)
    pr = planted_ranks or ranks
    pcore, pfac = planted_model(pr, dims, rng)
    z = planted_values(idx, pcore, pfac)
    if rating:
        g = 1
        for r in pr:
            g *= r
        val = np.clip(np.rint(3.0 + 1.25 * z / math.sqrt(g)), 1.0, 5.0)
    else:
        val = z.copy()
        if noise_var is not None:
            val += rng.standard_normal(z.shape[0]) * math.sqrt(noise_var)
        elif snr_db is not None:
            var = float(np.mean(z * z)) / (10.0 ** (snr_db / 10.0))
            val += rng.standard_normal(z.shape[0]) * math.sqrt(var)
    factors, core = initial_state(dims, ranks, rng)
    return {"idx": idx, "val": val, "factors": factors, "core": core,
            "planted": (pcore, pfac)}


# Workloads.  Sizes follow the configurations the method is exercised on:
#  1: 100^3, 1e4 entries, core 5^3, planted + N(0, 0.01) noise, L_F 0.01, FP64
#  2: (1e5)^3, 1e7 entries, core 10^3, planted, SNR 20 dB, L_F 0.01
#  3: 500k x 20k x 2k, Zipf 1.1 / 1.0 / uniform, 1e8 entries, ratings 1..5, L_1 0.1
#  4: 50k x 50k x 1000 x 24, Zipf 1.1 / 1.0, 5e7 entries, core 8^4, SNR 20 dB
WORKLOADS = {
    "planted-100^3-nnz1e4-r5": dict(dims=(100, 100, 100), nnz=10_000, ranks=(5, 5, 5),
                                    noise_var=0.01, reg=0, lam=0.01, seed=SEED_BASE + 1),
    "planted-1e5^3-nnz1e7-r10": dict(dims=(100_000,) * 3, nnz=10_000_000, ranks=(10, 10, 10),
                                     snr_db=20.0, reg=0, lam=0.01, seed=SEED_BASE + 2),
    "rating-zipf-500k.20k.2k-nnz1e8-r10": dict(dims=(500_000, 20_000, 2_000), nnz=100_000_000,
                                               ranks=(10, 10, 10), zipf=(1.1, 1.0, None),
                                               rating=True, reg=1, lam=0.1, seed=SEED_BASE + 3),
    "planted-zipf-50k.50k.1k.24-nnz5e7-r8": dict(dims=(50_000, 50_000, 1_000, 24), nnz=50_000_000,
                                                 ranks=(8, 8, 8, 8), zipf=(1.1, 1.0, None, None),
                                                 snr_db=20.0, reg=0, lam=0.01, seed=SEED_BASE + 4),
}


# Serving workload: ranks with a compiled kernel instance in 4..10 per order.
SERVING_RANKS = {3: (4, 5, 6, 7, 8, 9, 10), 4: (4, 5, 6, 7, 8, 9, 10)}


def rating_values(idx, dims, rng):
    """Cheap rating-shaped values for the serving stream: integers 1..5 from
    clip(rint(3 + 1.25 z)), z = sum of per-mode N(0, 1/N) effects of the entry's
    indices plus N(0, 0.25) noise (O(nnz N) to draw, unlike a planted Tucker
    model)."""
    N = len(dims)
    z = rng.standard_normal(idx.shape[0]) * 0.5
    for n in range(N):
        eff = rng.standard_normal(int(dims[n])) / math.sqrt(N)
        z += eff[idx[:, n]]
    return np.clip(np.rint(3.0 + 1.25 * z), 1.0, 5.0)


def serving_tensor(k, seed=SEED_BASE + 5, max_nnz=10_000_000):
    """Observed tensor k of the serving pool (own seeded generator, so the
    pool can be drawn in parallel): order 3 or 4 with equal probability,
    every dim log-uniform in [1e3, 1e5], nnz log-uniform in [1e4, max_nnz]
    capped at half the cells, first two modes bounded Zipf 1.0 and the others
    uniform, rating values (rating_values)."""
    rng = np.random.Generator(np.random.PCG64([seed, k]))
    N = 3 if rng.random() < 0.5 else 4
    dims = [int(round(10 ** rng.uniform(3, 5))) for _ in range(N)]
    cells = 1
    for d in dims:
        cells *= d
    nnz = int(round(10 ** rng.uniform(4, math.log10(max_nnz))))
    nnz = max(1, min(nnz, cells // 2))
    idx = observed_indices(dims, nnz, rng, [1.0, 1.0] + [None] * (N - 2))
    return {"idx": idx, "val": rating_values(idx, dims, rng), "dims": dims}


def serving_jobs(n_jobs, tensors, seed=SEED_BASE + 6):
    """Parameters of the serving job stream over a pool of tensors: each job
    draws a tensor, ranks uniform over SERVING_RANKS[N], L_F / L_1 with equal
    probability (lambda 0.01 / 0.1), FP32 / BF16 form with equal
    probability, 10 iterations, and a seed for its U[0, 1) initial state
    (serving_init).  The BF16 form differs from the FP32 form only in the
    order-3 factor sweep (matrix cores), so an order-4 job that draws BF16 is
    labelled and run as FP32.  Every job prunes with probability 1/2 (VeST^man
    toward 0.95, Sec. 3.3; the flag comes from a generator of its own, so the
    rest of the stream is unchanged by it)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rng_p = np.random.Generator(np.random.PCG64(seed + 1))
    jobs = []
    for i in range(n_jobs):
        k = int(rng.integers(0, len(tensors)))
        N = len(tensors[k]["dims"])
        J = int(rng.choice(SERVING_RANKS[N]))
        reg = int(rng.integers(0, 2))
        jobs.append({"tensor": k, "ranks": (J,) * N, "reg": reg, "lam": 0.01 if reg == 0 else 0.1,
                     "form": "FP32" if (rng.random() < 0.5 or N != 3) else "BF16", "iterations": 10,
                     "init_seed": (seed, i), "prune_target": 0.95 if rng_p.random() < 0.5 else 0.0})
    return jobs


def serving_init(job, dims):
    """U[0, 1) initial factors and core of a serving job."""
    return initial_state(dims, job["ranks"], np.random.Generator(np.random.PCG64(list(job["init_seed"]))))


def scaling_problem(order, dim, nnz, seed=SEED_BASE + 7, rank=3):
    """Synthetic tensor of the scalability runs (Sec. 4, Fig. 4a-c): every mode
    of size `dim`, ranks `rank`, `nnz` distinct entries drawn uniformly, values
    U[0, 1), initial state U[0, 1).  Distinctness: by flat index when the index
    space fits in 62 bits, otherwise by giving every entry its own mode-0 index
    (a seeded permutation; needs nnz <= dim)."""
    rng = np.random.default_rng(seed)
    N = int(order)
    if N * math.log2(max(dim, 2)) <= 62:
        total = dim ** N
        if nnz > total:
            raise ValueError("more entries than cells")
        flat = np.unique(rng.integers(0, total, size=nnz, dtype=np.int64))
        while flat.size < nnz:
            more = rng.integers(0, total, size=nnz - flat.size, dtype=np.int64)
            flat = np.unique(np.concatenate([flat, more]))
        flat = rng.permutation(flat)
        idx = np.empty((nnz, N), dtype=np.int32)
        for n in range(N - 1, -1, -1):
            idx[:, n] = flat % dim
            flat //= dim
    else:
        if nnz > dim:
            raise ValueError("distinct entries by mode-0 index need nnz <= dim")
        idx = np.empty((nnz, N), dtype=np.int32)
        idx[:, 0] = rng.permutation(dim)[:nnz]
        for n in range(1, N):
            idx[:, n] = rng.integers(0, dim, size=nnz, dtype=np.int32)
    val = rng.random(nnz)
    factors = [rng.random((dim, rank)) for _ in range(N)]
    core = rng.random((rank,) * N)
    return {"idx": idx, "val": val, "factors": factors, "core": core, "reg": 0, "lam": 0.01}


def workload(name, nnz=None, dims=None):
    """Build a named workload (optionally with a smaller nnz / dims)."""
    w = dict(WORKLOADS[name])
    if nnz is not None:
        w["nnz"] = nnz
    if dims is not None:
        w["dims"] = dims
    reg, lam = w.pop("reg"), w.pop("lam")
    p = make_problem(**w)
    p["reg"], p["lam"] = reg, lam
    return p
