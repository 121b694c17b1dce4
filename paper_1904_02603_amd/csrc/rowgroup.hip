// Row-group kernels over the per-mode layout of Omega:
//   OP_SWEEP  one pass of Alg. 4 for mode n (factor update, Eq. 9 / Eq. 13)
//   OP_KEYS   factor responsibility keys of mode n (Eq. 6)
//   OP_RESID  residual e = X - B over the core layout (Eq. 7, Alg. 3)
//
// One lane owns a slice of one row of mode n.  For every observed entry of
// the slice it gathers the N-1 other-mode factor rows, forms delta_alpha
// (Eq. 11) with the core operands streamed as wave-uniform scalar loads, and
// accumulates the row statistics in registers:
//   OP_SWEEP: c_j = sum X delta(j), V_jt = sum delta(j) delta(t)  (Eq. 9, 10)
//   OP_KEYS : s_j = sum e delta(j), q_j = sum delta(j)^2, with the residual
//             e = X - a^(n)_{i_n} . delta recomputed from the same delta
// The lanes of a row group are then summed by an xor butterfly and one lane
// runs the FP64 row epilogue.  Because delta does not depend on A^(n), the
// statistics are formed once per row and the Gauss-Seidel pass over j
// (ascending, skipping pruned elements) runs on them; rows are independent.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "internal.h"

namespace vest {

template <int N, int J, typename T>
struct RowArgs {
    const WaveInfo *waves;
    int32_t nwaves;
    int32_t reg;
    double lambda;
    const int32_t *row_order;
    const int32_t *oidx[N - 1];
    const T *xval;
    const T *fac[N - 1];      // other modes, ascending, compute type
    const uint32_t *omask[N - 1];  // their marking tables (gather form)
    T *Ag;                    // mode-n gather copy (stride gather_ld): own rows; OP_SWEEP refreshes it
    double *A;                // mode-n FP64 factor
    const uint32_t *mask;     // mode-n marking table
    double *partials;         // long-row chunk partials
    T *e;                     // OP_RESID: out
    T *ms;                    // OP_RESID: out, mode N-2 factor row of every slot (see ms_index)
    double *keys;             // OP_KEYS: out [I_n * J]
    double *rowbuf;           // OP_RESID_S0: per-row statistics of the first slab
    int32_t ldrb;
    const T *gt;              // gather form, staging outside LDS: core [o][j] ...
    const uint32_t *gnz;      // ... and its nonzero-column bits
};

template <int J, int OP>
__host__ __device__ constexpr int row_nacc() { return OP == OP_KEYS ? 2 * J : nacc_vc(J); }   // (OP_RESID: unused)

// FP64 epilogue of one row given its summed statistics s.
template <int N, int J, typename T, int OP, typename S>
__device__ __forceinline__ void row_epilogue(const RowArgs<N, J, T> &a, int row, const S (&s)[row_nacc<J, OP>()])
{
    double av[J];
    load_row<J, double>(a.A + (int64_t)row * J, av);
    const uint32_t mk = a.mask[row];
    if constexpr (OP == OP_SWEEP) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if ((mk >> j) & 1u) continue;
            double r = (double)s[j];
#pragma unroll
            for (int t = 0; t < J; ++t)
                if (t != j) r -= (double)s[J + sym<J>(j, t)] * av[t];
            av[j] = coord_min(a.reg, a.lambda, r, (double)s[J + sym<J>(j, j)]);
        }
        double *dst = a.A + (int64_t)row * J;
#pragma unroll
        for (int j = 0; j < J; ++j) dst[j] = av[j];
        T *dg = a.Ag + (int64_t)row * gather_ld(J, sizeof(T));
#pragma unroll
        for (int j = 0; j < J; ++j) dg[j] = (T)av[j];
    } else {
        // Delta(a_ij) = sum (2 e + a delta_j) a delta_j = 2 a s_j + a^2 q_j
        double *dst = a.keys + (int64_t)row * J;
#pragma unroll
        for (int j = 0; j < J; ++j)
            dst[j] = ((mk >> j) & 1u) ? HUGE_VAL : 2.0 * av[j] * (double)s[j] + av[j] * av[j] * (double)s[J + j];
    }
}

// Pruned-phase contraction (Eq. 11 restricted to nonzero terms).  The core
// is staged in LDS with the mode-n index innermost, Gt[(o_0 .. o_{N-2}) J + j]
// (o_m = index of the m-th other mode), plus one bit per core column
// (o_0 .. o_{N-2}) that has a nonzero value.  Each lane walks only the
// combinations of nonzero values of its entry's other-mode rows whose core
// column is nonzero, so the work per entry is proportional to the number of
// surviving terms instead of J^N.
// Up to order 4 the walk carries the running product w of the chosen factor
// values down to the last level and adds w * r * G into d (at most J^3 terms
// per sum).  From order 5 it is factored: level L returns the partial sum over
// its subtree, d_L[j] = sum_b r[L][b] d_{L+1}(b)[j], so that no floating-point
// sum has more than J terms (one running sum over the J^(N-1) columns of a
// high-order core loses accuracy with its length).
template <int L, int N, int J, typename T>
__device__ __forceinline__ void gather_level(const T *__restrict__ Gt, const uint32_t *__restrict__ Gnz,
                                             const T (&r)[N - 1][J], const uint32_t (&m)[N - 1], T w, int o,
                                             T (&d)[J])
{
    uint32_t bits = m[L];
    while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1;
        const T v = w * pick<J, T>(r[L], b);
        const int oo = o * J + b;
        if constexpr (L == N - 2) {
            if ((Gnz[oo >> 5] >> (oo & 31)) & 1u) {
                const T *g = Gt + oo * J;
#pragma unroll
                for (int j = 0; j < J; ++j) d[j] = vfma(v, g[j], d[j]);
            }
        } else {
            gather_level<L + 1, N, J, T>(Gt, Gnz, r, m, v, oo, d);
        }
    }
}

template <int L, int N, int J, typename T>
__device__ __forceinline__ void gather_level_factored(const T *__restrict__ Gt, const uint32_t *__restrict__ Gnz,
                                                      const T (&r)[N - 1][J], const uint32_t (&m)[N - 1], int o,
                                                      T (&d)[J])
{
#pragma unroll
    for (int j = 0; j < J; ++j) d[j] = T(0);
    uint32_t bits = m[L];
    while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1;
        const T x = pick<J, T>(r[L], b);
        const int oo = o * J + b;
        if constexpr (L == N - 2) {
            if ((Gnz[oo >> 5] >> (oo & 31)) & 1u) {
                const T *g = Gt + oo * J;
#pragma unroll
                for (int j = 0; j < J; ++j) d[j] = vfma(x, g[j], d[j]);
            }
        } else {
            T sub[J];
            gather_level_factored<L + 1, N, J, T>(Gt, Gnz, r, m, oo, sub);
#pragma unroll
            for (int j = 0; j < J; ++j) d[j] = vfma(x, sub[j], d[j]);
        }
    }
}

// delta of one entry in the gather form, given the unmarked-element bits
// m[k] of its other-mode rows (from the marking tables, one 32-bit word per
// row, small enough to stay in L2): the factor rows are fetched only when
// every other-mode row still has an unmarked element, otherwise delta = 0
// without touching them.
template <int N, int J, typename T>
__device__ __forceinline__ void delta_gather(const T *__restrict__ Gt, const uint32_t *__restrict__ Gnz,
                                             const T *const (&fac)[N - 1], const int32_t (&ii)[N - 1],
                                             const uint32_t (&mk)[N - 1], T (&r)[N - 1][J], T (&d)[J])
{
#pragma unroll
    for (int j = 0; j < J; ++j) d[j] = T(0);
    uint32_t m[N - 1];
    bool live = true;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        m[k] = mk[k];
        live = live && m[k] != 0u;
    }
    if (!live) return;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        load_grow<J, T>(fac[k] + (int64_t)ii[k] * gather_ld(J, sizeof(T)), r[k]);
        uint32_t b = 0;
#pragma unroll
        for (int t = 0; t < J; ++t) b |= (r[k][t] != T(0) ? 1u : 0u) << t;
        m[k] &= b;
    }
    if constexpr (N <= 4)
        gather_level<0, N, J, T>(Gt, Gnz, r, m, T(1), 0, d);
    else
        gather_level_factored<0, N, J, T>(Gt, Gnz, r, m, 0, d);
}

template <int N, int J, typename T>
__host__ __device__ constexpr size_t gather_lds_bytes()
{
    return gather_in_lds(N, J, (int)sizeof(T)) ? gather_stage_bytes(N, J, (int)sizeof(T)) : 0;
}

// Block-cooperative staging of the mode-permuted core Gp ([j][o], row-major)
// into Gt ([o][j]) and the nonzero-column bits.
template <int N, int J, typename T>
__device__ __forceinline__ void stage_core(const T *__restrict__ Gp, T *Gt, uint32_t *Gnz)
{
    constexpr int S = ipow(J, N - 1);
    constexpr int NW = (S + 31) / 32;
    for (int q = threadIdx.x; q < NW; q += blockDim.x) Gnz[q] = 0u;
    for (int q = threadIdx.x; q < S * J; q += blockDim.x) {
        const int j = q / S, o = q % S;
        Gt[o * J + j] = Gp[q];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < S; o += blockDim.x) {
        bool nz = false;
#pragma unroll
        for (int j = 0; j < J; ++j) nz |= Gt[o * J + j] != T(0);
        if (nz) atomicOr(&Gnz[o >> 5], 1u << (o & 31));
    }
    __syncthreads();
}

// Gather-form staging in the workspace for cores that exceed LDS: one block.
template <int N, int J, typename T>
__global__ void __launch_bounds__(1024) k_stage_core(const T *__restrict__ Gp, T *Gt, uint32_t *Gnz)
{
    stage_core<N, J, T>(Gp, Gt, Gnz);
}

// Dense OP_KEYS / OP_RESID steps, two entries per lane at a time (steps k
// and k + 1 of the lane's slice): one pass over the core operands serves both
// contractions (delta_vec2).  Padding slots and the missing partner of an odd
// last step are computed on row 0 and masked out of the results by selects;
// the statistics take the entries in slot order, as the one-entry loop does.
// The indices and values of the next pair are loaded ahead.
template <int N, int J, typename T, int OP>
__device__ __forceinline__ void pair_steps(const RowArgs<N, J, T> &a, const CoreBases<T> &Gb, const WaveInfo &wi,
                                           int lane, const T (&own)[J], T (&s)[row_nacc<J, OP>()])
{
    const int K = OP == OP_KEYS ? wi.klive : wi.K;   // keys: live entries only (the rest add zero)
    int32_t ia[N - 1], ib[N - 1];
    T xa = T(0), xb = T(0);
    auto load_pair = [&](int k, int32_t (&i0)[N - 1], T &x0, int32_t (&i1)[N - 1], T &x1) {
        const int64_t s0 = wi.base + (int64_t)(k < K ? k : K - 1) * kWave + lane;
        const int64_t s1 = wi.base + (int64_t)(k + 1 < K ? k + 1 : K - 1) * kWave + lane;
#pragma unroll
        for (int m = 0; m < N - 1; ++m) {
            i0[m] = ld_stream(a.oidx[m] + s0);
            i1[m] = ld_stream(a.oidx[m] + s1);
        }
        x0 = ld_stream(a.xval + s0);
        x1 = ld_stream(a.xval + s1);
    };
    if (K > 0) load_pair(0, ia, xa, ib, xb);
#pragma unroll 1
    for (int k = 0; k < K; k += 2) {
        const int64_t sla = wi.base + (int64_t)k * kWave + lane;
        const int64_t slb = sla + kWave;
        const bool hb = k + 1 < K;
        int32_t na[N - 1], nb[N - 1];
        T nxa, nxb;
        load_pair(k + 2, na, nxa, nb, nxb);
        const bool oka = ia[0] >= 0, okb = hb && ib[0] >= 0;
        T ra[N - 1][J], rb[N - 1][J];
#pragma unroll
        for (int m = 0; m < N - 1; ++m) {
            load_grow<J, T>(a.fac[m] + (int64_t)(oka ? ia[m] : 0) * gather_ld(J, sizeof(T)), ra[m]);
            load_grow<J, T>(a.fac[m] + (int64_t)(okb ? ib[m] : 0) * gather_ld(J, sizeof(T)), rb[m]);
        }
        T da[J], db[J];
        CoreBases<T> G = Gb;
        core_fence<N, J, T>(G);
        delta_vec2<N, J, T>(G, ra, rb, da, db);
        T ba = own[0] * da[0], bb = own[0] * db[0];
#pragma unroll
        for (int t = 1; t < J; ++t) {
            ba = vfma(own[t], da[t], ba);
            bb = vfma(own[t], db[t], bb);
        }
        const T ea = oka ? xa - ba : T(0), eb = okb ? xb - bb : T(0);
        if constexpr (OP == OP_KEYS) {
#pragma unroll
            for (int t = 0; t < J; ++t) {
                const T ua = oka ? da[t] : T(0), ub = okb ? db[t] : T(0);
                s[t] = vfma(ea, ua, s[t]);
                s[t] = vfma(eb, ub, s[t]);
                s[J + t] = vfma(ua, ua, s[J + t]);
                s[J + t] = vfma(ub, ub, s[J + t]);
            }
        } else {
            // without a partner the second store repeats the first (same
            // lane, same values), so both contractions stay unconditional
            const int64_t slc = hb ? slb : sla;
            st_stream(ea, a.e + sla);
            st_stream(hb ? eb : ea, a.e + slc);
            T wa[J], wc[J];
#pragma unroll
            for (int t = 0; t < J; ++t) {
                wa[t] = oka ? ra[N - 2][t] : T(0);
                const T vb = okb ? rb[N - 2][t] : T(0);
                wc[t] = hb ? vb : wa[t];
            }
            ms_store<J, T>(a.ms, sla, wa);
            ms_store<J, T>(a.ms, slc, wc);
        }
#pragma unroll
        for (int m = 0; m < N - 1; ++m) {
            ia[m] = na[m];
            ib[m] = nb[m];
        }
        xa = nxa;
        xb = nxb;
    }
}

// GA = false: dense factored contraction, core operands as scalar loads.
// GA = true : pruned-phase gather contraction from LDS (dynamic LDS of
//             gather_lds_bytes<N, J, T>() bytes).
template <int N, int J, typename T, int OP, bool GA, bool STAGE = true>
__device__ __forceinline__ void rowgroup_body(const RowArgs<N, J, T> &a, const T *__restrict__ Gp, int bx,
                                              char *smem)
{
    constexpr int NA = row_nacc<J, OP>();
    const T *Gt = a.gt;
    const uint32_t *Gnz = a.gnz;
    if constexpr (GA && gather_in_lds(N, J, (int)sizeof(T))) {
        // STAGE = false: the block staged the core already (k_rowgroup's
        // grid-stride form of the gather contraction)
        T *g = reinterpret_cast<T *>(smem);
        uint32_t *nz = reinterpret_cast<uint32_t *>(smem + (size_t)ipow(J, N) * sizeof(T));
        if constexpr (STAGE) stage_core<N, J, T>(Gp, g, nz);
        Gt = g;
        Gnz = nz;
    }
    const CoreBases<T> Gb = core_bases_if<N, J, T, !GA>(Gp);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = bx * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (wave >= a.nwaves) return;
    const WaveInfo wi = a.waves[wave];
    const int grp = lane >> wi.glog;
    const bool has_row = grp < wi.nrows;
    const int row = has_row ? a.row_order[wi.first + grp] : 0;

    T own[J];
    if constexpr (OP != OP_SWEEP) {
        if (has_row) load_grow<J, T>(a.Ag + (int64_t)row * gather_ld(J, sizeof(T)), own);
        else
#pragma unroll
            for (int j = 0; j < J; ++j) own[j] = T(0);
    }
    T s[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) s[v] = T(0);

    if constexpr (!GA && (OP == OP_KEYS || OP == OP_RESID)) {
        pair_steps<N, J, T, OP>(a, Gb, wi, lane, own, s);
    } else {
    // Software pipeline: the indices and value of step k + 1 (gather form:
    // k + 2) are loaded at the top of step k, and in the gather form the
    // marking words of step k + 1 as well, so a step waits for one memory
    // latency (its factor rows) instead of a chain of two or three.
    // Prefetches past the last step re-read that step (in range).
    constexpr uint32_t full = J == 32 ? 0xffffffffu : (1u << J) - 1u;
    constexpr int AHEAD = GA ? 2 : 1;
    // the gather-form sweep and the keys stop after the live entries (the
    // rest add zero); the residual passes write every slot.  The dense FP64
    // sweep at J = 10 sits at the 256-VGPR line of two waves per SIMD and the
    // live bound tips its allocation over it (a few AGPRs, one wave per
    // SIMD), so the dense sweep walks every slot: its dead entries, whose
    // other-mode rows are zero, add exact zeros.
    const int K = (OP == OP_KEYS || (OP == OP_SWEEP && GA)) ? wi.klive : wi.K;
    int32_t ci[N - 1], pi[N - 1];
    uint32_t cm[N - 1];
    T cx = T(0), px = T(0);
    auto load_step = [&](int k, int32_t (&ii)[N - 1], T &x) {
        const int64_t sl = wi.base + (int64_t)(k < K ? k : K - 1) * kWave + lane;
#pragma unroll
        for (int m = 0; m < N - 1; ++m) ii[m] = ld_stream(a.oidx[m] + sl);
        x = ld_stream(a.xval + sl);
    };
    auto load_marks = [&](const int32_t (&ii)[N - 1], uint32_t (&mm)[N - 1]) {
#pragma unroll
        for (int m = 0; m < N - 1; ++m) mm[m] = ii[0] >= 0 ? (~a.omask[m][ii[m]] & full) : 0u;
    };
    if (K > 0) {
        load_step(0, ci, cx);
        if constexpr (GA) {
            load_marks(ci, cm);
            load_step(1, pi, px);
        }
    }
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
        const int64_t sl = wi.base + (int64_t)k * kWave + lane;
        int32_t ni[N - 1];
        uint32_t nm[N - 1];
        T nx;
        load_step(k + AHEAD, ni, nx);
        if constexpr (GA) load_marks(pi, nm);
        if (ci[0] < 0) {
            if constexpr (OP == OP_RESID || OP == OP_RESID_S0) {
                st_stream(T(0), a.e + sl);
                T z[J];
#pragma unroll
                for (int t = 0; t < J; ++t) z[t] = T(0);
                ms_store<J, T>(a.ms, sl, z);
            }
        } else {
            T r[N - 1][J];
            T d[J];
            if constexpr (GA) {
                delta_gather<N, J, T>(Gt, Gnz, a.fac, ci, cm, r, d);
                if constexpr (OP == OP_RESID) {
                    // the slot copy of the mode N-2 row must hold the values
                    // even when delta vanished without loading them
                    load_grow<J, T>(a.fac[N - 2] + (int64_t)ci[N - 2] * gather_ld(J, sizeof(T)), r[N - 2]);
                }
            } else {
#pragma unroll
                for (int m = 0; m < N - 1; ++m)
                    load_grow<J, T>(a.fac[m] + (int64_t)ci[m] * gather_ld(J, sizeof(T)), r[m]);
                delta_vec<N, J, T>(Gb, r, d);
            }
            const T x = cx;
            if constexpr (OP == OP_SWEEP) {
#pragma unroll
                for (int t = 0; t < J; ++t) {
                    s[t] = vfma(x, d[t], s[t]);
#pragma unroll
                    for (int v = t; v < J; ++v) s[J + sym<J>(t, v)] = vfma(d[t], d[v], s[J + sym<J>(t, v)]);
                }
            } else {
                T b = own[0] * d[0];
#pragma unroll
                for (int t = 1; t < J; ++t) b = vfma(own[t], d[t], b);
                if constexpr (OP == OP_KEYS) {
                    const T ev = x - b;
#pragma unroll
                    for (int t = 0; t < J; ++t) {
                        s[t] = vfma(ev, d[t], s[t]);
                        s[J + t] = vfma(d[t], d[t], s[J + t]);
                    }
                } else {
                    const T ev = x - b;
                    st_stream(ev, a.e + sl);
                    ms_store<J, T>(a.ms, sl, r[N - 2]);
                    if constexpr (OP == OP_RESID_S0) {
                        // first slab (leading digits 0): w_t = prod_m a^(m)_{i_m 0} a^(N-2)_{i t},
                        // accumulated as the slab pass does
                        T p = T(1);
#pragma unroll
                        for (int m = 0; m < N - 2; ++m) p *= r[m][0];
                        T w[J];
#pragma unroll
                        for (int t = 0; t < J; ++t) w[t] = p * r[N - 2][t];
#pragma unroll
                        for (int t = 0; t < J; ++t) {
                            s[t] = vfma(ev, w[t], s[t]);
#pragma unroll
                            for (int v = t; v < J; ++v) s[J + sym<J>(t, v)] = vfma(w[t], w[v], s[J + sym<J>(t, v)]);
                        }
                    }
                }
            }
        }
        if constexpr (GA) {
#pragma unroll
            for (int m = 0; m < N - 1; ++m) {
                ci[m] = pi[m];
                pi[m] = ni[m];
                cm[m] = nm[m];
            }
            cx = px;
            px = nx;
        } else {
#pragma unroll
            for (int m = 0; m < N - 1; ++m) ci[m] = ni[m];
            cx = nx;
        }
    }
    }
    if constexpr (OP == OP_RESID) {
        return;
    } else if constexpr (OP == OP_RESID_S0) {
        group_reduce<NA, T>(s, wi.glog);
        if (wi.chunk >= 0) {
            store_partial<NA, T>(a.partials, wi.chunk, s, lane);
        } else if (has_row && (lane & ((1 << wi.glog) - 1)) == 0) {
            double *dst = a.rowbuf + (int64_t)row * a.ldrb;
#pragma unroll
            for (int v = 0; v < NA; ++v) dst[v] = (double)s[v];
        }
    } else {
        group_reduce<NA, T>(s, wi.glog);
        if (wi.chunk >= 0) {
            store_partial<NA, T>(a.partials, wi.chunk, s, lane);
            return;
        }
        if (has_row && (lane & ((1 << wi.glog) - 1)) == 0) row_epilogue<N, J, T, OP, T>(a, row, s);
    }
}

template <int N, int J, typename T, int OP, bool GA>
__global__ void __launch_bounds__(256) k_rowgroup(RowArgs<N, J, T> a, const T *__restrict__ Gp)
{
    extern __shared__ __align__(16) char smem[];
    if constexpr (GA && gather_in_lds(N, J, (int)sizeof(T))) {
        // gather form: the core is staged in LDS once per block, then the
        // block walks its share of the waves (grid of at most kGatherGrid
        // blocks), so the staging is not repeated for every four waves
        stage_core<N, J, T>(Gp, reinterpret_cast<T *>(smem),
                            reinterpret_cast<uint32_t *>(smem + (size_t)ipow(J, N) * sizeof(T)));
        for (int bx = blockIdx.x; bx * (int)(blockDim.x / kWave) < a.nwaves; bx += gridDim.x)
            rowgroup_body<N, J, T, OP, GA, false>(a, Gp, bx, smem);
    } else {
        rowgroup_body<N, J, T, OP, GA>(a, Gp, blockIdx.x, smem);
    }
}

// Several contexts of one shape in one launch (dense contraction): block b of
// the grid-stride loop is virtual block b - off[t] of task t (a context's
// RowArgs and permuted core), so one launch carries every job of a serving
// batch.
template <int N, int J, typename T>
struct RowTask {
    RowArgs<N, J, T> a;
    const T *Gp;
    const LongRow *longrows;
};

template <int N, int J, typename T, int OP>
__global__ void __launch_bounds__(256) k_rowgroup_multi(const RowTask<N, J, T> *__restrict__ tab,
                                                        const int32_t *__restrict__ off, int ntask, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const RowTask<N, J, T> tk = tab[t];   // arguments in registers, read once
        rowgroup_body<N, J, T, OP, false>(tk.a, tk.Gp, b - off[t], nullptr);
    }
}

// Rows longer than one chunk: sum the chunk partials in a fixed order, then
// run the same epilogue (one wave per long row).
template <int N, int J, typename T, int OP>
__device__ __forceinline__ void rowgroup_long_body(const RowArgs<N, J, T> &a, const LongRow *__restrict__ lr, int bx)
{
    constexpr int NA = row_nacc<J, OP>();
    __shared__ double sh[NA];
    const LongRow L = lr[bx];
    sum_partials<NA>(a.partials, L, sh, threadIdx.x);
    if (threadIdx.x == 0) {
        double s[NA];
#pragma unroll
        for (int v = 0; v < NA; ++v) s[v] = sh[v];
        row_epilogue<N, J, T, OP, double>(a, L.row, s);
    }
}

template <int N, int J, typename T, int OP>
__global__ void __launch_bounds__(64) k_rowgroup_long(RowArgs<N, J, T> a, const LongRow *__restrict__ lr)
{
    rowgroup_long_body<N, J, T, OP>(a, lr, blockIdx.x);
}

template <int N, int J, typename T, int OP>
__global__ void __launch_bounds__(64) k_rowgroup_long_multi(const RowTask<N, J, T> *__restrict__ tab,
                                                            const int32_t *__restrict__ off, int ntask, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const RowTask<N, J, T> tk = tab[t];
        rowgroup_long_body<N, J, T, OP>(tk.a, tk.longrows, b - off[t]);
        __syncthreads();   // the LDS sums are reused by the next long row
    }
}

// ------------------------------------------------------------ MFMA form
// Order 3, factor sweep.  For the 64 slots of one step of a wave the first
// stage of Eq. 11,
//     T_alpha[(j, j')] = sum_{j''} G[j][j'][j''] a^(q)_{i_q j''}
// (q = the last other mode, p the first), is the product of the core, read
// as a (J^2 x J) matrix, with the (J x 64) matrix of the entries' A^(q) rows:
// a 32 x 32 matrix-core tile has 32 pairs (j, j') as rows and one batch of
// 32 entries as columns (batch 0: the entries of lanes 0..31, batch 1: those
// of lanes 32..63).  A lane receives half of the rows of one column of each
// batch; one permlane32 swap per register pair gives every lane all rows of
// its own entry.  The second stage delta_j = sum_{j'} T[(j, j')] a^(p)_{i_p j'}
// and the row statistics c, V run on the vector ALU in FP32, the epilogue in
// FP64, as in the plain kernel.
//   MF_BF16: BF16 operands, FP32 accumulation (K = 16 per op).  Core and
//            A^(q) values are each split into x_hi = bf16(x) and
//            x_lo = bf16(x - x_hi), and the tile is the sum of the three
//            products lo.hi + hi.lo + hi.hi (the lo.lo term, of relative size
//            2^-18, is dropped), so the operands carry about 16 significant
//            bits instead of 8 (the split-BF16 scheme of Henry, Tang and
//            Heinecke, "Leveraging the bfloat16 artificial intelligence
//            datatype for higher-precision computations", ARITH 2019).
//   MF_F32 : FP32 operands (K = 2 per op)
enum { MF_BF16 = 0, MF_F32 = 1 };

__device__ __forceinline__ void swap32(uint32_t &lo, uint32_t &hi)
{
    // lanes 32..63 of lo trade places with lanes 0..31 of hi
    const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
    lo = r[0];
    hi = r[1];
}

__device__ __forceinline__ void swap32(float &lo, float &hi)
{
    uint32_t a = __float_as_uint(lo), b = __float_as_uint(hi);
    swap32(a, b);
    lo = __uint_as_float(a);
    hi = __uint_as_float(b);
}

template <int J, int MF>
__device__ __forceinline__ void rowgroup_mfma_body(const RowArgs<3, J, float> &a, const float *__restrict__ Gp, int bx)
{
    static_assert(J <= 16, "one K block of 16 (BF16) or J/2 steps of 2 (FP32)");
    constexpr int NA = nacc_vc(J);
    constexpr int NT = (J * J + 31) / 32;
    constexpr int KS = MF == MF_BF16 ? 1 : (J + 1) / 2;
    constexpr int NS = MF == MF_BF16 ? 2 : 1;  // hi / lo parts
    using AOp = typename std::conditional<MF == MF_BF16, bf16x8, float>::type;

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = bx * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (wave >= a.nwaves) return;  // whole waves only: the matrix ops need every lane
    const WaveInfo wi = a.waves[wave];
    const int grp = lane >> wi.glog;
    const bool has_row = grp < wi.nrows;
    const int row = has_row ? a.row_order[wi.first + grp] : 0;
    const int h = lane >> 5;

    // A operands: tile tau, row = pair P = 32 tau + (lane & 31); K index of
    // element e is 8h + e (BF16) or 2 step + h (FP32); zero outside J^2 x J.
    AOp ga[NS][NT][KS];
#pragma unroll
    for (int tau = 0; tau < NT; ++tau) {
        const int P = 32 * tau + (lane & 31);
        if constexpr (MF == MF_BF16) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * h + e;
                float v = 0.0f;
                if (P < J * J && k < J) v = Gp[P * J + k];
                const __bf16 hi = (__bf16)v;
                ga[0][tau][0][e] = hi;
                ga[1][tau][0][e] = (__bf16)(v - (float)hi);
            }
        } else {
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                const int k = 2 * st + h;
                float v = 0.0f;
                if (P < J * J && k < J) v = Gp[P * J + k];
                ga[0][tau][st] = v;
            }
        }
    }

    float s[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) s[v] = 0.0f;

    for (int k = 0; k < wi.klive; ++k) {   // live entries only (the rest add zero)
        const int64_t sl = wi.base + (int64_t)k * kWave + lane;
        const int32_t i0 = ld_stream(a.oidx[0] + sl);
        const int32_t i1 = ld_stream(a.oidx[1] + sl);  // 0 on padding slots
        const bool ok = i0 >= 0;
        float rp[J], rq[J];
        load_grow<J, float>(a.fac[0] + (int64_t)(ok ? i0 : 0) * gather_ld(J, 4), rp);
        load_grow<J, float>(a.fac[1] + (int64_t)i1 * gather_ld(J, 4), rq);
#pragma unroll
        for (int t = 0; t < J; ++t) rq[t] = ok ? rq[t] : 0.0f;  // zero column: T = 0, delta = 0
        const float x = ld_stream(a.xval + sl);                               // 0 on padding slots

        // B operands of the two batches from the lane's own row: lane l of
        // batch b must hold K range h of the entry of lane 32 b + (l & 31).
        AOp b0[NS][KS], b1[NS][KS];
        if constexpr (MF == MF_BF16) {
#pragma unroll
            for (int part = 0; part < NS; ++part) {
                bf16x8 k0, k1;  // K indices 0..7 and 8..15 of the own row
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float v0 = e < J ? rq[e] : 0.0f, v1 = 8 + e < J ? rq[8 + e] : 0.0f;
                    const __bf16 h0 = (__bf16)v0, h1 = (__bf16)v1;
                    k0[e] = part == 0 ? h0 : (__bf16)(v0 - (float)h0);
                    k1[e] = part == 0 ? h1 : (__bf16)(v1 - (float)h1);
                }
                uint32_t u0[4], u1[4];
                __builtin_memcpy(u0, &k0, 16);
                __builtin_memcpy(u1, &k1, 16);
#pragma unroll
                for (int w = 0; w < 4; ++w) swap32(u0[w], u1[w]);
                __builtin_memcpy(&b0[part][0], u0, 16);
                __builtin_memcpy(&b1[part][0], u1, 16);
            }
        } else {
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                b0[0][st] = rq[2 * st];
                b1[0][st] = 2 * st + 1 < J ? rq[2 * st + 1] : 0.0f;
                swap32(b0[0][st], b1[0][st]);
            }
        }

        float d[J];
#pragma unroll
        for (int t = 0; t < J; ++t) d[t] = 0.0f;
#pragma unroll
        for (int tau = 0; tau < NT; ++tau) {
            f32x16 D0 = {}, D1 = {};
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                if constexpr (MF == MF_BF16) {
                    // small terms first
                    D0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga[1][tau][st], b0[0][st], D0, 0, 0, 0);
                    D1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga[1][tau][st], b1[0][st], D1, 0, 0, 0);
                    D0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga[0][tau][st], b0[1][st], D0, 0, 0, 0);
                    D1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga[0][tau][st], b1[1][st], D1, 0, 0, 0);
                    D0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga[0][tau][st], b0[0][st], D0, 0, 0, 0);
                    D1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga[0][tau][st], b1[0][st], D1, 0, 0, 0);
                } else {
                    D0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ga[0][tau][st], b0[0][st], D0, 0, 0, 0);
                    D1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ga[0][tau][st], b1[0][st], D1, 0, 0, 0);
                }
            }
            // register r of half hh holds row 8 (r / 4) + 4 hh + r % 4 of the
            // tile; after the swap D0 holds the hh = 0 rows and D1 the hh = 1
            // rows of the lane's own entry.
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float lo = D0[r], hi = D1[r];
                swap32(lo, hi);
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int P = 32 * tau + 8 * (r / 4) + 4 * hh + r % 4;
                    if (P < J * J) d[P / J] = vfma(hh ? hi : lo, rp[P % J], d[P / J]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < J; ++t) {
            s[t] = vfma(x, d[t], s[t]);
#pragma unroll
            for (int v = t; v < J; ++v) s[J + sym<J>(t, v)] = vfma(d[t], d[v], s[J + sym<J>(t, v)]);
        }
    }
    group_reduce<NA, float>(s, wi.glog);
    if (wi.chunk >= 0) {
        store_partial<NA, float>(a.partials, wi.chunk, s, lane);
        return;
    }
    if (has_row && (lane & ((1 << wi.glog) - 1)) == 0) row_epilogue<3, J, float, OP_SWEEP, float>(a, row, s);
}

template <int J, int MF>
__global__ void __launch_bounds__(256) k_rowgroup_mfma(RowArgs<3, J, float> a, const float *__restrict__ Gp)
{
    rowgroup_mfma_body<J, MF>(a, Gp, blockIdx.x);
}

template <int J, int MF>
__global__ void __launch_bounds__(256) k_rowgroup_mfma_multi(const RowTask<3, J, float> *__restrict__ tab,
                                                             const int32_t *__restrict__ off, int ntask, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const RowTask<3, J, float> tk = tab[t];
        rowgroup_mfma_body<J, MF>(tk.a, tk.Gp, b - off[t]);
    }
}

// Kernel choice for the contraction of mode `mode` (the factors of the other
// modes enter).  AUTO compares costs in fused multiply-adds per entry: the
// dense contraction's sum_{m=2..N} J^m (a quarter of that on the matrix-core
// form) against the gather form's fixed cost G0 (its dependent loads of
// marking words and rows; 550, measured as half the dense FP64 cost at order
// 3, rank 10) plus 10 J per expected surviving term, E = prod_{k != mode}
// J d_k (d_k = unmarked fraction of A^(k)).
static bool use_gather(const vest_ctx *c, int mode, bool dense_on_mfma)
{
    if (!dense_form(c->N, c->J)) return true;
    if (c->kernel_policy == VEST_KERNEL_DENSE) return false;
    if (c->kernel_policy == VEST_KERNEL_GATHER) return true;
    const int N = c->N, J = c->J;
    double E = 1.0, D = 0.0, p = J;
    for (int k = 0; k < N; ++k) {
        if (k == mode) continue;
        const double size = (double)c->d.dims[k] * J;
        E *= J * (1.0 - (double)c->marked_fac[k] / size);
    }
    for (int m = 2; m <= N; ++m) D += (p *= J);
    if (dense_on_mfma) D *= 0.25;
    return 550.0 + 10.0 * J * E < D;
}

template <int N, int J, typename T>
static RowArgs<N, J, T> make_row_args(vest_ctx *c, int mode)
{
    const ModeLayout &L = c->lay[mode];
    RowArgs<N, J, T> a{};
    a.waves = L.waves;
    a.nwaves = L.nwaves;
    a.reg = c->d.reg;
    a.lambda = c->d.lambda;
    a.row_order = L.row_order;
    int m = 0;
    for (int k = 0; k < N; ++k) {
        if (k == mode) continue;
        a.oidx[m] = L.oidx[m];
        a.fac[m] = reinterpret_cast<const T *>(c->Ag[k]);
        a.omask[m] = c->fmask[k];
        ++m;
    }
    a.xval = reinterpret_cast<const T *>(L.xval);
    a.Ag = reinterpret_cast<T *>(c->Ag[mode]);
    a.A = c->A[mode];
    a.mask = c->fmask[mode];
    a.partials = c->partials;
    a.e = reinterpret_cast<T *>(c->e);
    a.ms = reinterpret_cast<T *>(c->ms);
    a.keys = c->key_fac[mode];
    a.rowbuf = c->rowbuf;
    a.ldrb = c->ldrb;
    return a;
}

template <int N, int J, typename T>
static hipError_t launch_rowgroup_t(vest_ctx *c, int mode, int op)
{
    const ModeLayout &L = c->lay[mode];
    RowArgs<N, J, T> a = make_row_args<N, J, T>(c, mode);
    const T *Gp = reinterpret_cast<const T *>(c->Gp[mode]);
    const int blocks = (L.nwaves + 3) / 4;
    const bool ga = use_gather(c, mode, (N == 3 && J <= 16 && std::is_same<T, float>::value && op == OP_SWEEP));
    const size_t lds = ga ? gather_lds_bytes<N, J, T>() : 0;
    if constexpr (!gather_in_lds(N, J, (int)sizeof(T))) {
        if (ga) {
            if (!c->gt || !c->gnz) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_stage_core<N, J, T>), dim3(1), dim3(1024), 0, c->stream, Gp,
                               reinterpret_cast<T *>(c->gt), c->gnz);
            a.gt = reinterpret_cast<const T *>(c->gt);
            a.gnz = c->gnz;
        }
    }
    if (ga && op == OP_RESID_S0) return hipErrorInvalidValue;   // dense form only (resid_fuses_slab0)
    if (blocks > 0) {
        bool done = false;
        if constexpr (N == 3 && J <= 16 && std::is_same<T, float>::value) {
            if (!ga && op == OP_SWEEP) {
                if (c->d.precision == VEST_BF16)
                    hipLaunchKernelGGL((k_rowgroup_mfma<J, MF_BF16>), dim3(blocks), dim3(256), 0, c->stream, a, Gp);
                else
                    hipLaunchKernelGGL((k_rowgroup_mfma<J, MF_F32>), dim3(blocks), dim3(256), 0, c->stream, a, Gp);
                done = true;
            }
        }
        if (done) {
        } else if (ga) {
            const int gb = gather_in_lds(N, J, (int)sizeof(T)) && blocks > kGatherGrid ? kGatherGrid : blocks;
            if (op == OP_SWEEP)
                hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_SWEEP, true>), dim3(gb), dim3(256), lds, c->stream, a, Gp);
            else if (op == OP_KEYS)
                hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_KEYS, true>), dim3(gb), dim3(256), lds, c->stream, a, Gp);
            else
                hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_RESID, true>), dim3(gb), dim3(256), lds, c->stream, a, Gp);
        } else if constexpr (dense_form(N, J)) {
            if (op == OP_SWEEP)
                hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_SWEEP, false>), dim3(blocks), dim3(256), 0, c->stream, a, Gp);
            else if (op == OP_KEYS)
                hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_KEYS, false>), dim3(blocks), dim3(256), 0, c->stream, a, Gp);
            else if (op == OP_RESID_S0)
                hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_RESID_S0, false>), dim3(blocks), dim3(256), 0, c->stream, a,
                                   Gp);
            else
                hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_RESID, false>), dim3(blocks), dim3(256), 0, c->stream, a, Gp);
        } else {
            return hipErrorInvalidValue;  // unreachable: use_gather is true without a dense instance
        }
    }
    // long rows of the sweep and the keys are finished here; the residual has
    // none to finish, and the first-slab sums of OP_RESID_S0 are finished by
    // the core sweep (its long-row kernel of the slab statistics)
    if (L.nlong > 0 && (op == OP_SWEEP || op == OP_KEYS)) {
        if (op == OP_SWEEP)
            hipLaunchKernelGGL((k_rowgroup_long<N, J, T, OP_SWEEP>), dim3(L.nlong), dim3(64), 0, c->stream, a,
                               L.longrows);
        else
            hipLaunchKernelGGL((k_rowgroup_long<N, J, T, OP_KEYS>), dim3(L.nlong), dim3(64), 0, c->stream, a,
                               L.longrows);
    }
    return hipGetLastError();
}

bool resid_fuses_slab0(const vest_ctx *c) { return !use_gather(c, c->N - 1, false); }

bool batch_dense_ok(const vest_ctx *c)
{
    for (int m = 0; m < c->N; ++m) {
        const bool mfma = c->N == 3 && c->J <= 16 && c->f32;
        if (use_gather(c, m, mfma) || use_gather(c, m, false)) return false;
    }
    return true;
}

template <int N, int J, typename T>
static bool plan_factor_batch_t(vest_ctx *const *cs, int n, int mode, int op, hipStream_t st, BatchArena &ba,
                                LaunchList &L)
{
    if (op != OP_SWEEP && op != OP_RESID_S0) return false;
    std::vector<RowTask<N, J, T>> tab(n);
    std::vector<int32_t> off(n + 1, 0), loff(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        vest_ctx *c = cs[i];
        tab[i].a = make_row_args<N, J, T>(c, mode);
        tab[i].Gp = reinterpret_cast<const T *>(c->Gp[mode]);
        tab[i].longrows = c->lay[mode].longrows;
        off[i + 1] = off[i] + (c->lay[mode].nwaves + 3) / 4;
        loff[i + 1] = loff[i] + (op == OP_SWEEP ? c->lay[mode].nlong : 0);
    }
    const size_t ot = ba.add(tab.data(), sizeof(RowTask<N, J, T>) * n);
    const size_t oo = ba.add(off.data(), 4 * (n + 1));
    const size_t ol = ba.add(loff.data(), 4 * (n + 1));
    if (ba.overflow) return false;
    const RowTask<N, J, T> *dt = ba.dptr<RowTask<N, J, T>>(ot);
    const int32_t *doff = ba.dptr<int32_t>(oo), *dloff = ba.dptr<int32_t>(ol);
    const int total = off[n], ltotal = loff[n];
    const bool bf16 = cs[0]->d.precision == VEST_BF16;
    L.push_back([=]() {
        const int grid = total < kBatchGrid ? total : kBatchGrid;
        if (total > 0) {
            bool done = false;
            if constexpr (N == 3 && J <= 16 && std::is_same<T, float>::value) {
                if (op == OP_SWEEP) {
                    const auto *mt = reinterpret_cast<const RowTask<3, J, float> *>(dt);
                    if (bf16)
                        hipLaunchKernelGGL((k_rowgroup_mfma_multi<J, MF_BF16>), dim3(grid), dim3(256), 0, st, mt, doff,
                                           n, total);
                    else
                        hipLaunchKernelGGL((k_rowgroup_mfma_multi<J, MF_F32>), dim3(grid), dim3(256), 0, st, mt, doff,
                                           n, total);
                    done = true;
                }
            }
            if constexpr (dense_form(N, J)) {
                if (!done) {
                    if (op == OP_SWEEP)
                        hipLaunchKernelGGL((k_rowgroup_multi<N, J, T, OP_SWEEP>), dim3(grid), dim3(256), 0, st, dt,
                                           doff, n, total);
                    else
                        hipLaunchKernelGGL((k_rowgroup_multi<N, J, T, OP_RESID_S0>), dim3(grid), dim3(256), 0, st, dt,
                                           doff, n, total);
                }
            }
        }
        if (ltotal > 0) {
            const int lg = ltotal < kBatchGrid ? ltotal : kBatchGrid;
            hipLaunchKernelGGL((k_rowgroup_long_multi<N, J, T, OP_SWEEP>), dim3(lg), dim3(64), 0, st, dt, dloff, n,
                               ltotal);
        }
    });
    return true;
}

bool plan_factor_batch(vest_ctx *const *cs, int n, int mode, int op, hipStream_t st, BatchArena &ba, LaunchList &L)
{
    const vest_ctx *c = cs[0];
    if (!dense_form(c->N, c->J)) return false;
#define VEST_CASE(NN, JJ)                                                                        \
    if (c->N == NN && c->J == JJ)                                                                \
        return c->f32 ? plan_factor_batch_t<NN, JJ, float>(cs, n, mode, op, st, ba, L)           \
                      : plan_factor_batch_t<NN, JJ, double>(cs, n, mode, op, st, ba, L);
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return false;
}

hipError_t launch_rowgroup(vest_ctx *c, int mode, int op)
{
#define VEST_CASE(NN, JJ)                                                                 \
    if (c->N == NN && c->J == JJ)                                                         \
        return c->f32 ? launch_rowgroup_t<NN, JJ, float>(c, mode, op) \
                                           : launch_rowgroup_t<NN, JJ, double>(c, mode, op);
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return hipErrorInvalidValue;
}

}  // namespace vest
