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
    const T *own;             // mode-n factor in compute type (OP_RESID)
    double *A;                // mode-n FP64 factor
    float *A32;               // FP32 copy refreshed by OP_SWEEP (may be null)
    const uint32_t *mask;     // mode-n marking table
    double *partials;         // long-row chunk partials
    T *e;                     // OP_RESID: out
    T *ms;                    // OP_RESID: out, mode N-2 factor row of every slot (see ms_index)
    double *keys;             // OP_KEYS: out [I_n * J]
};

template <int J, int OP>
__host__ __device__ constexpr int row_nacc() { return OP == OP_KEYS ? 2 * J : nacc_vc(J); }

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
        if (a.A32) {
            float *d32 = a.A32 + (int64_t)row * J;
#pragma unroll
            for (int j = 0; j < J; ++j) d32[j] = (float)av[j];
        }
    } else {
        // Delta(a_ij) = sum (2 e + a delta_j) a delta_j = 2 a s_j + a^2 q_j
        double *dst = a.keys + (int64_t)row * J;
#pragma unroll
        for (int j = 0; j < J; ++j)
            dst[j] = ((mk >> j) & 1u) ? HUGE_VAL : 2.0 * av[j] * (double)s[j] + av[j] * av[j] * (double)s[J + j];
    }
}

template <int N, int J, typename T, int OP, int U>
__global__ void __launch_bounds__(256) k_rowgroup(RowArgs<N, J, T> a, const T *__restrict__ Gp)
{
    constexpr int NA = row_nacc<J, OP>();
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (wave >= a.nwaves) return;
    const WaveInfo wi = a.waves[wave];
    const int grp = lane >> wi.glog;
    const bool has_row = grp < wi.nrows;
    const int row = has_row ? a.row_order[wi.first + grp] : 0;

    T own[J];
    if constexpr (OP == OP_RESID || OP == OP_KEYS) {
        if (has_row) load_row<J, T>(a.own + (int64_t)row * J, own);
        else
#pragma unroll
            for (int j = 0; j < J; ++j) own[j] = T(0);
    }
    T s[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) s[v] = T(0);

    // U entries per lane at a time: their index and value loads, then their
    // factor-row gathers, are issued together, and the contraction reuses
    // every core operand U times.  Slots past the lane's last entry are
    // clamped onto it (loaded, not used); padding slots are skipped.
    const int K = wi.K;
    if constexpr (U == 1) {
        for (int k = 0; k < K; ++k) {
            const int64_t sl = wi.base + (int64_t)k * kWave + lane;
            const int32_t i0 = a.oidx[0][sl];
            if (i0 < 0) {
                if constexpr (OP == OP_RESID) {
                    a.e[sl] = T(0);
#pragma unroll
                    for (int t = 0; t < J; ++t) a.ms[ms_index<J>(sl, t)] = T(0);
                }
                continue;
            }
            T r[N - 1][J];
            load_row<J, T>(a.fac[0] + (int64_t)i0 * J, r[0]);
#pragma unroll
            for (int m = 1; m < N - 1; ++m) load_row<J, T>(a.fac[m] + (int64_t)a.oidx[m][sl] * J, r[m]);
            T d[J];
            delta_vec<N, J, T>(Gp, r, d);
            const T x = a.xval[sl];
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
                    a.e[sl] = x - b;
#pragma unroll
                    for (int t = 0; t < J; ++t) a.ms[ms_index<J>(sl, t)] = r[N - 2][t];
                }
            }
        }
    } else
    for (int k0 = 0; k0 < K; k0 += U) {
        int64_t sl[U];
        int32_t ii[U][N - 1];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sl[u] = wi.base + (int64_t)(k0 + u < K ? k0 + u : K - 1) * kWave + lane;
#pragma unroll
            for (int m = 0; m < N - 1; ++m) ii[u][m] = a.oidx[m][sl[u]];
        }
        T r[U][N - 1][J];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = (k0 + u < K) && ii[u][0] >= 0;
#pragma unroll
            for (int m = 0; m < N - 1; ++m)
                load_row<J, T>(a.fac[m] + (int64_t)(ii[u][m] > 0 ? ii[u][m] : 0) * J, r[u][m]);
        }
        T x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = a.xval[sl[u]];
        T d[U][J];
        delta_vec_u<U, N, J, T>(Gp, r, d);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (OP == OP_RESID) {
                if (k0 + u < K) {
                    T b = own[0] * d[u][0];
#pragma unroll
                    for (int t = 1; t < J; ++t) b = vfma(own[t], d[u][t], b);
                    a.e[sl[u]] = ok[u] ? x[u] - b : T(0);
#pragma unroll
                    for (int t = 0; t < J; ++t) a.ms[ms_index<J>(sl[u], t)] = ok[u] ? r[u][N - 2][t] : T(0);
                }
                continue;
            }
            if (!ok[u]) continue;
            if constexpr (OP == OP_SWEEP) {
#pragma unroll
                for (int t = 0; t < J; ++t) {
                    s[t] = vfma(x[u], d[u][t], s[t]);
#pragma unroll
                    for (int v = t; v < J; ++v) s[J + sym<J>(t, v)] = vfma(d[u][t], d[u][v], s[J + sym<J>(t, v)]);
                }
            } else {
                T b = own[0] * d[u][0];
#pragma unroll
                for (int t = 1; t < J; ++t) b = vfma(own[t], d[u][t], b);
                const T ev = x[u] - b;
#pragma unroll
                for (int t = 0; t < J; ++t) {
                    s[t] = vfma(ev, d[u][t], s[t]);
                    s[J + t] = vfma(d[u][t], d[u][t], s[J + t]);
                }
            }
        }
    }
    if constexpr (OP == OP_RESID) {
        return;
    } else {
        group_reduce<NA, T>(s, wi.glog);
        if (wi.chunk >= 0) {
            store_partial<NA, T>(a.partials, wi.chunk, s, lane);
            return;
        }
        if (has_row && (lane & ((1 << wi.glog) - 1)) == 0) row_epilogue<N, J, T, OP, T>(a, row, s);
    }
}

// Rows longer than one chunk: sum the chunk partials in a fixed order, then
// run the same epilogue (one wave per long row).
template <int N, int J, typename T, int OP>
__global__ void __launch_bounds__(64) k_rowgroup_long(RowArgs<N, J, T> a, const LongRow *__restrict__ lr)
{
    constexpr int NA = row_nacc<J, OP>();
    __shared__ double sh[NA];
    const LongRow L = lr[blockIdx.x];
    sum_partials<NA>(a.partials, L, sh, threadIdx.x);
    if (threadIdx.x == 0) {
        double s[NA];
#pragma unroll
        for (int v = 0; v < NA; ++v) s[v] = sh[v];
        row_epilogue<N, J, T, OP, double>(a, L.row, s);
    }
}

template <int N, int J, typename T>
static hipError_t launch_rowgroup_t(vest_ctx *c, int mode, int op)
{
    const ModeLayout &L = c->lay[mode];
    const bool f32 = std::is_same<T, float>::value;
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
        a.fac[m] = f32 ? reinterpret_cast<const T *>(c->A32[k]) : reinterpret_cast<const T *>(c->A[k]);
        ++m;
    }
    a.xval = reinterpret_cast<const T *>(L.xval);
    a.own = f32 ? reinterpret_cast<const T *>(c->A32[mode]) : reinterpret_cast<const T *>(c->A[mode]);
    a.A = c->A[mode];
    a.A32 = f32 ? c->A32[mode] : nullptr;
    a.mask = c->fmask[mode];
    a.partials = c->partials;
    a.e = reinterpret_cast<T *>(c->e);
    a.ms = reinterpret_cast<T *>(c->ms);
    a.keys = c->key_fac[mode];
    const T *Gp = reinterpret_cast<const T *>(c->Gp[mode]);
    const int blocks = (L.nwaves + 3) / 4;
    if (blocks > 0) {
        // one entry per lane: with two, the compiler hoists the shared core
        // operands out of the loop and spills them to vector-register lanes
        constexpr int U = 1;
        if (op == OP_SWEEP)
            hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_SWEEP, U>), dim3(blocks), dim3(256), 0, c->stream, a, Gp);
        else if (op == OP_KEYS)
            hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_KEYS, U>), dim3(blocks), dim3(256), 0, c->stream, a, Gp);
        else
            hipLaunchKernelGGL((k_rowgroup<N, J, T, OP_RESID, U>), dim3(blocks), dim3(256), 0, c->stream, a, Gp);
    }
    if (L.nlong > 0 && op != OP_RESID) {
        if (op == OP_SWEEP)
            hipLaunchKernelGGL((k_rowgroup_long<N, J, T, OP_SWEEP>), dim3(L.nlong), dim3(64), 0, c->stream, a,
                               L.longrows);
        else
            hipLaunchKernelGGL((k_rowgroup_long<N, J, T, OP_KEYS>), dim3(L.nlong), dim3(64), 0, c->stream, a,
                               L.longrows);
    }
    return hipGetLastError();
}

hipError_t launch_rowgroup(vest_ctx *c, int mode, int op)
{
#define VEST_CASE(NN, JJ)                                                                 \
    if (c->N == NN && c->J == JJ)                                                         \
        return c->d.precision == VEST_FP32 ? launch_rowgroup_t<NN, JJ, float>(c, mode, op) \
                                           : launch_rowgroup_t<NN, JJ, double>(c, mode, op);
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return hipErrorInvalidValue;
}

}  // namespace vest
