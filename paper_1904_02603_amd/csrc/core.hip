// Core update (Eq. 12 / Eq. 14) and core responsibility keys (Eq. 5).
//
// The paper updates the core elements one after another in a fixed order
// (Sec. 3.5).  Done literally, every element costs one pass over Omega.  Here
// the same sequence of one-dimensional minimisations runs as an exact block
// Gauss-Seidel over "slabs": a slab is the set of J_{N-1} * J_N consecutive
// elements (flat order) that share the leading indices (j_1..j_{N-2}).  For a
// slab s with leading product p_s(alpha) = prod_{n<N-1} a^(n)_{i_n j_n} and
// w_{(t,u)}(alpha) = p_s(alpha) a^(N-1)_{i_{N-1} t} a^(N)_{i_N u}:
//   one pass over Omega, grouped by the mode-N index r (the core layout),
//   accumulates per row r
//     R_r[t]     = sum_alpha e_alpha p_s a^(N-1)_t
//     M_r[t,t']  = sum_alpha p_s^2 a^(N-1)_t a^(N-1)_t'
//   and the slab's Gram matrix and right-hand side follow exactly as
//     H[(t,u),(t',u')] = sum_r M_r[t,t'] a^(N)_{r u} a^(N)_{r u'}
//     rr[(t,u)]        = sum_r R_r[t] a^(N)_{r u}
//   (a dense product over rows: [R | M]^T [a | a a^T], "gram").  A single
//   wave then visits the slab's unpruned elements in flat order:
//     num_q = rr_q - sum_{p<q} H_qp D_p + G_q H_qq,   G_q <- rule(num_q, H_qq),
//   D_q = change of G_q, which is exactly the sequential update with the
//   residual corrected after every element.  The next slab's pass first applies
//   e -= sum_q D_q w_q to the residual.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "internal.h"

namespace vest {

template <int N, int J, typename T>
struct SlabArgs {
    static constexpr int NL = N > 2 ? N - 2 : 1;
    const WaveInfo *waves;
    int32_t nwaves;
    int32_t has_prev;
    const int32_t *row_order;
    const int32_t *oidx[N - 1];   // core layout: modes 0..N-2
    const T *colA[NL];            // column-major copies of modes 0..N-3
    int64_t dimA[NL];
    int32_t lead[NL];             // leading core indices of this slab
    int32_t lprev[NL];            // ... of the previous slab
    const T *Amid;                // mode N-2 factor, row-major
    const T *Alast;               // mode N-1 factor, row-major
    T *e;
    const double *dprev;          // [J][J] change of the previous slab's elements
    double *rowbuf;               // [I_{N-1}][gw]
    int32_t gw;
    double *partials;
};

template <int N, int J, typename T, bool ACC>
__global__ void __launch_bounds__(256) k_slab(SlabArgs<N, J, T> a)
{
    constexpr int NA = nacc_vc(J);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (wave >= a.nwaves) return;
    const WaveInfo wi = a.waves[wave];
    const int grp = lane >> wi.glog;
    const bool has_row = grp < wi.nrows;
    const int row = has_row ? a.row_order[wi.first + grp] : 0;

    T u[J];
    if (a.has_prev) {
        T al[J];
        if (has_row) load_row<J, T>(a.Alast + (int64_t)row * J, al);
        else
#pragma unroll
            for (int v = 0; v < J; ++v) al[v] = T(0);
#pragma unroll
        for (int t = 0; t < J; ++t) {
            T acc = (T)a.dprev[t * J] * al[0];
#pragma unroll
            for (int v = 1; v < J; ++v) acc = vfma((T)a.dprev[t * J + v], al[v], acc);
            u[t] = acc;
        }
    }
    T s[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) s[v] = T(0);

    for (int k = 0; k < wi.K; ++k) {
        const int64_t sl = wi.base + (int64_t)k * kWave + lane;
        int32_t ii[N - 1];
        ii[0] = a.oidx[0][sl];
        if (ii[0] < 0) continue;
#pragma unroll
        for (int m = 1; m < N - 1; ++m) ii[m] = a.oidx[m][sl];
        T mv[J];
        load_row<J, T>(a.Amid + (int64_t)ii[N - 2] * J, mv);
        T ev = a.e[sl];
        if (a.has_prev) {
            T pp = T(1);
#pragma unroll
            for (int m = 0; m < N - 2; ++m) pp *= a.colA[m][(int64_t)a.lprev[m] * a.dimA[m] + ii[m]];
            T du = mv[0] * u[0];
#pragma unroll
            for (int t = 1; t < J; ++t) du = vfma(mv[t], u[t], du);
            ev -= pp * du;
            a.e[sl] = ev;
        }
        if constexpr (ACC) {
            T p = T(1);
#pragma unroll
            for (int m = 0; m < N - 2; ++m) p *= a.colA[m][(int64_t)a.lead[m] * a.dimA[m] + ii[m]];
            T w[J];
#pragma unroll
            for (int t = 0; t < J; ++t) w[t] = p * mv[t];
#pragma unroll
            for (int t = 0; t < J; ++t) {
                s[t] = vfma(ev, w[t], s[t]);
#pragma unroll
                for (int v = t; v < J; ++v) s[J + sym<J>(t, v)] = vfma(w[t], w[v], s[J + sym<J>(t, v)]);
            }
        }
    }
    if constexpr (ACC) {
        group_reduce<NA, T>(s, wi.glog);
        if (wi.chunk >= 0) {
            store_partial<NA, T>(a.partials, wi.chunk, s, lane);
            return;
        }
        if (has_row && (lane & ((1 << wi.glog) - 1)) == 0) {
            double *dst = a.rowbuf + (int64_t)row * a.gw;
#pragma unroll
            for (int v = 0; v < NA; ++v) dst[v] = (double)s[v];
        }
    }
}

template <int J>
__global__ void __launch_bounds__(64) k_slab_long(const double *__restrict__ part, const LongRow *__restrict__ lr,
                                                  double *__restrict__ rowbuf, int gw)
{
    constexpr int NA = nacc_vc(J);
    __shared__ double sh[NA];
    const LongRow L = lr[blockIdx.x];
    sum_partials<NA>(part, L, sh, threadIdx.x);
    for (int v = threadIdx.x; v < NA; v += 64) rowbuf[(int64_t)L.row * gw + v] = sh[v];
}

// kp row r = [a_r (J) | packed a_r a_r^T (J(J+1)/2) | 0 padding]
template <int J>
__global__ void __launch_bounds__(256) k_kp(const double *__restrict__ A, int64_t I, int gw, double *__restrict__ kp)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= I) return;
    double a[J];
    load_row<J, double>(A + r * J, a);
    double *d = kp + r * gw;
#pragma unroll
    for (int t = 0; t < J; ++t) d[t] = a[t];
#pragma unroll
    for (int t = 0; t < J; ++t)
#pragma unroll
        for (int v = t; v < J; ++v) d[J + sym<J>(t, v)] = a[t] * a[v];
    for (int v = nacc_vc(J); v < gw; ++v) d[v] = 0.0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_colcopy(const double *__restrict__ A, int64_t I, int J, T *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= I * J) return;
    const int64_t j = q / I, i = q % I;
    out[q] = (T)A[i * J + j];
}

// Partial Gram of kGramRows rows: part[b] = sum_r rowbuf_r^T kp_r (gw x gw).
// Thread (ti, tj) owns an 8 x 8 tile; rows are staged through LDS.
template <int GW>
__global__ void __launch_bounds__(256) k_gram(const double *__restrict__ rb, const double *__restrict__ kp,
                                              int64_t nrows, double *__restrict__ part)
{
    constexpr int TB = GW / 8;
    constexpr int NT = TB * TB;
    constexpr int BR = 16;
    __shared__ double sx[BR][GW];
    __shared__ double sy[BR][GW];
    const int64_t r0 = (int64_t)blockIdx.x * kGramRows;
    const int64_t r1 = r0 + kGramRows < nrows ? r0 + kGramRows : nrows;
    const int t = threadIdx.x;
    const int ti = t / TB, tj = t % TB;
    double acc[8][8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[p][q] = 0.0;
    for (int64_t b0 = r0; b0 < r1; b0 += BR) {
        const int nb = (int)(r1 - b0 < BR ? r1 - b0 : BR);
        __syncthreads();
        for (int q = t; q < BR * GW; q += blockDim.x) {
            const int rr = q / GW, cc = q % GW;
            sx[rr][cc] = rr < nb ? rb[(b0 + rr) * GW + cc] : 0.0;
            sy[rr][cc] = rr < nb ? kp[(b0 + rr) * GW + cc] : 0.0;
        }
        __syncthreads();
        if (t < NT) {
            for (int rr = 0; rr < BR; ++rr) {
                double x[8], y[8];
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    x[p] = sx[rr][ti * 8 + p];
                    y[p] = sy[rr][tj * 8 + p];
                }
#pragma unroll
                for (int p = 0; p < 8; ++p)
#pragma unroll
                    for (int q = 0; q < 8; ++q) acc[p][q] = __builtin_fma(x[p], y[q], acc[p][q]);
            }
        }
    }
    if (t < NT) {
        double *o = part + (int64_t)blockIdx.x * GW * GW;
#pragma unroll
        for (int p = 0; p < 8; ++p)
#pragma unroll
            for (int q = 0; q < 8; ++q) o[(ti * 8 + p) * GW + tj * 8 + q] = acc[p][q];
    }
}

// Fixed-order sum of the gram partials.
__global__ void __launch_bounds__(256) k_gramsum(const double *__restrict__ part, int64_t nparts, int n,
                                                 double *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t c = 0;
    for (; c + 4 <= nparts; c += 4) {
        s0 += part[c * n + q];
        s1 += part[(c + 1) * n + q];
        s2 += part[(c + 2) * n + q];
        s3 += part[(c + 3) * n + q];
    }
    for (; c < nparts; ++c) s0 += part[c * n + q];
    out[q] = (s0 + s1) + (s2 + s3);
}

__device__ __forceinline__ int symr(int J, int t, int u)
{
    if (t > u) {
        const int x = t;
        t = u;
        u = x;
    }
    return t * J - t * (t - 1) / 2 + (u - t);
}

// Sequential updates of one slab (KEYS = false) or its core keys (KEYS = true).
template <int J, bool KEYS>
__global__ void __launch_bounds__(64) k_slabsolve(const double *__restrict__ gram, double *core,
                                                  const uint8_t *__restrict__ cmask, int64_t base, double lambda,
                                                  int reg, double *__restrict__ dprev, double *__restrict__ keys)
{
    constexpr int GW = gram_width(J);
    constexpr int B = J * J;
    constexpr int CPL = (B + kWave - 1) / kWave;
    __shared__ double sg[GW * GW];
    const int lane = threadIdx.x;
    for (int q = lane; q < GW * GW; q += kWave) sg[q] = gram[q];
    __syncthreads();
    auto H = [&](int q, int q2) {
        return sg[(J + symr(J, q / J, q2 / J)) * GW + J + symr(J, q % J, q2 % J)];
    };
    auto RR = [&](int q) { return sg[(q / J) * GW + (q % J)]; };

    if constexpr (KEYS) {
        // Delta(G_q) = sum (2 e + G_q w_q) G_q w_q = 2 G_q rr_q + G_q^2 H_qq  (Eq. 5)
        for (int q = lane; q < B; q += kWave) {
            const double g = core[base + q];
            keys[base + q] = cmask[base + q] ? HUGE_VAL : 2.0 * g * RR(q) + g * g * H(q, q);
        }
    } else {
        double corr[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) corr[c] = 0.0;
        for (int q = 0; q < B; ++q) {
            const int64_t flat = base + q;
            if (cmask[flat]) {
                if (lane == 0) dprev[q] = 0.0;
                continue;
            }
            const int oc = q / kWave;
            double mine = corr[0];
#pragma unroll
            for (int c = 1; c < CPL; ++c)
                if (oc == c) mine = corr[c];
            const double cq = __shfl(mine, q % kWave, kWave);
            const double hqq = H(q, q);
            const double g = core[flat];
            const double num = RR(q) - cq + g * hqq;
            const double nw = coord_min(reg, lambda, num, hqq);
            const double dq = nw - g;
            if (lane == 0) {
                core[flat] = nw;
                dprev[q] = dq;
            }
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int q2 = lane + c * kWave;
                if (q2 > q && q2 < B) corr[c] = __builtin_fma(H(q2, q), dq, corr[c]);
            }
        }
    }
}

template <int N, int J, typename T>
static hipError_t core_pass_t(vest_ctx *c, bool keys, double *key_out)
{
    const int last = N - 1;
    const ModeLayout &L = c->lay[last];
    const bool f32 = std::is_same<T, float>::value;
    constexpr int GW = gram_width(J);
    hipStream_t st = c->stream;
    const int64_t Ilast = c->d.dims[last];

    SlabArgs<N, J, T> a{};
    a.waves = L.waves;
    a.nwaves = L.nwaves;
    a.row_order = L.row_order;
    for (int m = 0; m < N - 1; ++m) a.oidx[m] = L.oidx[m];
    for (int m = 0; m < N - 2; ++m) {
        const int64_t I = c->d.dims[m];
        hipLaunchKernelGGL(k_colcopy<T>, dim3((unsigned)((I * J + 255) / 256)), dim3(256), 0, st, c->A[m], I, J,
                           reinterpret_cast<T *>(c->colA[m]));
        a.colA[m] = reinterpret_cast<const T *>(c->colA[m]);
        a.dimA[m] = I;
    }
    a.Amid = f32 ? reinterpret_cast<const T *>(c->A32[N - 2]) : reinterpret_cast<const T *>(c->A[N - 2]);
    a.Alast = f32 ? reinterpret_cast<const T *>(c->A32[last]) : reinterpret_cast<const T *>(c->A[last]);
    a.e = reinterpret_cast<T *>(c->e);
    a.dprev = c->dprev;
    a.rowbuf = c->rowbuf;
    a.gw = GW;
    a.partials = c->partials;
    hipLaunchKernelGGL(k_kp<J>, dim3((unsigned)((Ilast + 255) / 256)), dim3(256), 0, st, c->A[last], Ilast, GW,
                       c->kp);

    const int blocks = (L.nwaves + 3) / 4;
    const int64_t gchunks = (Ilast + kGramRows - 1) / kGramRows;
    const int nslab = ipow(J, N - 2);
    auto digits = [&](int s, int32_t *out) {
        for (int m = N - 3; m >= 0; --m) {
            out[m] = s % J;
            s /= J;
        }
    };
    for (int s = 0; s < nslab; ++s) {
        digits(s, a.lead);
        a.has_prev = (!keys && s > 0) ? 1 : 0;
        if (s > 0) digits(s - 1, a.lprev);
        if (blocks > 0) hipLaunchKernelGGL((k_slab<N, J, T, true>), dim3(blocks), dim3(256), 0, st, a);
        if (L.nlong > 0)
            hipLaunchKernelGGL(k_slab_long<J>, dim3(L.nlong), dim3(64), 0, st, c->partials, L.longrows, c->rowbuf,
                               GW);
        hipLaunchKernelGGL(k_gram<GW>, dim3((unsigned)gchunks), dim3(256), 0, st, c->rowbuf, c->kp, Ilast,
                           c->gram_part);
        hipLaunchKernelGGL(k_gramsum, dim3((GW * GW + 255) / 256), dim3(256), 0, st, c->gram_part, gchunks,
                           GW * GW, c->gram);
        const int64_t base = (int64_t)s * J * J;
        if (keys)
            hipLaunchKernelGGL((k_slabsolve<J, true>), dim3(1), dim3(64), 0, st, c->gram, c->core, c->cmask, base,
                               c->d.lambda, c->d.reg, c->dprev, key_out);
        else
            hipLaunchKernelGGL((k_slabsolve<J, false>), dim3(1), dim3(64), 0, st, c->gram, c->core, c->cmask, base,
                               c->d.lambda, c->d.reg, c->dprev, key_out);
    }
    if (!keys) {
        // apply the last slab's change to the residual
        a.has_prev = 1;
        digits(nslab - 1, a.lprev);
        if (blocks > 0) hipLaunchKernelGGL((k_slab<N, J, T, false>), dim3(blocks), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

static hipError_t core_pass(vest_ctx *c, bool keys, double *key_out)
{
#define VEST_CASE(NN, JJ)                                                                \
    if (c->N == NN && c->J == JJ)                                                        \
        return c->d.precision == VEST_FP32 ? core_pass_t<NN, JJ, float>(c, keys, key_out) \
                                           : core_pass_t<NN, JJ, double>(c, keys, key_out);
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_core_sweep(vest_ctx *c) { return core_pass(c, false, nullptr); }
hipError_t launch_core_keys(vest_ctx *c, double *core_key) { return core_pass(c, true, core_key); }

bool shape_supported(int N, int J)
{
#define VEST_CASE(NN, JJ) \
    if (N == NN && J == JJ) return true;
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return false;
}

}  // namespace vest
