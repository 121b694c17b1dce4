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
    const T *colA[NL];            // column-major copies of modes 0..N-3; at order 3 column pairs
                                  // (a_{i,s-1}, a_{i,s}) of mode 0 (see colcopy_body)
    const T *rowA[NL];            // gather copies of modes 0..N-3 (row stride gather_ld)
    int64_t dimA[NL];
    int32_t lead[NL];             // leading core indices of this slab
    int32_t lprev[NL];            // ... of the previous slab
    const T *ms;                  // mode N-2 factor row of every slot (see ms_index)
    const T *Alast;               // mode N-1 factor, gather copy (row stride gather_ld)
    T *e;
    const double *dprev;          // [J][J] change of the previous slab's elements
    double *rowbuf;               // [I_{N-1}][ldrb]
    int32_t ldrb;
    double *partials;
    double *wsum;                 // per wave: sum of e^2 after the correction (k_slab with E2)
    int32_t blead[kKeyAccMax / 2 * NL];  // k_slabkeys: leading indices of each slab of the batch
};

// The mode N-2 factor row of every entry is read from the slot-ordered copy
// written by the residual pass (coalesced, no gather).  Entries are taken U
// at a time per lane and every load of a batch is issued unconditionally (the
// slot is clamped into the wave's range), so a batch costs two memory
// latencies -- streamed loads, then the column gathers of the leading factors
// -- instead of a dependent chain per entry; padding slots are masked out of
// the arithmetic by selects.
// FP32 batches of four, FP64 of two (register budget).
template <typename T>
__host__ __device__ constexpr int slab_u() { return sizeof(T) == 4 ? 4 : 2; }

// With E2 every wave also writes the sum of e^2 over its entries, e taken
// after the previous slab's change (the residual this slab's statistics see).
template <int N, int J, typename T, bool ACC, bool E2 = false>
__device__ __forceinline__ void slab_body(const SlabArgs<N, J, T> &a, int bx)
{
    constexpr int NA = nacc_vc(J);
    constexpr int U = slab_u<T>();
    constexpr int NI = N > 2 ? N - 2 : 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = bx * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (wave >= a.nwaves) return;
    const WaveInfo wi = a.waves[wave];
    const int grp = lane >> wi.glog;
    const bool has_row = grp < wi.nrows;
    const int row = has_row ? a.row_order[wi.first + grp] : 0;

    T u[J];
    if (a.has_prev) {
        T al[J];
        if (has_row) load_grow<J, T>(a.Alast + (int64_t)row * gather_ld(J, sizeof(T)), al);
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
    double e2 = 0.0;

    // the leading indices of the next batch are loaded one batch ahead, so the
    // column gathers they address need not wait for them
    int32_t ii[U][NI];
    auto load_idx = [&](int k0, int32_t (&dst)[U][NI]) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int kk = k0 + q < wi.K ? k0 + q : wi.K - 1;
#pragma unroll
            for (int m = 0; m < NI; ++m) dst[q][m] = ld_stream(a.oidx[m] + wi.base + (int64_t)kk * kWave + lane);
        }
    };
    if (wi.K > 0) load_idx(0, ii);
    for (int k0 = 0; k0 < wi.K; k0 += U) {
        int64_t sl[U];
        int32_t ni[U][NI];
        T mv[U][J], ev[U];
        load_idx(k0 + U, ni);
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int kk = k0 + q < wi.K ? k0 + q : wi.K - 1;
            sl[q] = wi.base + (int64_t)kk * kWave + lane;
            ev[q] = ld_stream(a.e + sl[q]);
            ms_load<J, T>(a.ms, sl[q], mv[q]);
        }
        bool ok[U];
        T p[U], pp[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            ok[q] = (k0 + q < wi.K) && ii[q][0] >= 0;
            T pv = T(1), pr = T(1);
            if constexpr (N == 3) {
                // one aligned pair load: (a_{i,s-1}, a_{i,s}) of slab s = lead, whose previous
                // slab is s - 1; the apply-only pass reads the pair of the previous slab
                const int64_t i = ii[q][0] > 0 ? ii[q][0] : 0;
                const int64_t c = ACC ? a.lead[0] : a.lprev[0];
                typedef T t2 __attribute__((ext_vector_type(2)));
                const t2 pair = *reinterpret_cast<const t2 *>(a.colA[0] + 2 * (c * a.dimA[0] + i));
                if constexpr (ACC) pv = pair.y;
                if (a.has_prev) pr = ACC ? pair.x : pair.y;
            } else {
#pragma unroll
                for (int m = 0; m < N - 2; ++m) {
                    const int64_t i = ii[q][m] > 0 ? ii[q][m] : 0;
                    if constexpr (ACC) pv *= a.colA[m][(int64_t)a.lead[m] * a.dimA[m] + i];
                    if (a.has_prev) pr *= a.colA[m][(int64_t)a.lprev[m] * a.dimA[m] + i];
                }
            }
            p[q] = ok[q] ? pv : T(0);
            pp[q] = ok[q] ? pr : T(0);
            ev[q] = ok[q] ? ev[q] : T(0);
#pragma unroll
            for (int t = 0; t < J; ++t) mv[q][t] = ok[q] ? mv[q][t] : T(0);
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            T e = ev[q];
            if (a.has_prev) {
                T du = mv[q][0] * u[0];
#pragma unroll
                for (int t = 1; t < J; ++t) du = vfma(mv[q][t], u[t], du);
                e -= pp[q] * du;
                if (ok[q]) st_stream(e, a.e + sl[q]);
            }
            if constexpr (E2) e2 += (double)e * (double)e;   // zero for padding slots
            if constexpr (ACC) {
                T w[J];
#pragma unroll
                for (int t = 0; t < J; ++t) w[t] = p[q] * mv[q][t];
#pragma unroll
                for (int t = 0; t < J; ++t) {
                    s[t] = vfma(e, w[t], s[t]);
#pragma unroll
                    for (int v = t; v < J; ++v) s[J + sym<J>(t, v)] = vfma(w[t], w[v], s[J + sym<J>(t, v)]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int m = 0; m < NI; ++m) ii[q][m] = ni[q][m];
    }
    if constexpr (E2) {
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) e2 += __shfl_xor(e2, m);
        if (lane == 0) a.wsum[wave] = e2;
    }
    if constexpr (ACC) {
        group_reduce<NA, T>(s, wi.glog);
        if (wi.chunk >= 0) {
            store_partial<NA, T>(a.partials, wi.chunk, s, lane);
            return;
        }
        if (has_row && (lane & ((1 << wi.glog) - 1)) == 0) {
            double *dst = a.rowbuf + (int64_t)row * a.ldrb;
#pragma unroll
            for (int v = 0; v < NA; ++v) dst[v] = (double)s[v];
        }
    }
}

template <int N, int J, typename T, bool ACC, bool E2 = false>
__global__ void __launch_bounds__(256) k_slab(SlabArgs<N, J, T> a)
{
    slab_body<N, J, T, ACC, E2>(a, blockIdx.x);
}

// Several contexts of one shape in one launch (virtual block b - off[t] of
// task t; see k_rowgroup_multi).
template <int N, int J, typename T, bool ACC, bool E2 = false>
__global__ void __launch_bounds__(256) k_slab_multi(const SlabArgs<N, J, T> *__restrict__ tab,
                                                    const int32_t *__restrict__ off, int ntask, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const SlabArgs<N, J, T> a = tab[t];   // arguments in registers, read once
        slab_body<N, J, T, ACC, E2>(a, b - off[t]);
    }
}

// Core responsibility statistics of SB consecutive slabs in one pass:
// per row r and slab b,  R_b[t] = sum e p_b a^(N-1)_t  and, when WITH_D,
// D_b[t] = sum (p_b a^(N-1)_t)^2.  The residual is not modified.  Streamed
// loads as in k_slab.  The leading factor values p_b of the SB slabs come
// either from SB column gathers (column copies of the leading modes) or, in
// the ROWP form, from one gathered row per leading mode (one cache line) and
// an exact arithmetic pick of the slab's digit.
template <int N, int J, typename T, int SB, bool WITH_D>
__global__ void __launch_bounds__(256) k_slabkeys(SlabArgs<N, J, T> a, int nsb)
{
    constexpr int PER = WITH_D ? 2 * J : J;
    constexpr int NA = PER * SB;
    // Order 3: one leading row per entry (see above), FP32 one entry per batch
    // to keep the row and the picks in registers; with more leading modes the
    // rows and picks cost more registers than the column gathers save
    constexpr bool ROWP = N == 3;
    constexpr int U = (ROWP && sizeof(T) == 4) ? 1 : slab_u<T>();
    constexpr int NL = SlabArgs<N, J, T>::NL;
    constexpr int NI = N > 2 ? N - 2 : 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (wave >= a.nwaves) return;
    const WaveInfo wi = a.waves[wave];
    const int grp = lane >> wi.glog;
    const bool has_row = grp < wi.nrows;
    const int row = has_row ? a.row_order[wi.first + grp] : 0;
    T s[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) s[v] = T(0);
    int32_t ii[U][NI];   // leading indices, one batch ahead (as in k_slab)
    auto load_idx = [&](int k0, int32_t (&dst)[U][NI]) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int kk = k0 + q < wi.K ? k0 + q : wi.K - 1;
#pragma unroll
            for (int m = 0; m < NI; ++m) dst[q][m] = ld_stream(a.oidx[m] + wi.base + (int64_t)kk * kWave + lane);
        }
    };
    if (wi.K > 0) load_idx(0, ii);
    for (int k0 = 0; k0 < wi.K; k0 += U) {
        int64_t sl[U];
        int32_t ni[U][NI];
        T mv[U][J], ev[U], lr[U][NI][J];
        load_idx(k0 + U, ni);
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int kk = k0 + q < wi.K ? k0 + q : wi.K - 1;
            sl[q] = wi.base + (int64_t)kk * kWave + lane;
            ev[q] = ld_stream(a.e + sl[q]);
            ms_load<J, T>(a.ms, sl[q], mv[q]);
            if constexpr (ROWP) {
#pragma unroll
                for (int m = 0; m < N - 2; ++m)
                    load_grow<J, T>(a.rowA[m] + (int64_t)(ii[q][m] > 0 ? ii[q][m] : 0) * gather_ld(J, sizeof(T)),
                                    lr[q][m]);
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const bool ok = (k0 + q < wi.K) && ii[q][0] >= 0;
            const T evq = ok ? ev[q] : T(0);
            T mq[J];
#pragma unroll
            for (int t = 0; t < J; ++t) mq[t] = ok ? mv[q][t] : T(0);
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                if (b < nsb) {   // (no early exit: the accumulator indices stay compile-time)
                    T p = T(1);
#pragma unroll
                    for (int m = 0; m < N - 2; ++m) {
                        if constexpr (ROWP) {
                            p *= pick<J, T>(lr[q][m], a.blead[b * NL + m]);
                        } else {
                            const int64_t i = ii[q][m] > 0 ? ii[q][m] : 0;
                            p *= a.colA[m][(int64_t)a.blead[b * NL + m] * a.dimA[m] + i];
                        }
                    }
                    const T ep = evq * p;
#pragma unroll
                    for (int t = 0; t < J; ++t) {
                        s[b * PER + t] = vfma(ep, mq[t], s[b * PER + t]);
                        if constexpr (WITH_D) {
                            const T w = p * mq[t];
                            s[b * PER + J + t] = vfma(w, w, s[b * PER + J + t]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int m = 0; m < NI; ++m) ii[q][m] = ni[q][m];
    }
    group_reduce<NA, T>(s, wi.glog);
    if (wi.chunk >= 0) {
        store_partial<NA, T>(a.partials, wi.chunk, s, lane);
        return;
    }
    if (has_row && (lane & ((1 << wi.glog) - 1)) == 0) {
        double *dst = a.rowbuf + (int64_t)row * a.ldrb;
#pragma unroll
        for (int v = 0; v < NA; ++v) dst[v] = (double)s[v];
    }
}

template <int NA>
__device__ __forceinline__ void slab_long_body(const double *__restrict__ part, const LongRow *__restrict__ lr,
                                               double *__restrict__ rowbuf, int ldrb, int bx)
{
    __shared__ double sh[NA];
    const LongRow L = lr[bx];
    sum_partials<NA>(part, L, sh, threadIdx.x);
    for (int v = threadIdx.x; v < NA; v += 64) rowbuf[(int64_t)L.row * ldrb + v] = sh[v];
}

template <int NA>
__global__ void __launch_bounds__(64) k_slab_long(const double *__restrict__ part, const LongRow *__restrict__ lr,
                                                  double *__restrict__ rowbuf, int ldrb)
{
    slab_long_body<NA>(part, lr, rowbuf, ldrb, blockIdx.x);
}

struct SlabLongTask {
    const double *part;
    const LongRow *lr;
    double *rowbuf;
    int32_t ldrb;
};

template <int NA>
__global__ void __launch_bounds__(64) k_slab_long_multi(const SlabLongTask *__restrict__ tab,
                                                        const int32_t *__restrict__ off, int ntask, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const SlabLongTask tk = tab[t];
        slab_long_body<NA>(tk.part, tk.lr, tk.rowbuf, tk.ldrb, b - off[t]);
        __syncthreads();   // the LDS sums are reused by the next long row
    }
}

// kp row r = [a_r (J) | packed a_r a_r^T (J(J+1)/2) | 0 padding]
template <int J>
__device__ __forceinline__ void kp_body(const double *__restrict__ A, int64_t I, int gw, double *__restrict__ kp, int bx)
{
    const int64_t r = (int64_t)bx * blockDim.x + threadIdx.x;
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

template <int J>
__global__ void __launch_bounds__(256) k_kp(const double *__restrict__ A, int64_t I, int gw, double *__restrict__ kp)
{
    kp_body<J>(A, I, gw, kp, blockIdx.x);
}

struct KpTask {
    const double *A;
    int64_t I;
    int32_t gw;
    double *kp;
};

template <int J>
__global__ void __launch_bounds__(256) k_kp_multi(const KpTask *__restrict__ tab, const int32_t *__restrict__ off,
                                                  int ntask, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const KpTask tk = tab[t];
        kp_body<J>(tk.A, tk.I, tk.gw, tk.kp, b - off[t]);
    }
}

// kp2 row r = [a_r (J) | a_r^2 (J) | 0 padding]
template <int J>
__global__ void __launch_bounds__(256) k_kp2(const double *__restrict__ A, int64_t I, int w, double *__restrict__ kp)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= I) return;
    double a[J];
    load_row<J, double>(A + r * J, a);
    double *d = kp + r * w;
#pragma unroll
    for (int t = 0; t < J; ++t) {
        d[t] = a[t];
        d[J + t] = a[t] * a[t];
    }
    for (int v = 2 * J; v < w; ++v) d[v] = 0.0;
}

// Column-major copy of a leading factor for the core passes: out[j I + i] =
// a_{i j}.  With pair set (order 3, one leading mode, whose slabs s run in
// order) column s holds the pairs (a_{i,s-1}, a_{i,s}) -- a_{i,0} twice for
// s = 0 -- so that a slab pass reads both leading values of an entry with one
// aligned load: out[2 (s I + i) + {0, 1}].
template <typename T>
__device__ __forceinline__ void colcopy_body(const double *__restrict__ A, int64_t I, int J, int pair,
                                             T *__restrict__ out, int bx)
{
    const int64_t q = (int64_t)bx * blockDim.x + threadIdx.x;
    if (q >= I * J) return;
    const int64_t j = q / I, i = q % I;
    if (pair) {
        out[2 * q] = (T)A[i * J + (j > 0 ? j - 1 : 0)];
        out[2 * q + 1] = (T)A[i * J + j];
    } else {
        out[q] = (T)A[i * J + j];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_colcopy(const double *__restrict__ A, int64_t I, int J, int pair,
                                                 T *__restrict__ out)
{
    colcopy_body<T>(A, I, J, pair, out, blockIdx.x);
}

template <typename T>
struct ColTask {
    const double *A;
    int64_t I;
    int32_t J;
    int32_t pair;
    T *out;
};

template <typename T>
__global__ void __launch_bounds__(256) k_colcopy_multi(const ColTask<T> *__restrict__ tab,
                                                       const int32_t *__restrict__ off, int ntask, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const ColTask<T> tk = tab[t];
        colcopy_body<T>(tk.A, tk.I, tk.J, tk.pair, tk.out, b - off[t]);
    }
}

// Partial product of `rows` rows (a multiple of 32) on the FP64 matrix cores:
// part[b] = sum_r rb_r^T kp_r (W1 x W2).  Wave ti of the block owns the
// 16-row band ti of the output and every 16 x 16 tile along it; one
// v_mfma_f64_16x16x4 step consumes four rows r: lane l supplies
// A[l % 16][l / 16] = rb[r0 + l / 16][16 ti + l % 16] and
// B[l / 16][l % 16] = kp[r0 + l / 16][16 tj + l % 16], and tile element
// (i, j) ends in lane 16 (i % 4) + j, register i / 4.  The kp rows, read by
// every wave, are staged in LDS 32 at a time; columns past W1 / W2 and rows
// past nrows enter as zeros.
template <int W1, int W2>
__device__ __forceinline__ void gram_body(const double *__restrict__ rb, int ldrb, const double *__restrict__ kp,
                                          int ldkp, int64_t nrows, int rows, double *__restrict__ part, int bx)
{
    constexpr int T1 = (W1 + 15) / 16, T2 = (W2 + 15) / 16;
    constexpr int SUB = 32, W2P = 16 * T2, NT = 64 * T1;
    constexpr int PER = (SUB * W2P + NT - 1) / NT;
    static_assert(kGramRows % SUB == 0, "sub-blocks of 32 rows");
    __shared__ double skp[SUB * W2P];
    const int lane = threadIdx.x & (kWave - 1), ti = threadIdx.x / kWave;
    const int64_t r0 = (int64_t)bx * rows;
    const int ci = 16 * ti + (lane & 15);
    f64x4 acc[T2];
#pragma unroll
    for (int tj = 0; tj < T2; ++tj) acc[tj] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int s0 = 0; s0 < rows; s0 += SUB) {
        double v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = threadIdx.x + i * NT;
            const int rr = q / W2P, cc = q % W2P;
            const int64_t r = r0 + s0 + rr;
            v[i] = (q < SUB * W2P && r < nrows && cc < W2) ? kp[r * ldkp + cc] : 0.0;
        }
        double av[SUB / 4];
#pragma unroll
        for (int k = 0; k < SUB / 4; ++k) {
            const int64_t r = r0 + s0 + 4 * k + (lane >> 4);
            av[k] = (r < nrows && ci < W1) ? rb[r * ldrb + ci] : 0.0;
        }
        __syncthreads();  // the previous sub-block's reads of skp are done
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = threadIdx.x + i * NT;
            if (q < SUB * W2P) skp[q] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SUB / 4; ++k) {
            const int rr = 4 * k + (lane >> 4);
#pragma unroll
            for (int tj = 0; tj < T2; ++tj)
                acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[k], skp[rr * W2P + 16 * tj + (lane & 15)], acc[tj], 0,
                                                              0, 0);
        }
    }
    double *o = part + (int64_t)bx * W1 * W2;
#pragma unroll
    for (int tj = 0; tj < T2; ++tj) {
        const int j = 16 * tj + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 16 * ti + 4 * q + (lane >> 4);
            if (i < W1 && j < W2) o[i * W2 + j] = acc[tj][q];
        }
    }
}

template <int W1, int W2>
__global__ void __launch_bounds__(64 * ((W1 + 15) / 16)) k_gram(const double *__restrict__ rb, int ldrb,
                                                                 const double *__restrict__ kp, int ldkp,
                                                                 int64_t nrows, int rows, double *__restrict__ part)
{
    gram_body<W1, W2>(rb, ldrb, kp, ldkp, nrows, rows, part, blockIdx.x);
}

struct GramTask {
    const double *rb;
    const double *kp;
    double *part;
    int64_t nrows;
    int32_t ldrb, ldkp, rows;
};

template <int W1>
constexpr int gram_threads() { return 64 * ((W1 + 15) / 16); }

// Rows per gram partial: the smallest multiple of kGramRows that keeps the
// launch at about two waves per SIMD (1024 SIMDs); fewer, longer partials
// also shorten the fixed-order sum.  The workspace holds partials for
// kGramRows, so any larger choice fits.
template <int W1>
static int gram_rows(int64_t nrows)
{
    const int T1 = (W1 + 15) / 16;
    int rows = kGramRows;
    while (rows < 4096 && ((nrows + rows - 1) / rows) * T1 > 2048) rows *= 2;
    return rows;
}

// Partial Gram product of one slab in the core sweep, over `rows` rows of the
// last mode, on the FP64 matrix cores.  Of rb_r^T kp_r (rb_r = [R_r | M_r],
// kp_r = [a_r | (a a^T)_r]) the solve reads two blocks: M^T (a a^T), the slab's
// Gram matrix in symmetric-pair form (nm x nm, nm = J (J + 1) / 2), and R^T a,
// its right-hand side (J x J); the two cross blocks are not formed.  Wave ti
// owns the 16-row band ti of the M block and its TM tiles.  The R x a tile is
// shared: wave w takes the k-steps w, w + TM, ... of every 32-row sub-block
// and the TM accumulators are added in wave order at the end.  The next
// sub-block's operands are loaded before the current one's products are
// issued.  Partial layout: the M block (16 TM x 16 TM, row-major, padding
// rows and columns zero), then the 16 x 16 R x a tile.
template <int J>
__device__ __forceinline__ void gram_core_body(const double *__restrict__ rb, int ldrb, const double *__restrict__ kp,
                                               int ldkp, int64_t nrows, int rows, double *__restrict__ part, int bx)
{
    constexpr int NM = gram_nm(J), TM = gram_tm(J), MW = 16 * TM;
    constexpr int SUB = 32, KS = SUB / 4;   // rows per sub-block, k-steps per sub-block
    constexpr int KW = J + NM;              // staged kp columns: a, then a a^T
    constexpr int NT = 64 * TM;
    constexpr int PER = (SUB * KW + NT - 1) / NT;
    constexpr int KR = (KS + TM - 1) / TM;  // R x a k-steps of one wave per sub-block
    static_assert(kGramRows % SUB == 0, "sub-blocks of 32 rows");
    __shared__ double skp[SUB * KW];
    __shared__ double sred[TM][4][kWave];
    const int lane = threadIdx.x & (kWave - 1), ti = threadIdx.x / kWave;
    const int64_t r0 = (int64_t)bx * rows;
    const int cm = 16 * ti + (lane & 15);   // this lane's M column (A operand)
    const int cr = lane & 15;               // this lane's R column
    // B operand columns of the staged rows: tile tj reads a a^T pair 16 tj + (lane & 15)
    int bcol[TM];
    bool bok[TM];
#pragma unroll
    for (int tj = 0; tj < TM; ++tj) {
        bok[tj] = 16 * tj + (lane & 15) < NM;
        bcol[tj] = bok[tj] ? J + 16 * tj + (lane & 15) : 0;
    }
    const bool rok = cr < J;
    f64x4 acc[TM], racc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int tj = 0; tj < TM; ++tj) acc[tj] = f64x4{0.0, 0.0, 0.0, 0.0};
    double v[PER], am[KS], ar[KR];
    auto load = [&](int s0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = threadIdx.x + i * NT;
            const int rr = q / KW, cc = q % KW;
            const int64_t r = r0 + s0 + rr;
            v[i] = (q < SUB * KW && s0 + rr < rows && r < nrows) ? kp[r * ldkp + cc] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int rr = 4 * k + (lane >> 4);
            const int64_t r = r0 + s0 + rr;
            am[k] = (s0 + rr < rows && r < nrows && cm < NM) ? rb[r * ldrb + J + cm] : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) {
            const int k = ti + kk * TM;
            const int rr = 4 * k + (lane >> 4);
            const int64_t r = r0 + s0 + rr;
            ar[kk] = (k < KS && s0 + rr < rows && r < nrows && rok) ? rb[r * ldrb + cr] : 0.0;
        }
    };
    load(0);
    for (int s0 = 0; s0 < rows; s0 += SUB) {
        __syncthreads();   // the previous sub-block's reads of skp are done
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = threadIdx.x + i * NT;
            if (q < SUB * KW) skp[q] = v[i];
        }
        __syncthreads();
        double cam[KS], car[KR];
#pragma unroll
        for (int k = 0; k < KS; ++k) cam[k] = am[k];
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) car[kk] = ar[kk];
        if (s0 + SUB < rows) load(s0 + SUB);
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int rr = 4 * k + (lane >> 4);
#pragma unroll
            for (int tj = 0; tj < TM; ++tj) {
                const double b = bok[tj] ? skp[rr * KW + bcol[tj]] : 0.0;
                acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(cam[k], b, acc[tj], 0, 0, 0);
            }
        }
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) {
            const int k = ti + kk * TM;
            if (k < KS) {
                const int rr = 4 * k + (lane >> 4);
                const double b = rok ? skp[rr * KW + cr] : 0.0;
                racc = __builtin_amdgcn_mfma_f64_16x16x4f64(car[kk], b, racc, 0, 0, 0);
            }
        }
    }
    double *o = part + (int64_t)bx * gram_core_cells(J);
#pragma unroll
    for (int tj = 0; tj < TM; ++tj) {
        const int j = 16 * tj + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 16 * ti + 4 * q + (lane >> 4);
            o[i * MW + j] = acc[tj][q];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) sred[ti][q][lane] = racc[q];
    __syncthreads();
    if (ti == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double t = sred[0][q][lane];
            for (int w = 1; w < TM; ++w) t += sred[w][q][lane];
            o[MW * MW + (4 * q + (lane >> 4)) * 16 + (lane & 15)] = t;
        }
    }
}

template <int J>
__global__ void __launch_bounds__(64 * gram_tm(J)) k_gram_core(const double *__restrict__ rb, int ldrb,
                                                                const double *__restrict__ kp, int ldkp,
                                                                int64_t nrows, int rows, double *__restrict__ part)
{
    gram_core_body<J>(rb, ldrb, kp, ldkp, nrows, rows, part, blockIdx.x);
}

// One block per partial of every task (grid = total), no loop around the
// body: a task loop led the allocator to one wave per SIMD with AGPR copies,
// where the one-context kernel holds two waves at under 200 VGPRs.
template <int J>
__global__ void __launch_bounds__(64 * gram_tm(J)) k_gram_core_multi(const GramTask *__restrict__ tab,
                                                                      const int32_t *__restrict__ off, int ntask,
                                                                      int total)
{
    const int b = blockIdx.x;
    if (b >= total) return;
    const int t = task_of(off, ntask, b);
    const GramTask tk = tab[t];
    gram_core_body<J>(tk.rb, tk.ldrb, tk.kp, tk.ldkp, tk.nrows, tk.rows, tk.part, b - off[t]);
}

// Rows per partial of the core Gram product (as gram_rows, TM waves a block).
template <int J>
static int gram_core_rows(int64_t nrows)
{
    int rows = kGramRows;
    while (rows < 4096 && ((nrows + rows - 1) / rows) * gram_tm(J) > 2048) rows *= 2;
    return rows;
}

// Position in the slab's Gram layout (rows and columns of width gram_width:
// R x a at rows 0..J-1, columns 0..J-1; M x a a^T at rows and columns J..)
// of cell q of a core Gram partial, or -1 for padding.
template <int J>
__device__ __forceinline__ int gram_core_dst(int q)
{
    constexpr int NM = gram_nm(J), MW = 16 * gram_tm(J), GW = gram_width(J);
    if (q < MW * MW) {
        const int i = q / MW, j = q % MW;
        return (i < NM && j < NM) ? (J + i) * GW + J + j : -1;
    }
    const int i = (q - MW * MW) / 16, j = (q - MW * MW) % 16;
    return (i < J && j < J) ? i * GW + j : -1;
}

// Fixed-order sum of the gram partials: block b owns outputs 64 b .. 64 b + 63;
// wave w of the block sums partials w, w + 16, ... (coalesced across lanes),
// then the 16 wave sums are added in wave order.
template <typename Dst>
__device__ __forceinline__ void gramsum_map_body(const double *__restrict__ part, int64_t nparts, int n,
                                                 double *__restrict__ out, int bx, Dst dst)
{
    __shared__ double sh[16][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = bx * 64 + lane;
    double s0 = 0.0, s1 = 0.0;
    if (q < n) {
        int64_t c = w;
        for (; c + 16 < nparts; c += 32) {
            s0 += part[c * n + q];
            s1 += part[(c + 16) * n + q];
        }
        if (c < nparts) s0 += part[c * n + q];
    }
    sh[w][lane] = s0 + s1;
    __syncthreads();
    if (w == 0 && q < n) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t += sh[i][lane];
        const int d = dst(q);
        if (d >= 0) out[d] = t;
    }
}

__device__ __forceinline__ void gramsum_body(const double *__restrict__ part, int64_t nparts, int n,
                                             double *__restrict__ out, int bx)
{
    gramsum_map_body(part, nparts, n, out, bx, [](int q) { return q; });
}

__global__ void __launch_bounds__(1024) k_gramsum(const double *__restrict__ part, int64_t nparts, int n,
                                                  double *__restrict__ out)
{
    gramsum_body(part, nparts, n, out, blockIdx.x);
}

struct GsumTask {
    const double *part;
    int64_t nparts;
    int32_t n;
    double *out;
};

// Sum of core Gram partials, written into the slab's Gram layout.
template <int J>
__global__ void __launch_bounds__(1024) k_gramsum_core(const double *__restrict__ part, int64_t nparts,
                                                       double *__restrict__ out)
{
    gramsum_map_body(part, nparts, gram_core_cells(J), out, blockIdx.x, [](int q) { return gram_core_dst<J>(q); });
}

template <int J>
__global__ void __launch_bounds__(1024) k_gramsum_core_multi(const GsumTask *__restrict__ tab,
                                                             const int32_t *__restrict__ off, int ntask, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const GsumTask tk = tab[t];
        gramsum_map_body(tk.part, tk.nparts, gram_core_cells(J), tk.out, b - off[t],
                         [](int q) { return gram_core_dst<J>(q); });
        __syncthreads();
    }
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

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sequential updates of one slab's unmarked elements in flat order, one
// wave.  Lane l owns the elements q = l, l + 64, ...: it holds their
// constants (core value, rr_q, H_qq, reciprocal of the denominator), their
// running correction sum_{p<q} H_qp D_p and, once updated, their new value
// and change.  Element q's values reach the chain by readlane from the owner
// lane; the constants do not depend on the chain, so only the correction's
// read sits on it.  H lives in LDS; the column for the next element is read
// one element ahead.  A marked element goes through the same arithmetic with
// its change forced to zero (selects, no branch).  The diagonal of H is kept
// (it is sum w_q^2, reused by the core keys).
template <int J, int REG>
__device__ __forceinline__ void slabsolve_body(const double *__restrict__ gram, double *__restrict__ core,
                                               const uint8_t *__restrict__ cmask, int64_t base, double lambda,
                                               double *__restrict__ dprev, double *__restrict__ hdiag)
{
    constexpr int GW = gram_width(J);
    constexpr int B = J * J;
    constexpr int CPL = (B + kWave - 1) / kWave;
    __shared__ double sg[GW * GW];
    const int lane = threadIdx.x;
    {
        // all loads in flight before the LDS stores
        constexpr int NL = (GW * GW + kWave - 1) / kWave;
        double v[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = lane + i * kWave;
            v[i] = q < GW * GW ? gram[q] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = lane + i * kWave;
            if (q < GW * GW) sg[q] = v[i];
        }
    }
    __syncthreads();
    auto H = [&](int q, int q2) {
        return sg[(J + symr(J, q / J, q2 / J)) * GW + J + symr(J, q % J, q2 % J)];
    };
    double eg[CPL], er[CPL], eh[CPL], eiq[CPL], corr[CPL], nwv[CPL], dqv[CPL];
    uint64_t mbits[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int q = lane + c * kWave;
        const bool in = q < B;
        const double h = in ? H(q, q) : 0.0;
        eg[c] = in ? core[base + q] : 0.0;
        er[c] = in ? sg[(q / J) * GW + (q % J)] : 0.0;
        eh[c] = h;
        eiq[c] = REG == VEST_REG_LF ? 1.0 / (h + lambda) : (h > 0.0 ? 1.0 / (2.0 * h) : 0.0);
        corr[c] = 0.0;
        nwv[c] = eg[c];
        dqv[c] = 0.0;
        mbits[c] = __ballot(in && cmask[base + q] != 0);
        if (in) hdiag[base + q] = h;
    }
    // H(q2, q) for the lane's elements q2 = lane + 64 c, q = t J + u: the LDS
    // index is a per-lane row base for (t2, t), formed once per t, plus a
    // per-lane column offset for (u2, u), tabulated for every u; the loop over
    // u is unrolled so that the table index is a constant.  Out-of-range
    // pairs read cell 0 and are zeroed by a select.
    int t2[CPL], bcol[CPL][J];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int q2 = lane + c * kWave;
        t2[c] = q2 < B ? q2 / J : 0;
        const int u2 = q2 < B ? q2 % J : 0;
#pragma unroll
        for (int u = 0; u < J; ++u) bcol[c][u] = symr(J, u2, u);
    }
    auto rowbase = [&](int t, int (&ra)[CPL]) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) ra[c] = (J + symr(J, t2[c], t)) * GW + J;
    };
    auto hcol = [&](const int (&ra)[CPL], int u, int q, double (&hc)[CPL]) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int q2 = lane + c * kWave;
            const bool ok = q2 < B && q < B;
            const double x = sg[ok ? ra[c] + bcol[c][u] : 0];
            hc[c] = ok ? x : 0.0;
        }
    };
    int ra[CPL];
    rowbase(0, ra);
    double hcur[CPL];
    hcol(ra, 0, 0, hcur);
    for (int t = 0; t < J; ++t) {
        int rn[CPL];
        rowbase(t + 1 < J ? t + 1 : t, rn);
#pragma unroll
        for (int u = 0; u < J; ++u) {
            const int q = t * J + u;
            double hnxt[CPL];
            if (u + 1 < J)
                hcol(ra, u + 1, q + 1, hnxt);
            else
                hcol(rn, 0, q + 1, hnxt);
            const int oc = q / kWave, ol = q % kWave;
            uint64_t mb = mbits[0];
            double vg = eg[0], vr = er[0], vh = eh[0], vi = eiq[0], vc = corr[0];
#pragma unroll
            for (int c = 1; c < CPL; ++c)
                if (oc == c) {
                    mb = mbits[c];
                    vg = eg[c];
                    vr = er[c];
                    vh = eh[c];
                    vi = eiq[c];
                    vc = corr[c];
                }
            const bool dead = (mb >> ol) & 1ull;
            const double g = readlane_d(vg, ol), r = readlane_d(vr, ol), h = readlane_d(vh, ol),
                         iq = readlane_d(vi, ol);
            const double cc = readlane_d(vc, ol);
            // num_q = rr_q - sum_{p<q} H_qp D_p + G_q H_qq
            const double num = r - cc + g * h;
            double nw;
            if constexpr (REG == VEST_REG_LF) {
                nw = num * iq;
            } else {
                const double gg = -2.0 * num;
                const double up = (lambda - gg) * iq, dn = -(lambda + gg) * iq;
                nw = gg > lambda ? up : (gg < -lambda ? dn : 0.0);
            }
            nw = dead ? g : nw;
            const double dq = nw - g;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const bool own = c == oc && lane == ol;
                nwv[c] = own ? nw : nwv[c];
                dqv[c] = own ? dq : dqv[c];
                const int q2 = lane + c * kWave;
                corr[c] = (q2 > q && q2 < B) ? __builtin_fma(hcur[c], dq, corr[c]) : corr[c];
            }
#pragma unroll
            for (int c = 0; c < CPL; ++c) hcur[c] = hnxt[c];
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) ra[c] = rn[c];
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int q = lane + c * kWave;
        if (q < B) {
            core[base + q] = nwv[c];
            dprev[q] = dqv[c];
        }
    }
}

template <int J, int REG>
__global__ void __launch_bounds__(64) k_slabsolve(const double *__restrict__ gram, double *__restrict__ core,
                                                  const uint8_t *__restrict__ cmask, int64_t base, double lambda,
                                                  double *__restrict__ dprev, double *__restrict__ hdiag)
{
    slabsolve_body<J, REG>(gram, core, cmask, base, lambda, dprev, hdiag);
}

struct SolveTask {
    const double *gram;
    double *core;
    const uint8_t *cmask;
    double *dprev;
    double *hdiag;
    int64_t base;
    double lambda;
    int32_t reg;
};

// One block per context (grid = ntask); a launch solves the contexts of
// regulariser REG and leaves the others to the launch for theirs.  One body
// per kernel and no loop around it, as in k_slabsolve: both bodies in one
// kernel, or a task loop, spilled to scratch at J = 9, 10.
template <int J, int REG>
__global__ void __launch_bounds__(64) k_slabsolve_multi(const SolveTask *__restrict__ tab, int ntask)
{
    const int t = blockIdx.x;
    if (t >= ntask) return;
    const SolveTask tk = tab[t];
    if (tk.reg != REG) return;   // uniform over the block
    slabsolve_body<J, REG>(tk.gram, tk.core, tk.cmask, tk.base, tk.lambda, tk.dprev, tk.hdiag);
}

// SSE after the core sweep without applying its last slab's change D to the
// residual.  With e the residual the last slab's statistics were taken from,
// rr and H that slab's right-hand side and Gram matrix:
//   sum (e - sum_q D_q w_q)^2 = sum e^2 - 2 D . rr + D^T H D,
// sum e^2 being the per-wave sums of the last slab pass.  Fixed summation
// order (one block of 1024 threads: its inputs were just written from every
// XCD, so the block keeps many loads in flight).
template <int J>
__device__ __forceinline__ void sse_lag_body(const double *__restrict__ wsum, int nwaves,
                                             const double *__restrict__ gram, const double *__restrict__ dprev,
                                             double *__restrict__ out)
{
    constexpr int GW = gram_width(J), B = J * J;
    __shared__ double sh[1024];
    double s = 0.0;
#pragma unroll 8
    for (int w = threadIdx.x; w < nwaves; w += blockDim.x) s += wsum[w];
    // D^T H D over all element pairs, then - 2 D . rr
    double qf = 0.0;
#pragma unroll 8
    for (int k = threadIdx.x; k < B * B; k += blockDim.x) {
        const int q = k / B, p = k % B;
        const double dq = dprev[q], dp = dprev[p];
        if (dq != 0.0 && dp != 0.0)
            qf += dq * dp * gram[(J + symr(J, q / J, p / J)) * GW + J + symr(J, q % J, p % J)];
    }
    for (int q = threadIdx.x; q < B; q += blockDim.x) qf -= 2.0 * dprev[q] * gram[(q / J) * GW + q % J];
    const double S = block_sum(s, sh);
    __syncthreads();
    const double Q = block_sum(qf, sh);
    if (threadIdx.x == 0) out[0] = S + Q;
}

template <int J>
__global__ void __launch_bounds__(1024) k_sse_lag(const double *__restrict__ wsum, int nwaves,
                                                 const double *__restrict__ gram, const double *__restrict__ dprev,
                                                 double *__restrict__ out)
{
    sse_lag_body<J>(wsum, nwaves, gram, dprev, out);
}

struct SseTask {
    const double *wsum;
    const double *gram;
    const double *dprev;
    double *out;
    int32_t nwaves;
};

template <int J>
__global__ void __launch_bounds__(1024) k_sse_lag_multi(const SseTask *__restrict__ tab, int ntask)
{
    for (int t = blockIdx.x; t < ntask; t += gridDim.x) {
        const SseTask tk = tab[t];
        sse_lag_body<J>(tk.wsum, tk.nwaves, tk.gram, tk.dprev, tk.out);
        __syncthreads();
    }
}

// Core keys of a batch of slabs: Delta(G_q) = 2 G_q sum e w_q + G_q^2 sum w_q^2 (Eq. 5).
// sum w_q^2 comes from the batch product (WITH_D) or from the Gram diagonals
// kept by the last core sweep.
template <int J, bool WITH_D>
__global__ void __launch_bounds__(256) k_corekeys(const double *__restrict__ P, int w2, const double *__restrict__ core,
                                                  const uint8_t *__restrict__ cmask, const double *__restrict__ hdiag,
                                                  int64_t base, int nsb, double *__restrict__ keys)
{
    constexpr int PER = WITH_D ? 2 * J : J;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nsb * J * J) return;
    const int b = q / (J * J), t = (q / J) % J, u = q % J;
    const double r = P[(b * PER + t) * w2 + u];
    const double d = WITH_D ? P[(b * PER + J + t) * w2 + J + u] : hdiag[base + q];
    const double g = core[base + q];
    keys[base + q] = cmask[base + q] ? HUGE_VAL : 2.0 * g * r + g * g * d;
}

template <int N, int J, typename T, bool WITH_D>
static void core_keys_batches(vest_ctx *c, SlabArgs<N, J, T> a, double *key_out, hipStream_t st)
{
    constexpr int SB = key_slabs(N, J, WITH_D, (int)sizeof(T));
    constexpr int PER = WITH_D ? 2 * J : J;
    constexpr int W1 = round8(PER * SB), W2 = round8(2 * J);   // kp2 rows are [a | a^2] in both forms
    static_assert(SB <= kKeyAccMax / 2, "leading indices of a batch fit SlabArgs::blead");
    const ModeLayout &L = c->lay[N - 1];
    const int64_t Ilast = c->d.dims[N - 1];
    const int blocks = (L.nwaves + 3) / 4;
    const int grows = gram_rows<W1>(Ilast);
    const int64_t gchunks = (Ilast + grows - 1) / grows;
    const int nslab = ipow(J, N - 2);
    hipLaunchKernelGGL(k_kp2<J>, dim3((unsigned)((Ilast + 255) / 256)), dim3(256), 0, st, c->A[N - 1], Ilast, W2, c->kp);
    for (int s0 = 0; s0 < nslab; s0 += SB) {
        const int nsb = nslab - s0 < SB ? nslab - s0 : SB;
        for (int b = 0; b < nsb; ++b) {
            int s = s0 + b;
            for (int m = N - 3; m >= 0; --m) {
                a.blead[b * SlabArgs<N, J, T>::NL + m] = s % J;
                s /= J;
            }
        }
        if (blocks > 0)
            hipLaunchKernelGGL((k_slabkeys<N, J, T, SB, WITH_D>), dim3(blocks), dim3(256), 0, st, a, nsb);
        if (L.nlong > 0)
            hipLaunchKernelGGL(k_slab_long<PER * SB>, dim3(L.nlong), dim3(64), 0, st, a.partials, L.longrows,
                               c->rowbuf, c->ldrb);
        hipLaunchKernelGGL((k_gram<W1, W2>), dim3((unsigned)gchunks), dim3(gram_threads<W1>()), 0, st, c->rowbuf, c->ldrb, c->kp, W2,
                           Ilast, grows, c->gram_part);
        hipLaunchKernelGGL(k_gramsum, dim3((W1 * W2 + 63) / 64), dim3(1024), 0, st, c->gram_part, gchunks, W1 * W2,
                           c->gram);
        const int64_t base = (int64_t)s0 * J * J;
        hipLaunchKernelGGL((k_corekeys<J, WITH_D>), dim3((nsb * J * J + 255) / 256), dim3(256), 0, st, c->gram, W2,
                           c->core, c->cmask, c->hdiag, base, nsb, key_out);
    }
}

template <int N, int J, typename T>
static hipError_t core_pass_t(vest_ctx *c, bool keys, double *key_out, bool slab0_done, hipStream_t st,
                              double *partials)
{
    const int last = N - 1;
    const ModeLayout &L = c->lay[last];
    constexpr int GW = gram_width(J);
    const int64_t Ilast = c->d.dims[last];

    SlabArgs<N, J, T> a{};
    a.waves = L.waves;
    a.nwaves = L.nwaves;
    a.row_order = L.row_order;
    for (int m = 0; m < N - 1; ++m) a.oidx[m] = L.oidx[m];
    for (int m = 0; m < N - 2; ++m) {
        const int64_t I = c->d.dims[m];
        hipLaunchKernelGGL(k_colcopy<T>, dim3((unsigned)((I * J + 255) / 256)), dim3(256), 0, st, c->A[m], I, J,
                           N == 3 ? 1 : 0, reinterpret_cast<T *>(c->colA[m]));
        a.colA[m] = reinterpret_cast<const T *>(c->colA[m]);
        a.dimA[m] = I;
    }
    a.ms = reinterpret_cast<const T *>(c->ms);
    for (int m = 0; m < N - 2; ++m) a.rowA[m] = reinterpret_cast<const T *>(c->Ag[m]);
    a.Alast = reinterpret_cast<const T *>(c->Ag[last]);
    a.e = reinterpret_cast<T *>(c->e);
    a.dprev = c->dprev;
    a.rowbuf = c->rowbuf;
    a.ldrb = c->ldrb;
    a.partials = partials;
    a.wsum = c->wsum;

    const int blocks = (L.nwaves + 3) / 4;
    const int grows = gram_core_rows<J>(Ilast);
    const int64_t gchunks = (Ilast + grows - 1) / grows;
    const int nslab = ipow(J, N - 2);
    // with more than one slab the last slab's change is not applied to the
    // residual here (k_sse_lag forms the SSE); with one slab its statistics
    // may come from the residual pass, which does not sum e^2
    const bool lag = nslab > 1;
    auto digits = [&](int s, int32_t *out) {
        for (int m = N - 3; m >= 0; --m) {
            out[m] = s % J;
            s /= J;
        }
    };
    if (keys) {
        if (c->hdiag_valid)
            core_keys_batches<N, J, T, false>(c, a, key_out, st);
        else
            core_keys_batches<N, J, T, true>(c, a, key_out, st);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_kp<J>, dim3((unsigned)((Ilast + 255) / 256)), dim3(256), 0, st, c->A[last], Ilast, GW,
                       c->kp);
    for (int s = 0; s < nslab; ++s) {
        digits(s, a.lead);
        a.has_prev = s > 0 ? 1 : 0;
        if (s > 0) digits(s - 1, a.lprev);
        // the first slab's statistics may already come from the residual pass
        // (OP_RESID_S0); the last slab's pass also sums e^2 (see k_sse_lag)
        const bool lastp = lag && s == nslab - 1;
        if (!(s == 0 && slab0_done)) {
            const bool timed = c->slab_ev && c->slab_ev_n < c->slab_ev_cap;
            if (timed) hipEventRecord(c->slab_ev[2 * c->slab_ev_n], st);
            if (blocks > 0) {
                if (lastp)
                    hipLaunchKernelGGL((k_slab<N, J, T, true, true>), dim3(blocks), dim3(256), 0, st, a);
                else
                    hipLaunchKernelGGL((k_slab<N, J, T, true>), dim3(blocks), dim3(256), 0, st, a);
            }
            if (timed) hipEventRecord(c->slab_ev[2 * c->slab_ev_n++ + 1], st);
        }
        if (L.nlong > 0)
            hipLaunchKernelGGL(k_slab_long<nacc_vc(J)>, dim3(L.nlong), dim3(64), 0, st, partials, L.longrows,
                               c->rowbuf, c->ldrb);
        hipLaunchKernelGGL(k_gram_core<J>, dim3((unsigned)gchunks), dim3(64 * gram_tm(J)), 0, st, c->rowbuf, c->ldrb,
                           c->kp, GW, Ilast, grows, c->gram_part);
        hipLaunchKernelGGL(k_gramsum_core<J>, dim3((gram_core_cells(J) + 63) / 64), dim3(1024), 0, st, c->gram_part,
                           gchunks, c->gram);
        const int64_t base = (int64_t)s * J * J;
        if (c->d.reg == VEST_REG_LF)
            hipLaunchKernelGGL((k_slabsolve<J, VEST_REG_LF>), dim3(1), dim3(64), 0, st, c->gram, c->core, c->cmask,
                               base, c->d.lambda, c->dprev, c->hdiag);
        else
            hipLaunchKernelGGL((k_slabsolve<J, VEST_REG_L1>), dim3(1), dim3(64), 0, st, c->gram, c->core, c->cmask,
                               base, c->d.lambda, c->dprev, c->hdiag);
    }
    if (lag) {
        // the residual keeps lagging the last slab's change; its SSE is formed here
        hipLaunchKernelGGL(k_sse_lag<J>, dim3(1), dim3(1024), 0, st, c->wsum, L.nwaves, c->gram, c->dprev,
                           c->sse_lag);
        c->e_lag = true;
        return hipGetLastError();
    }
    // apply the last slab's change to the residual
    a.has_prev = 1;
    digits(nslab - 1, a.lprev);
    if (blocks > 0) hipLaunchKernelGGL((k_slab<N, J, T, false>), dim3(blocks), dim3(256), 0, st, a);
    c->e_lag = false;
    return hipGetLastError();
}

// Apply the core sweep's last slab change (dprev) to a lagging residual.
template <int N, int J, typename T>
static hipError_t lag_apply_t(vest_ctx *c)
{
    const int last = N - 1;
    const ModeLayout &L = c->lay[last];
    SlabArgs<N, J, T> a{};
    a.waves = L.waves;
    a.nwaves = L.nwaves;
    a.row_order = L.row_order;
    for (int m = 0; m < N - 1; ++m) a.oidx[m] = L.oidx[m];
    for (int m = 0; m < N - 2; ++m) {
        a.colA[m] = reinterpret_cast<const T *>(c->colA[m]);   // column copies made by the core sweep
        a.dimA[m] = c->d.dims[m];
    }
    a.ms = reinterpret_cast<const T *>(c->ms);
    for (int m = 0; m < N - 2; ++m) a.rowA[m] = reinterpret_cast<const T *>(c->Ag[m]);
    a.Alast = reinterpret_cast<const T *>(c->Ag[last]);
    a.e = reinterpret_cast<T *>(c->e);
    a.dprev = c->dprev;
    a.has_prev = 1;
    int s = ipow(J, N - 2) - 1;
    for (int m = N - 3; m >= 0; --m) {
        a.lprev[m] = s % J;
        s /= J;
    }
    const int blocks = (L.nwaves + 3) / 4;
    if (blocks > 0) hipLaunchKernelGGL((k_slab<N, J, T, false>), dim3(blocks), dim3(256), 0, c->stream, a);
    return hipGetLastError();
}

// The core sweep of several contexts of one shape, kernel by kernel as
// core_pass_t launches it for one (slab passes, long-row sums, Gram product,
// its sum and the sequential solve of every slab, then the SSE of the lagging
// residual, or with one slab its change applied), each launch carrying all
// the contexts.
template <int N, int J, typename T>
static bool plan_core_batch_t(vest_ctx *const *cs, int n, bool fused, hipStream_t st, BatchArena &ba, LaunchList &L)
{
    const int last = N - 1;
    constexpr int GW = gram_width(J);
    const int nslab = ipow(J, N - 2);
    std::vector<SlabArgs<N, J, T>> base(n);
    std::vector<KpTask> kp(n);
    std::vector<ColTask<T>> col;
    std::vector<SlabLongTask> sl(n);
    std::vector<GramTask> gr(n);
    std::vector<GsumTask> gs(n);
    std::vector<SseTask> sse(n);
    std::vector<int32_t> kpoff(n + 1, 0), coloff(1, 0), soff(n + 1, 0), sloff(n + 1, 0), groff(n + 1, 0),
        gsoff(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        vest_ctx *c = cs[i];
        const ModeLayout &Ly = c->lay[last];
        const int64_t Ilast = c->d.dims[last];
        SlabArgs<N, J, T> &a = base[i];
        a = SlabArgs<N, J, T>{};
        a.waves = Ly.waves;
        a.nwaves = Ly.nwaves;
        a.row_order = Ly.row_order;
        for (int m = 0; m < N - 1; ++m) a.oidx[m] = Ly.oidx[m];
        for (int m = 0; m < N - 2; ++m) {
            const int64_t I = c->d.dims[m];
            col.push_back(ColTask<T>{c->A[m], I, J, N == 3 ? 1 : 0, reinterpret_cast<T *>(c->colA[m])});
            coloff.push_back(coloff.back() + (int32_t)((I * J + 255) / 256));
            a.colA[m] = reinterpret_cast<const T *>(c->colA[m]);
            a.dimA[m] = I;
        }
        a.ms = reinterpret_cast<const T *>(c->ms);
        for (int m = 0; m < N - 2; ++m) a.rowA[m] = reinterpret_cast<const T *>(c->Ag[m]);
        a.Alast = reinterpret_cast<const T *>(c->Ag[last]);
        a.e = reinterpret_cast<T *>(c->e);
        a.dprev = c->dprev;
        a.rowbuf = c->rowbuf;
        a.ldrb = c->ldrb;
        a.partials = c->partials;
        a.wsum = c->wsum;
        sse[i] = SseTask{c->wsum, c->gram, c->dprev, c->sse_lag, Ly.nwaves};
        kp[i] = KpTask{c->A[last], Ilast, GW, c->kp};
        kpoff[i + 1] = kpoff[i] + (int32_t)((Ilast + 255) / 256);
        soff[i + 1] = soff[i] + (Ly.nwaves + 3) / 4;
        sl[i] = SlabLongTask{c->partials, Ly.longrows, c->rowbuf, c->ldrb};
        sloff[i + 1] = sloff[i] + Ly.nlong;
        const int grows = gram_core_rows<J>(Ilast);
        const int64_t gchunks = (Ilast + grows - 1) / grows;
        gr[i] = GramTask{c->rowbuf, c->kp, c->gram_part, Ilast, c->ldrb, GW, grows};
        groff[i + 1] = groff[i] + (int32_t)gchunks;
        gs[i] = GsumTask{c->gram_part, gchunks, gram_core_cells(J), c->gram};
        gsoff[i + 1] = gsoff[i] + (gram_core_cells(J) + 63) / 64;
    }
    auto digits = [&](int s, int32_t *out) {
        for (int m = N - 3; m >= 0; --m) {
            out[m] = s % J;
            s /= J;
        }
    };
    // per-slab tables: the slab pass's arguments and the solve's tasks
    std::vector<size_t> o_slab(nslab), o_solve(nslab);
    std::vector<SlabArgs<N, J, T>> tab(n);
    std::vector<SolveTask> sv(n);
    for (int s = 0; s < nslab; ++s) {
        for (int i = 0; i < n; ++i) {
            tab[i] = base[i];
            digits(s, tab[i].lead);
            tab[i].has_prev = s > 0 ? 1 : 0;
            if (s > 0) digits(s - 1, tab[i].lprev);
            vest_ctx *c = cs[i];
            sv[i] = SolveTask{c->gram, c->core, c->cmask, c->dprev, c->hdiag, (int64_t)s * J * J, c->d.lambda,
                              c->d.reg};
        }
        o_slab[s] = ba.add(tab.data(), sizeof(SlabArgs<N, J, T>) * n);
        o_solve[s] = ba.add(sv.data(), sizeof(SolveTask) * n);
    }
    for (int i = 0; i < n; ++i) {
        tab[i] = base[i];
        tab[i].has_prev = 1;
        digits(nslab - 1, tab[i].lprev);
    }
    const size_t o_final = ba.add(tab.data(), sizeof(SlabArgs<N, J, T>) * n);
    const size_t o_kp = ba.add(kp.data(), sizeof(KpTask) * n), o_kpoff = ba.add(kpoff.data(), 4 * (n + 1));
    const size_t o_col = col.empty() ? 0 : ba.add(col.data(), sizeof(ColTask<T>) * col.size());
    const size_t o_coloff = ba.add(coloff.data(), 4 * coloff.size());
    const size_t o_soff = ba.add(soff.data(), 4 * (n + 1));
    const size_t o_sl = ba.add(sl.data(), sizeof(SlabLongTask) * n), o_sloff = ba.add(sloff.data(), 4 * (n + 1));
    const size_t o_gr = ba.add(gr.data(), sizeof(GramTask) * n), o_groff = ba.add(groff.data(), 4 * (n + 1));
    const size_t o_gs = ba.add(gs.data(), sizeof(GsumTask) * n), o_gsoff = ba.add(gsoff.data(), 4 * (n + 1));
    const size_t o_sse = ba.add(sse.data(), sizeof(SseTask) * n);
    if (ba.overflow) return false;
    const bool lag = nslab > 1;   // as in core_pass_t
    int nlf = 0;   // contexts with the L_F regulariser (the rest L_1)
    for (int i = 0; i < n; ++i) nlf += cs[i]->d.reg == VEST_REG_LF ? 1 : 0;
    const BatchArena B = ba;
    const int ncol = (int)col.size();
    const int tcol = coloff.back(), tkp = kpoff[n], tslab = soff[n], tsl = sloff[n], tgr = groff[n], tgs = gsoff[n];
    auto grid = [](int total) { return total < kBatchGrid ? total : kBatchGrid; };
    L.push_back([=]() {
        if (tcol > 0)
            hipLaunchKernelGGL(k_colcopy_multi<T>, dim3(grid(tcol)), dim3(256), 0, st, B.dptr<ColTask<T>>(o_col),
                               B.dptr<int32_t>(o_coloff), ncol, tcol);
        if (tkp > 0)
            hipLaunchKernelGGL(k_kp_multi<J>, dim3(grid(tkp)), dim3(256), 0, st, B.dptr<KpTask>(o_kp),
                               B.dptr<int32_t>(o_kpoff), n, tkp);
        for (int s = 0; s < nslab; ++s) {
            if (!(s == 0 && fused) && tslab > 0) {
                if (lag && s == nslab - 1)
                    hipLaunchKernelGGL((k_slab_multi<N, J, T, true, true>), dim3(grid(tslab)), dim3(256), 0, st,
                                       B.dptr<SlabArgs<N, J, T>>(o_slab[s]), B.dptr<int32_t>(o_soff), n, tslab);
                else
                    hipLaunchKernelGGL((k_slab_multi<N, J, T, true>), dim3(grid(tslab)), dim3(256), 0, st,
                                       B.dptr<SlabArgs<N, J, T>>(o_slab[s]), B.dptr<int32_t>(o_soff), n, tslab);
            }
            if (tsl > 0)
                hipLaunchKernelGGL(k_slab_long_multi<nacc_vc(J)>, dim3(grid(tsl)), dim3(64), 0, st,
                                   B.dptr<SlabLongTask>(o_sl), B.dptr<int32_t>(o_sloff), n, tsl);
            hipLaunchKernelGGL(k_gram_core_multi<J>, dim3(tgr), dim3(64 * gram_tm(J)), 0, st,
                               B.dptr<GramTask>(o_gr), B.dptr<int32_t>(o_groff), n, tgr);
            hipLaunchKernelGGL(k_gramsum_core_multi<J>, dim3(grid(tgs)), dim3(1024), 0, st, B.dptr<GsumTask>(o_gs),
                               B.dptr<int32_t>(o_gsoff), n, tgs);
            if (nlf > 0)
                hipLaunchKernelGGL((k_slabsolve_multi<J, VEST_REG_LF>), dim3(n), dim3(64), 0, st,
                                   B.dptr<SolveTask>(o_solve[s]), n);
            if (nlf < n)
                hipLaunchKernelGGL((k_slabsolve_multi<J, VEST_REG_L1>), dim3(n), dim3(64), 0, st,
                                   B.dptr<SolveTask>(o_solve[s]), n);
        }
        if (lag)
            hipLaunchKernelGGL(k_sse_lag_multi<J>, dim3(grid(n)), dim3(1024), 0, st, B.dptr<SseTask>(o_sse), n);
        else if (tslab > 0)
            hipLaunchKernelGGL((k_slab_multi<N, J, T, false>), dim3(grid(tslab)), dim3(256), 0, st,
                               B.dptr<SlabArgs<N, J, T>>(o_final), B.dptr<int32_t>(o_soff), n, tslab);
    });
    return true;
}

bool plan_core_batch(vest_ctx *const *cs, int n, bool fused, hipStream_t st, BatchArena &ba, LaunchList &L)
{
    const vest_ctx *c = cs[0];
#define VEST_CASE(NN, JJ)                                                                    \
    if (c->N == NN && c->J == JJ)                                                            \
        return c->f32 ? plan_core_batch_t<NN, JJ, float>(cs, n, fused, st, ba, L)            \
                      : plan_core_batch_t<NN, JJ, double>(cs, n, fused, st, ba, L);
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return false;
}

static hipError_t core_pass(vest_ctx *c, bool keys, double *key_out, bool slab0_done, hipStream_t st,
                           double *partials)
{
#define VEST_CASE(NN, JJ)                                                                              \
    if (c->N == NN && c->J == JJ)                                                                      \
        return c->f32 ? core_pass_t<NN, JJ, float>(c, keys, key_out, slab0_done, st, partials)       \
                      : core_pass_t<NN, JJ, double>(c, keys, key_out, slab0_done, st, partials);
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_core_sweep(vest_ctx *c, bool slab0_done)
{
    return core_pass(c, false, nullptr, slab0_done, c->stream, c->partials);
}
hipError_t launch_core_keys(vest_ctx *c, double *core_key, hipStream_t st, double *partials)
{
    return core_pass(c, true, core_key, false, st, partials);
}
hipError_t launch_lag_apply(vest_ctx *c)
{
#define VEST_CASE(NN, JJ) \
    if (c->N == NN && c->J == JJ) return c->f32 ? lag_apply_t<NN, JJ, float>(c) : lag_apply_t<NN, JJ, double>(c);
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return hipErrorInvalidValue;
}

bool shape_supported(int N, int J)
{
#define VEST_CASE(NN, JJ) \
    if (N == NN && J == JJ) return true;
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return false;
}

}  // namespace vest
