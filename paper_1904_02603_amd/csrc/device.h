// Device-side building blocks shared by the libvest kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "internal.h"

namespace vest {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;   // matrix-core operand, 8 BF16
typedef __attribute__((ext_vector_type(16))) float f32x16;   // 32 x 32 tile accumulator slice
typedef __attribute__((ext_vector_type(4))) double f64x4;    // 16 x 16 FP64 tile accumulator slice

// Minimiser along one coordinate of  den x^2 - 2 num x + penalty(x)
// (the element-wise rules of Sec. 3.4, always in FP64):
//   L_F (Eq. 9 / Eq. 12): num / (den + lambda)
//   L_1 (Eq. 13 / Eq. 14): soft threshold with g = -2 num, d = 2 den.
__device__ __forceinline__ double coord_min(int reg, double lambda, double num, double den)
{
    if (reg == VEST_REG_LF) return num / (den + lambda);
    const double g = -2.0 * num, d = 2.0 * den;
    if (g > lambda) return (lambda - g) / d;
    if (g < -lambda) return -(lambda + g) / d;
    return 0.0;
}

// Index of (t, u), t <= u, in a packed upper triangle of a J x J matrix.
template <int J>
__host__ __device__ constexpr int sym(int t, int u)
{
    return t <= u ? t * J - t * (t - 1) / 2 + (u - t) : u * J - u * (u - 1) / 2 + (t - u);
}

// fma for both compute types
__device__ __forceinline__ double vfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float vfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Core operands are wave-uniform and read with scalar loads.  A scalar
// load's immediate offset reaches 4 KB, so the core is addressed through one
// base pointer per 4 KB window; each base is made opaque to the compiler,
// which would otherwise fold it back into one large offset and then
// materialise a separate 64-bit base for every load beyond the window (about
// forty extra scalar-register pairs, spilled, leaving no room to load the
// next operands while the current ones are consumed).  The pointers are in
// the constant address space so the loads stay scalar.
template <typename T>
struct CoreBases {
    static constexpr int W = 4096 / (int)sizeof(T);
    typedef const __attribute__((address_space(4))) T *CPtr;
    CPtr b[64];
};

template <int N, int J, typename T>
__device__ __forceinline__ CoreBases<T> core_bases(const T *__restrict__ Gp);

// The bases only where the dense contraction reads them (an empty set for the
// gather form, whose core may exceed the 64 windows).
template <int N, int J, typename T, bool USE>
__device__ __forceinline__ CoreBases<T> core_bases_if(const T *__restrict__ Gp)
{
    if constexpr (USE)
        return core_bases<N, J, T>(Gp);
    else
        return CoreBases<T>{};
}

template <int N, int J, typename T>
__device__ __forceinline__ CoreBases<T> core_bases(const T *__restrict__ Gp)
{
    constexpr int W = CoreBases<T>::W;
    static_assert((ipow(J, N) + W - 1) / W <= 64, "core windows");
    CoreBases<T> G;
#pragma unroll
    for (int k = 0; k < (ipow(J, N) + W - 1) / W; ++k) {
        uint64_t q = reinterpret_cast<uint64_t>(Gp + k * W);
        asm("" : "+s"(q));
        G.b[k] = (typename CoreBases<T>::CPtr)q;
    }
    return G;
}

// Re-launders the bases inside a loop: the core operands then count as
// loop-variant and their loads stay at their uses instead of being hoisted
// out of the loop (where hundreds of them would be kept live in scalar
// registers and spilled).
template <int N, int J, typename T>
__device__ __forceinline__ void core_fence(CoreBases<T> &G)
{
    constexpr int W = CoreBases<T>::W;
#pragma unroll
    for (int k = 0; k < (ipow(J, N) + W - 1) / W; ++k) {
        uint64_t q = reinterpret_cast<uint64_t>(G.b[k]);
        asm volatile("" : "+s"(q));
        G.b[k] = (typename CoreBases<T>::CPtr)q;
    }
}

template <int F, typename T>
__device__ __forceinline__ T core_at(const CoreBases<T> &G)
{
    constexpr int W = CoreBases<T>::W;
    return G.b[F / W][F % W];
}

// Contraction of one core slice with the rows of the other modes
// (Eq. 11): for the slice starting at flat offset F of the
// mode-n-permuted core, the sum over (o_D .. o_{NO-1}) of
// G[F + ...] * prod_m r[m][o_m], innermost mode first, terms added in
// ascending o.  All offsets are compile-time constants.
template <int NO, int J, int D, int F, typename T>
__device__ __forceinline__ T contract(const CoreBases<T> &G, const T (&r)[NO][J]);

template <int NO, int J, int D, int F, int O, typename T>
__device__ __forceinline__ T contract_rest(const CoreBases<T> &G, const T (&r)[NO][J], T acc)
{
    if constexpr (O == J) {
        return acc;
    } else {
        T v;
        if constexpr (D == NO - 1) v = core_at<F + O>(G);
        else v = contract<NO, J, D + 1, F + O * ipow(J, NO - 1 - D), T>(G, r);
        return contract_rest<NO, J, D, F, O + 1, T>(G, r, vfma(v, r[D][O], acc));
    }
}

template <int NO, int J, int D, int F, typename T>
__device__ __forceinline__ T contract(const CoreBases<T> &G, const T (&r)[NO][J])
{
    T v0;
    if constexpr (D == NO - 1) v0 = core_at<F>(G);
    else v0 = contract<NO, J, D + 1, F, T>(G, r);
    return contract_rest<NO, J, D, F, 1, T>(G, r, v0 * r[D][0]);
}

template <int N, int J, int j, typename T>
__device__ __forceinline__ void delta_from(const CoreBases<T> &G, const T (&r)[N - 1][J], T (&d)[J])
{
    if constexpr (j < J) {
        d[j] = contract<N - 1, J, 0, j * ipow(J, N - 1), T>(G, r);
        delta_from<N, J, j + 1, T>(G, r, d);
    }
}

// delta_alpha^{(n)} (Eq. 11) for one entry, given the permuted core Gp
// ([J_n][others ascending], row-major) and the N-1 other-mode factor rows.
template <int N, int J, typename T>
__device__ __forceinline__ void delta_vec(const CoreBases<T> &G, const T (&r)[N - 1][J], T (&d)[J])
{
    delta_from<N, J, 0, T>(G, r, d);
}

// The same contraction for two entries at once: every core operand is
// loaded once and feeds both.  The core is walked in blocks of J consecutive
// values (one innermost sum each, in the order delta_vec visits them); the
// loads of block B + 1 are issued before block B is consumed and a
// scheduling barrier closes every block, so the operands of at most two
// blocks are live in scalar registers (left to itself the scheduler would
// separate the two entries' chains and keep hundreds of operands live).
// Each entry's terms are added in the order of delta_vec, so both results
// equal the one-entry form bit for bit.
template <int F, int O, int J, typename T>
__device__ __forceinline__ void load_block(const CoreBases<T> &G, T (&out)[J])
{
    if constexpr (O < J) {
        out[O] = core_at<F + O>(G);
        load_block<F, O + 1, J, T>(G, out);
    }
}

template <int NO, int J, int B, typename T>
__device__ __forceinline__ void pair_step(const CoreBases<T> &G, const T (&ra)[NO][J], const T (&rb)[NO][J],
                                          T (&buf)[2][J], T (&acca)[NO], T (&accb)[NO], T (&da)[J], T (&db)[J])
{
    constexpr int NB = ipow(J, NO);   // blocks of J values in the J^(NO+1) core
    if constexpr (B + 1 < NB) load_block<(B + 1) * J, 0, J, T>(G, buf[(B + 1) & 1]);
    const T(&cur)[J] = buf[B & 1];
    T va = cur[0] * ra[NO - 1][0], vb = cur[0] * rb[NO - 1][0];
#pragma unroll
    for (int o = 1; o < J; ++o) {
        va = vfma(cur[o], ra[NO - 1][o], va);
        vb = vfma(cur[o], rb[NO - 1][o], vb);
    }
    // fold the finished innermost sum into the outer levels NO-2 .. 0
    bool up = true;
#pragma unroll
    for (int L = NO - 2; L >= 0; --L) {
        if (up) {
            const int o = (B / ipow(J, NO - 2 - L)) % J;
            if (o == 0) {
                acca[L] = va * ra[L][0];
                accb[L] = vb * rb[L][0];
            } else {
                acca[L] = vfma(va, ra[L][o], acca[L]);
                accb[L] = vfma(vb, rb[L][o], accb[L]);
            }
            up = o == J - 1;
            va = acca[L];
            vb = accb[L];
        }
    }
    if (up) {
        constexpr int j = B / ipow(J, NO - 1);
        da[j] = va;
        db[j] = vb;
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <int NO, int J, typename T, int... Bs>
__device__ __forceinline__ void pair_all(const CoreBases<T> &G, const T (&ra)[NO][J], const T (&rb)[NO][J],
                                         T (&buf)[2][J], T (&acca)[NO], T (&accb)[NO], T (&da)[J], T (&db)[J],
                                         std::integer_sequence<int, Bs...>)
{
    (pair_step<NO, J, Bs, T>(G, ra, rb, buf, acca, accb, da, db), ...);
}

template <int N, int J, typename T>
__device__ __forceinline__ void delta_vec2(const CoreBases<T> &G, const T (&ra)[N - 1][J], const T (&rb)[N - 1][J],
                                           T (&da)[J], T (&db)[J])
{
    T buf[2][J], acca[N - 1], accb[N - 1];
    load_block<0, 0, J, T>(G, buf[0]);
    pair_all<N - 1, J, T>(G, ra, rb, buf, acca, accb, da, db, std::make_integer_sequence<int, ipow(J, N - 1)>{});
}

// Sum over a block (blockDim.x a power of two) in a fixed LDS tree order.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// Task of virtual block b in a launch that carries several contexts:
// off[t] is the first virtual block of task t (off[0] = 0, nondecreasing);
// the last task whose first block is <= b (tasks without blocks are skipped).
__device__ __forceinline__ int task_of(const int32_t *__restrict__ off, int ntask, int b)
{
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Slot-ordered copy of a per-entry factor row, interleaved per wave: the J
// values of the 64 slots of one (wave, k) step form one contiguous block of
// 64 J elements (slot bases are multiples of 64).  Inside the block, 8-byte
// values (FP64) go value t of every lane in a 64-element run; 4-byte values
// (FP32) with J even go in pairs, values 2u and 2u + 1 of every lane in a run
// of 64 pairs.  Either way each load or store of a wave moves one contiguous
// 512-byte run of a single block.
template <int J, typename T>
__host__ __device__ constexpr bool ms_paired() { return sizeof(T) == 4 && J % 2 == 0; }

template <int J, typename T>
__host__ __device__ __forceinline__ int64_t ms_index(int64_t slot, int t)
{
    if constexpr (ms_paired<J, T>())
        return (slot >> 6) * (int64_t)(64 * J) + (t >> 1) * 128 + (slot & 63) * 2 + (t & 1);
    else
        return (slot >> 6) * (int64_t)(64 * J) + t * 64 + (slot & 63);
}

// Streams that every pass reads or writes once (entry indices, values, the
// residual, the slot copy of factor rows: hundreds of MB) go through the
// non-temporal hint, so that they do not evict the cache lines of the factor
// rows and columns that the same kernels gather.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_stream(T v, T *p) { __builtin_nontemporal_store(v, p); }

template <int J, typename T>
__device__ __forceinline__ void ms_load(const T *__restrict__ ms, int64_t slot, T (&v)[J])
{
    if constexpr (ms_paired<J, T>()) {
        typedef float f2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int u = 0; u < J / 2; ++u) {
            const f2 x = ld_stream(reinterpret_cast<const f2 *>(ms + ms_index<J, T>(slot, 2 * u)));
            v[2 * u] = x.x;
            v[2 * u + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int t = 0; t < J; ++t) v[t] = ld_stream(ms + ms_index<J, T>(slot, t));
    }
}

template <int J, typename T>
__device__ __forceinline__ void ms_store(T *__restrict__ ms, int64_t slot, const T (&v)[J])
{
    if constexpr (ms_paired<J, T>()) {
        typedef float f2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int u = 0; u < J / 2; ++u) {
            const f2 x = {v[2 * u], v[2 * u + 1]};
            st_stream(x, reinterpret_cast<f2 *>(ms + ms_index<J, T>(slot, 2 * u)));
        }
    } else {
#pragma unroll
        for (int t = 0; t < J; ++t) st_stream(v[t], ms + ms_index<J, T>(slot, t));
    }
}

// Load a factor row of J values with the widest aligned vector loads.
template <int J, typename T>
__device__ __forceinline__ void load_row(const T *__restrict__ p, T (&r)[J])
{
    constexpr int bytes = J * (int)sizeof(T);
    if constexpr (bytes % 16 == 0) {
        const uint4 *q = reinterpret_cast<const uint4 *>(__builtin_assume_aligned(p, 16));
#pragma unroll
        for (int v = 0; v < bytes / 16; ++v) {
            uint4 x = q[v];
            __builtin_memcpy(reinterpret_cast<char *>(r) + 16 * v, &x, 16);
        }
    } else if constexpr (bytes % 8 == 0) {
        const uint2 *q = reinterpret_cast<const uint2 *>(__builtin_assume_aligned(p, 8));
#pragma unroll
        for (int v = 0; v < bytes / 8; ++v) {
            uint2 x = q[v];
            __builtin_memcpy(reinterpret_cast<char *>(r) + 8 * v, &x, 8);
        }
    } else {
#pragma unroll
        for (int v = 0; v < J; ++v) r[v] = p[v];
    }
}

// r[b] for a per-lane (or runtime) b, as a sum with exactly one nonzero term (a select
// chain would be folded back into a dynamically indexed array, which lives
// in scratch memory).
template <int J, typename T>
__device__ __forceinline__ T pick(const T (&r)[J], int b)
{
    T v = r[0] * (b == 0 ? T(1) : T(0));
#pragma unroll
    for (int t = 1; t < J; ++t) v = vfma(r[t], b == t ? T(1) : T(0), v);
    return v;
}

// Load a row of a gather copy (16-byte aligned start): 16-byte loads, then
// the remainder in 8- and 4-byte pieces.
template <int J, typename T>
__device__ __forceinline__ void load_grow(const T *__restrict__ p, T (&r)[J])
{
    constexpr int bytes = J * (int)sizeof(T);
    const char *q = reinterpret_cast<const char *>(__builtin_assume_aligned(p, 16));
    char *d = reinterpret_cast<char *>(r);
#pragma unroll
    for (int v = 0; v < bytes / 16; ++v) {
        const uint4 x = reinterpret_cast<const uint4 *>(q)[v];
        __builtin_memcpy(d + 16 * v, &x, 16);
    }
    constexpr int o8 = bytes / 16 * 16;
    if constexpr (bytes - o8 >= 8) {
        const uint2 x = *reinterpret_cast<const uint2 *>(q + o8);
        __builtin_memcpy(d + o8, &x, 8);
    }
    constexpr int o4 = o8 + (bytes - o8 >= 8 ? 8 : 0);
    if constexpr (bytes - o4 >= 4) {
        const uint32_t x = *reinterpret_cast<const uint32_t *>(q + o4);
        __builtin_memcpy(d + o4, &x, 4);
    }
}

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int m)
{
    return __shfl_xor(v, m, kWave);
}

// Sum NA per-lane accumulators over the 2^glog lanes of each row group
// (xor butterfly: every lane of the group ends with the group total, summed
// in an order fixed by lane positions).
template <int NA, typename T>
__device__ __forceinline__ void group_reduce(T (&s)[NA], int glog)
{
    for (int b = 0; b < glog; ++b) {
        const int m = 1 << b;
#pragma unroll
        for (int v = 0; v < NA; ++v) s[v] += shfl_xor_t(s[v], m);
    }
}

// Long-row chunk: lane 0 stores the wave total (double) as one partial.
template <int NA, typename T>
__device__ __forceinline__ void store_partial(double *__restrict__ part, int chunk, const T (&s)[NA], int lane)
{
    if (lane == 0) {
        double *p = part + (int64_t)chunk * NA;
#pragma unroll
        for (int v = 0; v < NA; ++v) p[v] = (double)s[v];
    }
}

// Fixed-order sum of the partials of one long row into LDS (one wave);
// afterwards lane 0 can read all NA values.
template <int NA>
__device__ __forceinline__ void sum_partials(const double *__restrict__ part, const LongRow &lr,
                                             double *__restrict__ lds, int lane)
{
    for (int v = lane; v < NA; v += kWave) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int c = 0;
        for (; c + 4 <= lr.nchunks; c += 4) {
            const double *p = part + (int64_t)(lr.first_chunk + c) * NA + v;
            s0 += p[0];
            s1 += p[NA];
            s2 += p[2 * NA];
            s3 += p[3 * NA];
        }
        for (; c < lr.nchunks; ++c) s0 += part[(int64_t)(lr.first_chunk + c) * NA + v];
        lds[v] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
}

}  // namespace vest
