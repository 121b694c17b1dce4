// Small kernels: core permutation per mode, FP32 factor copies, loss
// reductions (Eq. 1 / 2 / 4), marking-table set-up and pruning (Sec. 3.3).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "device.h"
#include "internal.h"

namespace vest {

struct Shape {
    int32_t N;
    int32_t J;
};

// out[j_n][others ascending] = core[j_1..j_N]   (row-major both)
template <typename T>
__device__ __forceinline__ void permute_body(const double *__restrict__ core, Shape sh, int mode, int64_t G,
                                             T *__restrict__ out, int bx)
{
    const int64_t q = (int64_t)bx * blockDim.x + threadIdx.x;
    if (q >= G) return;
    // digits of q in the permuted order: position 0 is mode `mode`, then the
    // other modes ascending
    int32_t jv[VEST_MAX_ORDER];
    int64_t rest = q;
    for (int p = sh.N - 1; p >= 0; --p) {
        const int dgt = (int)(rest % sh.J);
        rest /= sh.J;
        int k;
        if (p == 0) k = mode;
        else k = (p - 1) < mode ? p - 1 : p;
        jv[k] = dgt;
    }
    int64_t flat = 0;
    for (int k = 0; k < sh.N; ++k) flat = flat * sh.J + jv[k];
    out[q] = (T)core[flat];
}

template <typename T>
__global__ void __launch_bounds__(256) k_permute(const double *__restrict__ core, Shape sh, int mode, int64_t G,
                                                 T *__restrict__ out)
{
    permute_body<T>(core, sh, mode, G, out, blockIdx.x);
}

template <typename T>
struct PermTask {
    const double *core;
    T *out;
    int64_t G;
    int32_t mode;
};

// the permuted cores of several contexts of one shape (all modes)
template <typename T>
__global__ void __launch_bounds__(256) k_permute_multi(const PermTask<T> *__restrict__ tab,
                                                       const int32_t *__restrict__ off, int ntask, int total, Shape sh)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int t = task_of(off, ntask, b);
        const PermTask<T> tk = tab[t];
        permute_body<T>(tk.core, sh, tk.mode, tk.G, tk.out, b - off[t]);
    }
}

template <typename T>
static bool plan_permute_batch_t(vest_ctx *const *cs, int n, hipStream_t st, BatchArena &ba, LaunchList &L)
{
    const int N = cs[0]->N;
    std::vector<PermTask<T>> tab;
    std::vector<int32_t> off(1, 0);
    for (int i = 0; i < n; ++i)
        for (int m = 0; m < N; ++m) {
            vest_ctx *c = cs[i];
            tab.push_back(PermTask<T>{c->core, reinterpret_cast<T *>(c->Gp[m]), c->G, m});
            off.push_back(off.back() + (int32_t)((c->G + 255) / 256));
        }
    const size_t ot = ba.add(tab.data(), sizeof(PermTask<T>) * tab.size());
    const size_t oo = ba.add(off.data(), 4 * off.size());
    if (ba.overflow) return false;
    const PermTask<T> *dt = ba.dptr<PermTask<T>>(ot);
    const int32_t *doff = ba.dptr<int32_t>(oo);
    const int ntask = (int)tab.size(), total = off.back();
    const Shape sh{N, cs[0]->J};
    L.push_back([=]() {
        if (total > 0)
            hipLaunchKernelGGL(k_permute_multi<T>, dim3(total < kBatchGrid ? total : kBatchGrid), dim3(256), 0, st,
                               dt, doff, ntask, total, sh);
    });
    return true;
}

bool plan_permute_batch(vest_ctx *const *cs, int n, hipStream_t st, BatchArena &ba, LaunchList &L)
{
    return cs[0]->f32 ? plan_permute_batch_t<float>(cs, n, st, ba, L) : plan_permute_batch_t<double>(cs, n, st, ba, L);
}

hipError_t launch_permute_core(vest_ctx *c, int mode)
{
    Shape sh{c->N, c->J};
    const unsigned blocks = (unsigned)((c->G + 255) / 256);
    if (c->f32)
        hipLaunchKernelGGL(k_permute<float>, dim3(blocks), dim3(256), 0, c->stream, c->core, sh, mode, c->G,
                           reinterpret_cast<float *>(c->Gp[mode]));
    else
        hipLaunchKernelGGL(k_permute<double>, dim3(blocks), dim3(256), 0, c->stream, c->core, sh, mode, c->G,
                           reinterpret_cast<double *>(c->Gp[mode]));
    return hipGetLastError();
}

// Gather copy of a factor: rows of J values at stride ld in the compute type,
// the padding zeroed.
template <typename T>
__global__ void __launch_bounds__(256) k_gcopy(const double *__restrict__ a, int64_t rows, int J, int ld,
                                               T *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * ld) return;
    const int64_t r = q / ld;
    const int j = (int)(q - r * ld);
    out[q] = j < J ? (T)a[r * J + j] : T(0);
}

hipError_t launch_gather_copy(vest_ctx *c, int mode)
{
    const int64_t rows = c->d.dims[mode];
    const int ld = gather_ld(c->J, c->tsize);
    const unsigned blocks = (unsigned)((rows * ld + 255) / 256);
    if (c->f32)
        hipLaunchKernelGGL(k_gcopy<float>, dim3(blocks), dim3(256), 0, c->stream, c->A[mode], rows, c->J, ld,
                           reinterpret_cast<float *>(c->Ag[mode]));
    else
        hipLaunchKernelGGL(k_gcopy<double>, dim3(blocks), dim3(256), 0, c->stream, c->A[mode], rows, c->J, ld,
                           reinterpret_cast<double *>(c->Ag[mode]));
    return hipGetLastError();
}

// ------------------------------------------------------------- reductions
// Deterministic sums: a fixed grid of kLossBlocks blocks, grid-stride order
// per thread, a fixed LDS tree per block, then one block over the partials.
template <typename T, int ABS>
__global__ void __launch_bounds__(256) k_sum(const T *__restrict__ v, int64_t n, double *__restrict__ partial)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = (double)v[i];
        s += ABS ? fabs(x) : x * x;
    }
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// out[g] = sum over arrays a in group g of the kLossBlocks partials of a.
// group_of[a] in {0, 1}; narr <= 16.
// With sse given, out[0] is *sse instead of the group-0 sum.
__global__ void __launch_bounds__(256) k_final(const double *__restrict__ partial, int narr, int ngroup0,
                                               double *__restrict__ out, const double *__restrict__ sse)
{
    __shared__ double sh[256];
    double s0 = 0.0, s1 = 0.0;
    for (int a = 0; a < narr; ++a)
        for (int b = threadIdx.x; b < kLossBlocks; b += blockDim.x) {
            const double v = partial[a * kLossBlocks + b];
            if (a < ngroup0) s0 += v;
            else s1 += v;
        }
    const double t0 = block_sum(s0, sh);
    __syncthreads();
    const double t1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        out[0] = sse ? *sse : t0;
        out[1] = t1;
    }
}

hipError_t launch_sumsq(hipStream_t s, const double *v, int64_t n, double *partial, double *out)
{
    hipLaunchKernelGGL((k_sum<double, 0>), dim3(kLossBlocks), dim3(256), 0, s, v, n, partial);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, partial, 1, 1, out, (const double *)nullptr);
    return hipGetLastError();
}

// dev_out[0] = SSE over the residual (or *sse, formed by the core sweep),
// dev_out[1] = sum of the regulariser terms (squares for L_F, absolute values
// for L_1) over core and factors.
hipError_t launch_loss(vest_ctx *c, double *dev_out, const double *sse)
{
    hipStream_t st = c->stream;
    double *part = c->red;
    const ModeLayout &L = c->lay[c->N - 1];
    if (sse)
        ;
    else if (c->f32)
        hipLaunchKernelGGL((k_sum<float, 0>), dim3(kLossBlocks), dim3(256), 0, st,
                           reinterpret_cast<const float *>(c->e), L.nslots, part);
    else
        hipLaunchKernelGGL((k_sum<double, 0>), dim3(kLossBlocks), dim3(256), 0, st,
                           reinterpret_cast<const double *>(c->e), L.nslots, part);
    const bool l1 = c->d.reg == VEST_REG_L1;
    int a = 1;
    auto reg = [&](const double *p, int64_t n) {
        if (l1)
            hipLaunchKernelGGL((k_sum<double, 1>), dim3(kLossBlocks), dim3(256), 0, st, p, n, part + a * kLossBlocks);
        else
            hipLaunchKernelGGL((k_sum<double, 0>), dim3(kLossBlocks), dim3(256), 0, st, p, n, part + a * kLossBlocks);
        ++a;
    };
    reg(c->core, c->G);
    for (int n = 0; n < c->N; ++n) reg(c->A[n], c->d.dims[n] * c->J);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, part, a, 1, dev_out, sse);
    return hipGetLastError();
}

// ------------------------------------------------------------- marking table
__global__ void __launch_bounds__(256) k_mask_factor(double *__restrict__ A, const uint32_t *__restrict__ mask,
                                                     int64_t I, int J, unsigned long long *__restrict__ count)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int hit = 0;
    if (q < I * J) {
        const int64_t i = q / J;
        const int j = (int)(q % J);
        if ((mask[i] >> j) & 1u) {
            A[q] = 0.0;
            hit = 1;
        }
    }
    const unsigned long long b = __ballot(hit);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

__global__ void __launch_bounds__(256) k_mask_core(double *__restrict__ core, const uint8_t *__restrict__ mask,
                                                   int64_t G, unsigned long long *__restrict__ count)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int hit = 0;
    if (q < G && mask[q]) {
        core[q] = 0.0;
        hit = 1;
    }
    const unsigned long long b = __ballot(hit);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

// counts_dev: N + 1 counters (factors, then core), zeroed by the caller.
hipError_t launch_mask_init(vest_ctx *c, int64_t *counts_dev)
{
    auto *cnt = reinterpret_cast<unsigned long long *>(counts_dev);
    for (int n = 0; n < c->N; ++n) {
        const int64_t m = c->d.dims[n] * c->J;
        hipLaunchKernelGGL(k_mask_factor, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c->stream, c->A[n],
                           c->fmask[n], c->d.dims[n], c->J, cnt + n);
    }
    hipLaunchKernelGGL(k_mask_core, dim3((unsigned)((c->G + 255) / 256)), dim3(256), 0, c->stream, c->core, c->cmask,
                       c->G, cnt + c->N);
    return hipGetLastError();
}

// ------------------------------------------------------------- pruning
// FP64 key -> unsigned integer with the same order (-0 and +0 equal).
// ------------------------------------------------------------------ prune
// The k unmarked elements with the smallest (key, flat index) of every tensor
// that prunes this step, all tensors at once, by radix selection over the
// 96-bit composite (order-preserving 64-bit image of the FP64 key, 32-bit flat
// index): eight rounds of 12-bit digits, most significant first.  A round
// counts the digit of every element whose higher digits equal the ones chosen
// so far (block-local LDS histograms added into one histogram per tensor);
// then one block per tensor takes the digit at which the running count reaches
// the k still to place.  The composites of a tensor are distinct, so after the
// last round exactly k of its elements lie at or below the chosen composite;
// they are zeroed and marked.  Marked elements carry +inf keys and never
// qualify (k never exceeds the unmarked count).
constexpr int kSelBits = 12, kSelBins = 1 << kSelBits, kSelRounds = 96 / kSelBits, kSelPerBlock = 4096;
typedef unsigned __int128 u128;

struct SelSeg {
    const double *key;
    double *val;        // core or factor values
    uint32_t *fmask;    // factor marking words (null for the core)
    uint8_t *cmask;     // core marks (null for a factor)
    int64_t n, k;
    int64_t block0;     // first block of this tensor in a pass
    int32_t J;
};
struct SelArgs {
    SelSeg seg[VEST_MAX_ORDER + 1];
    int32_t nseg;
    uint32_t *hist;     // [nseg][kSelBins]
    u128 *pref;         // [nseg] digits chosen so far
    int64_t *krem;      // [nseg] elements still to place
};

__device__ __forceinline__ u128 sel_composite(double k, int64_t i)
{
    if (k == 0.0) k = 0.0;   // -0 and +0 are one key
    uint64_t u = (uint64_t)__double_as_longlong(k);
    u = (u >> 63) ? ~u : (u | 0x8000000000000000ull);
    return ((u128)u << 32) | (uint32_t)i;
}

__device__ __forceinline__ int sel_segment(const SelArgs &a, int64_t b)
{
    int s = 0;
    while (s + 1 < a.nseg && a.seg[s + 1].block0 <= b) ++s;
    return s;
}

__global__ void __launch_bounds__(256) k_sel_init(SelArgs a)
{
    const int s = blockIdx.x;
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) a.hist[(int64_t)s * kSelBins + i] = 0u;
    if (threadIdx.x == 0) {
        a.pref[s] = 0;
        a.krem[s] = a.seg[s].k;
    }
}

__global__ void __launch_bounds__(256) k_sel_hist(SelArgs a, int round)
{
    __shared__ uint32_t h[kSelBins];
    const int s = sel_segment(a, blockIdx.x);
    if (a.krem[s] == 0) return;   // selection of this tensor already decided (k_sel_pick)
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const SelSeg &g = a.seg[s];
    const int64_t lo = ((int64_t)blockIdx.x - g.block0) * kSelPerBlock;
    const int64_t hi = lo + kSelPerBlock < g.n ? lo + kSelPerBlock : g.n;
    const int top = 96 - kSelBits * round;   // digits at and above `top` are chosen
    const u128 p = a.pref[s];
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const u128 c = sel_composite(g.key[i], i);
        if ((c >> top) == p) atomicAdd(&h[(uint32_t)(c >> (top - kSelBits)) & (kSelBins - 1)], 1u);
    }
    __syncthreads();
    uint32_t *gh = a.hist + (int64_t)s * kSelBins;
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x)
        if (h[i]) atomicAdd(&gh[i], h[i]);
}

// One block of 1024 threads per tensor, four bins per thread.
__global__ void __launch_bounds__(1024) k_sel_pick(SelArgs a, int round)
{
    __shared__ uint32_t part[1024];
    const int s = blockIdx.x, t = threadIdx.x;
    if (a.krem[s] == 0) return;   // decided in an earlier round; its bins are clean
    uint32_t *gh = a.hist + (int64_t)s * kSelBins;
    uint32_t c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = gh[4 * t + q];
    part[t] = c[0] + c[1] + c[2] + c[3];
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {   // inclusive scan of the thread sums
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int64_t krem = a.krem[s];
    int64_t run = t > 0 ? part[t - 1] : 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (run < krem && run + c[q] >= krem) {
            const u128 p = (a.pref[s] << kSelBits) | (u128)(4 * t + q);
            if (run + c[q] == krem) {
                // the whole bin is selected: every composite with this prefix
                // is at most the prefix followed by all-ones digits, and no
                // other composite above the smaller prefixes is; the selection
                // is decided and the later rounds are skipped
                const int rest = kSelBits * (kSelRounds - 1 - round);
                a.pref[s] = (p << rest) | (((u128)1 << rest) - 1);
                a.krem[s] = 0;
            } else {
                a.pref[s] = p;
                a.krem[s] = krem - run;
            }
        }
        run += c[q];
        gh[4 * t + q] = 0u;   // clean for the next round
    }
}

__global__ void __launch_bounds__(256) k_sel_mark(SelArgs a)
{
    const int s = sel_segment(a, blockIdx.x);
    const SelSeg &g = a.seg[s];
    const int64_t lo = ((int64_t)blockIdx.x - g.block0) * kSelPerBlock;
    const int64_t hi = lo + kSelPerBlock < g.n ? lo + kSelPerBlock : g.n;
    const u128 thr = a.pref[s];
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        if (sel_composite(g.key[i], i) > thr) continue;
        g.val[i] = 0.0;
        if (g.fmask) atomicOr(&g.fmask[i / g.J], 1u << (i % g.J));
        else g.cmask[i] = 1;
    }
}

// core_k for the core, factor_k[n] for mode n (0 = leave that tensor alone).
hipError_t launch_prune(vest_ctx *c, int64_t core_k, const int64_t *factor_k)
{
    hipStream_t st = c->stream;
    SelArgs a{};
    int64_t blocks = 0;
    auto add = [&](const double *key, double *val, uint32_t *fm, uint8_t *cm, int64_t n, int64_t k) {
        if (k <= 0) return;
        SelSeg &g = a.seg[a.nseg++];
        g.key = key;
        g.val = val;
        g.fmask = fm;
        g.cmask = cm;
        g.n = n;
        g.k = k;
        g.J = c->J;
        g.block0 = blocks;
        blocks += (n + kSelPerBlock - 1) / kSelPerBlock;
    };
    add(c->key_core, c->core, nullptr, c->cmask, c->G, core_k);
    for (int n = 0; n < c->N; ++n)
        add(c->key_fac[n], c->A[n], c->fmask[n], nullptr, c->d.dims[n] * c->J, factor_k[n]);
    if (a.nseg == 0) return hipSuccess;
    a.hist = c->sel_hist;
    a.pref = reinterpret_cast<u128 *>(c->sel_state);
    a.krem = reinterpret_cast<int64_t *>(c->sel_state + 16 * (VEST_MAX_ORDER + 1));
    hipLaunchKernelGGL(k_sel_init, dim3(a.nseg), dim3(256), 0, st, a);
    for (int r = 0; r < kSelRounds; ++r) {
        hipLaunchKernelGGL(k_sel_hist, dim3((unsigned)blocks), dim3(256), 0, st, a, r);
        hipLaunchKernelGGL(k_sel_pick, dim3(a.nseg), dim3(1024), 0, st, a, r);
    }
    hipLaunchKernelGGL(k_sel_mark, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace vest
