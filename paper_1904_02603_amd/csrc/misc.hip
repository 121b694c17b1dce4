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
__global__ void __launch_bounds__(256) k_permute(const double *__restrict__ core, Shape sh, int mode, int64_t G,
                                                 T *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ void __launch_bounds__(256) k_final(const double *__restrict__ partial, int narr, int ngroup0,
                                               double *__restrict__ out)
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
        out[0] = t0;
        out[1] = t1;
    }
}

hipError_t launch_sumsq(hipStream_t s, const double *v, int64_t n, double *partial, double *out)
{
    hipLaunchKernelGGL((k_sum<double, 0>), dim3(kLossBlocks), dim3(256), 0, s, v, n, partial);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, partial, 1, 1, out);
    return hipGetLastError();
}

// dev_out[0] = SSE over the residual, dev_out[1] = sum of the regulariser
// terms (squares for L_F, absolute values for L_1) over core and factors.
hipError_t launch_loss(vest_ctx *c, double *dev_out)
{
    hipStream_t st = c->stream;
    double *part = c->red;
    const ModeLayout &L = c->lay[c->N - 1];
    if (c->f32)
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
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, part, a, 1, dev_out);
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
__global__ void __launch_bounds__(256) k_keybits(const double *__restrict__ key, int64_t n,
                                                 uint64_t *__restrict__ kout, uint32_t *__restrict__ pout)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double k = key[q];
    if (k == 0.0) k = 0.0;
    uint64_t u = (uint64_t)__double_as_longlong(k);
    u = (u >> 63) ? ~u : (u | 0x8000000000000000ull);
    kout[q] = u;
    pout[q] = (uint32_t)q;
}

__global__ void __launch_bounds__(256) k_mark_core(const uint32_t *__restrict__ pos, int64_t k, double *__restrict__ core,
                                                   uint8_t *__restrict__ mask)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    const uint32_t q = pos[t];
    core[q] = 0.0;
    mask[q] = 1;
}

__global__ void __launch_bounds__(256) k_mark_factor(const uint32_t *__restrict__ pos, int64_t k, int J,
                                                     double *__restrict__ A, uint32_t *__restrict__ mask)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    const uint32_t q = pos[t];
    A[q] = 0.0;
    atomicOr(&mask[q / J], 1u << (q % J));
}

// Zero and mark the k unmarked elements with the smallest (key, flat index):
// marked elements carry +inf keys, and the LSD radix sort is stable over the
// index-ordered input, so equal keys stay in index order.
hipError_t launch_prune(vest_ctx *c, int tensor, int64_t k)
{
    hipStream_t st = c->stream;
    const int64_t n = tensor < 0 ? c->G : c->d.dims[tensor] * c->J;
    const double *key = tensor < 0 ? c->key_core : c->key_fac[tensor];
    hipLaunchKernelGGL(k_keybits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, key, n, c->pk_in, c->pv_in);
    size_t bytes = c->sort_tmp_bytes;
    hipError_t err = hipcub::DeviceRadixSort::SortPairs(c->sort_tmp, bytes, c->pk_in, c->pk_out, c->pv_in, c->pv_out,
                                                        (int)n, 0, 64, st);
    if (err != hipSuccess) return err;
    const unsigned blocks = (unsigned)((k + 255) / 256);
    if (tensor < 0)
        hipLaunchKernelGGL(k_mark_core, dim3(blocks), dim3(256), 0, st, c->pv_out, k, c->core, c->cmask);
    else
        hipLaunchKernelGGL(k_mark_factor, dim3(blocks), dim3(256), 0, st, c->pv_out, k, c->J, c->A[tensor],
                           c->fmask[tensor]);
    return hipGetLastError();
}

}  // namespace vest
