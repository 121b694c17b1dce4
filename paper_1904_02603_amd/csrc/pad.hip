// Unequal per-mode ranks (Table 1: J_n per mode).  The kernels are compiled
// for one uniform rank; a context with ranks J_1..J_N runs them at
// J = max J_n on workspace copies of the model in which every element outside
// the caller's model -- factor columns j >= J_n, core elements with some index
// j_n >= J_n -- is marked (Sec. 3.3: a marked element is zero and never
// updated again).  Those elements therefore contribute nothing to any delta,
// residual, update, key or loss, and the padded model equals the caller's.
// These kernels copy the caller's arrays in at vest_init and the caller's
// part back out after every call that changes it.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace vest {

struct RankArg {
    int32_t r[VEST_MAX_ORDER];
};

__global__ void __launch_bounds__(256) k_pad_factor_in(const double *__restrict__ u, int64_t I, int Ju, int J,
                                                       double *__restrict__ p)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= I * J) return;
    const int64_t i = q / J;
    const int j = (int)(q % J);
    p[q] = j < Ju ? u[i * Ju + j] : 0.0;
}

__global__ void __launch_bounds__(256) k_pad_factor_out(const double *__restrict__ p, int64_t I, int Ju, int J,
                                                        double *__restrict__ u)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= I * Ju) return;
    u[q] = p[(q / Ju) * J + q % Ju];
}

// bits j >= Ju of every row word marked
__global__ void __launch_bounds__(256) k_pad_mask_in(const uint32_t *__restrict__ u, int64_t I, int Ju,
                                                     uint32_t *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I) return;
    const uint32_t pad = Ju >= 32 ? 0u : ~((1u << Ju) - 1u);
    p[i] = u[i] | pad;
}

__global__ void __launch_bounds__(256) k_pad_mask_out(const uint32_t *__restrict__ p, int64_t I, int Ju,
                                                      uint32_t *__restrict__ u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I) return;
    const uint32_t keep = Ju >= 32 ? ~0u : (1u << Ju) - 1u;
    u[i] = p[i] & keep;
}

// flat index in the caller's core (ranks ur) of the padded element q (rank J
// in every mode), or -1 when q lies outside the caller's core
__device__ __forceinline__ int64_t user_flat(int64_t q, int N, int J, const RankArg &ur)
{
    int32_t j[VEST_MAX_ORDER];
    for (int n = N - 1; n >= 0; --n) {
        j[n] = (int32_t)(q % J);
        q /= J;
    }
    int64_t f = 0;
    for (int n = 0; n < N; ++n) {
        if (j[n] >= ur.r[n]) return -1;
        f = f * ur.r[n] + j[n];
    }
    return f;
}

__global__ void __launch_bounds__(256) k_pad_core_in(const double *__restrict__ u, const uint8_t *__restrict__ um,
                                                     int64_t G, int N, int J, RankArg ur, double *__restrict__ p,
                                                     uint8_t *__restrict__ pm)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= G) return;
    const int64_t f = user_flat(q, N, J, ur);
    p[q] = f >= 0 ? u[f] : 0.0;
    pm[q] = f >= 0 ? um[f] : (uint8_t)1;
}

// padded -> caller (values and, when um != nullptr, marks), by padded index
__global__ void __launch_bounds__(256) k_pad_core_out(const double *__restrict__ p, const uint8_t *__restrict__ pm,
                                                      int64_t G, int N, int J, RankArg ur, double *__restrict__ u,
                                                      uint8_t *__restrict__ um)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= G) return;
    const int64_t f = user_flat(q, N, J, ur);
    if (f < 0) return;
    u[f] = p[q];
    if (um) um[f] = pm[q];
}

static RankArg ranks_of(const vest_ctx *c)
{
    RankArg r{};
    for (int n = 0; n < c->N; ++n) r.r[n] = c->uranks[n];
    return r;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_pad_in(vest_ctx *c)
{
    hipStream_t st = c->stream;
    for (int n = 0; n < c->N; ++n) {
        const int64_t I = c->d.dims[n];
        hipLaunchKernelGGL(k_pad_factor_in, dim3(blocks_for(I * c->J)), dim3(256), 0, st, c->uA[n], I, c->uranks[n],
                           c->J, c->A[n]);
        hipLaunchKernelGGL(k_pad_mask_in, dim3(blocks_for(I)), dim3(256), 0, st, c->ufmask[n], I, c->uranks[n],
                           c->fmask[n]);
    }
    hipLaunchKernelGGL(k_pad_core_in, dim3(blocks_for(c->G)), dim3(256), 0, st, c->ucore, c->ucmask, c->G, c->N,
                       c->J, ranks_of(c), c->core, c->cmask);
    return hipGetLastError();
}

hipError_t launch_pad_out_factor(vest_ctx *c, int mode)
{
    const int64_t I = c->d.dims[mode];
    hipLaunchKernelGGL(k_pad_factor_out, dim3(blocks_for(I * c->uranks[mode])), dim3(256), 0, c->stream, c->A[mode],
                       I, c->uranks[mode], c->J, c->uA[mode]);
    return hipGetLastError();
}

hipError_t launch_pad_out_core(vest_ctx *c)
{
    hipLaunchKernelGGL(k_pad_core_out, dim3(blocks_for(c->G)), dim3(256), 0, c->stream, c->core, c->cmask, c->G,
                       c->N, c->J, ranks_of(c), c->ucore, (uint8_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_pad_out_masks(vest_ctx *c)
{
    for (int n = 0; n < c->N; ++n) {
        const int64_t I = c->d.dims[n];
        hipLaunchKernelGGL(k_pad_mask_out, dim3(blocks_for(I)), dim3(256), 0, c->stream, c->fmask[n], I,
                           c->uranks[n], c->ufmask[n]);
    }
    hipLaunchKernelGGL(k_pad_core_out, dim3(blocks_for(c->G)), dim3(256), 0, c->stream, c->core, c->cmask, c->G,
                       c->N, c->J, ranks_of(c), c->ucore, c->ucmask);
    return hipGetLastError();
}

hipError_t launch_pad_out_keys(vest_ctx *c, double *core_key, double *const *factor_key)
{
    for (int n = 0; n < c->N; ++n) {
        const int64_t I = c->d.dims[n];
        hipLaunchKernelGGL(k_pad_factor_out, dim3(blocks_for(I * c->uranks[n])), dim3(256), 0, c->stream,
                           c->pkey_fac[n], I, c->uranks[n], c->J, factor_key[n]);
    }
    hipLaunchKernelGGL(k_pad_core_out, dim3(blocks_for(c->G)), dim3(256), 0, c->stream, c->pkey_core, c->cmask, c->G,
                       c->N, c->J, ranks_of(c), core_key, (uint8_t *)nullptr);
    return hipGetLastError();
}

}  // namespace vest
