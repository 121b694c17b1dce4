// Output side of the method: the final column normalisation of Alg. 2, the
// sparse export of the pruned model, the reconstruction error on a held-out
// entry set, and magnitude keys for the value-pruning comparator.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "device.h"
#include "internal.h"

namespace vest {

// Squared norm of column t of an I x J row-major matrix: one block, fixed
// order (thread-strided partial sums, then a tree over the block).
__global__ void __launch_bounds__(256) k_colnorm2(const double *__restrict__ A, int64_t I, int J,
                                                   double *__restrict__ out)
{
    __shared__ double sh[256];
    const int t = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < I; i += 256) {
        const double a = A[i * J + t];
        s = __builtin_fma(a, a, s);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[t] = sh[0];
}

// A[i][t] /= ||column t|| for nonzero columns.
__global__ void __launch_bounds__(256) k_colscale(double *__restrict__ A, int64_t I, int J,
                                                   const double *__restrict__ n2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= I * J) return;
    const double nr = sqrt(n2[q % J]);
    if (nr > 0.0) A[q] = A[q] / nr;
}

// G[beta] *= ||column beta_n of A^(n)|| (mode n of the flat index).
__global__ void __launch_bounds__(256) k_corescale(double *__restrict__ core, int64_t G, int64_t stride, int J,
                                                    const double *__restrict__ n2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= G) return;
    core[q] *= sqrt(n2[(q / stride) % J]);
}

hipError_t launch_normalize(vest_ctx *c)
{
    hipStream_t st = c->stream;
    double *n2 = c->red;  // J doubles of scratch
    int64_t stride = c->G;
    for (int n = 0; n < c->N; ++n) {
        const int64_t I = c->d.dims[n];
        const int J = c->J;
        stride /= J;
        hipLaunchKernelGGL(k_colnorm2, dim3(J), dim3(256), 0, st, c->A[n], I, J, n2);
        hipLaunchKernelGGL(k_colscale, dim3((unsigned)((I * J + 255) / 256)), dim3(256), 0, st, c->A[n], I, J, n2);
        hipLaunchKernelGGL(k_corescale, dim3((unsigned)((c->G + 255) / 256)), dim3(256), 0, st, c->core, c->G, stride,
                           J, n2);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ sparse export
__global__ void __launch_bounds__(256) k_nzflag(const double *__restrict__ v, int64_t n, uint32_t *__restrict__ f)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) f[q] = v[q] != 0.0 ? 1u : 0u;
}

__global__ void __launch_bounds__(256) k_nzwrite(const double *__restrict__ v, int64_t n,
                                                  const uint32_t *__restrict__ f, const uint32_t *__restrict__ pos,
                                                  int64_t *__restrict__ oi, double *__restrict__ ov)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n && f[q]) {
        oi[pos[q]] = q;
        ov[pos[q]] = v[q];
    }
}

// total = last prefix + last flag
__global__ void k_nztotal(const uint32_t *__restrict__ f, const uint32_t *__restrict__ p, int64_t m,
                          uint64_t *__restrict__ out)
{
    if (threadIdx.x == 0) out[0] = (uint64_t)p[m - 1] + f[m - 1];
}

// Nonzero flags and their exclusive prefix of one tensor into the prune
// buffers (pv_in: flags, pv_out: positions); *count receives the total.
static hipError_t nz_scan(vest_ctx *c, const double *v, int64_t n, uint64_t *count_dev)
{
    hipStream_t st = c->stream;
    hipLaunchKernelGGL(k_nzflag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, n, c->pv_in);
    size_t tb = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, tb, c->pv_in, c->pv_out, (int)n, st);
    if (e != hipSuccess) return e;
    if (tb > c->sort_tmp_bytes) return hipErrorOutOfMemory;
    tb = c->sort_tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(c->sort_tmp, tb, c->pv_in, c->pv_out, (int)n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nztotal, dim3(1), dim3(64), 0, st, c->pv_in, c->pv_out, n, count_dev);
    return hipGetLastError();
}

hipError_t launch_count_nonzeros(vest_ctx *c, int64_t *counts)
{
    uint64_t *dev = reinterpret_cast<uint64_t *>(c->red);
    for (int n = 0; n <= c->N; ++n) {
        // the caller's arrays and flat order (the copies of a padded context
        // hold them as well, see pad.hip)
        const double *v = n < c->N ? c->uA[n] : c->ucore;
        const int64_t len = n < c->N ? c->d.dims[n] * c->uranks[n] : c->uG;
        hipError_t e = nz_scan(c, v, len, dev + n);
        if (e != hipSuccess) return e;
    }
    uint64_t h[VEST_MAX_ORDER + 1];
    hipError_t e = hipMemcpyAsync(h, dev, (c->N + 1) * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    for (int n = 0; n <= c->N; ++n) counts[n] = (int64_t)h[n];
    return e;
}

hipError_t launch_export(vest_ctx *c, int64_t *const *fi, double *const *fv, int64_t *ci, double *cv)
{
    uint64_t *dev = reinterpret_cast<uint64_t *>(c->red);
    for (int n = 0; n <= c->N; ++n) {
        const double *v = n < c->N ? c->uA[n] : c->ucore;
        const int64_t len = n < c->N ? c->d.dims[n] * c->uranks[n] : c->uG;
        hipError_t e = nz_scan(c, v, len, dev);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_nzwrite, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, c->stream, v, len, c->pv_in,
                           c->pv_out, n < c->N ? fi[n] : ci, n < c->N ? fv[n] : cv);
    }
    return hipGetLastError();
}

// ------------------------------------------------- held-out reconstruction
struct DimsIn {
    int64_t d[VEST_MAX_ORDER];
};
template <typename T>
struct FacIn {
    const T *p[VEST_MAX_ORDER];
};

// One level of the looped contraction over the other modes' indices
// o_L (order-8 shapes, where the unrolled dense form is not compiled),
// factored: level L returns the partial sum over its subtree,
// d_L[j] = sum_b r[L][b] d_{L+1}(b)[j], so that no floating-point sum has
// more than J terms; o is the flat index of the indices chosen so far.
template <int L, int N, int J, typename T>
__device__ __forceinline__ void heldout_level(const T *__restrict__ Gp, const T (&r)[N - 1][J], int o, T (&d)[J])
{
    constexpr int S = ipow(J, N - 1);
#pragma unroll
    for (int j = 0; j < J; ++j) d[j] = T(0);
#pragma nounroll
    for (int b = 0; b < J; ++b) {
        const T x = pick<J, T>(r[L], b);
        const int oo = o * J + b;
        if constexpr (L == N - 2) {
#pragma unroll
            for (int j = 0; j < J; ++j) d[j] = vfma(x, Gp[j * S + oo], d[j]);
        } else {
            T sub[J];
            heldout_level<L + 1, N, J, T>(Gp, r, oo, sub);
#pragma unroll
            for (int j = 0; j < J; ++j) d[j] = vfma(x, sub[j], d[j]);
        }
    }
}

// B(alpha) = a^(0)_{i_0} . delta^(0)_alpha (Eq. 7) for entries outside the
// layouts; per-block partial sums of (X - B)^2 and X^2, then a fixed-order
// total.  Out-of-range indices raise a flag instead of being read.
template <int N, int J, typename T>
__global__ void __launch_bounds__(256) k_heldout(const int32_t *__restrict__ idx, const double *__restrict__ val,
                                                  int64_t n, DimsIn dims, FacIn<T> fac, const T *__restrict__ Gp,
                                                  double *__restrict__ part, int32_t *__restrict__ flag)
{
    __shared__ double s1[256], s2[256];
    const CoreBases<T> Gb = core_bases_if<N, J, T, dense_form(N, J)>(Gp);
    double e2 = 0.0, x2 = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
        int32_t ii[N];
        bool ok = true;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            ii[m] = idx[q * N + m];
            ok = ok && ii[m] >= 0 && (int64_t)ii[m] < dims.d[m];
        }
        if (!ok) {
            flag[0] = 1;
            continue;
        }
        T r[N - 1][J];
#pragma unroll
        for (int m = 1; m < N; ++m) load_grow<J, T>(fac.p[m] + (int64_t)ii[m] * gather_ld(J, sizeof(T)), r[m - 1]);
        T own[J];
        load_grow<J, T>(fac.p[0] + (int64_t)ii[0] * gather_ld(J, sizeof(T)), own);
        T d[J];
        if constexpr (dense_form(N, J)) {
            delta_vec<N, J, T>(Gb, r, d);
        } else {
            // looped form: delta_j = sum_o Gp[j][o] prod_k r[k][o_k], o in flat
            // order over the other modes (mode 0's permuted core is row-major)
            heldout_level<0, N, J, T>(Gp, r, 0, d);
        }
        T b = own[0] * d[0];
#pragma unroll
        for (int t = 1; t < J; ++t) b = vfma(own[t], d[t], b);
        const double x = val[q];
        const double e = x - (double)b;
        e2 = __builtin_fma(e, e, e2);
        x2 = __builtin_fma(x, x, x2);
    }
    s1[threadIdx.x] = e2;
    s2[threadIdx.x] = x2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

__global__ void __launch_bounds__(256) k_heldout_total(const double *__restrict__ part, int nb, double *__restrict__ out)
{
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s1[0];
        out[1] = s2[0];
    }
}

template <int N, int J, typename T>
static hipError_t heldout_t(vest_ctx *c, const int32_t *idx, const double *val, int64_t n, double *dout)
{
    DimsIn dm{};
    FacIn<T> fa{};
    for (int m = 0; m < N; ++m) {
        dm.d[m] = c->d.dims[m];
        fa.p[m] = reinterpret_cast<const T *>(c->Ag[m]);
    }
    const int nb = kLossBlocks;
    hipLaunchKernelGGL((k_heldout<N, J, T>), dim3(nb), dim3(256), 0, c->stream, idx, val, n, dm, fa,
                       reinterpret_cast<const T *>(c->Gp[0]), c->red, c->flags);
    hipLaunchKernelGGL(k_heldout_total, dim3(1), dim3(256), 0, c->stream, c->red, nb, dout);
    return hipGetLastError();
}

hipError_t launch_heldout(vest_ctx *c, const int32_t *idx, const double *val, int64_t n, double *dout)
{
#define VEST_CASE(NN, JJ)                                                               \
    if (c->N == NN && c->J == JJ)                                                       \
        return c->f32 ? heldout_t<NN, JJ, float>(c, idx, val, n, dout)                   \
                      : heldout_t<NN, JJ, double>(c, idx, val, n, dout);
    VEST_SHAPES(VEST_CASE)
#undef VEST_CASE
    return hipErrorInvalidValue;
}

// ------------------------------------------------- value-pruning keys
// Comparator of Sec. 4: prune by magnitude.  key = |value|, +inf if marked.
__global__ void __launch_bounds__(256) k_absfac(const double *__restrict__ A, const uint32_t *__restrict__ mask,
                                                 int64_t n, int J, double *__restrict__ key)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    key[q] = ((mask[q / J] >> (q % J)) & 1u) ? HUGE_VAL : fabs(A[q]);
}

__global__ void __launch_bounds__(256) k_abscore(const double *__restrict__ core, const uint8_t *__restrict__ mask,
                                                  int64_t n, double *__restrict__ key)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    key[q] = mask[q] ? HUGE_VAL : fabs(core[q]);
}

hipError_t launch_value_keys(vest_ctx *c, double *core_key, double *const *fkey)
{
    hipStream_t st = c->stream;
    for (int n = 0; n < c->N; ++n) {
        const int64_t len = c->d.dims[n] * c->J;
        hipLaunchKernelGGL(k_absfac, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, c->A[n], c->fmask[n], len,
                           c->J, fkey[n]);
    }
    hipLaunchKernelGGL(k_abscore, dim3((unsigned)((c->G + 255) / 256)), dim3(256), 0, st, c->core, c->cmask, c->G,
                       core_key);
    return hipGetLastError();
}

}  // namespace vest
