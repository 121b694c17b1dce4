// Held-out reconstruction error of a Tucker model given as plain device
// arrays, for callers that cannot allocate device memory (vest_model_error_noalloc
// in vest.h).  Same quantity as vest_test_error: Eq. 4 over a set of entries,
// B(alpha) by Eq. 7.  No context and no workspace: the per-block partial sums
// live in a file-scope device array whose address is looked up once per
// device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"

namespace vest_noalloc {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kEntriesPerBlock = kThreads * kPerThread;
constexpr int kMaxBlocks = VEST_NOALLOC_MAX_ENTRIES / kEntriesPerBlock;
constexpr int kMaxDevices = 64;

// [block][3]: sum (X - B)^2, sum X^2, count of out-of-range entries.  Every
// call writes every slot it later reads, so nothing has to start at zero.
static __device__ __align__(256) double scratch[kMaxBlocks * 3];

struct Model {
    const double *A[VEST_MAX_ORDER];
    int64_t dims[VEST_MAX_ORDER];
    int32_t ranks[VEST_MAX_ORDER];
    int32_t N;
    int64_t G;
};

// B(alpha) = sum over core elements in flat order of G_beta * prod_n a^(n)_{i_n beta_n},
// evaluated factored from the last mode: acc[k] holds the sum over modes
// k..N-1 at fixed leading indices; when index k wraps, acc[k] times
// a^(k-1)_{i_{k-1} beta_{k-1}} is added to acc[k-1].
__device__ double reconstruct(const Model &m, const double *__restrict__ core, const int64_t *row)
{
    double acc[VEST_MAX_ORDER];
    int32_t jj[VEST_MAX_ORDER];
    for (int k = 0; k < m.N; ++k) {
        acc[k] = 0.0;
        jj[k] = 0;
    }
    const int last = m.N - 1;
    const double *al = m.A[last] + row[last];
    for (int64_t f = 0; f < m.G; ++f) {
        acc[last] = fma(al[jj[last]], core[f], acc[last]);
        int k = last;
        while (true) {
            if (++jj[k] < m.ranks[k]) break;
            jj[k] = 0;
            if (k == 0) break;
            acc[k - 1] = fma(m.A[k - 1][row[k - 1] + jj[k - 1]], acc[k], acc[k - 1]);
            acc[k] = 0.0;
            --k;
        }
    }
    return acc[0];
}

__global__ void __launch_bounds__(kThreads) k_partial(Model m, const double *__restrict__ core,
                                                      const int32_t *__restrict__ idx,
                                                      const double *__restrict__ val, int64_t n,
                                                      double *__restrict__ part)
{
    __shared__ double red[3][kThreads];
    double se = 0.0, xx = 0.0, bad = 0.0;
    for (int q = 0; q < kPerThread; ++q) {
        const int64_t e = (int64_t)blockIdx.x * kEntriesPerBlock + q * kThreads + threadIdx.x;
        if (e >= n) break;
        int64_t row[VEST_MAX_ORDER];
        bool ok = true;
        for (int k = 0; k < m.N; ++k) {
            const int32_t i = idx[e * m.N + k];
            ok = ok && i >= 0 && i < m.dims[k];
            row[k] = ok ? (int64_t)i * m.ranks[k] : 0;
        }
        const double x = val[e];
        if (!ok) {
            bad += 1.0;
            continue;
        }
        const double r = x - reconstruct(m, core, row);
        se = fma(r, r, se);
        xx = fma(x, x, xx);
    }
    red[0][threadIdx.x] = se;
    red[1][threadIdx.x] = xx;
    red[2][threadIdx.x] = bad;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int v = 0; v < 3; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[(int64_t)blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// One block: the block partials in a fixed tree (thread t takes blocks t,
// t + 256, ... in order), then out = {sse, sum X^2, RE, bad entries}.
__global__ void __launch_bounds__(kThreads) k_final(const double *__restrict__ part, int nblocks,
                                                    double *__restrict__ out)
{
    __shared__ double red[3][kThreads];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kThreads)
        for (int v = 0; v < 3; ++v) s[v] += part[(int64_t)b * 3 + v];
    for (int v = 0; v < 3; ++v) red[v][threadIdx.x] = s[v];
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int v = 0; v < 3; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double bad = red[2][0];
        const double sse = red[0][0], xx = red[1][0];
        out[0] = bad > 0 ? NAN : sse;
        out[1] = bad > 0 ? NAN : xx;
        out[2] = bad > 0 ? NAN : (xx > 0 ? sqrt(sse / xx) : 0.0);
        out[3] = bad;
    }
}

// Device address of `scratch` on each device, looked up on the first call
// made with that device current.
static std::mutex g_lock;
static double *g_scratch[kMaxDevices];

static hipError_t scratch_for_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace vest_noalloc

static int fail(const char *msg)
{
    vest::set_error("vest_model_error_noalloc: %s", msg);
    return VEST_EINVAL;
}

extern "C" int vest_model_error_noalloc(const vest_desc *desc, void *stream, const double *const *factors,
                                        const double *core, const int32_t *idx, const double *val, int64_t n,
                                        double *out)
{
    using namespace vest_noalloc;
    if (!desc || !factors || !core || !out) return fail("null argument");
    if (desc->order < 2 || desc->order > VEST_MAX_ORDER) return fail("order out of range");
    if (n < 0) return fail("negative entry count");
    if (n > VEST_NOALLOC_MAX_ENTRIES)
        return fail("entry set larger than VEST_NOALLOC_MAX_ENTRIES (the static scratch bound)");
    if (n > 0 && (!idx || !val)) return fail("null entry arrays");
    Model m{};
    m.N = desc->order;
    m.G = 1;
    for (int k = 0; k < m.N; ++k) {
        if (desc->dims[k] < 1 || desc->dims[k] >= (int64_t(1) << 31)) return fail("dimension out of range");
        if (desc->ranks[k] < 1 || desc->ranks[k] > VEST_MAX_RANK) return fail("rank out of range");
        if (!factors[k]) return fail("null factor pointer");
        m.A[k] = factors[k];
        m.dims[k] = desc->dims[k];
        m.ranks[k] = desc->ranks[k];
        m.G *= desc->ranks[k];
    }
    double *part = nullptr;
    hipError_t e = scratch_for_current_device(&part);
    if (e != hipSuccess) {
        fail(hipGetErrorString(e));
        return VEST_EDEVICE;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nblocks = (int)((n + kEntriesPerBlock - 1) / kEntriesPerBlock);
    if (nblocks > 0)
        hipLaunchKernelGGL(k_partial, dim3(nblocks), dim3(kThreads), 0, st, m, core, idx, val, n, part);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kThreads), 0, st, part, nblocks, out);
    e = hipGetLastError();
    if (e != hipSuccess) {
        fail(hipGetErrorString(e));
        return VEST_EDEVICE;
    }
    return VEST_OK;
}
