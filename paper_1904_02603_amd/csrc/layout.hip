// Validation of the observed tensor and construction of the per-mode
// row-group layouts (set-up, not part of a sweep).
//
//  1. index bounds and finiteness of every value;
//  2. Omega is a set (Table 1): a stable LSD radix sort by (i_1..i_N) puts
//     equal tuples next to each other;
//  3. per mode n: stable radix sort of the entry ids by i_n (ties keep the
//     canonical id order), row lengths, then the host assigns rows to
//     row-group classes and waves (see internal.h), and a scatter kernel
//     writes every entry into its slot.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace vest {

struct DimsArg {
    int64_t d[VEST_MAX_ORDER];
    int32_t N;
};

struct RowPlace {
    int64_t base;  // normal row: wave base slot; long row: index of its first wave
    int32_t glog;  // lanes per row (log2); -1 for a long row
    int32_t sub;   // row group within the wave
};

struct OidxArg {
    int32_t *p[VEST_MAX_ORDER];
};

__global__ void __launch_bounds__(256) k_validate(const int32_t *__restrict__ idx, const double *__restrict__ val,
                                                  int64_t nnz, DimsArg dm, int32_t *__restrict__ flags)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        for (int n = 0; n < dm.N; ++n) {
            const int32_t v = idx[e * dm.N + n];
            if (v < 0 || (int64_t)v >= dm.d[n]) atomicOr(&flags[0], 1);
        }
        if (!isfinite(val[e])) atomicOr(&flags[1], 1);
    }
}

__global__ void __launch_bounds__(256) k_iota(uint32_t *__restrict__ v, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) v[q] = (uint32_t)q;
}

__global__ void __launch_bounds__(256) k_gather_key(const int32_t *__restrict__ idx, int N, int n,
                                                    const uint32_t *__restrict__ perm, int64_t nnz,
                                                    uint32_t *__restrict__ keys)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) keys[q] = (uint32_t)idx[(int64_t)perm[q] * N + n];
}

__global__ void __launch_bounds__(256) k_dupcheck(const int32_t *__restrict__ idx, int N,
                                                  const uint32_t *__restrict__ perm, int64_t nnz,
                                                  int32_t *__restrict__ flags)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < 1 || q >= nnz) return;
    const int32_t *a = idx + (int64_t)perm[q] * N;
    const int32_t *b = idx + (int64_t)perm[q - 1] * N;
    bool same = true;
    for (int n = 0; n < N; ++n) same = same && (a[n] == b[n]);
    if (same) atomicOr(&flags[2], 1);
}

__global__ void __launch_bounds__(256) k_mode_key(const int32_t *__restrict__ idx, int N, int n, int64_t nnz,
                                                  uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) {
        keys[q] = (uint32_t)idx[q * N + n];
        vals[q] = (uint32_t)q;
    }
}

// Row lengths from the sorted row keys: every run of equal keys is one row.
// The first entry of a run records where it starts, the last one (after a
// kernel boundary) the length; no atomics, so rows of millions of entries (a
// Zipf-skewed mode) cost no more than short ones.
__global__ void __launch_bounds__(256) k_run_start(const uint32_t *__restrict__ keys, int64_t nnz,
                                                   uint32_t *__restrict__ start)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz && (q == 0 || keys[q] != keys[q - 1])) start[keys[q]] = (uint32_t)q;
}

__global__ void __launch_bounds__(256) k_run_len(const uint32_t *__restrict__ keys, int64_t nnz,
                                                 const uint32_t *__restrict__ start, uint32_t *__restrict__ counts)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz && (q == nnz - 1 || keys[q] != keys[q + 1])) counts[keys[q]] = (uint32_t)(q + 1) - start[keys[q]];
}

template <typename T>
__global__ void __launch_bounds__(256) k_scatter(const uint32_t *__restrict__ rows, const uint32_t *__restrict__ ids,
                                                 int64_t nnz, const int64_t *__restrict__ row_ptr,
                                                 const RowPlace *__restrict__ place, const WaveInfo *__restrict__ waves,
                                                 const int32_t *__restrict__ idx, int N, int mode,
                                                 const double *__restrict__ val, OidxArg oidx, T *__restrict__ xval,
                                                 int32_t *__restrict__ perm, int chunk)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const uint32_t r = rows[p];
    const uint32_t e = ids[p];
    const int64_t q = p - row_ptr[r];
    const RowPlace P = place[r];
    int64_t slot;
    if (P.glog >= 0) {
        const int64_t g = 1ll << P.glog;
        slot = P.base + (q >> P.glog) * kWave + ((int64_t)P.sub << P.glog) + (q & (g - 1));
    } else {
        slot = waves[P.base + q / chunk].base + (q % chunk);
    }
    int m = 0;
    for (int k = 0; k < N; ++k) {
        if (k == mode) continue;
        oidx.p[m][slot] = idx[(int64_t)e * N + k];
        ++m;
    }
    xval[slot] = (T)val[e];
    perm[slot] = (int32_t)e;
}

static int bits_for(int64_t v)
{
    int b = 1;
    while (b < 32 && (int64_t(1) << b) < v) ++b;
    return b;
}

static unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

#define CHECK_HIP(x)                         \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

// Host part of the row-group plan of one mode (see internal.h).
struct HostPlan {
    std::vector<WaveInfo> waves;
    std::vector<int32_t> row_order;
    std::vector<RowPlace> place;
    std::vector<LongRow> longrows;
    std::vector<int64_t> row_ptr;
    int64_t nslots = 0, maxlen = 0;
    int32_t nchunks = 0;
};

static void plan_mode(const std::vector<uint32_t> &cnt, int lt, HostPlan &hp)
{
    const int64_t I = (int64_t)cnt.size();
    const int64_t chunk = (int64_t)kWave * lt;   // long-row chunk
    std::vector<int32_t> cls[7], longs;
    for (int64_t r = 0; r < I; ++r) {
        const int64_t len = cnt[r];
        hp.maxlen = std::max<int64_t>(hp.maxlen, len);
        if (len > chunk) {
            longs.push_back((int32_t)r);
            continue;
        }
        int c = 0;
        while (((len + (int64_t(1) << c) - 1) >> c) > lt) ++c;
        cls[c].push_back((int32_t)r);
    }
    auto by_len = [&](int32_t a, int32_t b) { return cnt[a] > cnt[b]; };
    for (auto &v : cls) std::stable_sort(v.begin(), v.end(), by_len);
    std::stable_sort(longs.begin(), longs.end(), by_len);

    hp.place.assign(I, RowPlace{0, 0, 0});
    hp.row_order.clear();
    hp.waves.clear();
    hp.longrows.clear();
    int64_t slot = 0;
    for (int c = 0; c < 7; ++c) {
        const int per = kWave >> c;
        const std::vector<int32_t> &v = cls[c];
        for (size_t i = 0; i < v.size(); i += per) {
            const int nrows = (int)std::min<size_t>(per, v.size() - i);
            const int64_t lmax = cnt[v[i]];
            const int32_t K = (int32_t)((lmax + (int64_t(1) << c) - 1) >> c);
            WaveInfo w{};
            w.base = slot;
            w.K = K;
            w.glog = c;
            w.first = (int32_t)hp.row_order.size();
            w.nrows = nrows;
            w.chunk = -1;
            w.klive = K;
            for (int j = 0; j < nrows; ++j) {
                hp.place[v[i + j]] = RowPlace{slot, c, j};
                hp.row_order.push_back(v[i + j]);
            }
            hp.waves.push_back(w);
            slot += (int64_t)kWave * K;
        }
    }
    for (int32_t r : longs) {
        const int64_t len = cnt[r];
        const int32_t nch = (int32_t)((len + chunk - 1) / chunk);
        hp.place[r] = RowPlace{(int64_t)hp.waves.size(), -1, 0};
        hp.longrows.push_back(LongRow{r, hp.nchunks, nch, 0});
        const int32_t pos = (int32_t)hp.row_order.size();
        hp.row_order.push_back(r);
        for (int32_t ch = 0; ch < nch; ++ch) {
            const int64_t n = std::min<int64_t>(chunk, len - (int64_t)ch * chunk);
            WaveInfo w{};
            w.base = slot;
            w.K = (int32_t)((n + kWave - 1) / kWave);
            w.glog = 6;
            w.first = pos;
            w.nrows = 1;
            w.chunk = hp.nchunks++;
            w.klive = w.K;
            hp.waves.push_back(w);
            slot += (int64_t)kWave * w.K;
        }
    }
    hp.nslots = slot;
    hp.row_ptr.assign(I + 1, 0);
    for (int64_t r = 0; r < I; ++r) hp.row_ptr[r + 1] = hp.row_ptr[r] + cnt[r];
}

hipError_t build_layouts(vest_ctx *c, const int32_t *idx, const double *val, char *scratch, size_t scratch_bytes,
                         int *bad)
{
    *bad = 0;
    const int N = c->N;
    const int64_t nnz = c->d.nnz;
    hipStream_t st = c->stream;
    int64_t Imax = 0;
    for (int n = 0; n < N; ++n) Imax = std::max<int64_t>(Imax, c->d.dims[n]);

    Bump b{scratch, 0, scratch_bytes};
    auto *ka = (uint32_t *)b.take(nnz * 4), *kb = (uint32_t *)b.take(nnz * 4);
    auto *va = (uint32_t *)b.take(nnz * 4), *vb = (uint32_t *)b.take(nnz * 4);
    auto *counts = (uint32_t *)b.take(Imax * 4);
    auto *place = (RowPlace *)b.take(Imax * sizeof(RowPlace));
    auto *rptr = (int64_t *)b.take((Imax + 1) * 8);
    if (!ka || !kb || !va || !vb || !counts || !place || !rptr) return hipErrorOutOfMemory;

    // 1. bounds and finiteness
    DimsArg dm{};
    dm.N = N;
    for (int n = 0; n < N; ++n) dm.d[n] = c->d.dims[n];
    CHECK_HIP(hipMemsetAsync(c->flags, 0, 64, st));
    hipLaunchKernelGGL(k_validate, dim3(std::min<int64_t>(grid_for(nnz), 4096)), dim3(256), 0, st, idx, val, nnz, dm,
                       c->flags);
    int32_t fl[16] = {};
    CHECK_HIP(hipMemcpyAsync(fl, c->flags, 64, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipStreamSynchronize(st));
    if (fl[0]) { *bad = 1; return hipSuccess; }
    if (fl[1]) { *bad = 2; return hipSuccess; }

    // 2. duplicates: lexicographic order by stable LSD passes, last mode first
    hipLaunchKernelGGL(k_iota, dim3(grid_for(nnz)), dim3(256), 0, st, va, nnz);
    for (int n = N - 1; n >= 0; --n) {
        hipLaunchKernelGGL(k_gather_key, dim3(grid_for(nnz)), dim3(256), 0, st, idx, N, n, va, nnz, ka);
        size_t tb = c->sort_tmp_bytes;
        CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(c->sort_tmp, tb, ka, kb, va, vb, (int)nnz, 0,
                                                     bits_for(c->d.dims[n]), st));
        std::swap(va, vb);
    }
    hipLaunchKernelGGL(k_dupcheck, dim3(grid_for(nnz)), dim3(256), 0, st, idx, N, va, nnz, c->flags);
    CHECK_HIP(hipMemcpyAsync(fl, c->flags, 64, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipStreamSynchronize(st));
    if (fl[2]) { *bad = 3; return hipSuccess; }

    // 3. per-mode layouts
    std::vector<uint32_t> cnt;
    for (int n = 0; n < N; ++n) {
        const int64_t I = c->d.dims[n];
        ModeLayout &L = c->lay[n];
        hipLaunchKernelGGL(k_mode_key, dim3(grid_for(nnz)), dim3(256), 0, st, idx, N, n, nnz, ka, va);
        size_t tb = c->sort_tmp_bytes;
        CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(c->sort_tmp, tb, ka, kb, va, vb, (int)nnz, 0, bits_for(I), st));
        CHECK_HIP(hipMemsetAsync(counts, 0, I * 4, st));
        // run starts go to the row-placement buffer, which is written only later
        auto *start = reinterpret_cast<uint32_t *>(place);
        hipLaunchKernelGGL(k_run_start, dim3(grid_for(nnz)), dim3(256), 0, st, kb, nnz, start);
        hipLaunchKernelGGL(k_run_len, dim3(grid_for(nnz)), dim3(256), 0, st, kb, nnz, start, counts);
        cnt.assign(I, 0);
        CHECK_HIP(hipMemcpyAsync(cnt.data(), counts, I * 4, hipMemcpyDeviceToHost, st));
        CHECK_HIP(hipStreamSynchronize(st));

        HostPlan hp;
        auto fits = [&] {
            return hp.nslots <= L.cap_slots && (int64_t)hp.waves.size() <= L.cap_waves &&
                   (int64_t)hp.longrows.size() <= L.cap_long && hp.nchunks <= L.cap_chunks;
        };
        int lt = lane_target_for(nnz);
        plan_mode(cnt, lt, hp);
        if (!fits() && lt != kLaneTargetLarge) {   // a compaction of a context sized for the larger target
            hp = HostPlan();
            lt = kLaneTargetLarge;
            plan_mode(cnt, lt, hp);
        }
        if (!fits()) return hipErrorOutOfMemory;
        L.lane_target = lt;
        L.nslots = hp.nslots;
        L.npad = hp.nslots - nnz;
        L.nwaves = (int32_t)hp.waves.size();
        L.nlong = (int32_t)hp.longrows.size();
        L.nchunks = hp.nchunks;
        L.maxlen = hp.maxlen;
        CHECK_HIP(hipMemcpyAsync(L.waves, hp.waves.data(), hp.waves.size() * sizeof(WaveInfo),
                                 hipMemcpyHostToDevice, st));
        CHECK_HIP(hipMemcpyAsync(L.row_order, hp.row_order.data(), hp.row_order.size() * 4, hipMemcpyHostToDevice,
                                 st));
        if (!hp.longrows.empty())
            CHECK_HIP(hipMemcpyAsync(L.longrows, hp.longrows.data(), hp.longrows.size() * sizeof(LongRow),
                                     hipMemcpyHostToDevice, st));
        CHECK_HIP(hipMemcpyAsync(place, hp.place.data(), I * sizeof(RowPlace), hipMemcpyHostToDevice, st));
        CHECK_HIP(hipMemcpyAsync(rptr, hp.row_ptr.data(), (I + 1) * 8, hipMemcpyHostToDevice, st));

        const int64_t ns = hp.nslots;
        CHECK_HIP(hipMemsetAsync(L.oidx[0], 0xff, ns * 4, st));
        for (int m = 1; m < N - 1; ++m) CHECK_HIP(hipMemsetAsync(L.oidx[m], 0, ns * 4, st));
        CHECK_HIP(hipMemsetAsync(L.xval, 0, ns * c->tsize, st));
        CHECK_HIP(hipMemsetAsync(L.perm, 0xff, ns * 4, st));
        OidxArg oa{};
        for (int m = 0; m < N - 1; ++m) oa.p[m] = L.oidx[m];
        if (c->f32)
            hipLaunchKernelGGL(k_scatter<float>, dim3(grid_for(nnz)), dim3(256), 0, st, kb, vb, nnz, rptr, place,
                               L.waves, idx, N, n, val, oa, reinterpret_cast<float *>(L.xval), L.perm,
                               kWave * lt);
        else
            hipLaunchKernelGGL(k_scatter<double>, dim3(grid_for(nnz)), dim3(256), 0, st, kb, vb, nnz, rptr, place,
                               L.waves, idx, N, n, val, oa, reinterpret_cast<double *>(L.xval), L.perm,
                               kWave * lt);
        CHECK_HIP(hipGetLastError());
        // the host vectors above are read by pending copies: wait before reuse
        CHECK_HIP(hipStreamSynchronize(st));
    }

    return hipGetLastError();
}

// ------------------------------------------------------------ compaction
// An entry is dead once some mode's row of it is fully marked: its
// reconstruction B(alpha) and every delta, core weight and key term of it
// are zero for good (marks never clear).  One wave per wave of the mode-0
// layout marks the live slots and sums X^2 of the dead ones.
struct MaskArg {
    const uint32_t *p[VEST_MAX_ORDER];
};

template <typename T>
__global__ void __launch_bounds__(64) k_live(const WaveInfo *__restrict__ waves, const int32_t *__restrict__ row_order,
                                             OidxArg oidx, const T *__restrict__ xval, MaskArg mk, int N,
                                             uint32_t full, uint32_t *__restrict__ flags, double *__restrict__ dsq)
{
    __shared__ double sh[64];
    const WaveInfo wi = waves[blockIdx.x];
    const int lane = threadIdx.x;
    const int grp = lane >> wi.glog;
    const int32_t row = grp < wi.nrows ? row_order[wi.first + grp] : 0;
    double acc = 0.0;
    for (int k = 0; k < wi.K; ++k) {
        const int64_t s = wi.base + (int64_t)k * 64 + lane;
        uint32_t alive = 0;
        if (oidx.p[0][s] >= 0) {
            bool ok = (~mk.p[0][row] & full) != 0u;
            for (int m = 1; m < N; ++m) ok = ok && (~mk.p[m][oidx.p[m - 1][s]] & full) != 0u;
            alive = ok ? 1u : 0u;
            if (!ok) {
                const double x = (double)xval[s];
                acc += x * x;
            }
        }
        flags[s] = alive;
    }
    sh[lane] = acc;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (lane < w) sh[lane] += sh[lane + w];
        __syncthreads();
    }
    if (lane == 0) dsq[blockIdx.x] = sh[0];
}

template <typename T>
__global__ void __launch_bounds__(64) k_gather_live(const WaveInfo *__restrict__ waves,
                                                    const int32_t *__restrict__ row_order, OidxArg oidx,
                                                    const T *__restrict__ xval, int N,
                                                    const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos,
                                                    int32_t *__restrict__ idx, double *__restrict__ val)
{
    const WaveInfo wi = waves[blockIdx.x];
    const int lane = threadIdx.x;
    const int grp = lane >> wi.glog;
    const int32_t row = grp < wi.nrows ? row_order[wi.first + grp] : 0;
    for (int k = 0; k < wi.K; ++k) {
        const int64_t s = wi.base + (int64_t)k * 64 + lane;
        if (!flags[s]) continue;
        const int64_t q = pos[s];
        idx[q * N] = row;
        for (int m = 1; m < N; ++m) idx[q * N + m] = oidx.p[m - 1][s];
        val[q] = (double)xval[s];
    }
}

__global__ void k_sum_fixed(const double *__restrict__ part, int64_t n, double *__restrict__ out)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

hipError_t launch_compact(vest_ctx *c, int32_t **idx_out, double **val_out, int64_t *live, double *dead_sq)
{
    const int N = c->N;
    const ModeLayout &L = c->lay[0];
    hipStream_t st = c->stream;
    const int64_t ns = L.nslots;
    Bump b{(char *)c->stage, 0, c->stage_bytes};
    auto *flags = (uint32_t *)b.take(ns * 4);
    auto *pos = (uint32_t *)b.take(ns * 4);
    auto *dsq = (double *)b.take((size_t)L.nwaves * 8 + 8);
    auto *idx = (int32_t *)b.take((size_t)c->d.nnz * N * 4);
    auto *val = (double *)b.take((size_t)c->d.nnz * 8);
    if (!flags || !pos || !dsq || !idx || !val) return hipErrorOutOfMemory;
    OidxArg oa{};
    for (int m = 0; m < N - 1; ++m) oa.p[m] = L.oidx[m];
    MaskArg mk{};
    for (int n = 0; n < N; ++n) mk.p[n] = c->fmask[n];
    const uint32_t full = c->J == 32 ? 0xffffffffu : (1u << c->J) - 1u;
    if (L.nwaves > 0) {
        if (c->f32)
            hipLaunchKernelGGL(k_live<float>, dim3(L.nwaves), dim3(64), 0, st, L.waves, L.row_order, oa,
                               reinterpret_cast<const float *>(L.xval), mk, N, full, flags, dsq);
        else
            hipLaunchKernelGGL(k_live<double>, dim3(L.nwaves), dim3(64), 0, st, L.waves, L.row_order, oa,
                               reinterpret_cast<const double *>(L.xval), mk, N, full, flags, dsq);
    }
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, dsq, (int64_t)L.nwaves, dsq + L.nwaves);
    size_t tb = 0;
    CHECK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, flags, pos, (int)ns, st));
    if (tb > c->sort_tmp_bytes) return hipErrorOutOfMemory;
    tb = c->sort_tmp_bytes;
    CHECK_HIP(hipcub::DeviceScan::ExclusiveSum(c->sort_tmp, tb, flags, pos, (int)ns, st));
    if (L.nwaves > 0) {
        if (c->f32)
            hipLaunchKernelGGL(k_gather_live<float>, dim3(L.nwaves), dim3(64), 0, st, L.waves, L.row_order, oa,
                               reinterpret_cast<const float *>(L.xval), N, flags, pos, idx, val);
        else
            hipLaunchKernelGGL(k_gather_live<double>, dim3(L.nwaves), dim3(64), 0, st, L.waves, L.row_order, oa,
                               reinterpret_cast<const double *>(L.xval), N, flags, pos, idx, val);
    }
    CHECK_HIP(hipGetLastError());
    uint32_t tail[2] = {0, 0};
    double d = 0.0;
    CHECK_HIP(hipMemcpyAsync(&tail[0], pos + ns - 1, 4, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipMemcpyAsync(&tail[1], flags + ns - 1, 4, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipMemcpyAsync(&d, dsq + L.nwaves, 8, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipStreamSynchronize(st));
    *live = (int64_t)tail[0] + tail[1];
    *dead_sq = d;
    *idx_out = idx;
    *val_out = val;
    return hipSuccess;
}

// Live partition (see internal.h).  One wave per layout wave; lane l reads
// its K <= 16 slots (indices, value, canonical id), marks each live or dead
// and writes them back live first, in order, then dead; klive of the wave is
// the largest live count of its lanes.  Dead entries contribute exactly zero
// to the factor sweeps and keys (delta = 0), so stopping at klive changes no
// result.  Padding slots count as dead and already sit at the end.
constexpr int kLiveMaxK = 16;

// LDS bytes of one wave's staging: its K <= kLiveMaxK steps of indices,
// canonical id and value, one column per lane
template <int N, typename T>
constexpr size_t live_lds_bytes() { return (size_t)kLiveMaxK * kWave * ((N - 1) * 4 + 4 + sizeof(T)); }

// One wave per block.  Each lane reads its K slots, decides which entries are
// live, and places every entry at its new step in an LDS column of its own
// (a dynamically indexed per-lane array; no lane reads another's column).  It
// then writes back in step order, so each store of the wave covers one
// contiguous row of 64 slots, and only from the lane's first moved step on
// (a slot keeps its entry up to the lane's first dead one).
template <int N, typename T>
__global__ void __launch_bounds__(kWave) k_live_partition(WaveInfo *__restrict__ waves, int nwaves, OidxArg oidx,
                                                          T *__restrict__ xval, int32_t *__restrict__ perm,
                                                          MaskArg masks, uint32_t full)
{
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x;
    const int w = blockIdx.x;
    if (w >= nwaves) return;
    const WaveInfo wi = waves[w];
    if (wi.K > kLiveMaxK) {   // not met with lane targets <= 16; such a wave keeps every step
        if (lane == 0) waves[w].klive = wi.K;
        return;
    }
    const int K = wi.K;
    int32_t id[kLiveMaxK][N - 1], pv[kLiveMaxK];
    T xv[kLiveMaxK];
    bool live[kLiveMaxK];
    int nlive = 0;
#pragma unroll
    for (int k = 0; k < kLiveMaxK; ++k) {
        live[k] = false;
        if (k < K) {
            const int64_t sl = wi.base + (int64_t)k * kWave + lane;
#pragma unroll
            for (int m = 0; m < N - 1; ++m) id[k][m] = oidx.p[m][sl];
            xv[k] = xval[sl];
            pv[k] = perm[sl];
            bool ok = id[k][0] >= 0;
#pragma unroll
            for (int m = 0; m < N - 1; ++m) ok = ok && ((~masks.p[m][ok ? id[k][m] : 0]) & full) != 0u;
            live[k] = ok;
            nlive += ok ? 1 : 0;
        }
    }
    T *sx = reinterpret_cast<T *>(smem);                                         // [kLiveMaxK][64]
    int32_t *sp = reinterpret_cast<int32_t *>(smem + (size_t)kLiveMaxK * kWave * sizeof(T));   // [kLiveMaxK][64]
    int32_t *si = sp + kLiveMaxK * kWave;                                        // [N-1][kLiveMaxK][64]
    int nl = 0, nd = nlive, first = K;
#pragma unroll
    for (int k = 0; k < kLiveMaxK; ++k) {
        if (k < K) {
            const int dst = live[k] ? nl++ : nd++;
            if (dst != k && k < first) first = k;
            const int c = dst * kWave + lane;
            sx[c] = xv[k];
            sp[c] = pv[k];
#pragma unroll
            for (int m = 0; m < N - 1; ++m) si[m * kLiveMaxK * kWave + c] = id[k][m];
        }
    }
    for (int k = first; k < K; ++k) {
        const int c = k * kWave + lane;
        const int64_t sl = wi.base + (int64_t)k * kWave + lane;
#pragma unroll
        for (int m = 0; m < N - 1; ++m) oidx.p[m][sl] = si[m * kLiveMaxK * kWave + c];
        xval[sl] = sx[c];
        perm[sl] = sp[c];
    }
    int kl = nlive;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const int o = __shfl_xor(kl, d);
        kl = o > kl ? o : kl;
    }
    if (lane == 0) waves[w].klive = kl;
}

template <int N>
static hipError_t live_partition_n(vest_ctx *c, hipStream_t st)
{
    const uint32_t full = c->J >= 32 ? 0xffffffffu : (1u << c->J) - 1u;
    for (int n = 0; n < N; ++n) {
        ModeLayout &L = c->lay[n];
        if (L.nwaves == 0) continue;
        OidxArg oa{};
        MaskArg ma{};
        for (int m = 0; m < N - 1; ++m) {
            oa.p[m] = L.oidx[m];
            ma.p[m] = c->fmask[m < n ? m : m + 1];
        }
        if (c->f32)
            hipLaunchKernelGGL((k_live_partition<N, float>), dim3(L.nwaves), dim3(kWave), (live_lds_bytes<N, float>()),
                               st, L.waves, L.nwaves, oa, reinterpret_cast<float *>(L.xval), L.perm, ma, full);
        else
            hipLaunchKernelGGL((k_live_partition<N, double>), dim3(L.nwaves), dim3(kWave), (live_lds_bytes<N, double>()),
                               st, L.waves, L.nwaves, oa, reinterpret_cast<double *>(L.xval), L.perm, ma, full);
    }
    return hipGetLastError();
}

hipError_t launch_live_partition(vest_ctx *c, hipStream_t st)
{
    switch (c->N) {
    case 2: return live_partition_n<2>(c, st);
    case 3: return live_partition_n<3>(c, st);
    case 4: return live_partition_n<4>(c, st);
    case 5: return live_partition_n<5>(c, st);
    case 6: return live_partition_n<6>(c, st);
    case 7: return live_partition_n<7>(c, st);
    case 8: return live_partition_n<8>(c, st);
    case 9: return live_partition_n<9>(c, st);
    case 10: return live_partition_n<10>(c, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace vest
