// Entry points of the C ABI declared in include/vest.h.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace vest {

static thread_local char g_err[512];

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

static int device_error(vest_ctx *c, hipError_t e, const char *where)
{
    set_error("%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
    if (c) c->dead = true;
    return VEST_EDEVICE;
}

int check_desc(const vest_desc *d)
{
    if (!d) { set_error("null descriptor"); return VEST_EINVAL; }
    if (d->order < 2 || d->order > VEST_MAX_ORDER) { set_error("order %d outside 2..%d", d->order, VEST_MAX_ORDER); return VEST_EINVAL; }
    if (d->reg != VEST_REG_LF && d->reg != VEST_REG_L1) { set_error("unknown regulariser %d", d->reg); return VEST_EINVAL; }
    if (d->precision != VEST_FP64 && d->precision != VEST_FP32 && d->precision != VEST_BF16) { set_error("unknown precision %d", d->precision); return VEST_EINVAL; }
    if (d->reserved != 0) { set_error("reserved field must be 0"); return VEST_EINVAL; }
    if (!(d->lambda > 0.0) || !std::isfinite(d->lambda)) { set_error("lambda must be finite and > 0"); return VEST_EINVAL; }
    if (d->nnz < 1 || d->nnz >= (int64_t(1) << 31)) { set_error("nnz %lld outside 1..2^31-1", (long long)d->nnz); return VEST_EINVAL; }
    for (int n = 0; n < d->order; ++n) {
        if (d->dims[n] < 1 || d->dims[n] >= (int64_t(1) << 31)) { set_error("dims[%d] out of range", n); return VEST_EINVAL; }
        if (d->ranks[n] < 1 || d->ranks[n] > VEST_MAX_RANK) { set_error("ranks[%d] outside 1..%d", n, VEST_MAX_RANK); return VEST_EINVAL; }
    }
    // unequal ranks run padded to the largest (pad.hip): sizes checked at it
    const int J = max_rank(d);
    int64_t G = 1;
    for (int n = 0; n < d->order; ++n) G *= J;
    for (int n = 0; n < d->order; ++n)
        if (d->dims[n] * J >= (int64_t(1) << 31) || G >= (int64_t(1) << 31)) {
            set_error("tensor of %d-th factor or core too large", n);
            return VEST_EINVAL;
        }
    if (!shape_supported(d->order, J)) {
        set_error("no kernel instance for order %d, rank %d", d->order, J);
        return VEST_EUNSUPPORTED;
    }
    return VEST_OK;
}

int max_rank(const vest_desc *d)
{
    int J = 0;
    for (int n = 0; n < d->order; ++n) J = d->ranks[n] > J ? d->ranks[n] : J;
    return J;
}

// The descriptor the kernels run on: every rank set to the largest.
static vest_desc uniform_desc(const vest_desc *d)
{
    vest_desc u = *d;
    const int J = max_rank(d);
    for (int n = 0; n < d->order; ++n) u.ranks[n] = J;
    return u;
}

int plan_workspace(const vest_desc *d, Plan *p)
{
    const int N = d->order, J = d->ranks[0];
    const int64_t nnz = d->nnz;
    int64_t G = 1, Imax = 0, maxt = 0;
    for (int n = 0; n < N; ++n) {
        G *= J;
        Imax = d->dims[n] > Imax ? d->dims[n] : Imax;
        maxt = d->dims[n] * J > maxt ? d->dims[n] * J : maxt;
    }
    maxt = G > maxt ? G : maxt;
    p->max_tensor = maxt;
    for (int n = 0; n < N; ++n) {
        // class-c waves (c >= 1) hold rows longer than LT 2^(c-1): at most
        // 2 nnz / (64 LT) + 1 waves per class; long rows add at most
        // 2 nnz / (64 LT) chunk waves
        // rounding pads a row of L entries by less than 2 L / LT slots, each
        // length class's last wave by at most 64 LT; the wave and chunk
        // counts are bounded at the smaller target (both layouts fit)
        const int64_t lt = lane_target_for(nnz), ch = (int64_t)kWave * kLaneTargetSmall;
        p->slot_bound[n] = nnz + 2 * nnz / lt + 1024 * lt + 1024;
        p->wave_bound[n] = d->dims[n] / 64 + nnz / (32 * kLaneTargetSmall) + 2 * nnz / ch + 16;
        p->long_bound[n] = nnz / ch + 1;
    }
    p->chunk_bound = 2 * nnz / ((int64_t)kWave * kLaneTargetSmall) + 1;
    p->gram_chunks = (d->dims[N - 1] + kGramRows - 1) / kGramRows;
    size_t t1 = 0, t2 = 0;
    hipError_t e1 = hipcub::DeviceRadixSort::SortPairs(nullptr, t1, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                       (uint32_t *)nullptr, (uint32_t *)nullptr, (int)nnz);
    hipError_t e2 = hipcub::DeviceRadixSort::SortPairs(nullptr, t2, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                                       (uint32_t *)nullptr, (uint32_t *)nullptr, (int)maxt);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        set_error("radix-sort scratch query failed (no HIP device?)");
        return VEST_EDEVICE;
    }
    p->sort_tmp = (t1 > t2 ? t1 : t2) + 256;
    p->scratch_bytes = (size_t)nnz * 4 * 4 + (size_t)Imax * (4 + 16 + 8) + 8 + 16 * 256;
    return VEST_OK;
}

// Assign every workspace region (also used with base = nullptr to size it).
static bool carve(vest_ctx *c, const Plan &p, Bump &b, char **scratch)
{
    const int N = c->N, J = c->J;
    const size_t ts = (size_t)c->tsize;
    bool ok = true;
    auto take = [&](size_t bytes) {
        void *q = b.take(bytes ? bytes : 1);
        ok = ok && (q != nullptr || b.base == nullptr);
        return q;
    };
    for (int n = 0; n < N; ++n) {
        ModeLayout &L = c->lay[n];
        const int64_t sb = p.slot_bound[n];
        L.cap_slots = L.nslots = sb;
        L.cap_waves = L.nwaves = (int32_t)p.wave_bound[n];
        L.cap_long = L.nlong = (int32_t)p.long_bound[n];
        L.cap_chunks = L.nchunks = (int32_t)p.chunk_bound;
        L.waves = (WaveInfo *)take(p.wave_bound[n] * sizeof(WaveInfo));
        L.row_order = (int32_t *)take(c->d.dims[n] * 4);
        for (int m = 0; m < N - 1; ++m) L.oidx[m] = (int32_t *)take(sb * 4);
        L.xval = take(sb * ts);
        L.perm = (int32_t *)take(sb * 4);
        L.longrows = (LongRow *)take(p.long_bound[n] * sizeof(LongRow));
    }
    // e and ms are contiguous; together they also stage a compaction
    // (vest_compact): mode-0 slot flags and positions, wave partials, the
    // live entries' indices and values
    const size_t e_bytes = (size_t)p.slot_bound[N - 1] * ts;
    size_t ms_bytes = (size_t)(p.slot_bound[N - 1] + 63) / 64 * 64 * J * ts;
    const size_t stage_need = 2 * ((size_t)p.slot_bound[0] * 4 + 256) + ((size_t)p.wave_bound[0] * 8 + 264) +
                              ((size_t)c->d.nnz * N * 4 + 256) + ((size_t)c->d.nnz * 8 + 256);
    if (e_bytes + 256 + ms_bytes < stage_need) ms_bytes = stage_need - e_bytes;
    c->e = take(e_bytes);
    c->ms = take(ms_bytes);
    c->stage = c->e;
    c->stage_bytes = (size_t)((char *)c->ms - (char *)c->e) + ms_bytes;
    c->hdiag = (double *)take(c->G * 8);
    for (int n = 0; n < N; ++n) c->Gp[n] = take(c->G * ts);
    for (int n = 0; n < N; ++n) c->Ag[n] = take(c->d.dims[n] * gather_ld(J, (int)ts) * ts);
    for (int m = 0; m + 2 < N; ++m) c->colA[m] = take(c->d.dims[m] * J * ts * (N == 3 ? 2 : 1));   // order 3: pairs
    const int gw = gram_width(J);
    const int64_t Il = c->d.dims[N - 1];
    c->ldrb = rowbuf_width(N, J, (int)ts);
    int64_t gsq = (int64_t)gw * gw > (int64_t)keys_width(N, J, (int)ts) * round8(2 * J)
                      ? (int64_t)gw * gw
                      : (int64_t)keys_width(N, J, (int)ts) * round8(2 * J);
    if (gsq < gram_core_cells(J)) gsq = gram_core_cells(J);
    // (keys_width x round8(2J) also bounds the R-only batches: round8(J S) x round8(J))
    c->rowbuf = (double *)take(Il * c->ldrb * 8);
    c->kp = (double *)take(Il * gw * 8);
    c->gram_part = (double *)take(p.gram_chunks * gsq * 8);
    c->gram = (double *)take(gsq * 8);
    c->dprev = (double *)take(J * J * 8);
    int na = nacc_vc(J) > 2 * J ? nacc_vc(J) : 2 * J;
    na = na > keys_nacc(N, J, (int)ts) ? na : keys_nacc(N, J, (int)ts);
    c->partials = (double *)take(p.chunk_bound * na * 8);
    c->wsum = (double *)take(p.wave_bound[N - 1] * 8);
    c->partials_side = (double *)take(p.chunk_bound * na * 8);
    if (!gather_in_lds(N, J, (int)ts)) {
        c->gt = take((size_t)c->G * ts);
        c->gnz = (uint32_t *)take(((size_t)(c->G / J) + 31) / 32 * 4);
    }
    if (c->padded) {
        for (int n = 0; n < N; ++n) {
            c->A[n] = (double *)take(c->d.dims[n] * J * 8);
            c->fmask[n] = (uint32_t *)take(c->d.dims[n] * 4);
            c->pkey_fac[n] = (double *)take(c->d.dims[n] * J * 8);
        }
        c->core = (double *)take(c->G * 8);
        c->cmask = (uint8_t *)take(c->G);
        c->pkey_core = (double *)take(c->G * 8);
    }
    c->red = (double *)take((16 * kLossBlocks + 64) * 8);
    c->sse_lag = c->red + 16 * kLossBlocks + 32;
    c->flags = (int32_t *)take(64);
    c->sel_hist = (uint32_t *)take((size_t)(VEST_MAX_ORDER + 1) * 4096 * 4);
    c->sel_state = (char *)take((size_t)(VEST_MAX_ORDER + 1) * 24);
    c->pv_in = (uint32_t *)take(p.max_tensor * 4);
    c->pv_out = (uint32_t *)take(p.max_tensor * 4);
    c->sort_tmp = take(p.sort_tmp);
    c->sort_tmp_bytes = p.sort_tmp;
    *scratch = (char *)take(p.scratch_bytes);
    return ok;
}

static void fill_ctx_shape(vest_ctx *c, const vest_desc *d)
{
    c->d = uniform_desc(d);
    c->N = d->order;
    c->J = max_rank(d);
    c->G = 1;
    c->uG = 1;
    c->padded = false;
    for (int n = 0; n < c->N; ++n) {
        c->G *= c->J;
        c->uG *= d->ranks[n];
        c->uranks[n] = d->ranks[n];
        c->padded = c->padded || d->ranks[n] != c->J;
    }
    c->f32 = d->precision != VEST_FP64;
    c->tsize = c->f32 ? 4 : 8;
}

#define CALL_HIP(c, x, where)                                       \
    do {                                                            \
        hipError_t e_ = (x);                                        \
        if (e_ != hipSuccess) return device_error((c), e_, where); \
    } while (0)

static int ensure_gp(vest_ctx *c, int mode)
{
    if (c->gp_version[mode] != c->core_version) {
        CALL_HIP(c, launch_permute_core(c, mode), "permute core");
        c->gp_version[mode] = c->core_version;
    }
    return VEST_OK;
}

// Refresh every mode's permuted core right after the core changed, so that a
// factor sweep launches exactly one kernel.
static int refresh_gp(vest_ctx *c)
{
    for (int n = 0; n < c->N; ++n) {
        int rc = ensure_gp(c, n);
        if (rc) return rc;
    }
    return VEST_OK;
}

static int ensure_ag(vest_ctx *c)
{
    for (int n = 0; n < c->N; ++n)
        if (!c->ag_valid[n]) {
            CALL_HIP(c, launch_gather_copy(c, n), "gather copy");
            c->ag_valid[n] = true;
        }
    return VEST_OK;
}

static int ensure_residual(vest_ctx *c)
{
    if (c->e_valid && c->ms_valid) {
        if (c->e_lag) {
            CALL_HIP(c, launch_lag_apply(c), "residual catch-up");
            c->e_lag = false;
        }
        return VEST_OK;
    }
    int rc = ensure_ag(c);
    if (rc) return rc;
    rc = ensure_gp(c, c->N - 1);
    if (rc) return rc;
    CALL_HIP(c, launch_rowgroup(c, c->N - 1, OP_RESID), "residual");
    c->e_valid = true;
    c->ms_valid = true;
    c->e_lag = false;
    return VEST_OK;
}

// Live partition of the layouts once marks have changed (before a factor
// sweep or the factor keys read klive).  It moves entries of the core layout,
// so the residual and its slot copy must be formed again.
// Fraction of dead entries in the worst mode layout if the marks were spread
// at random: a mode-n entry is dead when one of its other-mode rows is fully
// marked, and a row of J elements of a factor with marked fraction f is fully
// marked with probability f^J.
static double dead_estimate(const vest_ctx *c)
{
    double p[VEST_MAX_ORDER];
    for (int k = 0; k < c->N; ++k) {
        const double f = (double)c->marked_fac[k] / ((double)c->d.dims[k] * c->J);
        p[k] = std::pow(f, c->J);
    }
    double worst = 0.0;
    for (int n = 0; n < c->N; ++n) {
        double alive = 1.0;
        for (int k = 0; k < c->N; ++k)
            if (k != n) alive *= 1.0 - p[k];
        worst = std::max(worst, 1.0 - alive);
    }
    return worst;
}

// The partition costs about one gather sweep per mode, and skipping it is
// exact: marks never clear, so the steps past an older partition's klive hold
// dead entries still.  It runs when the estimate of dead entries has grown by
// kLiveStep since the last partition (a VeST^man ramp partitions a few times,
// not after every prune step).
static constexpr double kLiveStep = 0.1;

static int ensure_live(vest_ctx *c, hipStream_t st)
{
    if (!c->live_stale) return VEST_OK;
    const double est = dead_estimate(c);
    if (est < c->live_dead_est + kLiveStep) return VEST_OK;   // stays stale: re-checked after more marks
    CALL_HIP(c, launch_live_partition(c, st), "live partition");
    c->live_stale = false;
    c->live_dead_est = est;
    c->e_valid = false;
    c->ms_valid = false;
    c->e_lag = false;
    return VEST_OK;
}

static int live(vest_ctx *c)
{
    if (!c) { set_error("null context"); return VEST_EINVAL; }
    if (c->dead) { set_error("context is unusable after a device error"); return VEST_EDEVICE; }
    return VEST_OK;
}

}  // namespace vest

using namespace vest;

extern "C" {

const char *vest_strerror(int code)
{
    switch (code) {
    case VEST_OK: return "ok";
    case VEST_EINVAL: return "invalid argument or input data";
    case VEST_ENOSPC: return "workspace too small";
    case VEST_EDEVICE: return "HIP device error";
    case VEST_ESTATE: return "call out of order";
    case VEST_EUNSUPPORTED: return "no kernel instance for this order and rank";
    default: return "unknown error";
    }
}

const char *vest_last_error(void) { return g_err; }

int vest_workspace_bytes(const vest_desc *desc, size_t *bytes)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!bytes) { set_error("null output"); return VEST_EINVAL; }
    Plan p;
    const vest_desc ud = uniform_desc(desc);
    rc = plan_workspace(&ud, &p);
    if (rc) return rc;
    vest_ctx tmp;
    fill_ctx_shape(&tmp, desc);
    Bump b{nullptr, 0, ~size_t(0)};
    char *scr = nullptr;
    carve(&tmp, p, b, &scr);
    *bytes = b.off + 256;
    return VEST_OK;
}

int vest_init(const vest_desc *desc, void *stream, const int32_t *idx, const double *val, double *const *factors,
              double *core, uint32_t *const *factor_mask, uint8_t *core_mask, void *workspace, size_t ws_bytes,
              vest_ctx **out)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!out || !idx || !val || !factors || !core || !factor_mask || !core_mask || !workspace) {
        set_error("null pointer argument");
        return VEST_EINVAL;
    }
    for (int n = 0; n < desc->order; ++n)
        if (!factors[n] || !factor_mask[n]) { set_error("null factor or mask pointer (mode %d)", n); return VEST_EINVAL; }
    if (((uintptr_t)workspace & 255) != 0) { set_error("workspace must be 256-byte aligned"); return VEST_EINVAL; }
    Plan p;
    const vest_desc ud = uniform_desc(desc);
    rc = plan_workspace(&ud, &p);
    if (rc) return rc;
    size_t need = 0;
    {
        vest_ctx tmp;
        fill_ctx_shape(&tmp, desc);
        Bump b{nullptr, 0, ~size_t(0)};
        char *scr = nullptr;
        carve(&tmp, p, b, &scr);
        need = b.off + 256;
    }
    if (ws_bytes < need) {
        set_error("workspace of %zu bytes, %zu needed", ws_bytes, need);
        return VEST_ENOSPC;
    }
    vest_ctx *c = new (std::nothrow) vest_ctx();
    if (!c) { set_error("out of host memory"); return VEST_EINVAL; }
    fill_ctx_shape(c, desc);
    c->stream = (hipStream_t)stream;
    hipError_t he = hipGetDevice(&c->device);
    if (he != hipSuccess) { int r = device_error(nullptr, he, "hipGetDevice"); delete c; return r; }
    for (int n = 0; n < c->N; ++n) {
        c->A[n] = c->uA[n] = factors[n];
        c->fmask[n] = c->ufmask[n] = factor_mask[n];
    }
    c->core = c->ucore = core;
    c->cmask = c->ucmask = core_mask;
    Bump b{(char *)workspace, 0, ws_bytes};   // a padded context re-points A, core and masks into it
    char *scratch = nullptr;
    if (!carve(c, p, b, &scratch)) { delete c; set_error("workspace carve failed"); return VEST_ENOSPC; }

    c->scratch = scratch;
    c->scratch_bytes = p.scratch_bytes;
    int bad = 0;
    he = build_layouts(c, idx, val, scratch, p.scratch_bytes, &bad);
    if (he != hipSuccess) { int r = device_error(nullptr, he, "layout"); delete c; return r; }
    if (bad) {
        const char *why[] = {"", "index out of range", "non-finite value", "duplicate index tuple (Omega is a set)"};
        set_error("invalid observed tensor: %s", why[bad]);
        delete c;
        return VEST_EINVAL;
    }
    // ||X||^2 over Omega
    double *dout = c->red + 16 * kLossBlocks;
    he = launch_sumsq(c->stream, val, desc->nnz, c->red, dout);
    double hx[2] = {0, 0};
    if (he == hipSuccess) he = hipMemcpyAsync(hx, dout, 16, hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) { int r = device_error(nullptr, he, "norm"); delete c; return r; }
    c->xnorm2 = hx[0];

    // marking table: zero the marked elements, count the marks
    int64_t *cnt = reinterpret_cast<int64_t *>(c->red + 16 * kLossBlocks + 8);
    int64_t hc[VEST_MAX_ORDER + 1] = {};
    he = hipMemsetAsync(cnt, 0, (c->N + 1) * 8, c->stream);
    if (he == hipSuccess && c->padded) he = launch_pad_in(c);
    if (he == hipSuccess) he = launch_mask_init(c, cnt);
    if (he == hipSuccess && c->padded) {   // marked elements of the caller's arrays are zero too
        for (int n = 0; n < c->N && he == hipSuccess; ++n) he = launch_pad_out_factor(c, n);
        if (he == hipSuccess) he = launch_pad_out_core(c);
    }
    if (he == hipSuccess) he = hipMemcpyAsync(hc, cnt, (c->N + 1) * 8, hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess) he = hipMemsetAsync(c->rowbuf, 0, c->d.dims[c->N - 1] * c->ldrb * 8, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) { int r = device_error(nullptr, he, "masks"); delete c; return r; }
    for (int n = 0; n < c->N; ++n) {
        c->marked_fac[n] = hc[n];
        if (hc[n] > 0) c->live_stale = true;   // rows may start fully marked
    }
    c->marked_core = hc[c->N];
    c->core_version = 1;
    for (int n = 0; n < c->N; ++n) c->ag_valid[n] = false;
    if ((rc = ensure_ag(c)) || (rc = refresh_gp(c))) { delete c; return rc; }
    *out = c;
    return VEST_OK;
}

int vest_sweep_factor(vest_ctx *c, int32_t mode)
{
    int rc = live(c);
    if (rc) return rc;
    if (mode < 0 || mode >= c->N) { set_error("mode %d outside 0..%d", mode, c->N - 1); return VEST_EINVAL; }
    if ((rc = ensure_live(c, c->stream))) return rc;
    if ((rc = ensure_ag(c))) return rc;
    if ((rc = ensure_gp(c, mode))) return rc;
    CALL_HIP(c, launch_rowgroup(c, mode, OP_SWEEP), "factor sweep");
    if (c->padded) CALL_HIP(c, launch_pad_out_factor(c, mode), "padded copy-out");
    c->e_valid = false;
    c->ms_valid = false;
    c->hdiag_valid = false;
    return VEST_OK;
}

int vest_sweep_core(vest_ctx *c)
{
    int rc = live(c);
    if (rc) return rc;
    // when the residual has to be formed anyway, its pass also accumulates
    // the first slab's statistics (dense form)
    bool fused = false;
    if (!(c->e_valid && c->ms_valid)) {
        if ((rc = ensure_ag(c)) || (rc = ensure_gp(c, c->N - 1))) return rc;
        fused = resid_fuses_slab0(c);
        CALL_HIP(c, launch_rowgroup(c, c->N - 1, fused ? OP_RESID_S0 : OP_RESID), "residual");
        c->e_valid = true;
        c->ms_valid = true;
        c->e_lag = false;
    } else if ((rc = ensure_residual(c))) {   // a residual lagging the previous core sweep catches up
        return rc;
    }
    CALL_HIP(c, launch_core_sweep(c, fused), "core sweep");   // sets e_lag
    if (c->padded) CALL_HIP(c, launch_pad_out_core(c), "padded copy-out");
    c->core_version++;
    c->e_valid = true;
    c->hdiag_valid = true;
    return refresh_gp(c);
}

int vest_iterate_many(vest_ctx *const *cs, int32_t n, void *stream, void *dev_table, void *host_table,
                      size_t table_bytes)
{
    if (!cs || n < 1 || !dev_table || !host_table) { set_error("bad batch arguments"); return VEST_EINVAL; }
    for (int i = 0; i < n; ++i) {
        int rc = live(cs[i]);
        if (rc) return rc;
    }
    const vest_ctx *c0 = cs[0];
    for (int i = 0; i < n; ++i) {
        const vest_ctx *c = cs[i];
        bool fits = c->N == c0->N && c->J == c0->J && c->f32 == c0->f32 && c->d.precision == c0->d.precision &&
                    !c->padded && !c->slab_ev && batch_dense_ok(c) && resid_fuses_slab0(c);
        for (int m = 0; m < c->N && fits; ++m) fits = c->ag_valid[m] && c->gp_version[m] == c->core_version;
        for (int j = 0; j < i && fits; ++j) fits = cs[j] != c;
        if (!fits) {
            set_error("context %d does not fit the batched path (shape, form, marks or state)", i);
            return VEST_EUNSUPPORTED;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        int rc = ensure_live(cs[i], st);
        if (rc) return rc;
    }
    BatchArena ba;
    ba.host = (char *)host_table;
    ba.dev = (char *)dev_table;
    ba.cap = table_bytes;
    LaunchList L;
    bool ok = true;
    for (int m = 0; m < c0->N && ok; ++m) ok = plan_factor_batch(cs, n, m, OP_SWEEP, st, ba, L);
    ok = ok && plan_factor_batch(cs, n, c0->N - 1, OP_RESID_S0, st, ba, L);
    ok = ok && plan_core_batch(cs, n, true, st, ba, L);
    ok = ok && plan_permute_batch(cs, n, st, ba, L);
    if (!ok) {
        set_error("batch tables exceed %zu bytes or the shape has no batched path", table_bytes);
        return VEST_EUNSUPPORTED;
    }
    hipError_t e = hipMemcpyAsync(dev_table, host_table, ba.used, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        for (auto &f : L) f();
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        for (int i = 0; i < n; ++i) cs[i]->dead = true;
        return device_error(nullptr, e, "batched iteration");
    }
    for (int i = 0; i < n; ++i) {
        vest_ctx *c = cs[i];
        c->core_version++;
        for (int m = 0; m < c->N; ++m) c->gp_version[m] = c->core_version;
        c->e_valid = true;
        c->ms_valid = true;
        c->e_lag = ipow(c->J, c->N - 2) > 1;   // as in the single-context core sweep
        c->hdiag_valid = true;
    }
    return VEST_OK;
}

int vest_responsibility(vest_ctx *c, double *core_key, double *const *factor_key)
{
    int rc = live(c);
    if (rc) return rc;
    if (!core_key || !factor_key) { set_error("null key pointer"); return VEST_EINVAL; }
    for (int n = 0; n < c->N; ++n)
        if (!factor_key[n]) { set_error("null factor key pointer (mode %d)", n); return VEST_EINVAL; }
    if ((rc = ensure_live(c, c->stream))) return rc;
    if ((rc = ensure_residual(c))) return rc;
    for (int n = 0; n < c->N; ++n)
        if ((rc = ensure_gp(c, n))) return rc;
    // The core keys stream the entries (HBM-bound) while the factor keys are
    // bound by the vector ALU; they share no buffer they write (the core keys
    // take their own long-row partials), so for large contexts they run on a
    // second stream, forked from and joined back into the context's stream.
    double *const *ukey_fac = factor_key;
    double *ukey_core = core_key;
    if (c->padded) {   // keys of the padded model, copied out at the end
        core_key = c->pkey_core;
        factor_key = c->pkey_fac;
    }
    const bool two = c->d.nnz >= kSideStreamMinNnz;
    if (two && !c->side) {
        CALL_HIP(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "side stream");
        CALL_HIP(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming), "fork event");
        CALL_HIP(c, hipEventCreateWithFlags(&c->join, hipEventDisableTiming), "join event");
    }
    c->key_core = core_key;
    if (two) {
        CALL_HIP(c, hipEventRecord(c->fork, c->stream), "fork");
        CALL_HIP(c, hipStreamWaitEvent(c->side, c->fork, 0), "fork wait");
        CALL_HIP(c, launch_core_keys(c, core_key, c->side, c->partials_side), "core keys");
        CALL_HIP(c, hipEventRecord(c->join, c->side), "join");
    }
    for (int n = 0; n < c->N; ++n) {
        c->key_fac[n] = factor_key[n];
        CALL_HIP(c, launch_rowgroup(c, n, OP_KEYS), "factor keys");
    }
    if (two)
        CALL_HIP(c, hipStreamWaitEvent(c->stream, c->join, 0), "join wait");
    else
        CALL_HIP(c, launch_core_keys(c, core_key, c->stream, c->partials), "core keys");
    if (c->padded) CALL_HIP(c, launch_pad_out_keys(c, ukey_core, ukey_fac), "padded key copy-out");
    c->keys_pending = true;
    return VEST_OK;
}

int vest_prune(vest_ctx *c, int64_t core_k, const int64_t *factor_k)
{
    int rc = live(c);
    if (rc) return rc;
    if (!c->keys_pending) { set_error("vest_prune needs keys from vest_responsibility"); return VEST_ESTATE; }
    if (!factor_k) { set_error("null factor counts"); return VEST_EINVAL; }
    if (core_k < 0 || core_k > c->G - c->marked_core) { set_error("core count %lld out of range", (long long)core_k); return VEST_EINVAL; }
    for (int n = 0; n < c->N; ++n)
        if (factor_k[n] < 0 || factor_k[n] > c->d.dims[n] * c->J - c->marked_fac[n]) {
            set_error("factor count %lld of mode %d out of range", (long long)factor_k[n], n);
            return VEST_EINVAL;
        }
    CALL_HIP(c, launch_prune(c, core_k, factor_k), "prune");
    if (c->padded) {
        for (int n = 0; n < c->N; ++n)
            if (factor_k[n] > 0) CALL_HIP(c, launch_pad_out_factor(c, n), "padded copy-out");
        CALL_HIP(c, launch_pad_out_masks(c), "padded copy-out");
    }
    if (core_k > 0) {
        c->marked_core += core_k;
        c->core_version++;
    }
    for (int n = 0; n < c->N; ++n)
        if (factor_k[n] > 0) {
            c->marked_fac[n] += factor_k[n];
            c->ag_valid[n] = false;
            c->ms_valid = false;
            c->hdiag_valid = false;
            c->live_stale = true;
        }
    c->e_valid = false;
    c->keys_pending = false;
    if ((rc = ensure_ag(c))) return rc;
    return refresh_gp(c);
}

int vest_loss(vest_ctx *c, double *out)
{
    int rc = live(c);
    if (rc) return rc;
    if (!out) { set_error("null output"); return VEST_EINVAL; }
    // after a core sweep the SSE is already formed (the residual lags)
    const bool lagged = c->e_valid && c->ms_valid && c->e_lag;
    if (!lagged && (rc = ensure_residual(c))) return rc;
    double *dout = c->red + 16 * kLossBlocks;
    CALL_HIP(c, launch_loss(c, dout, lagged ? c->sse_lag : nullptr), "loss");
    // the two sums come back through pinned host memory (a direct copy, no
    // pageable staging), allocated on the first call, freed by vest_destroy
    if (!c->host_red) CALL_HIP(c, hipHostMalloc((void **)&c->host_red, 64, hipHostMallocDefault), "pinned buffer");
    CALL_HIP(c, hipMemcpyAsync(c->host_red, dout, 16, hipMemcpyDeviceToHost, c->stream), "loss copy");
    CALL_HIP(c, hipStreamSynchronize(c->stream), "loss sync");
    const double h[2] = {c->host_red[0], c->host_red[1]};
    out[0] = h[0] + c->sse_dead;
    out[1] = c->xnorm2;
    out[2] = c->d.lambda * h[1];
    out[3] = out[0] + out[2];
    out[4] = c->xnorm2 > 0 ? std::sqrt(out[0] / c->xnorm2) : 0.0;
    return VEST_OK;
}

int vest_compact(vest_ctx *c, int64_t *live_out)
{
    int rc = live(c);
    if (rc) return rc;
    int32_t *idx = nullptr;
    double *val = nullptr;
    int64_t nlive = 0;
    double dsq = 0.0;
    CALL_HIP(c, launch_compact(c, &idx, &val, &nlive, &dsq), "compaction");
    if (live_out) *live_out = nlive;
    if (nlive == c->d.nnz || nlive == 0) return VEST_OK;  // nothing to drop / keep the layout
    c->d.nnz = nlive;
    int bad = 0;
    // the build scratch carved for the original entry count bounds the one
    // the smaller build needs
    hipError_t he = build_layouts(c, idx, val, c->scratch, c->scratch_bytes, &bad);
    if (he != hipSuccess) return device_error(c, he, "compaction layout");
    if (bad) { set_error("compaction produced an invalid entry set (%d)", bad); c->dead = true; return VEST_EDEVICE; }
    c->sse_dead += dsq;
    c->e_valid = false;
    c->ms_valid = false;
    c->hdiag_valid = false;
    // every entry left is live in every layout (none has a fully marked row)
    // and the rebuilt layouts start with every step live
    c->live_stale = false;
    c->live_dead_est = dead_estimate(c);
    return VEST_OK;
}

int vest_normalize(vest_ctx *c)
{
    int rc = live(c);
    if (rc) return rc;
    CALL_HIP(c, launch_normalize(c), "normalisation");
    if (c->padded) {
        for (int n = 0; n < c->N; ++n) CALL_HIP(c, launch_pad_out_factor(c, n), "padded copy-out");
        CALL_HIP(c, launch_pad_out_core(c), "padded copy-out");
    }
    c->core_version++;
    for (int n = 0; n < c->N; ++n) c->ag_valid[n] = false;
    c->e_valid = false;
    c->ms_valid = false;
    c->hdiag_valid = false;
    c->keys_pending = false;
    if ((rc = ensure_ag(c))) return rc;
    return refresh_gp(c);
}

int vest_count_nonzeros(vest_ctx *c, int64_t *counts)
{
    int rc = live(c);
    if (rc) return rc;
    if (!counts) { set_error("null output"); return VEST_EINVAL; }
    CALL_HIP(c, launch_count_nonzeros(c, counts), "nonzero count");
    return VEST_OK;
}

int vest_export(vest_ctx *c, int64_t *const *fac_idx, double *const *fac_val, int64_t *core_idx, double *core_val)
{
    int rc = live(c);
    if (rc) return rc;
    if (!fac_idx || !fac_val || !core_idx || !core_val) { set_error("null output"); return VEST_EINVAL; }
    for (int n = 0; n < c->N; ++n)
        if (!fac_idx[n] || !fac_val[n]) { set_error("null output of mode %d", n); return VEST_EINVAL; }
    CALL_HIP(c, launch_export(c, fac_idx, fac_val, core_idx, core_val), "export");
    return VEST_OK;
}

int vest_test_error(vest_ctx *c, const int32_t *idx, const double *val, int64_t n, double *out)
{
    int rc = live(c);
    if (rc) return rc;
    if (!out || (n > 0 && (!idx || !val)) || n < 0) { set_error("bad held-out arguments"); return VEST_EINVAL; }
    double h[2] = {0.0, 0.0};
    int32_t fl[16] = {};
    if (n > 0) {
        for (int m = 0; m < c->N; ++m)
            if ((rc = ensure_gp(c, m))) return rc;
        if ((rc = ensure_ag(c))) return rc;
        double *dout = c->red + 16 * kLossBlocks;
        CALL_HIP(c, hipMemsetAsync(c->flags, 0, 64, c->stream), "flags");
        CALL_HIP(c, launch_heldout(c, idx, val, n, dout), "held-out error");
        CALL_HIP(c, hipMemcpyAsync(h, dout, 16, hipMemcpyDeviceToHost, c->stream), "held-out copy");
        CALL_HIP(c, hipMemcpyAsync(fl, c->flags, 64, hipMemcpyDeviceToHost, c->stream), "flag copy");
        CALL_HIP(c, hipStreamSynchronize(c->stream), "held-out sync");
        if (fl[0]) { set_error("held-out index out of range"); return VEST_EINVAL; }
    }
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[1] > 0 ? std::sqrt(h[0] / h[1]) : 0.0;
    return VEST_OK;
}

int vest_value_keys(vest_ctx *c, double *core_key, double *const *factor_key)
{
    int rc = live(c);
    if (rc) return rc;
    if (!core_key || !factor_key) { set_error("null key pointer"); return VEST_EINVAL; }
    for (int n = 0; n < c->N; ++n)
        if (!factor_key[n]) { set_error("null factor key pointer (mode %d)", n); return VEST_EINVAL; }
    if (c->padded) {
        CALL_HIP(c, launch_value_keys(c, c->pkey_core, c->pkey_fac), "value keys");
        CALL_HIP(c, launch_pad_out_keys(c, core_key, factor_key), "padded key copy-out");
        for (int n = 0; n < c->N; ++n) c->key_fac[n] = c->pkey_fac[n];
        c->key_core = c->pkey_core;
    } else {
        CALL_HIP(c, launch_value_keys(c, core_key, factor_key), "value keys");
        for (int n = 0; n < c->N; ++n) c->key_fac[n] = factor_key[n];
        c->key_core = core_key;
    }
    c->keys_pending = true;
    return VEST_OK;
}

int vest_set_kernel(vest_ctx *c, int32_t kernel)
{
    if (!c) { set_error("null context"); return VEST_EINVAL; }
    if (kernel != VEST_KERNEL_AUTO && kernel != VEST_KERNEL_DENSE && kernel != VEST_KERNEL_GATHER) {
        set_error("unknown kernel policy %d", kernel);
        return VEST_EINVAL;
    }
    c->kernel_policy = kernel;
    return VEST_OK;
}

int vest_layout_stats(vest_ctx *c, int32_t mode, int64_t *out)
{
    if (!c || !out || mode < 0 || mode >= c->N) { set_error("bad argument"); return VEST_EINVAL; }
    const ModeLayout &L = c->lay[mode];
    out[0] = L.nslots;
    out[1] = L.npad;
    out[2] = L.nwaves;
    out[3] = L.nlong;
    out[4] = L.nchunks;
    out[5] = L.maxlen;
    out[6] = c->d.dims[mode];
    out[7] = c->d.nnz;
    return VEST_OK;
}

static void drop_slab_events(vest_ctx *c)
{
    for (int i = 0; i < 2 * c->slab_ev_cap; ++i) (void)hipEventDestroy(c->slab_ev[i]);
    delete[] c->slab_ev;
    c->slab_ev = nullptr;
    c->slab_ev_cap = c->slab_ev_n = 0;
}

int vest_slab_timing(vest_ctx *c, int32_t enable)
{
    int rc = live(c);
    if (rc) return rc;
    if (c->slab_ev) {
        CALL_HIP(c, hipStreamSynchronize(c->stream), "timing sync");
        drop_slab_events(c);
    }
    if (!enable) return VEST_OK;
    const int cap = 1024;
    c->slab_ev = new hipEvent_t[2 * cap];
    for (int i = 0; i < 2 * cap; ++i) {
        const hipError_t e = hipEventCreate(&c->slab_ev[i]);
        if (e != hipSuccess) {
            c->slab_ev_cap = i / 2;
            if (i % 2) (void)hipEventDestroy(c->slab_ev[i - 1]);
            drop_slab_events(c);
            set_error("event creation failed: %s", hipGetErrorString(e));
            return VEST_EDEVICE;
        }
    }
    c->slab_ev_cap = cap;
    c->slab_ev_n = 0;
    return VEST_OK;
}

int vest_slab_time(vest_ctx *c, double *ms, int64_t *launches)
{
    int rc = live(c);
    if (rc) return rc;
    if (!ms || !launches) { set_error("null output"); return VEST_EINVAL; }
    double total = 0.0;
    for (int i = 0; i < c->slab_ev_n; ++i) {
        CALL_HIP(c, hipEventSynchronize(c->slab_ev[2 * i + 1]), "timing sync");
        float t = 0.0f;
        CALL_HIP(c, hipEventElapsedTime(&t, c->slab_ev[2 * i], c->slab_ev[2 * i + 1]), "elapsed time");
        total += t;
    }
    *ms = total;
    *launches = c->slab_ev_n;
    c->slab_ev_n = 0;
    return VEST_OK;
}

int vest_destroy(vest_ctx *c)
{
    if (!c) return VEST_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (c->side) {
        const hipError_t e2 = hipStreamSynchronize(c->side);
        if (e == hipSuccess) e = e2;
        (void)hipStreamDestroy(c->side);
        (void)hipEventDestroy(c->fork);
        (void)hipEventDestroy(c->join);
    }
    if (c->slab_ev) drop_slab_events(c);
    if (c->host_red && c->host_red_owned) (void)hipHostFree(c->host_red);
    delete c;
    if (e != hipSuccess) return device_error(nullptr, e, "destroy");
    return VEST_OK;
}

}  // extern "C"
