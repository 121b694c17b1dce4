// Internal declarations of libvest (not part of the C ABI).
//
// Data layout in HBM (per context, all inside the caller's workspace):
//
//  * Per mode n, a "row-group" layout of Omega grouped by the mode-n index
//    (Omega^{(n)}_{i_n}, Table 1).  Rows are grouped into classes by length:
//    a row of L entries gets g = 2^c lanes of one 64-lane wavefront, the
//    smallest power of two with ceil(L / g) <= LT (the layout's lane target,
//    lane_target_for); 64/g rows share a wave.  Inside a class rows are
//    ordered by decreasing length, so the lanes of a wave carry nearly equal
//    work.  Rows longer than 64 LT are cut into chunks of 64 LT entries, one
//    wave each, whose partial sums are combined in a fixed order by a
//    finishing kernel.
//    Entry (k, lane) of wave w lives in slot waves[w].base + 64 k + lane, so
//    the k-th entries of the 64 lanes are contiguous: every index / value load
//    of a wave is one coalesced 256-byte (or 512-byte) transaction.  Lane l of
//    a row group takes the row's entries l, l + g, l + 2g, ...  Padding slots
//    carry -1 in the first index array.
//  * Per slot: the N-1 other-mode indices (int32, one array per mode, modes
//    ascending), the value X_alpha (double or float), the canonical entry id.
//  * The residual e = X - B lives in the slot order of mode N-1 (the "core
//    layout").
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>
#include <type_traits>
#include <vector>

#include "vest.h"

// (order, uniform rank) pairs with compiled kernel instances.  A context with
// unequal per-mode ranks runs the instance of its largest rank (pad.hip).
#define VEST_SHAPES(X) X(2, 2) X(2, 3) X(3, 2) X(3, 3) X(3, 4) X(3, 5) X(3, 6) X(3, 7) X(3, 8) X(3, 9) \
    X(3, 10) X(4, 2) X(4, 3) X(4, 4) X(4, 5) X(4, 6) X(4, 7) X(4, 8) X(4, 9) X(4, 10) X(5, 3) X(6, 3) X(7, 3)   \
    X(8, 3) X(9, 3) X(10, 3)

// The dense contraction of Eq. 11 is unrolled per (N, J) up to 4096 core
// elements (order 4 at rank 8, order 7 at rank 3); beyond, every factor pass
// runs the looped gather form.
__host__ __device__ constexpr int dense_pow(int b, int e) { return e == 0 ? 1 : b * dense_pow(b, e - 1); }
__host__ __device__ constexpr bool dense_form(int N, int J) { return J > 0 && dense_pow(J, N) <= 4096; }

namespace vest {

constexpr int kWave = 64;
// Entries per lane of a row group (the layout's lane target LT): 16 from 2^22
// entries, 8 below, where the shorter per-wave loops and the extra waves pay
// (measured: 16 best at 10^7 entries, 8 up to 30 % faster on 10^6-entry and
// compacted sets).  Rows longer than 64 LT entries are cut into chunks of
// 64 LT.  Workspace bounds hold for both targets.
constexpr int kLaneTargetSmall = 8, kLaneTargetLarge = 16;
constexpr int64_t kLaneTargetLargeFrom = int64_t(1) << 22;
inline int lane_target_for(int64_t nnz) { return nnz >= kLaneTargetLargeFrom ? kLaneTargetLarge : kLaneTargetSmall; }
constexpr int kGramRows = 128;                    // rows per gram partial
constexpr int kGatherGrid = 1024;                 // blocks of a gather-form pass (core staged once per block)
constexpr int kLossBlocks = 1024;                 // fixed grid of the loss reductions
constexpr int64_t kSideStreamMinNnz = 1 << 20;    // entries from which the key passes overlap

struct WaveInfo {
    int64_t base;   // slot of (k = 0, lane 0)
    int32_t K;      // entries per lane (trip count)
    int32_t glog;   // log2(lanes per row), 0..6
    int32_t first;  // position in row_order of the wave's first row
    int32_t nrows;  // rows in this wave
    int32_t chunk;  // long-row chunk id (partial slot) or -1
    int32_t klive;  // steps that hold live entries (<= K; see launch_live_partition)
};
static_assert(sizeof(WaveInfo) == 32, "WaveInfo layout");

struct LongRow {
    int32_t row;
    int32_t first_chunk;
    int32_t nchunks;
    int32_t pad_;
};

struct ModeLayout {
    // capacities of the workspace regions (fixed at carve time)
    int64_t cap_slots = 0;
    int32_t cap_waves = 0, cap_long = 0, cap_chunks = 0;
    // current layout
    int64_t nslots = 0;
    int64_t npad = 0;
    int32_t nwaves = 0;
    int32_t nlong = 0;
    int32_t nchunks = 0;
    int64_t maxlen = 0;
    int32_t lane_target = kLaneTargetLarge;   // LT of the current layout
    WaveInfo *waves = nullptr;
    int32_t *row_order = nullptr;
    int32_t *oidx[VEST_MAX_ORDER] = {};
    void *xval = nullptr;
    int32_t *perm = nullptr;
    LongRow *longrows = nullptr;
};

// Operations of the row-group kernel.
// OP_RESID_S0: the residual pass of the core layout that also accumulates the
// first slab's statistics (the first slab pass of the core sweep, fused)
enum RowOp { OP_SWEEP = 0, OP_KEYS = 1, OP_RESID = 2, OP_RESID_S0 = 3 };

// Number of per-row accumulators of an operation.
__host__ __device__ constexpr int nacc_vc(int J) { return J * (J + 1) / 2 + J; }
__host__ __device__ constexpr int round8(int x) { return (x + 7) / 8 * 8; }
__host__ __device__ constexpr int gram_width(int J) { return round8(nacc_vc(J)); }
// The core sweep's Gram product keeps two blocks of rb^T kp: the slab's
// Gram matrix in symmetric-pair form (gram_nm x gram_nm, in 16 x 16 tiles,
// gram_tm per side) and its right-hand side (one 16 x 16 tile); its partials
// hold gram_core_cells values.
__host__ __device__ constexpr int gram_nm(int J) { return J * (J + 1) / 2; }
__host__ __device__ constexpr int gram_tm(int J) { return (gram_nm(J) + 15) / 16; }
__host__ __device__ constexpr int gram_core_cells(int J) { return 256 * gram_tm(J) * gram_tm(J) + 256; }

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// The gather form stages the core with the mode-n index innermost plus one bit
// per core column.  Up to 64 KB it is staged in each workgroup's LDS; larger
// stagings (orders 9 and 10 at rank 3: 157 KB and 472 KB in FP64) are written
// once per pass into the workspace and read through the cache.
__host__ __device__ constexpr size_t gather_stage_bytes(int N, int J, int tsize)
{
    return (size_t)ipow(J, N) * tsize + ((size_t)ipow(J, N - 1) + 31) / 32 * 4;
}
__host__ __device__ constexpr bool gather_in_lds(int N, int J, int tsize)
{
    return gather_stage_bytes(N, J, tsize) <= 65536;
}

// Core-key passes handle key_slabs(N, J, d, tsize) slabs at once (J or 2 J
// accumulators each, at most key_acc(tsize) per lane so that nothing spills,
// never more than the J^(N-2) slabs there are): 64 FP64 or 128 FP32 values.
constexpr int kKeyAccMax = 128;
__host__ __device__ constexpr int key_acc(int tsize) { return tsize == 4 ? 128 : 64; }
__host__ __device__ constexpr int key_slabs(int N, int J, bool with_d, int tsize)
{
    return key_acc(tsize) / ((with_d ? 2 : 1) * J) < 1 ? 1
           : (key_acc(tsize) / ((with_d ? 2 : 1) * J) > ipow(J, N - 2) ? ipow(J, N - 2)
                                                                       : key_acc(tsize) / ((with_d ? 2 : 1) * J));
}
__host__ __device__ constexpr int keys_width(int N, int J, int tsize)
{
    return round8(2 * J * key_slabs(N, J, true, tsize)) > round8(J * key_slabs(N, J, false, tsize))
               ? round8(2 * J * key_slabs(N, J, true, tsize))
               : round8(J * key_slabs(N, J, false, tsize));
}
__host__ __device__ constexpr int keys_nacc(int N, int J, int tsize)
{
    return 2 * J * key_slabs(N, J, true, tsize) > J * key_slabs(N, J, false, tsize)
               ? 2 * J * key_slabs(N, J, true, tsize)
               : J * key_slabs(N, J, false, tsize);
}
// Row stride (elements) of the gather copies of the factors: the row's bytes
// rounded up to a power of two (at least 16), so that with a 256-byte aligned
// base no row straddles a 128-byte cache line and a random row costs one line.
__host__ __device__ constexpr int gather_ld(int J, int tsize)
{
    int b = 16;
    while (b < J * tsize) b *= 2;
    return b / tsize;
}
__host__ __device__ constexpr int rowbuf_width(int N, int J, int tsize)
{
    return gram_width(J) > keys_width(N, J, tsize) ? gram_width(J) : keys_width(N, J, tsize);
}

}  // namespace vest

// The context (opaque in the C ABI).
struct vest_ctx {
    vest_desc d{};
    hipStream_t stream = nullptr;
    int device = 0;
    int N = 0, J = 0;                 // uniform rank of the kernel instance
    int64_t G = 0;                    // |G|
    int tsize = 8;                    // bytes of the compute type
    bool f32 = false;                 // compute type is float (FP32 and BF16 forms)
    int kernel_policy = 0;            // VEST_KERNEL_AUTO / _DENSE / _GATHER

    // model state the kernels work on: the caller's arrays, or, when the
    // per-mode ranks differ, padded copies in the workspace (see `padded`)
    double *A[VEST_MAX_ORDER] = {};
    double *core = nullptr;
    uint32_t *fmask[VEST_MAX_ORDER] = {};
    uint8_t *cmask = nullptr;

    // Unequal per-mode ranks J_n: the kernels run on the uniform rank
    // J = max J_n with every element outside the caller's J_1 x .. x J_N
    // model marked (pruned, value 0) in workspace copies of the factors,
    // core and marking tables.  Marked elements are zero and never updated,
    // so the padded model is the caller's model exactly; every call that
    // changes the state copies the caller's part back (pad.hip).
    bool padded = false;
    int32_t uranks[VEST_MAX_ORDER] = {};
    int64_t uG = 0;                   // prod J_n of the caller's core
    double *uA[VEST_MAX_ORDER] = {};
    double *ucore = nullptr;
    uint32_t *ufmask[VEST_MAX_ORDER] = {};
    uint8_t *ucmask = nullptr;
    double *pkey_core = nullptr;      // padded keys (the ones vest_prune reads)
    double *pkey_fac[VEST_MAX_ORDER] = {};

    // workspace-resident derived state
    vest::ModeLayout lay[VEST_MAX_ORDER];
    void *e = nullptr;                // residual, core-layout slot order (T)
    void *ms = nullptr;               // mode N-2 factor row of every core-layout slot (T)
    double *hdiag = nullptr;          // diagonal of every slab's Gram matrix [|G|]
    void *Gp[VEST_MAX_ORDER] = {};    // core permuted for each mode (T)
    void *Ag[VEST_MAX_ORDER] = {};    // gather copies of the factors (T, row stride gather_ld)
    void *colA[VEST_MAX_ORDER] = {};  // column-major factor copies, modes < N-2 (T; order 3: column pairs)
    double *rowbuf = nullptr;         // [I_{N-1}][ldrb]
    int ldrb = 0;
    double *kp = nullptr;             // [I_{N-1}][gram_width]
    double *gram_part = nullptr;      // [nchunks][gw*gw]
    double *gram = nullptr;           // [gw*gw]
    double *dprev = nullptr;          // [J*J] last slab's core change
    double *wsum = nullptr;           // [waves of the last mode] sum of e^2 per wave of the last slab pass
    double *sse_lag = nullptr;        // SSE after the core sweep while e lags its last slab (device)
    double *partials = nullptr;       // long-row chunk partials
    double *partials_side = nullptr;  // ... of the core keys while they run on `side`
    void *gt = nullptr;               // gather-form core staging when it exceeds LDS (T, [o][j])
    uint32_t *gnz = nullptr;          // ... and its nonzero-column bits
    double *red = nullptr;            // reduction scratch [4 * kLossBlocks + 16]
    int32_t *flags = nullptr;         // device error flags [16]
    uint32_t *pv_in = nullptr, *pv_out = nullptr;  // nonzero flags / positions (export)
    uint32_t *sel_hist = nullptr;     // prune selection: [N + 1][4096] digit counts
    char *sel_state = nullptr;        // prune selection: chosen digits and counts per tensor
    void *sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    double *host_red = nullptr;       // pinned host mirror of small results
    bool host_red_owned = true;       // allocated by the context (else lent by a server)

    // bookkeeping
    double xnorm2 = 0.0;
    double sse_dead = 0.0;            // sum X^2 of the entries dropped by vest_compact
    void *stage = nullptr;            // compaction staging (spans the e and ms regions)
    size_t stage_bytes = 0;
    char *scratch = nullptr;          // layout-build scratch
    size_t scratch_bytes = 0;
    int64_t marked_core = 0;
    int64_t marked_fac[VEST_MAX_ORDER] = {};
    uint64_t core_version = 1;
    uint64_t gp_version[VEST_MAX_ORDER] = {};
    bool ag_valid[VEST_MAX_ORDER] = {};
    bool e_valid = false;
    bool live_stale = false;          // marks changed since the layouts' live partition
    double live_dead_est = 0.0;       // dead-entry estimate at that partition (ensure_live)
    // e lacks the change of the core sweep's last slab (held in dprev); the
    // SSE it would have is in sse_lag, and the change is applied to e only
    // when something reads e
    bool e_lag = false;
    bool ms_valid = false;            // ms matches the current factors
    bool hdiag_valid = false;         // hdiag matches the current factors
    bool keys_pending = false;
    double *key_core = nullptr;
    double *key_fac[VEST_MAX_ORDER] = {};
    bool dead = false;
    hipEvent_t *slab_ev = nullptr;    // vest_slab_timing: start / end event pairs
    int slab_ev_cap = 0, slab_ev_n = 0;
    // vest_responsibility runs the core keys (HBM-bound) on a second stream
    // beside the factor keys (ALU-bound); created on first use for large
    // contexts only
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

namespace vest {

// ---------------------------------------------------------------- launchers
// (defined in the .hip files; return hipSuccess or the first HIP error)
bool shape_supported(int N, int J);

hipError_t launch_rowgroup(vest_ctx *c, int mode, int op);       // OP_SWEEP / OP_KEYS / OP_RESID / OP_RESID_S0
bool resid_fuses_slab0(const vest_ctx *c);                       // OP_RESID_S0 applies (dense form)
hipError_t launch_core_sweep(vest_ctx *c, bool slab0_done);
hipError_t launch_normalize(vest_ctx *c);
hipError_t launch_count_nonzeros(vest_ctx *c, int64_t *counts);  // synchronises
hipError_t launch_export(vest_ctx *c, int64_t *const *fi, double *const *fv, int64_t *ci, double *cv);
hipError_t launch_heldout(vest_ctx *c, const int32_t *idx, const double *val, int64_t n, double *dout);
hipError_t launch_value_keys(vest_ctx *c, double *core_key, double *const *fkey);
// Live entries of the mode-0 layout re-assembled into (idx, val) in `stage`;
// *live and *dead_sq (sum X^2 of the dropped ones) on return (synchronises).
hipError_t launch_compact(vest_ctx *c, int32_t **idx, double **val, int64_t *live, double *dead_sq);
hipError_t launch_core_keys(vest_ctx *c, double *core_key, hipStream_t st, double *partials);
hipError_t launch_permute_core(vest_ctx *c, int mode);
hipError_t launch_gather_copy(vest_ctx *c, int mode);
hipError_t launch_loss(vest_ctx *c, double *dev_out3, const double *sse);   // sse, reg (device); sse given or summed over e
hipError_t launch_lag_apply(vest_ctx *c);   // apply the core sweep's last slab change to e
// Live partition of every mode's layout after marks changed: each lane's
// entries with no fully marked other-mode row (those whose delta can be
// nonzero) move ahead of the others, in order, and every wave records in
// klive the steps that hold them; factor sweeps and factor keys stop there.
hipError_t launch_live_partition(vest_ctx *c, hipStream_t st);
hipError_t launch_prune(vest_ctx *c, int64_t core_k, const int64_t *factor_k);  // all tensors at once
hipError_t launch_sumsq(hipStream_t s, const double *v, int64_t n, double *partial, double *out);
hipError_t launch_mask_init(vest_ctx *c, int64_t *counts_dev);
hipError_t build_layouts(vest_ctx *c, const int32_t *idx, const double *val, char *scratch,
                         size_t scratch_bytes, int *bad);
// padded contexts (pad.hip): caller arrays -> workspace copies, and back
hipError_t launch_pad_in(vest_ctx *c);
hipError_t launch_pad_out_factor(vest_ctx *c, int mode);
hipError_t launch_pad_out_core(vest_ctx *c);
hipError_t launch_pad_out_masks(vest_ctx *c);
hipError_t launch_pad_out_keys(vest_ctx *c, double *core_key, double *const *factor_key);

// ------------------------------------------------------- batched contexts
// One Alg. 2 iteration of several contexts of one shape (serving): every
// kernel of the iteration runs once for all of them, its launch carrying a
// table of per-context tasks (virtual blocks b - off[t] of task t).  The
// tables are written to a host staging area, uploaded once, then the recorded
// launches are issued.
struct BatchArena {
    char *host = nullptr;   // staging (pinned)
    char *dev = nullptr;    // device mirror
    size_t cap = 0, used = 0;
    bool overflow = false;
    size_t add(const void *p, size_t n)
    {
        const size_t o = (used + 255) & ~size_t(255);
        if (o + n > cap) {
            overflow = true;
            return 0;
        }
        std::memcpy(host + o, p, n);
        used = o + n;
        return o;
    }
    template <class X>
    X *dptr(size_t off) const { return reinterpret_cast<X *>(dev + off); }
};
using LaunchList = std::vector<std::function<void()>>;
constexpr int kBatchGrid = 2048;      // blocks of a multi-context launch (grid-stride over tasks)

// Factor pass (OP_SWEEP with its long-row finish, or OP_RESID_S0) of mode
// `mode` for every context; core sweep with the first slab's sums taken from
// OP_RESID_S0 when `fused`; permuted cores of every mode.  false if a context
// does not fit the batched (dense-contraction) path.
bool plan_factor_batch(vest_ctx *const *cs, int n, int mode, int op, hipStream_t st, BatchArena &ba, LaunchList &L);
bool plan_core_batch(vest_ctx *const *cs, int n, bool fused, hipStream_t st, BatchArena &ba, LaunchList &L);
bool plan_permute_batch(vest_ctx *const *cs, int n, hipStream_t st, BatchArena &ba, LaunchList &L);
bool batch_dense_ok(const vest_ctx *c);   // every factor pass of c would run the dense contraction

// ---------------------------------------------------------------- workspace
struct Plan {
    size_t total = 0;
    size_t scratch_bytes = 0;     // init-time scratch
    size_t sort_tmp = 0;          // radix-sort scratch
    int64_t slot_bound[VEST_MAX_ORDER] = {};
    int64_t wave_bound[VEST_MAX_ORDER] = {};
    int64_t long_bound[VEST_MAX_ORDER] = {};
    int64_t chunk_bound = 0;
    int64_t gram_chunks = 0;
    int64_t max_tensor = 0;
};
int plan_workspace(const vest_desc *d, Plan *p);

// Bump allocator over the workspace.
struct Bump {
    char *base;
    size_t off, cap;
    void *take(size_t bytes) {
        size_t o = (off + 255) & ~size_t(255);
        if (o + bytes > cap) return nullptr;
        off = o + bytes;
        return base + o;
    }
};

void set_error(const char *fmt, ...);
int check_desc(const vest_desc *d);   // VEST_OK or the code vest_init would return for the descriptor
int max_rank(const vest_desc *d);     // the uniform rank the kernels of a context run at

}  // namespace vest
