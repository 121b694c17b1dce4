/*
 * vest.h -- C ABI of the MI355X (gfx950) VeST hot-path library, libvest.so.
 *
 * VeST (M. Park, J.-G. Jang, L. Sael, "VeST: Very Sparse Tucker Factorization
 * of Large-Scale Tensors", arXiv:1904.02603) fits a partially observed N-order
 * tensor X (observed entries Omega) with a Tucker model: core G (J_1 x .. x
 * J_N) and factor matrices A^(n) (I_n x J_n), minimising Eq. 1 (L_F) or Eq. 2
 * (L_1) by element-wise coordinate descent (Sec. 3.4), and prunes elements of
 * low responsibility (Sec. 3.2-3.3).  This library runs the per-iteration
 * steps of Alg. 2 on the GPU; the host decides the schedule.
 *
 * Conventions shared by every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller, except where
 *     a comment says "host".  The library never frees caller memory.
 *   - Indices are 0-based.  idx is entry-major: idx[e*N + n] is the mode-n
 *     index of observed entry e; entry e is "canonical entry id" e.
 *   - Factor matrices are row-major FP64: A_n[i*J_n + j] = a^(n)_{i j}.
 *   - The core is row-major FP64 with the last mode fastest: the flat index of
 *     (j_1..j_N) is ((j_1*J_2 + j_2)*J_3 + j_3)... ("flat order").
 *   - Marking table (Sec. 3.3): factor_mask[n][i] bit j set = a^(n)_{ij}
 *     pruned; core_mask[flat] != 0 = core element pruned.  Pruned elements are
 *     zero and are never updated again.
 *   - Every call enqueues on the stream given to vest_init and returns without
 *     waiting, except vest_init and vest_loss, which synchronise that stream.
 *   - Return value: VEST_OK (0) or a negative VEST_E* code; vest_last_error()
 *     gives a message for the last failing call on the calling thread.
 *   - A context is not thread-safe.  Distinct contexts on distinct streams are
 *     independent.
 */
#ifndef VEST_H
#define VEST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VEST_MAX_ORDER 10
#define VEST_MAX_RANK 32

enum {
    VEST_OK = 0,
    VEST_EINVAL = -1,   /* bad argument or input data (nothing of the caller's was modified) */
    VEST_ENOSPC = -2,   /* workspace too small                                         */
    VEST_EDEVICE = -3,  /* HIP runtime error; the context must be destroyed             */
    VEST_ESTATE = -4,   /* call out of order (e.g. vest_prune before vest_responsibility) */
    VEST_EUNSUPPORTED = -5 /* valid problem, but no kernel instance for (order, max rank): ranks 2..10
                              at orders 3 and 4, 2..3 at order 2, 3 at orders 5..10 */
};

enum { VEST_REG_LF = 0, VEST_REG_L1 = 1 };   /* Eq. 1 / Eq. 2 */

/* Arithmetic of the delta contraction and of the row / residual sums.  The
 * per-coordinate division, the soft threshold and the responsibility keys
 * are FP64 in every form; factors and core stay FP64.
 *   VEST_FP64  FP64 throughout
 *   VEST_FP32  FP32 contraction and sums (order-3 factor sweeps run the first
 *              contraction stage on FP32 matrix cores)
 *   VEST_BF16  as VEST_FP32, except that in the order-3 factor sweep the
 *              first contraction stage runs on BF16 matrix cores with FP32
 *              accumulation: core and last other-mode factor row are each
 *              split into two BF16 parts (hi + lo) and three products are
 *              summed, about 16 significant operand bits */
enum { VEST_FP64 = 0, VEST_FP32 = 1, VEST_BF16 = 2 };

typedef struct {
    int32_t order;                     /* N, 2..VEST_MAX_ORDER                         */
    int32_t reg;                       /* VEST_REG_LF or VEST_REG_L1                   */
    int32_t precision;                 /* VEST_FP64, VEST_FP32 or VEST_BF16            */
    int32_t reserved;                  /* must be 0                                    */
    double lambda;                     /* lambda > 0, one value for core and factors
                                          (Eq. 1 / Eq. 2, Table 1)                     */
    int64_t nnz;                       /* |Omega| >= 1                                 */
    int64_t dims[VEST_MAX_ORDER];      /* I_n >= 1, I_n < 2^31                         */
    int32_t ranks[VEST_MAX_ORDER];     /* J_n, 1..VEST_MAX_RANK; may differ per mode
                                          (Table 1): the context then runs the kernels
                                          of J = max J_n on a padded copy of the model
                                          in its workspace, every element outside the
                                          caller's J_1 x .. x J_N model marked, and
                                          copies the caller's part back after every
                                          call that changes it                           */
} vest_desc;

typedef struct vest_ctx vest_ctx;      /* opaque, library-owned host object */

/* Upper bound of the device workspace vest_init needs for this problem
 * (indices re-laid out per mode, residuals, reduction scratch, sort scratch).
 * Depends only on the descriptor, so a scheduler can admit jobs by footprint.
 * Needs a HIP device (the sort scratch size is queried from the runtime). */
int vest_workspace_bytes(const vest_desc *desc, size_t *bytes /* host out */);

/* Validate the observed tensor and build the per-mode layouts of Omega
 * (Omega^{(n)}_{i_n} of Table 1: entries grouped by their mode-n index, ties
 * in canonical id order) inside the workspace.
 *   idx          nnz*N int32, entry-major (read during the call only)
 *   val          nnz FP64 observed values X_alpha (read during the call only)
 *   factors      host array of N device pointers, A_n with I_n*J_n FP64;
 *                in: initial values (initialisation of Alg. 2), out: the model state
 *   core         prod(J_n) FP64, in/out
 *   factor_mask  host array of N device pointers, I_n uint32 words each
 *                (requires J_n <= 32); may hold earlier marks (resume)
 *   core_mask    prod(J_n) bytes
 *   workspace    >= vest_workspace_bytes(desc) bytes, 256-byte aligned,
 *                owned by the caller, used exclusively by this context
 * Fails with VEST_EINVAL (index out of range, duplicate index tuple -- Omega is
 * a set --, non-finite value, lambda <= 0, bad order/rank) before writing any
 * caller buffer other than the workspace.  On success, marked elements of the
 * factors and core are set to zero.  Synchronises the stream.
 * stream is a hipStream_t (NULL = the default stream). */
int vest_init(const vest_desc *desc, void *stream,
              const int32_t *idx, const double *val,
              double *const *factors, double *core,
              uint32_t *const *factor_mask, uint8_t *core_mask,
              void *workspace, size_t ws_bytes, vest_ctx **out /* host out */);

/* One pass of Alg. 4 for mode n: every row i of A^(n) is updated element by
 * element, j ascending, Gauss-Seidel in place, skipping marked elements, with
 * Eq. 9 (L_F) or Eq. 13 (L_1, soft threshold).  Rows are independent, so the
 * result equals the sequential sweep. */
int vest_sweep_factor(vest_ctx *ctx, int32_t mode);

/* One pass of the core update: every unmarked core element in flat order,
 * sequentially (Sec. 3.5), with Eq. 12 (L_F) or Eq. 14 (L_1).  Executed as an
 * exact block Gauss-Seidel (same sequence of one-dimensional minimisations,
 * different rounding). */
int vest_sweep_core(vest_ctx *ctx);

/* Responsibility keys of every element from one snapshot of the state
 * (Sec. 3.2, Eq. 5 and Eq. 6), as Delta(e) = SSE(with e set to 0) - SSE =
 * ||X||^2 (RE(e)^2 - RE^2), which orders elements exactly as Resp(e) of
 * Eq. 3 does when RE > 0.  Marked elements get +infinity.
 *   core_key     prod(J_n) FP64 out
 *   factor_key   host array of N device pointers, I_n*J_n FP64 out each
 * The buffers must stay valid until the next vest_prune.  From 2^20 entries
 * the core keys run on a second stream that the context creates on first use
 * (forked from and joined back into the context's stream with events, so the
 * keys are complete in the order of the context's stream, as for every call);
 * vest_destroy releases it. */
int vest_responsibility(vest_ctx *ctx, double *core_key, double *const *factor_key);

/* Prune (Sec. 3.3, Alg. 3 last step): in the core and in each factor matrix
 * independently, zero and mark the k unmarked elements with the smallest
 * (key, flat index) of the last vest_responsibility call.
 *   factor_k     host array of N counts.
 * VEST_ESTATE if no keys are pending; VEST_EINVAL if a count is negative or
 * exceeds that tensor's unmarked elements. */
int vest_prune(vest_ctx *ctx, int64_t core_k, const int64_t *factor_k);

/* Loss and normalised reconstruction error of the current state (Eq. 1 /
 * Eq. 2, Eq. 4; ||X|| over Omega):
 *   out[0] SSE = sum_Omega (X - B)^2    out[1] ||X||^2 over Omega
 *   out[2] regulariser term             out[3] loss = out[0] + out[2]
 *   out[4] RE = sqrt(out[0] / out[1])
 * Right after vest_sweep_core, out[0] is formed from the last core slab's
 * statistics (sum e^2 - 2 D.rr + D^T H D with D that slab's change; equal to
 * the direct sum up to rounding order) instead of a pass over the residual.
 * out is a host array of 5 doubles.  Synchronises the stream. */
int vest_loss(vest_ctx *ctx, double *out);

/* Final step of Alg. 2: every factor matrix gets unit-length columns,
 * A^(n) <- A^(n) diag(1 / ||a^(n)_{:t}||), and the core absorbs the norms,
 * G <- G x_n diag(||a^(n)_{:t}||), modes in order; a zero column stays zero
 * (its core slice is scaled by 0).  The reconstruction is unchanged. */
int vest_normalize(vest_ctx *ctx);

/* Number of nonzero values of each factor matrix and of the core (host out,
 * N + 1 values, modes in order then the core).  Synchronises the stream. */
int vest_count_nonzeros(vest_ctx *ctx, int64_t *counts);

/* Sparse export of the model (the output of Alg. 2): for each factor matrix
 * the flat indices i*J_n + j and the values of its nonzero elements in
 * ascending flat order, and the same for the core (flat order of vest.h).
 * Device outputs, sized by vest_count_nonzeros; fac_idx / fac_val are host
 * arrays of N device pointers. */
int vest_export(vest_ctx *ctx, int64_t *const *fac_idx, double *const *fac_val, int64_t *core_idx,
                double *core_val);

/* Loss terms of the current model on another set of entries (a held-out
 * test set; Eq. 4 over that set): idx n*N int32 entry-major, val n FP64,
 * device arrays.  out (host, 3 doubles): sum (X - B)^2, sum X^2, RE.
 * VEST_EINVAL for an index out of range.  Synchronises the stream. */
int vest_test_error(vest_ctx *ctx, const int32_t *idx, const double *val, int64_t n, double *out);

/* Allocation-free variant of vest_test_error, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops or
 * harnesses that forbid hipMalloc): the same loss terms of a model given as
 * plain device arrays, with no context and no workspace.
 *   desc       host; order, dims and ranks are read (ranks may differ per
 *              mode); nnz, reg, lambda and precision are ignored
 *   stream     hipStream_t the kernels are enqueued on (NULL = default)
 *   factors    host array of N device pointers, A_n row-major I_n x J_n FP64
 *   core       prod(J_n) FP64, flat order
 *   idx, val   n*N int32 entry-major and n FP64, device
 *   out        DEVICE, 4 doubles: sum (X - B)^2, sum X^2, RE, and the number
 *              of entries with an index out of range (the first three are
 *              NaN when it is not 0)
 * Only enqueues (two kernels, no copy, no synchronisation, no allocation by
 * the library or the runtime).  Per-block partial sums live in a static
 * device array of the library, 3 * 8 bytes per 1024 entries, so n is limited
 * to VEST_NOALLOC_MAX_ENTRIES (VEST_EINVAL beyond, before anything is
 * enqueued).  Each GPU has one such array, kept until the process ends and
 * shared by every call on that GPU: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller.  Every
 * call writes each partial it reads, so no clearing is needed.  Returns
 * VEST_EINVAL for a bad argument and VEST_EDEVICE for a launch error. */
#define VEST_NOALLOC_MAX_ENTRIES (1 << 24)
int vest_model_error_noalloc(const vest_desc *desc, void *stream, const double *const *factors,
                             const double *core, const int32_t *idx, const double *val, int64_t n,
                             double *out);

/* Keys of the value-pruning comparator: |value| of every unmarked element,
 * +infinity for marked ones, written like vest_responsibility's keys and
 * made the pending keys of the next vest_prune (which then removes the
 * smallest-magnitude elements). */
int vest_value_keys(vest_ctx *ctx, double *core_key, double *const *factor_key);

/* Drop from the per-mode layouts the observed entries that can no longer
 * contribute: those with a fully marked factor row in some mode (Sec. 3.3;
 * marks never clear).  Their reconstruction, every delta term, core weight
 * and key contribution are zero for good, so every later call returns the
 * same results with or without them (up to rounding order); their residual
 * stays X_alpha and sum X^2 over them is kept for vest_loss.  Rebuilds the
 * layouts inside the workspace from the kept entries (no caller array is
 * needed) and synchronises the stream.  *live (may be NULL) receives the
 * number of entries kept; nothing changes when all are live or none is. */
int vest_compact(vest_ctx *ctx, int64_t *live);

/* Contraction kernel of the factor sweeps, factor keys and residual passes
 * (Eq. 11):
 *   VEST_KERNEL_AUTO    per call, from the marked fractions of the factors
 *                       (default)
 *   VEST_KERNEL_DENSE   dense factored contraction over all of G
 *   VEST_KERNEL_GATHER  pruned-phase form: only terms whose other-mode factor
 *                       values are nonzero and whose core column
 *                       G[.., j_n = any, ..] is nonzero; the core is staged in
 *                       LDS
 * Both forms compute the same sums up to rounding order.  From order 8 the
 * dense form is not compiled and every setting runs the gather form.
 * VEST_EINVAL for an unknown value. */
enum { VEST_KERNEL_AUTO = 0, VEST_KERNEL_DENSE = 1, VEST_KERNEL_GATHER = 2 };
int vest_set_kernel(vest_ctx *ctx, int32_t kernel);

/* Layout statistics of mode n (host out, 8 values): slots, padding slots,
 * waves, long rows, long-row chunks, max row length, rows, nnz. */
int vest_layout_stats(vest_ctx *ctx, int32_t mode, int64_t *out);

/* Instrumentation: kernel timing of the slab passes of the core sweep (the
 * accumulating passes of Sec. 3.5's element updates grouped by slab, J^(N-2)
 * launches per core sweep).  While enabled, each launch is bracketed by two
 * HIP events on the context's stream (up to 1024 launches are recorded);
 * vest_slab_time waits for the recorded launches, returns their summed
 * duration in milliseconds and their count (host out), and clears the record.
 * Enabling creates the events (the only allocation), disabling destroys them;
 * VEST_EDEVICE if event creation fails. */
int vest_slab_timing(vest_ctx *ctx, int32_t enable);
int vest_slab_time(vest_ctx *ctx, double *ms, int64_t *launches);

/* Release the context (not the workspace or any caller buffer).  Waits for
 * the context's queued work. */
int vest_destroy(vest_ctx *ctx);

const char *vest_strerror(int code);
const char *vest_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VEST_H */
