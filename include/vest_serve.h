/*
 * vest_serve.h -- request loop of libvest: many VeST factorization jobs of
 * uneven order, size and rank share one GPU.
 *
 * A server owns one device arena of a fixed size and a fixed number of job
 * slots (one HIP stream each).  Jobs are queued on submission and admitted
 * in arrival order, later jobs filling in when the head of the queue does not
 * fit, as soon as a slot is free and the job's device footprint (observed
 * tensor, model state, marking tables, the vest_init workspace and, for a
 * pruning job, its keys) fits in the free part of the arena.  An admitted job keeps its state resident.
 * Admitted jobs of one class -- same order, rank and precision, entry counts
 * within a factor of 4 -- advance together:
 * the loop enqueues one batched iteration of Alg. 2 (every factor sweep,
 * Alg. 4, then the core sweep, Eq. 12 / Eq. 14; vest_iterate_many) for all
 * idle jobs of the class on the class's stream, every kernel of it launched
 * once for the whole class; classes run on separate streams, so the work of
 * all admitted jobs overlaps on the device.  A job the batched path does not
 * take (unequal ranks) runs its iterations alone on its slot's stream.  A finished job's factors, core
 * and loss (Eq. 1 / Eq. 2, Eq. 4) are copied to host memory owned by the
 * server and its device memory returns to the arena.  Every kernel of the
 * library sums in a fixed order, so a job's result does not depend on what
 * else runs beside it.
 *
 * Threading: a server is driven by one host thread (vest_server_progress is
 * not re-entrant).  The server runs two helper threads of its own that upload
 * admitted jobs and build their layouts (vest_init, which waits for the job's
 * stream), so the driving thread keeps enqueueing the other jobs' iterations
 * meanwhile; a job stays QUEUED until that has finished.  All host
 * pointers of a job must stay valid until the job has left the QUEUED state.
 */
#ifndef VEST_SERVE_H
#define VEST_SERVE_H

#include "vest.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vest_server vest_server;   /* opaque, library-owned host object */

enum { VEST_JOB_QUEUED = 0, VEST_JOB_ACTIVE = 1, VEST_JOB_DONE = 2, VEST_JOB_FAILED = 3 };

typedef struct {
    vest_desc desc;                 /* problem, as for vest_init                  */
    const int32_t *idx;             /* host, nnz*N int32, entry-major             */
    const double *val;              /* host, nnz FP64                             */
    const double *const *factors;   /* host array of N host arrays, I_n*J_n FP64,
                                       initial factors                            */
    const double *core;             /* host, prod(J_n) FP64, initial core         */
    int32_t iterations;             /* iterations of Alg. 2 (>= 1)                */
    int32_t reserved;               /* must be 0                                  */
    double prune_target;            /* 0: no pruning.  In (0, 1): VeST^man toward
                                       this sparsity (Sec. 3.3): after each
                                       iteration t but the last, while the marked
                                       fraction of all elements is below it,
                                       responsibility keys and one prune step of
                                       ceil(pr_t |T|) new marks per tensor,
                                       pr_t = min(0.01 t, 0.1), each tensor capped
                                       at ceil(target |T|) marks.  Equal ranks
                                       only; such a job iterates alone on its
                                       slot's stream and reserves its keys
                                       (prod J_n + sum I_n J_n doubles) in the
                                       arena.                                      */
} vest_job;

/* One iteration of Alg. 2 (the factor sweep of every mode, Alg. 4, then the
 * core sweep, Eq. 12 / Eq. 14) for n contexts of one shape -- same order,
 * rank and precision -- in one sequence of launches: every kernel of the
 * iteration runs once for all the contexts, its launch carrying a table of
 * per-context tasks that a grid-stride loop walks (virtual block b of the
 * launch is a block of one context's work).  Each context's arithmetic is the
 * same as vest_sweep_factor / vest_sweep_core run on it alone, so its results
 * do not depend on the batch it runs in.
 *   ctxs         host array of n distinct contexts
 *   stream       hipStream_t all launches go to; the caller orders the
 *                contexts' own earlier work before it
 *   dev_table    device buffer of table_bytes for the task tables
 *   host_table   host staging of table_bytes (pinned memory recommended);
 *                it is copied to dev_table on `stream` and must not be
 *                modified until that copy has completed
 * VEST_EUNSUPPORTED, with nothing enqueued, when a context does not fit the
 * batched path (unequal ranks, marks that make a factor pass take the gather
 * contraction, instrumentation on, a different shape) or the tables exceed
 * table_bytes; the caller then runs the contexts one by one. */
int vest_iterate_many(vest_ctx *const *ctxs, int32_t n, void *stream, void *dev_table, void *host_table,
                      size_t table_bytes);

/* Create a server with an arena of device_bytes (allocated once, on the
 * current device) and `slots` concurrent jobs (1..256). */
int vest_server_create(size_t device_bytes, int32_t slots, vest_server **out /* host out */);

/* Queue a job; its arrival time is the time of this call.  VEST_ENOSPC if its
 * footprint exceeds the whole arena, VEST_EINVAL for a bad descriptor,
 * iteration count or prune target (checked as vest_init does, without
 * touching the data). */
int vest_server_submit(vest_server *s, const vest_job *job, int64_t *id /* host out */);

/* One scheduling pass: retire jobs whose last iteration has completed, make
 * active the jobs whose upload and vest_init a helper thread has finished,
 * hand queued jobs that fit (arena blocks and a slot assigned here) to the
 * helper threads, enqueue the next iteration of every active job whose
 * previous one has completed.  Waits for the GPU only inside the retirement
 * (loss and result copies) of a job.
 * *completed (may be NULL) receives the number of jobs retired by this pass. */
int vest_server_progress(vest_server *s, int32_t *completed);

/* State of a job and its times in seconds since the server was created:
 * times[0] arrival, times[1] admission (arena blocks and slot assigned),
 * times[2] completion (-1 if not yet).
 * For a failed job *state is VEST_JOB_FAILED and *error the VEST_E* code. */
int vest_server_status(vest_server *s, int64_t id, int32_t *state, int32_t *error, double times[3]);

/* Copy a finished job's results to caller memory (any of the pointers may be
 * NULL) and release them:  factors = host array of N host arrays,
 * core = prod(J_n) doubles, loss = 5 doubles as vest_loss.  VEST_ESTATE if
 * the job has not finished (or was fetched already). */
int vest_server_fetch(vest_server *s, int64_t id, double *const *factors, double *core, double *loss);

/* out[0] queued (with those being uploaded and initialised), out[1] active,
 * out[2] finished (not fetched), out[3] arena
 * bytes in use, out[4] arena size, out[5] largest free block, out[6] batched
 * iterations issued, out[7] job-iterations they carried. */
int vest_server_stats(vest_server *s, int64_t *out /* 8 values */);

/* Wait for all enqueued work and release everything (unfetched results too). */
int vest_server_destroy(vest_server *s);

#ifdef __cplusplus
}
#endif

#endif /* VEST_SERVE_H */
