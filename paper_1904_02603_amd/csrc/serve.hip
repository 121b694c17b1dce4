// Request loop of libvest (include/vest_serve.h): admission by device
// footprint into one arena, one stream per job slot; a job's upload and
// vest_init (layout build, which waits for its stream) run on an admission
// worker thread while the progress thread keeps the other jobs' iterations
// flowing; admitted jobs of one
// class (order, rank, precision, entry count within a factor of 4) advance
// together, one batched
// iteration of Alg. 2 at a time (vest_iterate_many: every kernel of the
// iteration launched once for the whole class), classes on streams of their
// own; a job that does not fit the batched path runs alone on its slot's
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"
#include "vest_serve.h"

namespace {

using vest::set_error;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of adjacent free blocks.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        used_ = 0;
        size_ = size;
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = align_up(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n;
            const size_t start = it->first + n;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = align_up(n ? n : 1);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &f : free_) m = f.second > m ? f.second : m;
        return m;
    }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, size_ = 0;
};

// One device allocation of a job: offset and size inside the arena.
struct Block {
    size_t off = 0, bytes = 0;
    bool live = false;
};

struct Job {
    int64_t id = 0;
    vest_job in{};
    int N = 0;
    int64_t G = 1;
    int32_t state = VEST_JOB_QUEUED;
    int32_t error = 0;
    double t_arrive = -1, t_admit = -1, t_done = -1;
    size_t ws_bytes = 0;
    // device blocks: 0 workspace, 1 factors, 2 core, 3 factor masks, 4 core
    // mask, 5 idx, 6 val (5 and 6 only until vest_init has returned), 7 the
    // responsibility keys of a pruning job (core, then each factor matrix)
    static constexpr int kBlocks = 8;
    Block blk[kBlocks];
    vest_ctx *ctx = nullptr;
    int slot = -1;
    int klass = -1;          // shape class (batched iterations), -1 until admitted
    int32_t iters_done = 0;
    int32_t prune_steps = 0;
    // admission on the worker thread: init_rc is valid once init_done is set
    std::atomic<int> init_done{0};
    int init_rc = 0;
    bool inflight = false;   // an iteration is enqueued and not yet complete
    bool in_batch = false;   // ... as part of its class's batch (else on its slot stream)
    // results (host)
    std::vector<double> res_fac, res_core;
    double loss[5] = {0, 0, 0, 0, 0};
    bool fetched = false;

    size_t fac_elems() const
    {
        size_t s = 0;
        for (int n = 0; n < N; ++n) s += (size_t)in.desc.dims[n] * in.desc.ranks[n];
        return s;
    }
    size_t mask_words() const
    {
        size_t s = 0;
        for (int n = 0; n < N; ++n) s += (size_t)in.desc.dims[n];
        return s;
    }
    size_t block_bytes(int b) const
    {
        switch (b) {
        case 0: return ws_bytes;
        case 1: return fac_elems() * 8;
        case 2: return (size_t)G * 8;
        case 3: return mask_words() * 4;
        case 4: return (size_t)G;
        case 5: return (size_t)in.desc.nnz * N * 4;
        case 6: return (size_t)in.desc.nnz * 8;
        default: return in.prune_target > 0.0 ? ((size_t)G + fac_elems()) * 8 : 0;
        }
    }
    size_t footprint() const
    {
        size_t s = 0;
        for (int b = 0; b < kBlocks; ++b)
            if (block_bytes(b)) s += align_up(block_bytes(b));
        return s;
    }
};

}  // namespace

// Jobs of one shape advance in batched iterations on the class's stream; the
// task tables of a batch are staged in pinned host memory and mirrored in a
// device buffer (both allocated when the class first appears).
struct Klass {
    int N = 0, J = 0, precision = 0, bucket = 0;
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    char *dev = nullptr;         // device table buffer
    char *host = nullptr;        // pinned staging of the tables
    bool usable = false;         // buffers in place
    bool inflight = false;
    std::vector<int64_t> batch;  // jobs of the batch in flight
};

constexpr size_t kClassTable = 1u << 20;
constexpr int kAdmissionThreads = 2;   // concurrent uploads + layout builds

struct vest_server {
    char *base = nullptr;
    Arena arena;
    std::vector<Klass> classes;
    double *pinned_loss = nullptr;   // the host buffer vest_loss of a retiring job reads into
    int64_t batches = 0, batched_job_iters = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<int64_t> slot_job;   // job id per slot, -1 if free
    std::map<int64_t, std::unique_ptr<Job>> jobs;
    std::deque<int64_t> queue;
    std::vector<int64_t> admitting;   // upload and vest_init in progress on the worker
    std::vector<int64_t> active;
    int64_t next_id = 1;
    // admission workers: take jobs whose arena blocks and slot are assigned
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job *> todo;
    bool stop = false;
    int device = 0;
    std::chrono::steady_clock::time_point t0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    char *ptr(const Block &b) const { return base + b.off; }
};

namespace {

int hip_fail(hipError_t e, const char *where)
{
    set_error("%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
    return VEST_EDEVICE;
}

void release_blocks(vest_server *s, Job &j)
{
    for (auto &b : j.blk)
        if (b.live) {
            s->arena.release(b.off, b.bytes);
            b.live = false;
        }
}

// Pointers of a job's blocks in the form vest_init takes.
struct JobPtrs {
    double *fac[VEST_MAX_ORDER];
    uint32_t *fmask[VEST_MAX_ORDER];
    double *core;
    uint8_t *cmask;
};

JobPtrs job_ptrs(vest_server *s, Job &j)
{
    JobPtrs p{};
    double *f = (double *)s->ptr(j.blk[1]);
    uint32_t *m = (uint32_t *)s->ptr(j.blk[3]);
    for (int n = 0; n < j.N; ++n) {
        p.fac[n] = f;
        p.fmask[n] = m;
        f += (size_t)j.in.desc.dims[n] * j.in.desc.ranks[n];
        m += (size_t)j.in.desc.dims[n];
    }
    p.core = (double *)s->ptr(j.blk[2]);
    p.cmask = (uint8_t *)s->ptr(j.blk[4]);
    return p;
}

// Arena blocks of a queued job; false (nothing held) if the arena cannot
// hold it now.  Progress thread.
bool alloc_blocks(vest_server *s, Job &j)
{
    for (int b = 0; b < Job::kBlocks; ++b) {
        j.blk[b].bytes = j.block_bytes(b);
        if (!j.blk[b].bytes) continue;
        if (!s->arena.alloc(j.blk[b].bytes, &j.blk[b].off)) {
            release_blocks(s, j);
            return false;
        }
        j.blk[b].live = true;
    }
    return true;
}

// Upload and initialise a job whose blocks and slot are assigned (worker
// thread; touches only the job, its slot's stream and its arena blocks).
// On failure the slot's stream is drained before returning.
int init_job(vest_server *s, Job &j)
{
    const int slot = j.slot;
    hipStream_t st = s->streams[slot];
    JobPtrs p = job_ptrs(s, j);
    const vest_desc &d = j.in.desc;
    hipError_t e = hipMemcpyAsync(s->ptr(j.blk[5]), j.in.idx, j.blk[5].bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->ptr(j.blk[6]), j.in.val, j.blk[6].bytes, hipMemcpyHostToDevice, st);
    for (int n = 0; n < j.N && e == hipSuccess; ++n)
        e = hipMemcpyAsync(p.fac[n], j.in.factors[n], (size_t)d.dims[n] * d.ranks[n] * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p.core, j.in.core, (size_t)j.G * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->ptr(j.blk[3]), 0, j.blk[3].bytes, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->ptr(j.blk[4]), 0, j.blk[4].bytes, st);
    int rc = e == hipSuccess ? VEST_OK : hip_fail(e, "job upload");
    if (rc == VEST_OK)
        rc = vest_init(&d, st, (const int32_t *)s->ptr(j.blk[5]), (const double *)s->ptr(j.blk[6]), p.fac, p.core,
                       p.fmask, p.cmask, s->ptr(j.blk[0]), j.ws_bytes, &j.ctx);
    if (rc != VEST_OK) (void)hipStreamSynchronize(st);
    return rc;
}

void admission_worker(vest_server *s)
{
    (void)hipSetDevice(s->device);   // the current device is per host thread
    for (;;) {
        Job *j = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->todo.empty(); });
            if (s->stop) return;
            j = s->todo.front();
            s->todo.pop_front();
        }
        j->init_rc = init_job(s, *j);
        j->init_done.store(1, std::memory_order_release);
    }
}

// A job the worker has finished with: the observed tensor now lives in the
// workspace layouts (vest_init waited for its stream), so its blocks go back
// to the arena; the job becomes active or fails.  Progress thread.
void finish_admission(vest_server *s, Job &j)
{
    for (int b = 5; b < 7; ++b)
        if (j.blk[b].live) {
            s->arena.release(j.blk[b].off, j.blk[b].bytes);
            j.blk[b].live = false;
        }
    if (j.init_rc != VEST_OK) {
        release_blocks(s, j);
        s->slot_job[j.slot] = -1;
        j.slot = -1;
        j.state = VEST_JOB_FAILED;
        j.error = j.init_rc;
        j.t_done = s->now();
        return;
    }
    j.state = VEST_JOB_ACTIVE;
}

// Jobs of a class advance in lockstep, so a class also bounds the spread of
// its jobs' sizes: entries within a factor of 4 (a small job is not held back
// by a large one's iterations).
int size_bucket(int64_t nnz)
{
    int b = 0;
    while (nnz >= 4) {
        nnz >>= 2;
        ++b;
    }
    return b;
}

int klass_of(vest_server *s, const Job &j)
{
    const int N = j.N, J = j.in.desc.ranks[0], pr = j.in.desc.precision, sb = size_bucket(j.in.desc.nnz);
    for (size_t k = 0; k < s->classes.size(); ++k) {
        const Klass &K = s->classes[k];
        if (K.N == N && K.J == J && K.precision == pr && K.bucket == sb) return (int)k;
    }
    Klass K;
    K.N = N;
    K.J = J;
    K.precision = pr;
    K.bucket = sb;
    hipError_t e = hipStreamCreateWithFlags(&K.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&K.event, hipEventDisableTiming);
    // the tables live outside the arena, which is the jobs' budget
    if (e == hipSuccess && hipMalloc((void **)&K.dev, kClassTable) == hipSuccess &&
        hipHostMalloc((void **)&K.host, kClassTable, hipHostMallocDefault) == hipSuccess)
        K.usable = true;
    s->classes.push_back(K);
    return (int)s->classes.size() - 1;
}

// VeST^man of a pruning job (Sec. 3.3, the schedule of paper_1904_02603_amd
// /schedule.py): after iteration t (t < iterations) and while the marked
// fraction of all elements is below the target, one prune step of
// ceil(pr_t |T|) new marks per tensor, pr_t = min(0.01 t, 0.1), each tensor
// capped at ceil(target |T|) marks; keys from vest_responsibility.
int64_t prune_count(int t, int64_t size, int64_t marked, double target)
{
    const double pr = std::min(0.01 * t, 0.1);
    const int64_t want = (int64_t)std::ceil(pr * (double)size - 1e-12);
    const int64_t room = std::min(size - marked, (int64_t)std::ceil(target * (double)size - 1e-12) - marked);
    return std::max<int64_t>(0, std::min(want, room));
}

int prune_step(vest_server *s, Job &j)
{
    const int t = j.iters_done;
    if (!(j.in.prune_target > 0.0) || t < 1 || t >= j.in.iterations) return VEST_OK;
    vest_ctx *c = j.ctx;
    int64_t marked = c->marked_core, total = j.G;
    for (int n = 0; n < j.N; ++n) {
        marked += c->marked_fac[n];
        total += (int64_t)j.in.desc.dims[n] * j.in.desc.ranks[n];
    }
    if ((double)marked >= j.in.prune_target * (double)total) return VEST_OK;
    double *keys = (double *)s->ptr(j.blk[7]);
    double *fk[VEST_MAX_ORDER];
    int64_t kf[VEST_MAX_ORDER];
    double *q = keys + j.G;
    for (int n = 0; n < j.N; ++n) {
        const int64_t sz = (int64_t)j.in.desc.dims[n] * j.in.desc.ranks[n];
        fk[n] = q;
        q += sz;
        kf[n] = prune_count(t, sz, c->marked_fac[n], j.in.prune_target);
    }
    const int64_t kc = prune_count(t, j.G, c->marked_core, j.in.prune_target);
    int rc = vest_responsibility(c, keys, fk);
    if (rc == VEST_OK) rc = vest_prune(c, kc, kf);
    if (rc == VEST_OK) j.prune_steps++;
    return rc;
}

int enqueue_iteration(vest_server *s, Job &j)
{
    int rc = prune_step(s, j);   // the prune step that follows the previous iteration
    for (int n = 0; n < j.N && rc == VEST_OK; ++n) rc = vest_sweep_factor(j.ctx, n);
    if (rc == VEST_OK) rc = vest_sweep_core(j.ctx);
    if (rc != VEST_OK) return rc;
    hipError_t e = hipEventRecord(s->events[j.slot], s->streams[j.slot]);
    if (e != hipSuccess) return hip_fail(e, "event record");
    j.inflight = true;
    j.in_batch = false;
    return VEST_OK;
}

// One batched iteration of every idle job of class k that has iterations
// left; jobs the batched path does not take run alone.  Returns the jobs
// that failed (to be retired by the caller).
std::vector<int64_t> enqueue_class(vest_server *s, int k)
{
    Klass &K = s->classes[k];
    std::vector<int64_t> failed, ids;
    std::vector<vest_ctx *> cs;
    for (int64_t id : s->active) {
        Job &j = *s->jobs[id];
        if (j.klass == k && !j.inflight && j.iters_done < j.in.iterations) {
            if (j.in.prune_target > 0.0) {   // pruning jobs run alone on their slot stream
                if (enqueue_iteration(s, j) != VEST_OK) failed.push_back(id);
                continue;
            }
            ids.push_back(id);
            cs.push_back(j.ctx);
        }
    }
    if (ids.empty() || K.inflight) return failed;
    int rc = VEST_EUNSUPPORTED;
    if (K.usable)
        rc = vest_iterate_many(cs.data(), (int32_t)cs.size(), K.stream, K.dev, K.host, kClassTable);
    if (rc == VEST_OK) {
        hipError_t e = hipEventRecord(K.event, K.stream);
        if (e == hipSuccess) {
            K.inflight = true;
            K.batch = ids;
            for (int64_t id : ids) {
                Job &j = *s->jobs[id];
                j.inflight = true;
                j.in_batch = true;
            }
            s->batches++;
            s->batched_job_iters += (int64_t)ids.size();
            return failed;
        }
        rc = hip_fail(e, "event record");
        for (int64_t id : ids) failed.push_back(id);
        return failed;
    }
    // not batched: each job alone on its slot's stream
    for (int64_t id : ids) {
        Job &j = *s->jobs[id];
        if (enqueue_iteration(s, j) != VEST_OK) failed.push_back(id);
    }
    return failed;
}

// Loss, result copies, release.  Synchronises the job's stream.
void retire(vest_server *s, Job &j)
{
    hipStream_t st = s->streams[j.slot];
    j.ctx->host_red = s->pinned_loss;   // server-owned; not freed by vest_destroy
    j.ctx->host_red_owned = false;
    int rc = vest_loss(j.ctx, j.loss);
    if (rc == VEST_OK) {
        JobPtrs p = job_ptrs(s, j);
        j.res_fac.resize(j.fac_elems());
        j.res_core.resize((size_t)j.G);
        hipError_t e = hipMemcpyAsync(j.res_fac.data(), p.fac[0], j.res_fac.size() * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(j.res_core.data(), p.core, j.res_core.size() * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "result copy");
    }
    vest_destroy(j.ctx);
    j.ctx = nullptr;
    release_blocks(s, j);
    s->slot_job[j.slot] = -1;
    j.slot = -1;
    j.state = rc == VEST_OK ? VEST_JOB_DONE : VEST_JOB_FAILED;
    j.error = rc;
    j.t_done = s->now();
}

}  // namespace

extern "C" {

int vest_server_create(size_t device_bytes, int32_t slots, vest_server **out)
{
    if (!out || slots < 1 || slots > 256 || device_bytes < kAlign) {
        set_error("bad server arguments (slots %d, %zu bytes)", slots, device_bytes);
        return VEST_EINVAL;
    }
    vest_server *s = new (std::nothrow) vest_server();
    if (!s) { set_error("out of host memory"); return VEST_EINVAL; }
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc((void **)&s->base, device_bytes);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "server arena");
    }
    s->arena.reset(device_bytes / kAlign * kAlign);
    if (hipHostMalloc((void **)&s->pinned_loss, 64, hipHostMallocDefault) != hipSuccess) s->pinned_loss = nullptr;
    s->streams.assign(slots, nullptr);
    s->events.assign(slots, nullptr);
    s->slot_job.assign(slots, -1);
    for (int i = 0; i < slots && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        vest_server_destroy(s);
        return hip_fail(e, "server streams");
    }
    try {
        for (int w = 0; w < kAdmissionThreads; ++w) s->workers.emplace_back(admission_worker, s);
    } catch (...) {
        vest_server_destroy(s);
        set_error("cannot start the admission thread");
        return VEST_EINVAL;
    }
    *out = s;
    return VEST_OK;
}

int vest_server_submit(vest_server *s, const vest_job *job, int64_t *id)
{
    if (!s || !job || !id) { set_error("null argument"); return VEST_EINVAL; }
    int rc = vest::check_desc(&job->desc);
    if (rc) return rc;
    if (job->iterations < 1 || job->reserved != 0) { set_error("iterations must be >= 1, reserved 0"); return VEST_EINVAL; }
    if (!(job->prune_target >= 0.0 && job->prune_target < 1.0)) { set_error("prune_target outside [0, 1)"); return VEST_EINVAL; }
    if (job->prune_target > 0.0)
        for (int n = 1; n < job->desc.order; ++n)
            if (job->desc.ranks[n] != job->desc.ranks[0]) {
                set_error("a pruning job needs equal ranks");
                return VEST_EINVAL;
            }
    if (!job->idx || !job->val || !job->factors || !job->core) { set_error("null job array"); return VEST_EINVAL; }
    for (int n = 0; n < job->desc.order; ++n)
        if (!job->factors[n]) { set_error("null factor %d", n); return VEST_EINVAL; }
    std::unique_ptr<Job> j(new (std::nothrow) Job());
    if (!j) { set_error("out of host memory"); return VEST_EINVAL; }
    j->in = *job;
    j->N = job->desc.order;
    for (int n = 0; n < j->N; ++n) j->G *= job->desc.ranks[n];
    rc = vest_workspace_bytes(&job->desc, &j->ws_bytes);
    if (rc) return rc;
    if (j->footprint() > s->arena.size()) {
        set_error("job footprint %zu bytes exceeds the arena of %zu", j->footprint(), s->arena.size());
        return VEST_ENOSPC;
    }
    j->id = s->next_id++;
    j->t_arrive = s->now();
    *id = j->id;
    s->queue.push_back(j->id);
    s->jobs[j->id] = std::move(j);
    return VEST_OK;
}

int vest_server_progress(vest_server *s, int32_t *completed)
{
    if (!s) { set_error("null server"); return VEST_EINVAL; }
    int32_t done = 0;
    // 1. batches that completed
    for (Klass &K : s->classes) {
        if (!K.inflight) continue;
        hipError_t q = hipEventQuery(K.event);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return hip_fail(q, "event query");
        for (int64_t id : K.batch) {
            Job &j = *s->jobs[id];
            j.inflight = false;
            j.in_batch = false;
            ++j.iters_done;
        }
        K.inflight = false;
        K.batch.clear();
    }
    // 2. single iterations that completed; retire finished jobs
    std::vector<int64_t> still;
    for (int64_t id : s->active) {
        Job &j = *s->jobs[id];
        if (j.inflight && !j.in_batch) {
            hipError_t q = hipEventQuery(s->events[j.slot]);
            if (q == hipErrorNotReady) {
                still.push_back(id);
                continue;
            }
            if (q != hipSuccess) return hip_fail(q, "event query");
            j.inflight = false;
            ++j.iters_done;
        }
        if (j.inflight) {   // its class's batch is still running
            still.push_back(id);
            continue;
        }
        if (j.iters_done >= j.in.iterations) {
            retire(s, j);
            ++done;
            continue;
        }
        still.push_back(id);
    }
    s->active.swap(still);
    // 3. admissions the worker finished
    std::vector<int64_t> pending;
    for (int64_t id : s->admitting) {
        Job &j = *s->jobs[id];
        if (!j.init_done.load(std::memory_order_acquire)) {
            pending.push_back(id);
            continue;
        }
        finish_admission(s, j);
        if (j.state == VEST_JOB_ACTIVE) {
            j.klass = klass_of(s, j);
            s->active.push_back(j.id);
        } else {
            ++done;  // failed at admission
        }
    }
    s->admitting.swap(pending);
    // 4. admit queued jobs in arrival order (later jobs fill in when the head
    //    does not fit yet): blocks and slot here, upload and vest_init on the
    //    worker
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        int slot = -1;
        for (size_t k = 0; k < s->slot_job.size(); ++k)
            if (s->slot_job[k] < 0) { slot = (int)k; break; }
        if (slot < 0) break;
        Job &j = *s->jobs[*it];
        if (j.footprint() > s->arena.size() - s->arena.used() || !alloc_blocks(s, j)) {
            ++it;
            continue;
        }
        j.slot = slot;
        s->slot_job[slot] = j.id;
        j.t_admit = s->now();
        s->admitting.push_back(j.id);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->todo.push_back(&j);
        }
        s->cv.notify_one();
        it = s->queue.erase(it);
    }
    // 5. the next iteration of every idle job, batched per class
    for (size_t k = 0; k < s->classes.size(); ++k) {
        std::vector<int64_t> failed = enqueue_class(s, (int)k);
        if (failed.empty()) continue;
        (void)hipStreamSynchronize(s->classes[k].stream);
        for (int64_t id : failed) {
            Job &j = *s->jobs[id];
            const int32_t err = j.ctx && j.ctx->dead ? VEST_EDEVICE : VEST_EUNSUPPORTED;
            j.inflight = false;
            retire(s, j);
            j.state = VEST_JOB_FAILED;
            j.error = err;
            ++done;
            s->active.erase(std::find(s->active.begin(), s->active.end(), id));
        }
    }
    if (completed) *completed = done;
    return VEST_OK;
}

int vest_server_status(vest_server *s, int64_t id, int32_t *state, int32_t *error, double *times)
{
    if (!s) { set_error("null server"); return VEST_EINVAL; }
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) { set_error("unknown job %lld", (long long)id); return VEST_EINVAL; }
    const Job &j = *it->second;
    if (state) *state = j.state;
    if (error) *error = j.error;
    if (times) {
        times[0] = j.t_arrive;
        times[1] = j.t_admit;
        times[2] = j.t_done;
    }
    return VEST_OK;
}

int vest_server_fetch(vest_server *s, int64_t id, double *const *factors, double *core, double *loss)
{
    if (!s) { set_error("null server"); return VEST_EINVAL; }
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) { set_error("unknown job %lld", (long long)id); return VEST_EINVAL; }
    Job &j = *it->second;
    if (j.state != VEST_JOB_DONE || j.fetched) { set_error("job %lld has no results to fetch", (long long)id); return VEST_ESTATE; }
    if (factors) {
        size_t off = 0;
        for (int n = 0; n < j.N; ++n) {
            const size_t len = (size_t)j.in.desc.dims[n] * j.in.desc.ranks[n];
            if (factors[n]) std::memcpy(factors[n], j.res_fac.data() + off, len * 8);
            off += len;
        }
    }
    if (core) std::memcpy(core, j.res_core.data(), j.res_core.size() * 8);
    if (loss) std::memcpy(loss, j.loss, sizeof(j.loss));
    j.fetched = true;
    std::vector<double>().swap(j.res_fac);
    std::vector<double>().swap(j.res_core);
    return VEST_OK;
}

int vest_server_stats(vest_server *s, int64_t *out)
{
    if (!s || !out) { set_error("null argument"); return VEST_EINVAL; }
    int64_t finished = 0;
    for (auto &kv : s->jobs)
        if (kv.second->state == VEST_JOB_DONE && !kv.second->fetched) ++finished;
    out[0] = (int64_t)(s->queue.size() + s->admitting.size());
    out[1] = (int64_t)s->active.size();
    out[2] = finished;
    out[3] = (int64_t)s->arena.used();
    out[4] = (int64_t)s->arena.size();
    out[5] = (int64_t)s->arena.largest();
    out[6] = s->batches;
    out[7] = s->batched_job_iters;
    return VEST_OK;
}

int vest_server_destroy(vest_server *s)
{
    if (!s) return VEST_OK;
    {   // admissions in progress complete first
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (std::thread &t : s->workers)
        if (t.joinable()) t.join();
    for (int64_t id : s->admitting) {
        Job &j = *s->jobs[id];
        if (j.init_done.load(std::memory_order_acquire) && j.ctx) vest_destroy(j.ctx);
        j.ctx = nullptr;
    }
    for (hipStream_t st : s->streams)
        if (st) hipStreamSynchronize(st);
    for (Klass &K : s->classes)
        if (K.stream) hipStreamSynchronize(K.stream);
    for (int64_t id : s->active) {
        Job &j = *s->jobs[id];
        if (j.ctx) vest_destroy(j.ctx);
        j.ctx = nullptr;
    }
    for (Klass &K : s->classes) {
        if (K.stream) {
            hipStreamSynchronize(K.stream);
            hipStreamDestroy(K.stream);
        }
        if (K.event) hipEventDestroy(K.event);
        if (K.host) hipHostFree(K.host);
        if (K.dev) hipFree(K.dev);
    }
    if (s->pinned_loss) hipHostFree(s->pinned_loss);
    for (hipEvent_t ev : s->events)
        if (ev) hipEventDestroy(ev);
    for (hipStream_t st : s->streams)
        if (st) hipStreamDestroy(st);
    if (s->base) hipFree(s->base);
    delete s;
    return VEST_OK;
}

}  // extern "C"
