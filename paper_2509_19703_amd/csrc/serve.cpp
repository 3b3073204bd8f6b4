// Request server: continuous batching of layout-preparation jobs
// (partial-BFS kNN + membership of one graph per job) on one device.
//
// gumap_submit copies a job's host CSR into pinned host memory (a pool
// reserved at creation) and queues it.  When the pool is full it waits, for a
// bounded time, while inputs of earlier jobs are still held there (each is
// returned as soon as it is uploaded); only then does it fall back to
// pageable memory, whose uploads are several times slower.
// A scheduler thread runs a pipeline on three streams:
//   admission   queued jobs are admitted first-come-first-served while their
//               device bytes fit the budget, a slot is free and their result
//               fits the pinned result pool; the CSR is uploaded (and, if the
//               job is not canonical, canonicalised) on the copy stream and an
//               event marks the upload;
//   iterations  one launch of the jobs kernel over row chunks taken from
//               every admitted job with rows left (oldest job first, up to a
//               row budget); the compute stream waits for the uploads of the
//               jobs it includes, and up to two iterations are in flight, so
//               jobs that arrive while one runs join the next;
//   retirement  when the iteration holding a job's last rows completes, its
//               results are copied to pinned host memory on a third stream;
//               when that copy completes the job is done and its device space
//               is returned.
// Every row of a job is computed by the same per-row code whatever shares the
// launch, so a result does not depend on the mix of jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gumap.h"
#include "kernels.h"
#include "runtime.h"

namespace {

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over [0, capacity).
class SlabAllocator {
public:
    explicit SlabAllocator(size_t capacity = 0) { reset(capacity); }
    void reset(size_t capacity)
    {
        free_.clear();
        if (capacity) free_[0] = capacity;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes ? bytes : 1, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1, 256);
        auto it = free_.emplace(off, bytes).first;
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

private:
    std::map<size_t, size_t> free_;
};

enum JobState { kQueued, kAdmitted, kDownloading, kDone };

// An event shared by the jobs whose copies it follows: one record per batch
// of uploads or downloads instead of one per job (records interleaved with
// every copy slow down uploads that overlap downloads in the other direction).
struct SharedEvent {
    hipEvent_t ev = nullptr;
    ~SharedEvent()
    {
        if (ev) (void)hipEventDestroy(ev);
    }
};
typedef std::shared_ptr<SharedEvent> EventRef;

// Records a fresh event on `s`; null on failure.
EventRef record_event(hipStream_t s)
{
    auto r = std::make_shared<SharedEvent>();
    if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(r->ev, s) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return r;
}

// hipEventQuery, asked once per event within one pass over many jobs.
struct QueryCache {
    std::map<SharedEvent *, bool> seen;
    bool done(const EventRef &r)
    {
        auto it = seen.find(r.get());
        if (it != seen.end()) return it->second;
        const hipError_t q = hipEventQuery(r->ev);
        if (q != hipSuccess && q != hipErrorNotReady) (void)hipGetLastError();
        return seen[r.get()] = (q != hipErrorNotReady);
    }
};

struct Job {
    uint64_t ticket = 0;
    JobState state = kQueued;
    int status = GUMAP_OK;
    int32_t n = 0, nnz = 0, k = 0;
    bool weights = false;
    uint32_t flags = 0;
    // host input: pinned pool slice, or pageable copy when the pool was full
    int32_t *in_rp = nullptr, *in_col = nullptr;
    size_t in_off = 0, in_bytes = 0;
    bool in_pinned = false;
    std::vector<int32_t> pg_rp, pg_col;
    // host results (pinned pool slice, or pageable memory when the pool is full)
    size_t out_off = 0, out_bytes = 0;
    bool out_pinned = false;
    std::vector<char> pg_out;
    int32_t *r_ids = nullptr;
    uint8_t *r_hops = nullptr;
    float *r_w = nullptr, *r_rho = nullptr, *r_sigma = nullptr;
    // device
    size_t bytes = 0, slab_off = 0;
    gm::DevJob dev{};
    EventRef up_done, down_done;   // upload and result download complete
    bool waited = false;           // compute stream already waits for the upload
    bool input_freed = false;
    int32_t next_row = 0;
    int64_t last_iter = -1;
    uint64_t t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
};

size_t job_device_bytes(int32_t n, int32_t nnz, int32_t k, bool weights, bool needs_canon)
{
    size_t b = align_up((size_t)(n + 1) * 4, 256) + align_up((size_t)std::max(nnz, 1) * 4, 256);
    b += align_up((size_t)n * k * 4, 256) + align_up((size_t)n * k, 256);
    if (weights) b += align_up((size_t)n * k * 4, 256) + 2 * align_up((size_t)n * 4, 256);
    if (needs_canon) {
        b += align_up((size_t)(n + 1) * 4, 256) + align_up((size_t)std::max(nnz, 1) * 4, 256);
        b += align_up(gm::canon_scratch_bytes(n, nnz), 256) + 512;
    }
    return b;
}

size_t job_result_bytes(int32_t n, int32_t k, bool weights)
{
    size_t b = align_up((size_t)n * k * 4, 256) + align_up((size_t)n * k, 256);
    if (weights) b += align_up((size_t)n * k * 4, 256) + 2 * align_up((size_t)n * 4, 256);
    return b;
}

size_t job_input_bytes(int32_t n, int32_t nnz)
{
    return align_up((size_t)(n + 1) * 4, 256) + align_up((size_t)std::max(nnz, 1) * 4, 256);
}

constexpr int kInFlight = 2;
constexpr int kPoolWaitMs = 200;   // longest wait of a submission for pinned pool space

// Host copies of submitted CSRs, split into 1 MiB parts over a few
// persistent threads plus the caller: one thread reaches only a fraction of
// the host's memory bandwidth on multi-megabyte copies from cold memory.
// Parts are claimed with a compare-and-swap on (generation, index), so a
// worker that wakes late never takes a part of a later copy.
class CopyPool {
public:
    explicit CopyPool(int workers)
    {
        for (int i = 0; i < workers; ++i) th_.emplace_back([this] { work(); });
    }
    ~CopyPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    void copy(void *dst, const void *src, size_t bytes)
    {
        if (th_.empty() || bytes < 2 * kPart) {
            std::memcpy(dst, src, bytes);
            return;
        }
        std::lock_guard<std::mutex> call(call_mu_);   // one copy at a time
        uint32_t gen;
        {
            std::lock_guard<std::mutex> lk(mu_);
            dst_ = (char *)dst;
            src_ = (const char *)src;
            bytes_ = bytes;
            parts_ = (uint32_t)((bytes + kPart - 1) / kPart);
            gen = ++gen_;
            done_.store(0);
            next_.store((uint64_t)gen << 32);
        }
        cv_.notify_all();
        run_parts(gen, (char *)dst, (const char *)src, bytes, parts_);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return done_.load() == parts_; });
    }

    // memset split over as many threads as the pool holds
    void fill(void *dst, int value, size_t bytes)
    {
        const size_t parts = (bytes + kPart * 16 - 1) / (kPart * 16);
        std::vector<std::thread> th;
        std::atomic<size_t> next{0};
        auto run = [&] {
            for (size_t i; (i = next.fetch_add(1)) < parts;) {
                const size_t off = i * kPart * 16;
                std::memset((char *)dst + off, value, std::min(kPart * 16, bytes - off));
            }
        };
        for (size_t i = 0; i < th_.size(); ++i) th.emplace_back(run);
        run();
        for (auto &t : th) t.join();
    }

private:
    static constexpr size_t kPart = 1u << 20;

    void run_parts(uint32_t gen, char *dst, const char *src, size_t bytes, uint32_t parts)
    {
        for (;;) {
            uint64_t v = next_.load();
            for (;;) {
                if ((uint32_t)(v >> 32) != gen || (uint32_t)v >= parts) return;
                if (next_.compare_exchange_weak(v, v + 1)) break;
            }
            const size_t off = (size_t)(uint32_t)v * kPart;
            std::memcpy(dst + off, src + off, std::min(kPart, bytes - off));
            if (done_.fetch_add(1) + 1 == parts) {
                std::lock_guard<std::mutex> lk(mu_);
                done_cv_.notify_all();
            }
        }
    }
    void work()
    {
        uint32_t seen = 0;
        for (;;) {
            uint32_t gen, parts;
            char *dst;
            const char *src;
            size_t bytes;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen = gen_;
                dst = dst_;
                src = src_;
                bytes = bytes_;
                parts = parts_;
            }
            run_parts(gen, dst, src, bytes, parts);
        }
    }

    std::mutex call_mu_, mu_;
    std::condition_variable cv_, done_cv_;
    std::vector<std::thread> th_;
    char *dst_ = nullptr;
    const char *src_ = nullptr;
    size_t bytes_ = 0;
    uint32_t parts_ = 0, gen_ = 0;
    std::atomic<uint64_t> next_{0};
    std::atomic<uint32_t> done_{0};
    bool stop_ = false;
};

}  // namespace

struct gumap_server {
    size_t budget = 0;
    int32_t max_slots = 0;
    bool no_device = false;
    int device = 0;
    char *slab = nullptr;               // device
    SlabAllocator alloc;
    char *host_pool = nullptr;          // pinned (or plain memory without a device)
    size_t host_pool_bytes = 0;
    SlabAllocator host_alloc;
    hipStream_t compute = nullptr, copy = nullptr, d2h = nullptr, meta = nullptr;
    // per in-flight iteration slot
    hipEvent_t iter_done[kInFlight] = {}, table_done[kInFlight] = {};
    gm::DevJob *d_jobs[kInFlight] = {};
    gm::JobChunk *d_chunks[kInFlight] = {};
    unsigned long long *d_counter[kInFlight] = {};
    gm::DevJob *h_jobs[kInFlight] = {};
    gm::JobChunk *h_chunks[kInFlight] = {};
    int32_t table_cap = 0, chunk_cap = 0;
    int64_t iter_rows = 0;
    int blocks = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::condition_variable cv_space;  // pinned pool space returned
    size_t pinned_inputs = 0;          // pool bytes held by inputs not yet uploaded
    std::deque<std::shared_ptr<Job>> queue;               // waiting for admission
    std::vector<std::shared_ptr<Job>> admitted;           // resident, rows left or in flight
    std::vector<std::shared_ptr<Job>> downloading;
    std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool kick = false;                 // a submission or a released result may unblock admission
    std::thread worker;
    std::unique_ptr<CopyPool> copier;
    gumap_server_stats stats{};
    size_t resident = 0;

    struct Flight {
        int64_t iter;
        int slot;
        std::vector<std::shared_ptr<Job>> jobs;        // jobs with rows in it
        std::vector<std::shared_ptr<Job>> finishing;   // jobs whose last rows are in it
    };
    // Device-free scheduler only: the executor reports this iteration as
    // failed, as a device error would (test hook, GUMAP_SERVE_NODEV_FAIL_ITER).
    int64_t fail_iter = -1;
    std::deque<Flight> flights;
    int64_t iter_count = 0;

    void run();
    int stage(Job &j);
    void finish_locked(const std::shared_ptr<Job> &j, int status);
    void free_input_locked(Job &j);
    bool launch_iteration();
    bool retire_iterations();
    bool poll_downloads();
};

void gumap_server::free_input_locked(Job &j)
{
    if (j.input_freed) return;
    if (j.in_pinned) {
        host_alloc.release(j.in_off, j.in_bytes);
        pinned_inputs -= j.in_bytes;
        cv_space.notify_all();
    }
    j.pg_rp.clear();
    j.pg_rp.shrink_to_fit();
    j.pg_col.clear();
    j.pg_col.shrink_to_fit();
    j.in_rp = j.in_col = nullptr;
    j.input_freed = true;
}

void gumap_server::finish_locked(const std::shared_ptr<Job> &j, int status)
{
    j->status = status;
    j->state = kDone;
    j->t_done = now_ns();
    resident -= j->bytes;
    alloc.release(j->slab_off, j->bytes);
    free_input_locked(*j);
    if (status != GUMAP_OK && j->out_pinned) {
        host_alloc.release(j->out_off, j->out_bytes);
        j->out_pinned = false;
    }
    j->up_done.reset();
    j->down_done.reset();
    if (status == GUMAP_OK) stats.completed++;
    else stats.failed++;
    cv_done.notify_all();
}

// Upload (and canonicalise / validate) an admitted job.  Scheduler thread.
int gumap_server::stage(Job &j)
{
    if (no_device) return GUMAP_OK;
    char *base = slab + j.slab_off;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += align_up(bytes ? bytes : 1, 256);
        return p;
    };
    int32_t *rp = (int32_t *)take((size_t)(j.n + 1) * 4);
    int32_t *col = (int32_t *)take((size_t)std::max(j.nnz, 1) * 4);
    j.dev.ids = (int32_t *)take((size_t)j.n * j.k * 4);
    j.dev.hops = (uint8_t *)take((size_t)j.n * j.k);
    j.dev.weights = j.dev.rho = j.dev.sigma = nullptr;
    if (j.weights) {
        j.dev.weights = (float *)take((size_t)j.n * j.k * 4);
        j.dev.rho = (float *)take((size_t)j.n * 4);
        j.dev.sigma = (float *)take((size_t)j.n * 4);
    }
    // results come back in one copy: the host result region mirrors this layout
    if (j.n > 0 && ((char *)j.dev.hops - (char *)j.dev.ids != (char *)j.r_hops - (char *)j.r_ids ||
                    (j.weights && (char *)j.dev.sigma - (char *)j.dev.ids != (char *)j.r_sigma - (char *)j.r_ids)))
        return gm::set_error(GUMAP_EINVAL, "internal: result layouts differ");
    j.dev.n = j.n;
    j.dev.k = j.k;
    j.dev.row_ptr = rp;
    j.dev.col = col;
    hipError_t e = hipSuccess;
    if (j.in_pinned) {
        // the pinned slice has the device layout (row_ptr, then col_idx at the
        // next 256-byte boundary): one copy
        const size_t bytes = align_up((size_t)(j.n + 1) * 4, 256) + (size_t)j.nnz * 4;
        if (e == hipSuccess) e = hipMemcpyAsync(rp, j.in_rp, bytes, hipMemcpyHostToDevice, copy);
    } else {
        if (e == hipSuccess) e = hipMemcpyAsync(rp, j.in_rp, (size_t)(j.n + 1) * 4, hipMemcpyHostToDevice, copy);
        if (e == hipSuccess && j.nnz)
            e = hipMemcpyAsync(col, j.in_col, (size_t)j.nnz * 4, hipMemcpyHostToDevice, copy);
    }
    if (e != hipSuccess) return gm::hip_status(e, "job upload");
    if (!(j.flags & GUMAP_CSR_SORTED) || (j.flags & GUMAP_VALIDATE)) {
        int32_t *crp = (int32_t *)take((size_t)(j.n + 1) * 4);
        int32_t *ccol = (int32_t *)take((size_t)std::max(j.nnz, 1) * 4);
        void *scratch = take(gm::canon_scratch_bytes(j.n, j.nnz));
        int *err = (int *)take(256);
        if (j.flags & GUMAP_VALIDATE) {
            e = hipMemsetAsync(err, 0, sizeof(int), copy);
            if (e == hipSuccess) e = gm::launch_validate_structure(j.n, j.nnz, rp, col, err, copy);
            int bad = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, copy);
            if (e == hipSuccess) e = hipStreamSynchronize(copy);
            if (e != hipSuccess) return gm::hip_status(e, "job validate");
            if (bad) return gm::set_error(GUMAP_EGRAPH, "malformed CSR");
        }
        if (!(j.flags & GUMAP_CSR_SORTED)) {
            e = gm::launch_canonicalize(j.n, j.nnz, rp, col, crp, ccol, scratch, copy);
            if (e != hipSuccess) return gm::hip_status(e, "job canonicalize");
            j.dev.row_ptr = crp;
            j.dev.col = ccol;
        }
        if (j.flags & GUMAP_VALIDATE) {
            e = hipMemsetAsync(err, 0, sizeof(int), copy);
            if (e == hipSuccess) e = gm::launch_check_symmetric(j.n, j.dev.row_ptr, j.dev.col, err, copy);
            int bad = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, copy);
            if (e == hipSuccess) e = hipStreamSynchronize(copy);
            if (e != hipSuccess) return gm::hip_status(e, "job validate");
            if (bad) return gm::set_error(GUMAP_EGRAPH, "CSR is not symmetric");
        }
    }
    return GUMAP_OK;
}

// Enqueue one iteration if a slot is free and rows are waiting.
bool gumap_server::launch_iteration()
{
    if ((int)flights.size() >= kInFlight) return false;
    const int slot = (int)(iter_count % kInFlight);
    std::vector<std::shared_ptr<Job>> table;
    std::vector<gm::JobChunk> chunks;
    Flight fl;
    fl.iter = iter_count;
    fl.slot = slot;
    int max_k = 1;
    {
        std::lock_guard<std::mutex> lk(mu);
        int64_t rows_left = iter_rows;
        for (auto &j : admitted) {
            if (j->next_row >= j->n && j->n > 0) continue;
            if (j->last_iter >= 0 && j->n == 0) continue;
            if (rows_left <= 0 || (int32_t)table.size() >= table_cap) break;
            const int32_t job_idx = (int32_t)table.size();
            const int32_t step = gm::batch_chunk_rows(j->k);
            int32_t r = j->next_row;
            while (r < j->n && rows_left > 0 && (int32_t)chunks.size() < chunk_cap) {
                const int32_t e = std::min(j->n, r + step);
                chunks.push_back(gm::JobChunk{job_idx, r, e, 0});
                rows_left -= e - r;
                r = e;
            }
            if (r == j->next_row && j->n > 0) break;
            if (j->t_start == 0) j->t_start = now_ns();
            table.push_back(j);
            max_k = std::max(max_k, j->k);
            j->next_row = r;
            j->last_iter = iter_count;
            if (r >= j->n) fl.finishing.push_back(j);
            fl.jobs.push_back(j);
        }
        if (table.empty()) return false;
        stats.iterations++;
    }
    if (!no_device) {
        hipError_t e = hipSuccess;
        SharedEvent *last = nullptr;
        for (auto &j : table) {
            if (!j->waited) {
                if (j->up_done.get() != last) e = hipStreamWaitEvent(compute, j->up_done->ev, 0);
                last = j->up_done.get();
                j->waited = true;
                if (e != hipSuccess) break;
            }
        }
        for (size_t i = 0; i < table.size(); ++i) h_jobs[slot][i] = table[i]->dev;
        std::copy(chunks.begin(), chunks.end(), h_chunks[slot]);
        // the iteration's tables go up on a stream of their own: a copy
        // queued behind the running kernel on the compute stream would hold
        // up the job uploads that share its copy engine
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_jobs[slot], h_jobs[slot], table.size() * sizeof(gm::DevJob), hipMemcpyHostToDevice, meta);
        if (e == hipSuccess && !chunks.empty())
            e = hipMemcpyAsync(d_chunks[slot], h_chunks[slot], chunks.size() * sizeof(gm::JobChunk),
                               hipMemcpyHostToDevice, meta);
        if (e == hipSuccess) e = hipEventRecord(table_done[slot], meta);
        if (e == hipSuccess) e = hipStreamWaitEvent(compute, table_done[slot], 0);
        if (e == hipSuccess) e = gm::launch_batch_reset(d_counter[slot], compute);
        if (e == hipSuccess)
            e = gm::launch_partial_jobs(d_jobs[slot], d_chunks[slot], (int32_t)chunks.size(), max_k,
                                        d_counter[slot], blocks, compute);
        if (e == hipSuccess) e = hipEventRecord(iter_done[slot], compute);
        if (e != hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &j : table)
                if (j->state == kAdmitted) {
                    admitted.erase(std::remove(admitted.begin(), admitted.end(), j), admitted.end());
                    finish_locked(j, GUMAP_EDEVICE);
                }
            (void)hipGetLastError();
            return false;
        }
    }
    flights.push_back(std::move(fl));
    ++iter_count;
    return true;
}

// Completed iterations: start the result downloads of jobs they finished.
bool gumap_server::retire_iterations()
{
    std::vector<std::shared_ptr<Job>> started, failed;
    bool popped = false;
    while (!flights.empty()) {
        Flight &fl = flights.front();
        bool iter_failed = false;
        if (!no_device) {
            hipError_t q = hipEventQuery(iter_done[fl.slot]);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) {
                (void)hipGetLastError();
                iter_failed = true;
            }
        } else {
            iter_failed = fl.iter == fail_iter;
        }
        if (iter_failed) {
            // the executor reported an error: every job with rows in the
            // iteration ends with GUMAP_EDEVICE, the others go on
            for (auto &j : fl.jobs)
                if (j->state == kAdmitted && std::find(failed.begin(), failed.end(), j) == failed.end())
                    failed.push_back(j);
            flights.pop_front();
            popped = true;
            continue;
        }
        for (auto &j : fl.finishing) {
            if (j->last_iter != fl.iter || j->state != kAdmitted) continue;
            if (std::find(failed.begin(), failed.end(), j) != failed.end()) continue;
            const size_t nk = (size_t)j->n * j->k;
            hipError_t e = hipSuccess;
            if (!no_device && j->n > 0) {
                // host and device result regions share one layout (ids, hops,
                // weights, rho, sigma at 256-byte boundaries): one copy
                const size_t bytes = j->weights ? (size_t)((char *)j->r_sigma - (char *)j->r_ids) + (size_t)j->n * 4
                                                : (size_t)((char *)j->r_hops - (char *)j->r_ids) + nk;
                // issued as a one-row 2D copy: some HIP runtimes run linear
                // device-to-host copies as shader blits, which stall the DMA
                // engine carrying the uploads; the 2D form goes to DMA, so
                // downloads and uploads overlap on the full-duplex link
                e = hipMemcpy2DAsync(j->r_ids, bytes, j->dev.ids, bytes, bytes, 1, hipMemcpyDeviceToHost, d2h);
            }
            if (e != hipSuccess) {
                (void)hipGetLastError();
                failed.push_back(j);
            } else {
                started.push_back(j);
            }
        }
        flights.pop_front();
        popped = true;
    }
    if (started.empty() && failed.empty()) return popped;
    EventRef ev;
    if (!no_device && !started.empty()) {
        ev = record_event(d2h);
        if (!ev) {
            failed.insert(failed.end(), started.begin(), started.end());
            started.clear();
        }
    }
    std::lock_guard<std::mutex> lk(mu);
    for (auto &j : failed) {
        if (j->state != kAdmitted) continue;
        admitted.erase(std::remove(admitted.begin(), admitted.end(), j), admitted.end());
        finish_locked(j, GUMAP_EDEVICE);
    }
    for (auto &j : started) {
        admitted.erase(std::remove(admitted.begin(), admitted.end(), j), admitted.end());
        j->down_done = ev;
        j->state = kDownloading;
        downloading.push_back(j);
    }
    return true;
}

bool gumap_server::poll_downloads()
{
    // events are queried without the lock (only this thread changes the
    // admitted and downloading lists), so submissions are not held up
    std::vector<std::shared_ptr<Job>> ready, uploaded;
    QueryCache qc;
    for (auto &j : downloading)
        if (no_device || !j->down_done || qc.done(j->down_done)) ready.push_back(j);
    for (auto &j : admitted) {
        if (j->input_freed || !j->up_done) continue;
        if (qc.done(j->up_done)) uploaded.push_back(j);
    }
    if (ready.empty() && uploaded.empty()) return false;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &j : ready) {
        downloading.erase(std::find(downloading.begin(), downloading.end(), j));
        finish_locked(j, GUMAP_OK);
    }
    // inputs of uploaded jobs go back to the pool
    for (auto &j : uploaded) free_input_locked(*j);
    return !ready.empty();
}

void gumap_server::run()
{
    if (!no_device) (void)hipSetDevice(device);
    for (;;) {
        std::vector<std::shared_ptr<Job>> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            const bool busy = !flights.empty() || !downloading.empty();
            if (!busy && !stop) cv_work.wait_for(lk, std::chrono::milliseconds(2), [&] { return stop || kick; });
            kick = false;
            if (stop && flights.empty() && downloading.empty()) break;
            // admission: first come first served, no overtaking
            while (!stop && !queue.empty()) {
                auto &j = queue.front();
                if (max_slots > 0 && (int32_t)admitted.size() >= max_slots) break;
                size_t off = 0, hoff = 0;
                if (resident + j->bytes > budget) break;
                if (!alloc.alloc(j->bytes, &off)) break;
                j->slab_off = off;
                char *hb;
                if (host_alloc.alloc(j->out_bytes, &hoff)) {
                    j->out_pinned = true;
                    j->out_off = hoff;
                    hb = host_pool + hoff;
                } else {
                    j->pg_out.assign(j->out_bytes, 0);
                    hb = j->pg_out.data();
                }
                char *const out_base = hb;
                const size_t nk = (size_t)j->n * j->k;
                j->r_ids = (int32_t *)hb;
                hb += align_up(nk * 4, 256);
                j->r_hops = (uint8_t *)hb;
                hb += align_up(nk, 256);
                if (j->weights) {
                    j->r_w = (float *)hb;
                    hb += align_up(nk * 4, 256);
                    j->r_rho = (float *)hb;
                    hb += align_up((size_t)j->n * 4, 256);
                    j->r_sigma = (float *)hb;
                }
                if (no_device) std::memset(out_base, 0, j->out_bytes);
                resident += j->bytes;
                stats.peak_resident_bytes = std::max<uint64_t>(stats.peak_resident_bytes, resident);
                j->state = kAdmitted;
                j->t_admit = now_ns();
                fresh.push_back(j);
                queue.pop_front();
            }
        }
        std::vector<std::shared_ptr<Job>> staged;
        for (auto &j : fresh) {
            const int st = stage(*j);
            if (st == GUMAP_OK) {
                staged.push_back(j);
                continue;
            }
            (void)hipGetLastError();
            std::lock_guard<std::mutex> lk(mu);
            finish_locked(j, st);
        }
        if (!staged.empty()) {
            // one event marks the uploads of the whole batch
            EventRef up = no_device ? nullptr : record_event(copy);
            std::lock_guard<std::mutex> lk(mu);
            for (auto &j : staged) {
                if (!no_device && !up) {
                    gm::set_error(GUMAP_EDEVICE, "upload event");
                    finish_locked(j, GUMAP_EDEVICE);
                    continue;
                }
                j->up_done = up;
                if (no_device) j->waited = true;
                admitted.push_back(j);
            }
        }
        bool progress = !fresh.empty();
        progress |= retire_iterations();
        progress |= poll_downloads();
        bool stopping;
        {
            std::lock_guard<std::mutex> lk(mu);
            stopping = stop;
        }
        if (!stopping)
            while (launch_iteration()) progress = true;
        if (!progress && (!flights.empty() || !downloading.empty()))
            std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    if (!no_device) {
        (void)hipStreamSynchronize(compute);
        (void)hipStreamSynchronize(copy);
        (void)hipStreamSynchronize(d2h);
        (void)hipStreamSynchronize(meta);
    }
}

extern "C" {

gumap_server *gumap_server_create(size_t hbm_budget_bytes, int32_t max_slots, uint32_t flags, int *status)
{
    auto fail = [&](int st) -> gumap_server * {
        if (status) *status = st;
        return nullptr;
    };
    gm::clear_error();
    if (hbm_budget_bytes == 0 || max_slots < 0 || (flags & ~GUMAP_SERVER_NO_DEVICE))
        return fail(gm::set_error(GUMAP_EINVAL, "bad server arguments"));
    auto *s = new gumap_server();
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->no_device = (flags & GUMAP_SERVER_NO_DEVICE) != 0;
    if (s->no_device) {
        const char *fi = getenv("GUMAP_SERVE_NODEV_FAIL_ITER");
        if (fi && *fi) s->fail_iter = strtoll(fi, nullptr, 10);
    }
    s->alloc.reset(hbm_budget_bytes);
    s->stats.budget_bytes = hbm_budget_bytes;
    s->iter_rows = (int64_t)gm::env_size("GUMAP_SERVE_ITER_ROWS", 1 << 20);
    s->table_cap = 4096;
    s->chunk_cap = (int32_t)std::min<int64_t>(1 << 22, s->iter_rows + s->table_cap);
    s->host_pool_bytes = gm::env_size("GUMAP_SERVE_HOST_POOL_MB", s->no_device ? 256 : 16384) << 20;
    s->host_alloc.reset(s->host_pool_bytes);
    hipError_t e = hipSuccess;
    if (s->no_device) {
        s->host_pool = (char *)malloc(s->host_pool_bytes);
        if (!s->host_pool) e = hipErrorOutOfMemory;
    } else {
        e = hipGetDevice(&s->device);
        if (e == hipSuccess) e = hipMalloc((void **)&s->slab, hbm_budget_bytes);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s->host_pool, s->host_pool_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->d2h, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->meta, hipStreamNonBlocking);
        for (int i = 0; i < kInFlight && e == hipSuccess; ++i) {
            e = hipEventCreateWithFlags(&s->iter_done[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s->table_done[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipMalloc((void **)&s->d_jobs[i], (size_t)s->table_cap * sizeof(gm::DevJob));
            if (e == hipSuccess) e = hipMalloc((void **)&s->d_chunks[i], (size_t)s->chunk_cap * sizeof(gm::JobChunk));
            if (e == hipSuccess) e = hipMalloc((void **)&s->d_counter[i], 256);
            if (e == hipSuccess)
                e = hipHostMalloc((void **)&s->h_jobs[i], (size_t)s->table_cap * sizeof(gm::DevJob), hipHostMallocDefault);
            if (e == hipSuccess)
                e = hipHostMalloc((void **)&s->h_chunks[i], (size_t)s->chunk_cap * sizeof(gm::JobChunk), hipHostMallocDefault);
        }
        if (e == hipSuccess) s->blocks = gm::partial_batch_max_blocks();
    }
    if (e != hipSuccess) {
        const int st = gm::hip_status(e, "server setup");
        (void)hipGetLastError();
        gumap_server_destroy(s);
        return fail(st);
    }
    {
        const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
        const int def = std::max(0, std::min(7, hw / 2 - 1));
        s->copier.reset(new CopyPool((int)std::min<size_t>(31, gm::env_size("GUMAP_SERVE_COPY_THREADS", (size_t)def))));
        // the first CPU write to each page of pinned memory is about ten
        // times slower than later ones: touch the whole pool now, so that
        // submissions copy at full speed
        s->copier->fill(s->host_pool, 0, s->host_pool_bytes);
    }
    s->worker = std::thread([s] { s->run(); });
    if (status) *status = GUMAP_OK;
    return s;
}

int gumap_submit(gumap_server *s, const gumap_job *job, uint64_t *ticket)
{
    gm::clear_error();
    if (!s || !job || !ticket) return gm::set_error(GUMAP_EINVAL, "NULL argument");
    if (job->n < 0 || job->nnz < 0) return gm::set_error(GUMAP_EINVAL, "negative n or nnz");
    if (job->k < 1 || job->k > GUMAP_MAX_K) return gm::set_error(GUMAP_EINVAL, "k outside [1, 254]");
    if ((job->n > 0 && !job->row_ptr) || (job->nnz > 0 && !job->col_idx))
        return gm::set_error(GUMAP_EINVAL, "NULL CSR array");
    if (job->flags & ~(GUMAP_CSR_SORTED | GUMAP_VALIDATE)) return gm::set_error(GUMAP_EINVAL, "unknown flags");
    auto j = std::make_shared<Job>();
    j->t_submit = now_ns();   // latency counts the copy into the pool
    j->n = job->n;
    j->nnz = job->nnz;
    j->k = job->k;
    j->weights = job->want_weights != 0;
    j->flags = job->flags;
    const bool needs_canon = !(job->flags & GUMAP_CSR_SORTED) || (job->flags & GUMAP_VALIDATE);
    j->bytes = job_device_bytes(j->n, j->nnz, j->k, j->weights, needs_canon);
    j->out_bytes = job_result_bytes(j->n, j->k, j->weights);
    if (j->bytes > s->budget)
        return gm::set_error(GUMAP_E2BIG, "job needs %zu device bytes, budget is %zu", j->bytes, s->budget);
    // copy the CSR now: into the pinned pool when it has room (waiting up to
    // kPoolWaitMs while earlier inputs still held there are being uploaded),
    // else into pageable memory
    j->in_bytes = job_input_bytes(j->n, j->nnz);
    {
        std::unique_lock<std::mutex> lk(s->mu);
        j->in_pinned = s->host_alloc.alloc(j->in_bytes, &j->in_off);
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(kPoolWaitMs);
        while (!j->in_pinned && s->pinned_inputs > 0 && j->in_bytes <= s->host_pool_bytes && !s->stop) {
            const bool timed_out = s->cv_space.wait_until(lk, deadline) == std::cv_status::timeout;
            j->in_pinned = s->host_alloc.alloc(j->in_bytes, &j->in_off);
            if (timed_out) break;
        }
        if (j->in_pinned) s->pinned_inputs += j->in_bytes;
    }
    if (j->in_pinned) {
        j->in_rp = (int32_t *)(s->host_pool + j->in_off);
        j->in_col = (int32_t *)(s->host_pool + j->in_off + align_up((size_t)(j->n + 1) * 4, 256));
    } else {
        j->pg_rp.resize((size_t)j->n + 1);
        j->pg_col.resize((size_t)std::max(j->nnz, 1));
        j->in_rp = j->pg_rp.data();
        j->in_col = j->pg_col.data();
    }
    if (j->n > 0) s->copier->copy(j->in_rp, job->row_ptr, (size_t)(j->n + 1) * 4);
    else j->in_rp[0] = 0;
    if (j->nnz > 0) s->copier->copy(j->in_col, job->col_idx, (size_t)j->nnz * 4);
    std::lock_guard<std::mutex> lk(s->mu);
    j->ticket = s->next_ticket++;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    s->stats.submitted++;
    *ticket = j->ticket;
    s->kick = true;
    s->cv_work.notify_one();
    return GUMAP_OK;
}

static void fill_result(const Job &j, gumap_result *out)
{
    out->status = j.status;
    out->n = j.n;
    out->k = j.k;
    const bool ok = j.status == GUMAP_OK;
    out->nbr_ids = ok ? j.r_ids : nullptr;
    out->nbr_hops = ok ? j.r_hops : nullptr;
    out->weights = ok && j.weights ? j.r_w : nullptr;
    out->rho = ok && j.weights ? j.r_rho : nullptr;
    out->sigma = ok && j.weights ? j.r_sigma : nullptr;
    out->t_submit_ns = j.t_submit;
    out->t_admit_ns = j.t_admit;
    out->t_start_ns = j.t_start;
    out->t_done_ns = j.t_done;
}

int gumap_poll(gumap_server *s, uint64_t ticket, gumap_result *out)
{
    if (!s || !out) return gm::set_error(GUMAP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return gm::set_error(GUMAP_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state != kDone) return GUMAP_PENDING;
    fill_result(*it->second, out);
    return it->second->status;
}

int gumap_wait(gumap_server *s, uint64_t ticket, int64_t timeout_ms, gumap_result *out)
{
    if (!s || !out) return gm::set_error(GUMAP_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return gm::set_error(GUMAP_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    std::shared_ptr<Job> j = it->second;
    auto ready = [&] { return j->state == kDone; };
    if (timeout_ms < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return GUMAP_PENDING;
    fill_result(*j, out);
    return j->status;
}

int gumap_release(gumap_server *s, uint64_t ticket)
{
    if (!s) return gm::set_error(GUMAP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return gm::set_error(GUMAP_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state != kDone) return GUMAP_PENDING;
    Job &j = *it->second;
    if (j.out_pinned) {
        s->host_alloc.release(j.out_off, j.out_bytes);
        s->cv_space.notify_all();
    }
    j.out_pinned = false;
    s->jobs.erase(it);
    s->kick = true;
    s->cv_work.notify_one();   // result space freed: admission may proceed
    return GUMAP_OK;
}

int gumap_server_get_stats(gumap_server *s, gumap_server_stats *out)
{
    if (!s || !out) return gm::set_error(GUMAP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->queued = s->queue.size();
    out->running = s->admitted.size() + s->downloading.size();
    out->resident_bytes = s->resident;
    return GUMAP_OK;
}

void gumap_server_destroy(gumap_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_space.notify_all();
    if (s->worker.joinable()) s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &kv : s->jobs) {
            Job &j = *kv.second;
            j.up_done.reset();
            j.down_done.reset();
        }
        s->jobs.clear();
        s->queue.clear();
        s->admitted.clear();
        s->downloading.clear();
    }
    if (s->no_device) {
        free(s->host_pool);
    } else {
        if (s->slab) (void)hipFree(s->slab);
        if (s->host_pool) (void)hipHostFree(s->host_pool);
        for (int i = 0; i < kInFlight; ++i) {
            if (s->d_jobs[i]) (void)hipFree(s->d_jobs[i]);
            if (s->d_chunks[i]) (void)hipFree(s->d_chunks[i]);
            if (s->d_counter[i]) (void)hipFree(s->d_counter[i]);
            if (s->h_jobs[i]) (void)hipHostFree(s->h_jobs[i]);
            if (s->h_chunks[i]) (void)hipHostFree(s->h_chunks[i]);
            if (s->iter_done[i]) (void)hipEventDestroy(s->iter_done[i]);
            if (s->table_done[i]) (void)hipEventDestroy(s->table_done[i]);
        }
        if (s->compute) (void)hipStreamDestroy(s->compute);
        if (s->copy) (void)hipStreamDestroy(s->copy);
        if (s->d2h) (void)hipStreamDestroy(s->d2h);
        if (s->meta) (void)hipStreamDestroy(s->meta);
    }
    delete s;
}

}  // extern "C"
