// Request server: continuous batching of layout-preparation jobs
// (partial-BFS kNN + membership per job graph) on one device.
//
// Jobs arrive through gumap_submit with host CSR arrays, which are copied at
// once.  A scheduler thread admits queued jobs first-come-first-served while
// their device bytes fit the budget (and a slot is free), copies their CSR
// into a device slab that was reserved once at creation, and runs device
// iterations: each iteration is one launch of the jobs kernel over a list of
// row chunks taken from every admitted job that still has rows to do, up to
// a row budget per iteration, oldest job first.  Jobs admitted while an
// iteration runs join the next one.  When all rows of a job are done its
// results are copied to host buffers, its slab space is returned and it is
// marked done.  Every row of a job is computed by the same per-row code
// whatever else shares the launch, so a result does not depend on the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
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

// First-fit allocator over [0, capacity) of the slab.
class SlabAllocator {
public:
    explicit SlabAllocator(size_t capacity) { if (capacity) free_[0] = capacity; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes, 256);
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

enum JobState { kQueued, kRunning, kDone };

struct Job {
    uint64_t ticket = 0;
    JobState state = kQueued;
    int status = GUMAP_OK;
    int32_t n = 0, nnz = 0, k = 0;
    bool weights = false;
    uint32_t flags = 0;
    std::vector<int32_t> h_rp, h_col;                 // host input copy
    std::vector<int32_t> r_ids;                       // host results
    std::vector<uint8_t> r_hops;
    std::vector<float> r_w, r_rho, r_sigma;
    size_t bytes = 0, slab_off = 0;
    int32_t next_row = 0, rows_done = 0;              // scheduling progress
    gm::DevJob dev{};
    uint64_t t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
};

// Device bytes a job holds while resident.
size_t job_bytes(int32_t n, int32_t nnz, int32_t k, bool weights, bool sorted)
{
    size_t b = align_up((size_t)(n + 1) * 4, 256) + align_up((size_t)std::max(nnz, 1) * 4, 256);
    b += align_up((size_t)n * k * 4, 256) + align_up((size_t)n * k, 256);
    if (weights) b += align_up((size_t)n * k * 4, 256) + 2 * align_up((size_t)n * 4, 256);
    if (!sorted) {
        b += align_up((size_t)(n + 1) * 4, 256) + align_up((size_t)std::max(nnz, 1) * 4, 256);
        b += align_up(gm::canon_scratch_bytes(n, nnz), 256) + 512;
    }
    return b;
}

}  // namespace

struct gumap_server {
    size_t budget = 0;
    int32_t max_slots = 0;
    bool no_device = false;
    int device = 0;
    char *slab = nullptr;
    SlabAllocator alloc{0};
    hipStream_t compute = nullptr, copy = nullptr;
    hipEvent_t iter_done = nullptr;
    gm::DevJob *d_jobs = nullptr;            // job table of the running iteration
    gm::JobChunk *d_chunks = nullptr;
    unsigned long long *d_counter = nullptr;
    gm::DevJob *h_jobs = nullptr;            // pinned staging
    gm::JobChunk *h_chunks = nullptr;
    int32_t table_cap = 0, chunk_cap = 0;
    int64_t iter_rows = 0;
    int blocks = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Job>> queue;               // waiting for admission
    std::vector<std::shared_ptr<Job>> running;            // admitted, rows pending or in flight
    std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    gumap_server_stats stats{};
    size_t resident = 0;
    std::string fatal;

    void run();
    bool admit_locked(std::vector<std::shared_ptr<Job>> &admitted);
    int stage_job(Job &j);
    void finish_job(const std::shared_ptr<Job> &j, int status);
};

int gumap_server::stage_job(Job &j)
{
    // called without the lock; j is owned by the scheduler while running
    if (no_device) return GUMAP_OK;
    hipError_t e = hipSuccess;
    char *base = slab + j.slab_off;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += align_up(bytes, 256);
        return p;
    };
    int32_t *rp = (int32_t *)take((size_t)(j.n + 1) * 4);
    int32_t *col = (int32_t *)take((size_t)std::max(j.nnz, 1) * 4);
    j.dev.ids = (int32_t *)take((size_t)j.n * j.k * 4);
    j.dev.hops = (uint8_t *)take((size_t)j.n * j.k);
    j.dev.weights = nullptr;
    j.dev.rho = j.dev.sigma = nullptr;
    if (j.weights) {
        j.dev.weights = (float *)take((size_t)j.n * j.k * 4);
        j.dev.rho = (float *)take((size_t)j.n * 4);
        j.dev.sigma = (float *)take((size_t)j.n * 4);
    }
    j.dev.n = j.n;
    j.dev.k = j.k;
    e = hipMemcpyAsync(rp, j.h_rp.data(), (size_t)(j.n + 1) * 4, hipMemcpyHostToDevice, copy);
    if (e == hipSuccess && j.nnz)
        e = hipMemcpyAsync(col, j.h_col.data(), (size_t)j.nnz * 4, hipMemcpyHostToDevice, copy);
    if (e != hipSuccess) return gm::hip_status(e, "job upload");
    j.dev.row_ptr = rp;
    j.dev.col = col;
    if (!(j.flags & GUMAP_CSR_SORTED) || (j.flags & GUMAP_VALIDATE)) {
        int32_t *crp = (int32_t *)take((size_t)(j.n + 1) * 4);
        int32_t *ccol = (int32_t *)take((size_t)std::max(j.nnz, 1) * 4);
        void *scratch = take(gm::canon_scratch_bytes(j.n, j.nnz));
        int *err = (int *)scratch;  // structural check uses the first word of the canon scratch
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
            // symmetry (and order, when claimed) of the canonical rows
            int *err2 = (int *)(base + off);
            (void)take(256);
            e = hipMemsetAsync(err2, 0, sizeof(int), copy);
            if (e == hipSuccess) e = gm::launch_check_symmetric(j.n, j.dev.row_ptr, j.dev.col, err2, copy);
            int bad = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(&bad, err2, sizeof(int), hipMemcpyDeviceToHost, copy);
            if (e == hipSuccess) e = hipStreamSynchronize(copy);
            if (e != hipSuccess) return gm::hip_status(e, "job validate");
            if (bad) return gm::set_error(GUMAP_EGRAPH, "CSR is not symmetric");
        }
    }
    return GUMAP_OK;
}

bool gumap_server::admit_locked(std::vector<std::shared_ptr<Job>> &admitted)
{
    bool any = false;
    while (!queue.empty()) {
        auto &j = queue.front();
        if (max_slots > 0 && (int32_t)running.size() + (int32_t)admitted.size() >= max_slots) break;
        size_t off = 0;
        if (resident + j->bytes > budget || !alloc.alloc(j->bytes, &off)) break;  // FIFO: no overtaking
        j->slab_off = off;
        resident += j->bytes;
        stats.peak_resident_bytes = std::max<uint64_t>(stats.peak_resident_bytes, resident);
        j->state = kRunning;
        j->t_admit = now_ns();
        admitted.push_back(j);
        queue.pop_front();
        any = true;
    }
    return any;
}

void gumap_server::finish_job(const std::shared_ptr<Job> &j, int status)
{
    // lock held by caller
    j->status = status;
    j->state = kDone;
    j->t_done = now_ns();
    resident -= j->bytes;
    alloc.release(j->slab_off, j->bytes);
    j->h_rp.clear();
    j->h_rp.shrink_to_fit();
    j->h_col.clear();
    j->h_col.shrink_to_fit();
    if (status == GUMAP_OK) stats.completed++;
    else stats.failed++;
    cv_done.notify_all();
}

void gumap_server::run()
{
    if (!no_device) (void)hipSetDevice(device);
    bool iteration_running = false;
    for (;;) {
        std::vector<std::shared_ptr<Job>> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (!iteration_running) {
                cv_work.wait_for(lk, std::chrono::milliseconds(2), [&] {
                    return stop || !queue.empty() || !running.empty();
                });
            }
            if (stop && !iteration_running) break;
            admit_locked(admitted);
        }
        // stage admitted jobs (uploads overlap the running iteration)
        for (auto &j : admitted) {
            int st = stage_job(*j);
            std::lock_guard<std::mutex> lk(mu);
            if (st != GUMAP_OK) {
                finish_job(j, st);
            } else {
                running.push_back(j);
            }
        }
        if (iteration_running) {
            if (!no_device) {
                hipError_t q = hipEventQuery(iter_done);
                if (q == hipErrorNotReady) {
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
                    continue;
                }
                if (q != hipSuccess) {
                    std::lock_guard<std::mutex> lk(mu);
                    fatal = hipGetErrorString(q);
                    for (auto &j : running) finish_job(j, GUMAP_EDEVICE);
                    running.clear();
                    iteration_running = false;
                    continue;
                }
            }
            iteration_running = false;
        }
        // No iteration is in flight now: every scheduled row is complete, so
        // jobs whose rows were all scheduled are finished.
        std::vector<std::shared_ptr<Job>> finished;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &j : running)
                if (j->rows_done >= j->n) finished.push_back(j);
        }
        for (auto &j : finished) {
            int st = GUMAP_OK;
            size_t nk = (size_t)j->n * j->k;
            j->r_ids.resize(nk);
            j->r_hops.resize(nk);
            if (j->weights) {
                j->r_w.resize(nk);
                j->r_rho.resize(j->n);
                j->r_sigma.resize(j->n);
            }
            if (!no_device && j->n > 0) {
                hipError_t e = hipMemcpyAsync(j->r_ids.data(), j->dev.ids, nk * 4, hipMemcpyDeviceToHost, copy);
                if (e == hipSuccess) e = hipMemcpyAsync(j->r_hops.data(), j->dev.hops, nk, hipMemcpyDeviceToHost, copy);
                if (e == hipSuccess && j->weights) {
                    e = hipMemcpyAsync(j->r_w.data(), j->dev.weights, nk * 4, hipMemcpyDeviceToHost, copy);
                    if (e == hipSuccess) e = hipMemcpyAsync(j->r_rho.data(), j->dev.rho, (size_t)j->n * 4, hipMemcpyDeviceToHost, copy);
                    if (e == hipSuccess) e = hipMemcpyAsync(j->r_sigma.data(), j->dev.sigma, (size_t)j->n * 4, hipMemcpyDeviceToHost, copy);
                }
                if (e == hipSuccess) e = hipStreamSynchronize(copy);
                if (e != hipSuccess) st = gm::hip_status(e, "job download");
            }
            std::lock_guard<std::mutex> lk(mu);
            running.erase(std::remove(running.begin(), running.end(), j), running.end());
            finish_job(j, st);
        }
        // next iteration: chunks from every running job with rows left
        std::vector<std::shared_ptr<Job>> table;
        std::vector<gm::JobChunk> chunks;
        int max_k = 1;
        {
            std::lock_guard<std::mutex> lk(mu);
            int64_t rows_left = iter_rows;
            for (auto &j : running) {
                if (j->next_row >= j->n || rows_left <= 0) continue;
                if ((int32_t)table.size() >= table_cap) break;
                const int32_t job_idx = (int32_t)table.size();
                const int32_t step = gm::batch_chunk_rows(j->k);
                int32_t r = j->next_row;
                while (r < j->n && rows_left > 0 && (int32_t)chunks.size() < chunk_cap) {
                    int32_t e = std::min(j->n, r + step);
                    chunks.push_back(gm::JobChunk{job_idx, r, e, 0});
                    rows_left -= e - r;
                    r = e;
                }
                if (r == j->next_row) break;
                if (j->t_start == 0) j->t_start = now_ns();
                table.push_back(j);
                max_k = std::max(max_k, j->k);
                j->rows_done += r - j->next_row;   // counted done once this iteration completes
                j->next_row = r;
            }
            if (!chunks.empty()) stats.iterations++;
        }
        if (chunks.empty()) continue;
        if (!no_device) {
            for (size_t i = 0; i < table.size(); ++i) h_jobs[i] = table[i]->dev;
            std::copy(chunks.begin(), chunks.end(), h_chunks);
            hipError_t e = hipStreamSynchronize(copy);   // staged uploads must land first
            if (e == hipSuccess) e = hipMemcpyAsync(d_jobs, h_jobs, table.size() * sizeof(gm::DevJob), hipMemcpyHostToDevice, compute);
            if (e == hipSuccess) e = hipMemcpyAsync(d_chunks, h_chunks, chunks.size() * sizeof(gm::JobChunk), hipMemcpyHostToDevice, compute);
            if (e == hipSuccess) e = gm::launch_batch_reset(d_counter, compute);
            if (e == hipSuccess)
                e = gm::launch_partial_jobs(d_jobs, d_chunks, (int32_t)chunks.size(), max_k, d_counter, blocks, compute);
            if (e == hipSuccess) e = hipEventRecord(iter_done, compute);
            if (e != hipSuccess) {
                std::lock_guard<std::mutex> lk(mu);
                fatal = hipGetErrorString(e);
                for (auto &j : running) finish_job(j, GUMAP_EDEVICE);
                running.clear();
                continue;
            }
        }
        iteration_running = true;
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
    s->alloc = SlabAllocator(hbm_budget_bytes);
    s->stats.budget_bytes = hbm_budget_bytes;
    s->iter_rows = (int64_t)gm::env_size("GUMAP_SERVE_ITER_ROWS", 1 << 20);
    s->table_cap = 4096;
    s->chunk_cap = (int32_t)std::min<int64_t>(1 << 22, s->iter_rows + s->table_cap);
    if (!s->no_device) {
        hipError_t e = hipGetDevice(&s->device);
        if (e == hipSuccess) e = hipMalloc((void **)&s->slab, hbm_budget_bytes);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->iter_done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc((void **)&s->d_jobs, (size_t)s->table_cap * sizeof(gm::DevJob));
        if (e == hipSuccess) e = hipMalloc((void **)&s->d_chunks, (size_t)s->chunk_cap * sizeof(gm::JobChunk));
        if (e == hipSuccess) e = hipMalloc((void **)&s->d_counter, 256);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_jobs, (size_t)s->table_cap * sizeof(gm::DevJob), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_chunks, (size_t)s->chunk_cap * sizeof(gm::JobChunk), hipHostMallocDefault);
        if (e != hipSuccess) {
            int st = gm::hip_status(e, "server setup");
            (void)hipGetLastError();
            if (s->slab) (void)hipFree(s->slab);
            if (s->d_jobs) (void)hipFree(s->d_jobs);
            if (s->d_chunks) (void)hipFree(s->d_chunks);
            if (s->d_counter) (void)hipFree(s->d_counter);
            if (s->h_jobs) (void)hipHostFree(s->h_jobs);
            if (s->h_chunks) (void)hipHostFree(s->h_chunks);
            if (s->iter_done) (void)hipEventDestroy(s->iter_done);
            if (s->compute) (void)hipStreamDestroy(s->compute);
            if (s->copy) (void)hipStreamDestroy(s->copy);
            delete s;
            return fail(st);
        }
        s->blocks = gm::partial_batch_max_blocks();
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
    j->n = job->n;
    j->nnz = job->nnz;
    j->k = job->k;
    j->weights = job->want_weights != 0;
    j->flags = job->flags;
    const bool needs_canon = !(job->flags & GUMAP_CSR_SORTED) || (job->flags & GUMAP_VALIDATE);
    j->bytes = job_bytes(j->n, j->nnz, j->k, j->weights, !needs_canon);
    if (j->bytes > s->budget)
        return gm::set_error(GUMAP_E2BIG, "job needs %zu device bytes, budget is %zu", j->bytes, s->budget);
    j->h_rp.assign(job->row_ptr, job->row_ptr + (job->n > 0 ? job->n + 1 : 0));
    if (job->n == 0) j->h_rp.assign(1, 0);
    if (job->nnz) j->h_col.assign(job->col_idx, job->col_idx + job->nnz);
    j->t_submit = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    j->ticket = s->next_ticket++;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    s->stats.submitted++;
    *ticket = j->ticket;
    s->cv_work.notify_one();
    return GUMAP_OK;
}

static void fill_result(const Job &j, gumap_result *out)
{
    out->status = j.status;
    out->n = j.n;
    out->k = j.k;
    const bool ok = j.status == GUMAP_OK;
    out->nbr_ids = ok ? j.r_ids.data() : nullptr;
    out->nbr_hops = ok ? j.r_hops.data() : nullptr;
    out->weights = ok && j.weights ? j.r_w.data() : nullptr;
    out->rho = ok && j.weights ? j.r_rho.data() : nullptr;
    out->sigma = ok && j.weights ? j.r_sigma.data() : nullptr;
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
    s->jobs.erase(it);
    return GUMAP_OK;
}

int gumap_server_get_stats(gumap_server *s, gumap_server_stats *out)
{
    if (!s || !out) return gm::set_error(GUMAP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->queued = s->queue.size();
    out->running = s->running.size();
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
    if (s->worker.joinable()) s->worker.join();
    if (!s->no_device) {
        (void)hipStreamSynchronize(s->compute);
        (void)hipStreamSynchronize(s->copy);
        (void)hipFree(s->slab);
        (void)hipFree(s->d_jobs);
        (void)hipFree(s->d_chunks);
        (void)hipFree(s->d_counter);
        (void)hipHostFree(s->h_jobs);
        (void)hipHostFree(s->h_chunks);
        (void)hipEventDestroy(s->iter_done);
        (void)hipStreamDestroy(s->compute);
        (void)hipStreamDestroy(s->copy);
    }
    delete s;
}

}  // extern "C"
