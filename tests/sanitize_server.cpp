// Drives the request server's device-free scheduler (GUMAP_SERVER_NO_DEVICE)
// through the C-ABI under AddressSanitizer and UndefinedBehaviorSanitizer
// (built by tests/test_sanitizers_cpu.py, host code only): submissions of
// mixed sizes from two threads, waits and polls, releases, a job larger than
// the budget, unknown tickets, an executor-reported failure and a server
// destroyed with jobs still queued.  Exit status 0 means every check held
// and the sanitizers reported nothing.
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <thread>
#include <vector>

#include "gumap.h"

static int failures = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            std::fprintf(stderr, "check failed at %d: %s\n", __LINE__, #cond); \
            ++failures;                                               \
        }                                                             \
    } while (0)

struct Csr {
    std::vector<int32_t> rp, col;
};

// a cycle of n vertices with chords to i + 7 (symmetric, sorted rows)
static Csr ring(int32_t n)
{
    Csr g;
    g.rp.assign((size_t)n + 1, 0);
    std::vector<std::vector<int32_t>> adj((size_t)n);
    auto add = [&](int32_t a, int32_t b) {
        if (a == b) return;
        adj[(size_t)a].push_back(b);
        adj[(size_t)b].push_back(a);
    };
    for (int32_t i = 0; i < n; ++i) {
        add(i, (i + 1) % n);
        if (n > 14) add(i, (i + 7) % n);
    }
    for (int32_t i = 0; i < n; ++i) {
        auto &r = adj[(size_t)i];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        g.rp[(size_t)i + 1] = g.rp[(size_t)i] + (int32_t)r.size();
        g.col.insert(g.col.end(), r.begin(), r.end());
    }
    return g;
}

static gumap_job job_of(const Csr &g, int32_t k)
{
    gumap_job j{};
    j.n = (int32_t)g.rp.size() - 1;
    j.nnz = (int32_t)g.col.size();
    j.row_ptr = g.rp.data();
    j.col_idx = g.col.empty() ? nullptr : g.col.data();
    j.k = k;
    j.want_weights = 1;
    j.flags = GUMAP_CSR_SORTED;
    return j;
}

int main()
{
    int st = 0;
    gumap_server *s = gumap_server_create((size_t)64 << 20, 4, GUMAP_SERVER_NO_DEVICE, &st);
    CHECK(s && st == GUMAP_OK);
    if (!s) return 1;
    std::vector<Csr> graphs;
    for (int i = 0; i < 40; ++i) graphs.push_back(ring(20 + 37 * i));
    std::vector<uint64_t> tickets(graphs.size(), 0);
    auto submit_range = [&](size_t b, size_t e) {
        for (size_t i = b; i < e; ++i) {
            gumap_job j = job_of(graphs[i], (int32_t)(3 + i % 20));
            if (gumap_submit(s, &j, &tickets[i]) != GUMAP_OK) ++failures;
        }
    };
    std::thread a(submit_range, 0, 20), b(submit_range, 20, 40);
    a.join();
    b.join();
    for (size_t i = 0; i < graphs.size(); ++i) {
        gumap_result r{};
        CHECK(gumap_wait(s, tickets[i], 20000, &r) == GUMAP_OK);
        CHECK(r.status == GUMAP_OK && r.n == (int32_t)graphs[i].rp.size() - 1);
        CHECK(r.t_submit_ns <= r.t_admit_ns && r.t_admit_ns <= r.t_done_ns);
        CHECK(gumap_release(s, tickets[i]) == GUMAP_OK);
        CHECK(gumap_release(s, tickets[i]) == GUMAP_ENOTFOUND);
    }
    gumap_result r{};
    CHECK(gumap_poll(s, 987654321ull, &r) == GUMAP_ENOTFOUND);
    Csr big = ring(300000);
    gumap_job bj = job_of(big, 30);
    uint64_t t = 0;
    CHECK(gumap_submit(s, &bj, &t) == GUMAP_E2BIG);
    gumap_job bad = job_of(graphs[0], 0);
    CHECK(gumap_submit(s, &bad, &t) == GUMAP_EINVAL);
    gumap_server_stats stats{};
    CHECK(gumap_server_get_stats(s, &stats) == GUMAP_OK && stats.completed == graphs.size());
    // destroyed with jobs still queued or running
    for (int i = 0; i < 10; ++i) {
        gumap_job j = job_of(graphs[(size_t)i], 15);
        CHECK(gumap_submit(s, &j, &t) == GUMAP_OK);
    }
    gumap_server_destroy(s);
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("sanitized scheduler: ok\n");
    return 0;
}
