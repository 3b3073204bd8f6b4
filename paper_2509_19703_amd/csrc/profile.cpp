// Event-pair timing of the library's kernel launches (see gumap_profile.h).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gumap_profile.h"
#include "profile.h"

namespace gm {

namespace {

struct Pending {
    std::string name;
    hipEvent_t start = nullptr, stop = nullptr;
    double bytes = 0.0, extra = 0.0;
};

struct Totals {
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0, extra = 0.0;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<std::string> only;   // names recorded (all when empty)
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, Totals> totals;
    std::vector<std::string> order;

    hipEvent_t get_event()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        // timing events need no system-scope fence (the host reads them only
        // after the stream has drained), which keeps each record cheaper
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }
};

Profiler &prof()
{
    static Profiler p;
    return p;
}

}  // namespace

bool prof_on() { return prof().on; }

int prof_begin(const char *name, hipStream_t s)
{
    Profiler &p = prof();
    if (!p.on) return -1;
    if (!p.only.empty()) {
        bool listed = false;
        for (const std::string &o : p.only) listed |= o == name;
        if (!listed) return -1;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return -1;   // never record profiling events into a captured graph
    }
    std::lock_guard<std::mutex> lk(p.mu);
    Pending x;
    x.name = name;
    x.start = p.get_event();
    x.stop = p.get_event();
    if (!x.start || !x.stop || hipEventRecord(x.start, s) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    p.pending.push_back(x);
    return (int)p.pending.size() - 1;
}

void prof_end(int mark, hipStream_t s, double bytes)
{
    if (mark < 0) return;
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (mark >= (int)p.pending.size()) return;
    p.pending[mark].bytes = bytes;
    if (hipEventRecord(p.pending[mark].stop, s) != hipSuccess) (void)hipGetLastError();
}

void prof_set_bytes(int mark, double bytes)
{
    if (mark < 0) return;
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (mark < (int)p.pending.size()) p.pending[mark].bytes = bytes;
}

void prof_set_extra(int mark, double bytes)
{
    if (mark < 0) return;
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (mark < (int)p.pending.size()) p.pending[mark].extra = bytes;
}

void prof_resolve()
{
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    for (Pending &x : p.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(x.stop) == hipSuccess && hipEventElapsedTime(&ms, x.start, x.stop) == hipSuccess) {
            auto it = p.totals.find(x.name);
            if (it == p.totals.end()) {
                p.order.push_back(x.name);
                it = p.totals.emplace(x.name, Totals{}).first;
            }
            it->second.launches += 1;
            it->second.ms += ms;
            it->second.bytes += x.bytes;
            it->second.extra += x.extra;
        } else {
            (void)hipGetLastError();
        }
        p.pool.push_back(x.start);
        p.pool.push_back(x.stop);
    }
    p.pending.clear();
}

}  // namespace gm

extern "C" {

void gumap_profile_enable(int on) { gm::prof().on = on != 0; }

void gumap_profile_only(const char *names)
{
    gm::Profiler &p = gm::prof();
    std::lock_guard<std::mutex> lk(p.mu);
    p.only.clear();
    if (!names) return;
    std::string cur;
    for (const char *c = names;; ++c) {
        if (*c == ',' || *c == '\0') {
            if (!cur.empty()) p.only.push_back(cur);
            cur.clear();
            if (*c == '\0') break;
        } else {
            cur.push_back(*c);
        }
    }
}

void gumap_profile_reset(void)
{
    gm::Profiler &p = gm::prof();
    std::lock_guard<std::mutex> lk(p.mu);
    p.totals.clear();
    p.order.clear();
}

int gumap_profile_count(void)
{
    gm::Profiler &p = gm::prof();
    std::lock_guard<std::mutex> lk(p.mu);
    return (int)p.order.size();
}

int gumap_profile_entry(int i, const char **name, int64_t *launches, double *total_ms, double *alg_bytes)
{
    gm::Profiler &p = gm::prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (i < 0 || i >= (int)p.order.size()) return -1;
    const std::string &nm = p.order[i];
    const gm::Totals &t = p.totals[nm];
    if (name) *name = nm.c_str();
    if (launches) *launches = t.launches;
    if (total_ms) *total_ms = t.ms;
    if (alg_bytes) *alg_bytes = t.bytes;
    return 0;
}

int gumap_profile_extra(int i, double *extra_bytes)
{
    gm::Profiler &p = gm::prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (i < 0 || i >= (int)p.order.size()) return -1;
    if (extra_bytes) *extra_bytes = p.totals[p.order[i]].extra;
    return 0;
}

}  // extern "C"
