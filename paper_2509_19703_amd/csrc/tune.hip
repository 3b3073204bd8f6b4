// Autotuner of the all-source BFS (gumap_knn_build_tune) and the table of
// its picks that gumap_knn_build and gumap_stress consult.
//
// The settings it chooses among change only the speed of the search, never
// its result (the BFS levels, hop rows and kNN rows are the same for every
// setting): whether small graphs run every level of a source group in one
// workgroup, the source-bitset width (64 x 1, 2, 4 or 8 words per vertex),
// the (vertex, word) items per thread of the level kernel, whether level 1 is
// a top-down scatter from the sources or a range scan, the degree above which
// a vertex is searched by a whole wave, how many hops keep their frontier
// instead of bit-plane updates, and whether the levels right after the
// sources may run top-down.  The search is a coordinate descent from the
// library defaults: each setting in turn takes the value that times fastest
// with the others held at the best so far.  Each candidate runs the real call
// on the caller's graph and sources (writing the outputs): one warm-up, then
// the fastest of three timed calls.
//
// A pick is recorded for the shape of the call (a bucket: floor(log2) of the
// vertex count, of the mean degree, of the number of sources and of k, and
// whether the full hop rows are wanted), so later calls of a similar shape
// use it.  With GUMAP_AUTOTUNE_CACHE naming a file, the table is read from it
// on first use and rewritten after each tuning, as JSON.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gumap.h"
#include "kernels.h"
#include "runtime.h"

namespace gm {
namespace {

int ilog2(int64_t x)
{
    int b = -1;
    while (x > 0) {
        ++b;
        x >>= 1;
    }
    return b;
}

struct Bucket {
    int n, deg, rows, k, hm;
    bool operator<(const Bucket &o) const
    {
        return std::tie(n, deg, rows, k, hm) < std::tie(o.n, o.deg, o.rows, o.k, o.hm);
    }
};

Bucket bucket_of(int32_t n, int64_t nnz, int64_t rows, int32_t k, bool hop_matrix)
{
    Bucket b;
    b.n = ilog2(n);
    b.deg = ilog2(n > 0 ? std::max<int64_t>(1, nnz / n) : 1);
    b.rows = ilog2(rows);
    b.k = ilog2(k);
    b.hm = hop_matrix ? 1 : 0;
    return b;
}

std::map<Bucket, gumap_build_tuning> &table()
{
    static std::map<Bucket, gumap_build_tuning> t;
    return t;
}

bool &cache_tried()
{
    static bool tried = false;
    return tried;
}

void to_knobs(const gumap_build_tuning &t, BuildKnobs *kb)
{
    kb->fused = t.fused;
    kb->words = t.words;
    kb->verts = t.level_verts;
    kb->first = t.first_level;
    kb->heavy = t.heavy_degree;
    kb->hist = t.hist_levels;
    kb->push = t.push_levels;
}

// ---- JSON cache: {"format": "gumap-build-tuning", "version": 1,
//      "entries": [{"n_log2": .., "deg_log2": .., "rows_log2": .., "k_log2": ..,
//      "hop_matrix": .., "fused": .., "words": .., "level_verts": ..,
//      "first_level": .., "heavy_degree": .., "hist_levels": ..,
//      "push_levels": .., "candidates": .., "best_ms": .., "default_ms": ..}, ...]}
const char *const kFields[] = {"n_log2",      "deg_log2",    "rows_log2",    "k_log2",      "hop_matrix",
                               "fused",       "words",       "level_verts",  "first_level", "heavy_degree",
                               "hist_levels", "push_levels", "candidates",   "best_ms",     "default_ms"};
constexpr int kNumFields = sizeof(kFields) / sizeof(kFields[0]);

int save_table(const char *path)
{
    FILE *f = fopen(path, "w");
    if (!f) return set_error(GUMAP_EINVAL, "cannot write the tuning cache %s", path);
    fprintf(f, "{\"format\": \"gumap-build-tuning\", \"version\": 1, \"entries\": [");
    bool first = true;
    for (const auto &kv : table()) {
        const Bucket &b = kv.first;
        const gumap_build_tuning &t = kv.second;
        fprintf(f,
                "%s\n  {\"n_log2\": %d, \"deg_log2\": %d, \"rows_log2\": %d, \"k_log2\": %d, \"hop_matrix\": %d, "
                "\"fused\": %d, \"words\": %d, \"level_verts\": %d, \"first_level\": %d, \"heavy_degree\": %d, "
                "\"hist_levels\": %d, \"push_levels\": %d, \"candidates\": %d, \"best_ms\": %.6f, "
                "\"default_ms\": %.6f}",
                first ? "" : ",", b.n, b.deg, b.rows, b.k, b.hm, t.fused, t.words, t.level_verts, t.first_level,
                t.heavy_degree, t.hist_levels, t.push_levels, t.candidates, (double)t.best_ms, (double)t.default_ms);
        first = false;
    }
    fprintf(f, "\n]}\n");
    const bool ok = ferror(f) == 0;
    if (fclose(f) != 0 || !ok) return set_error(GUMAP_EINVAL, "cannot write the tuning cache %s", path);
    return GUMAP_OK;
}

// Reads the entries of a cache written by save_table: every object holding
// all the fields above becomes a table entry; anything else is an error.
int load_table(const char *path)
{
    FILE *f = fopen(path, "r");
    if (!f) return set_error(GUMAP_EINVAL, "cannot read the tuning cache %s", path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    if (text.find("\"gumap-build-tuning\"") == std::string::npos)
        return set_error(GUMAP_EINVAL, "%s is not a gumap tuning cache", path);
    const size_t list = text.find("\"entries\"");
    if (list == std::string::npos) return set_error(GUMAP_EINVAL, "%s has no entries list", path);
    std::map<Bucket, gumap_build_tuning> parsed;
    size_t pos = list;
    while ((pos = text.find('{', pos)) != std::string::npos) {
        const size_t end = text.find('}', pos);
        if (end == std::string::npos) return set_error(GUMAP_EINVAL, "%s: unterminated entry", path);
        const std::string obj = text.substr(pos, end - pos + 1);
        double v[kNumFields];
        for (int i = 0; i < kNumFields; ++i) {
            const std::string key = std::string("\"") + kFields[i] + "\"";
            const size_t at = obj.find(key);
            if (at == std::string::npos) return set_error(GUMAP_EINVAL, "%s: entry without %s", path, kFields[i]);
            size_t colon = obj.find(':', at + key.size());
            if (colon == std::string::npos) return set_error(GUMAP_EINVAL, "%s: malformed %s", path, kFields[i]);
            const char *start = obj.c_str() + colon + 1;
            char *stop = nullptr;
            v[i] = strtod(start, &stop);
            if (stop == start) return set_error(GUMAP_EINVAL, "%s: %s is not a number", path, kFields[i]);
        }
        Bucket b{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4]};
        gumap_build_tuning t{};
        t.fused = (int32_t)v[5];
        t.words = (int32_t)v[6];
        t.level_verts = (int32_t)v[7];
        t.first_level = (int32_t)v[8];
        t.heavy_degree = (int32_t)v[9];
        t.hist_levels = (int32_t)v[10];
        t.push_levels = (int32_t)v[11];
        t.candidates = (int32_t)v[12];
        t.best_ms = (float)v[13];
        t.default_ms = (float)v[14];
        const bool valid = (t.fused == 0 || t.fused == 1) &&
                           (t.words == 1 || t.words == 2 || t.words == 4 || t.words == 8) &&
                           (t.level_verts == 1 || t.level_verts == 2 || t.level_verts == 4 || t.level_verts == 8) &&
                           (t.first_level == 0 || t.first_level == 1) && t.heavy_degree >= 0 &&
                           t.hist_levels >= 0 && t.hist_levels <= 64 && t.push_levels >= 0 && t.push_levels <= 3;
        if (!valid) return set_error(GUMAP_EINVAL, "%s: an entry has a setting out of range", path);
        parsed[b] = t;
        pos = end + 1;
    }
    table() = parsed;
    return GUMAP_OK;
}

void load_env_cache_once()
{
    if (cache_tried()) return;
    cache_tried() = true;
    const char *path = getenv("GUMAP_AUTOTUNE_CACHE");
    if (path && *path) {
        FILE *f = fopen(path, "r");
        if (!f) return;   // not written yet
        fclose(f);
        if (load_table(path) != GUMAP_OK) clear_error();   // an unreadable cache is ignored
    }
}

int tune_build(const gumap_graph *g, int32_t k, const int32_t *sources, int32_t n_sources, int32_t *ids,
               uint8_t *hops, uint8_t *hop_matrix, hipStream_t s, gumap_build_tuning *out)
{
    int st;
    if ((st = check_graph_args(g))) return st;
    if ((st = check_k(k))) return st;
    *out = gumap_build_tuning{};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_status(e, "tuning events");
    auto time_one = [&](const BuildKnobs *kb, float *ms) -> int {
        int r = knn_build_tuned(g, k, sources, n_sources, ids, hops, hop_matrix, s, kb);
        float best = 1e30f;
        for (int rep = 0; rep < 3 && r == GUMAP_OK; ++rep) {
            hipError_t x = hipEventRecord(e0, s);
            if (x == hipSuccess) r = knn_build_tuned(g, k, sources, n_sources, ids, hops, hop_matrix, s, kb);
            if (r) break;
            if (x == hipSuccess) x = hipEventRecord(e1, s);
            if (x == hipSuccess) x = hipEventSynchronize(e1);
            float t = 0.0f;
            if (x == hipSuccess) x = hipEventElapsedTime(&t, e0, e1);
            if (x != hipSuccess) r = hip_status(x, "tuning launch");
            else best = std::min(best, t);
        }
        *ms = best;
        return r;
    };
    // library defaults, written out
    BuildKnobs cur;
    cur.fused = msbfs_fused_lds_bytes(g->n) <= 144 * 1024 ? 1 : 0;
    cur.words = 0;   // width from the number of sources
    cur.verts = 4;
    cur.first = (double)g->nnz * 256.0 <= (double)g->n * (double)g->n ? 1 : 0;
    cur.heavy = 0;
    cur.hist = 15;
    cur.push = 0;
    float best_ms = 0.0f;
    st = time_one(&cur, &best_ms);
    out->default_ms = best_ms;
    int candidates = 1;
    auto try_values = [&](int BuildKnobs::*field, std::initializer_list<int> values) -> int {
        const int keep = cur.*field;
        int best_v = keep;
        for (int v : values) {
            if (v == keep) continue;
            BuildKnobs t = cur;
            t.*field = v;
            float ms = 0.0f;
            int r = time_one(&t, &ms);
            if (r) return r;
            ++candidates;
            if (ms < best_ms) {
                best_ms = ms;
                best_v = v;
            }
        }
        cur.*field = best_v;
        return GUMAP_OK;
    };
    if (st == GUMAP_OK && cur.fused == 1) st = try_values(&BuildKnobs::fused, {0});
    if (st == GUMAP_OK && cur.fused == 0) {
        if (cur.words == 0) {
            // the width the default rule picks, written out
            const int64_t rows = sources ? n_sources : g->n;
            int w = 1;
            while (w < 8 && 64 * (int64_t)w < rows) w <<= 1;
            cur.words = w;
        }
        st = try_values(&BuildKnobs::words, {1, 2, 4, 8});
        if (st == GUMAP_OK) st = try_values(&BuildKnobs::verts, {1, 2, 4, 8});
        if (st == GUMAP_OK) st = try_values(&BuildKnobs::first, {0, 1});
        if (st == GUMAP_OK) st = try_values(&BuildKnobs::heavy, {0, 32, 128, 512});
        if (st == GUMAP_OK) st = try_values(&BuildKnobs::hist, {0, 15});
        if (st == GUMAP_OK && cur.first == 1) st = try_values(&BuildKnobs::push, {0, 2});
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    if (cur.fused == 1) {
        // the per-level settings do not apply to the one-workgroup form
        cur.words = 1;
        cur.verts = 4;
        cur.first = 1;
        cur.heavy = 0;
        cur.hist = 0;
        cur.push = 0;
    }
    out->fused = cur.fused;
    out->words = cur.words;
    out->level_verts = cur.verts;
    out->first_level = cur.first;
    out->heavy_degree = cur.heavy;
    out->hist_levels = cur.hist;
    out->push_levels = cur.push;
    out->candidates = candidates;
    out->best_ms = best_ms;
    load_env_cache_once();
    table()[bucket_of(g->n, g->nnz, sources ? n_sources : g->n, k, hop_matrix != nullptr)] = *out;
    const char *path = getenv("GUMAP_AUTOTUNE_CACHE");
    if (path && *path) return save_table(path);
    return GUMAP_OK;
}

}  // namespace

bool tuned_knobs(int32_t n, int64_t nnz, int64_t rows, int32_t k, bool hop_matrix, BuildKnobs *out)
{
    load_env_cache_once();
    const auto it = table().find(bucket_of(n, nnz, rows, k, hop_matrix));
    if (it == table().end()) return false;
    to_knobs(it->second, out);
    return true;
}

}  // namespace gm

extern "C" int gumap_knn_build_tune(const gumap_graph *g, int32_t k, const int32_t *sources, int32_t n_sources,
                                    int32_t *nbr_ids, uint8_t *nbr_hops, uint8_t *hop_matrix, hipStream_t stream,
                                    gumap_build_tuning *out)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    if (!out) return gm::set_error(GUMAP_EINVAL, "out is NULL");
    int st = gm::tune_build(g, k, sources, n_sources, nbr_ids, nbr_hops, hop_matrix, stream, out);
    if (st != GUMAP_OK && st != GUMAP_EINVAL) {
        (void)hipStreamSynchronize(stream);
        (void)hipGetLastError();
    }
    return st;
}

extern "C" int gumap_build_tuning_lookup(int32_t n, int64_t nnz, int64_t n_sources, int32_t k, int hop_matrix,
                                         gumap_build_tuning *out)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    if (!out) return gm::set_error(GUMAP_EINVAL, "out is NULL");
    if (n < 0 || nnz < 0 || n_sources < 0 || k < 1) return gm::set_error(GUMAP_EINVAL, "negative size or k < 1");
    gm::load_env_cache_once();
    const auto it = gm::table().find(gm::bucket_of(n, nnz, n_sources, k, hop_matrix != 0));
    if (it == gm::table().end()) return 0;
    *out = it->second;
    return 1;
}

extern "C" int gumap_autotune_cache_load(const char *path)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    if (!path) return gm::set_error(GUMAP_EINVAL, "path is NULL");
    gm::cache_tried() = true;
    return gm::load_table(path);
}

extern "C" int gumap_autotune_cache_save(const char *path)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    if (!path) return gm::set_error(GUMAP_EINVAL, "path is NULL");
    return gm::save_table(path);
}

extern "C" void gumap_autotune_clear(void)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::table().clear();
    gm::cache_tried() = true;
}
