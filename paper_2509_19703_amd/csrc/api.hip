// C-ABI of libgumap: argument checks, scratch management and the launch
// sequences of the plain calls (gumap_knn_build, gumap_knn_partial,
// gumap_membership), of the batched call and its captured plan, of the
// drawing metrics (gumap_stress, gumap_neighborhood), of the layout step
// (gumap_fuzzy_union, gumap_edge_shuffle, gumap_grad_sample,
// gumap_spectral_layout) and of the sparsifier (gumap_effective_resistance,
// gumap_sparsify_select).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gumap.h"
#include "kernels.h"
#include "profile.h"
#include "runtime.h"
#include "util.h"

namespace gm {

// ------------------------------------------------------------ errors ---
static thread_local std::string t_error;

int set_error(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_error = buf;
    return status;
}

void clear_error() { t_error.clear(); }
const char *last_error() { return t_error.c_str(); }

int hip_status(hipError_t e, const char *what)
{
    if (e == hipSuccess) return GUMAP_OK;
    if (e == hipErrorOutOfMemory) return set_error(GUMAP_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return set_error(GUMAP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// --------------------------------------------------------- scratch -----
std::mutex &api_mutex()
{
    static std::mutex m;
    return m;
}

namespace {

struct DeviceScratch {
    void *ptr[kScratchSlots] = {};
    size_t size[kScratchSlots] = {};
    void *host = nullptr;
    size_t host_size = 0;
    hipStream_t side = nullptr;          // default priority; copies that overlap the caller's kernels
    hipEvent_t ev_ready = nullptr, ev_copied = nullptr;
};

DeviceScratch &scratch_of(int dev)
{
    static DeviceScratch per_dev[64];
    return per_dev[dev & 63];
}

}  // namespace

int scratch_get(int slot, size_t bytes, void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    DeviceScratch &d = scratch_of(dev);
    if (bytes == 0) bytes = 256;
    if (d.size[slot] < bytes) {
        if (d.ptr[slot]) {
            (void)hipDeviceSynchronize();
            (void)hipFree(d.ptr[slot]);
            d.ptr[slot] = nullptr;
            d.size[slot] = 0;
        }
        size_t want = bytes + bytes / 8;
        e = hipMalloc(&d.ptr[slot], want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            d.ptr[slot] = nullptr;
            return set_error(GUMAP_ENOMEM, "device scratch of %zu bytes: %s", want, hipGetErrorString(e));
        }
        d.size[slot] = want;
    }
    *out = d.ptr[slot];
    return GUMAP_OK;
}

// The current device's side stream and its two events (created on first use).
int side_stream_get(hipStream_t *side, hipEvent_t *ready, hipEvent_t *copied)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    DeviceScratch &d = scratch_of(dev);
    if (!d.side) {
        hipStream_t st = nullptr;
        hipEvent_t a = nullptr, b = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (b) (void)hipEventDestroy(b);
            if (a) (void)hipEventDestroy(a);
            if (st) (void)hipStreamDestroy(st);
            return hip_status(e, "side stream");
        }
        d.side = st;
        d.ev_ready = a;
        d.ev_copied = b;
    }
    *side = d.side;
    *ready = d.ev_ready;
    *copied = d.ev_copied;
    return GUMAP_OK;
}

int host_scratch_get(size_t bytes, void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    DeviceScratch &d = scratch_of(dev);
    if (bytes == 0) bytes = 256;
    if (d.host_size < bytes) {
        if (d.host) (void)hipHostFree(d.host);
        d.host = nullptr;
        d.host_size = 0;
        e = hipHostMalloc(&d.host, bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            d.host = nullptr;
            return set_error(GUMAP_ENOMEM, "pinned host scratch of %zu bytes", bytes);
        }
        d.host_size = bytes;
    }
    *out = d.host;
    return GUMAP_OK;
}

size_t env_size(const char *name, size_t dflt)
{
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    char *end = nullptr;
    unsigned long long x = strtoull(v, &end, 10);
    return end && end != v ? (size_t)x : dflt;
}

size_t knob(const char *name, int kb_value, size_t dflt)
{
    const char *v = getenv(name);
    if (v && *v) return env_size(name, dflt);
    return kb_value >= 0 ? (size_t)kb_value : dflt;
}

// Reads a device int flag (after the stream drains).
int read_flag(const int *dflag, int *out, hipStream_t s)
{
    void *h = nullptr;
    int st = host_scratch_get(64, &h);
    if (st) return st;
    hipError_t e = hipMemcpyAsync(h, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "reading device flag");
    *out = *(int *)h;
    return GUMAP_OK;
}

// ------------------------------------------------------- CSR ingest ----
int prepare_graph(const gumap_graph *g, hipStream_t s, CanonCsr *out)
{
    const int32_t n = g->n, nnz = g->nnz;
    out->n = n;
    out->row_ptr = g->row_ptr;
    out->col = g->col_idx;
    if (n == 0) return GUMAP_OK;
    int *err = nullptr;
    int st;
    if (g->flags & GUMAP_VALIDATE) {
        st = scratch_get(kSlotFlags, 256, (void **)&err);
        if (st) return st;
        hipError_t e = hipMemsetAsync(err, 0, sizeof(int), s);
        if (e == hipSuccess) e = launch_validate_structure(n, nnz, g->row_ptr, g->col_idx, err, s);
        if (e != hipSuccess) return hip_status(e, "validate");
        int bad = 0;
        if ((st = read_flag(err, &bad, s))) return st;
        if (bad) return set_error(GUMAP_EGRAPH, "malformed CSR (check bits 0x%x)", bad);
    }
    if (!(g->flags & GUMAP_CSR_SORTED)) {
        int32_t *rp = nullptr, *col = nullptr;
        void *tmp = nullptr;
        if ((st = scratch_get(kSlotCanonRp, (size_t)(n + 1) * sizeof(int32_t), (void **)&rp))) return st;
        if ((st = scratch_get(kSlotCanonCol, (size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t), (void **)&col))) return st;
        if ((st = scratch_get(kSlotCanonTmp, canon_scratch_bytes(n, nnz), &tmp))) return st;
        hipError_t e = launch_canonicalize(n, nnz, g->row_ptr, g->col_idx, rp, col, tmp, s);
        if (e != hipSuccess) return hip_status(e, "canonicalize");
        out->row_ptr = rp;
        out->col = col;
    }
    if (g->flags & GUMAP_VALIDATE) {
        hipError_t e = hipMemsetAsync(err, 0, sizeof(int), s);
        if (e == hipSuccess && (g->flags & GUMAP_CSR_SORTED)) e = check_sorted(n, out->row_ptr, out->col, err, s);
        if (e == hipSuccess) e = launch_check_symmetric(n, out->row_ptr, out->col, err, s);
        if (e != hipSuccess) return hip_status(e, "validate");
        int bad = 0;
        if ((st = read_flag(err, &bad, s))) return st;
        if (bad) return set_error(GUMAP_EGRAPH, "%s", (bad & 32) ? "rows not sorted/unique or self-loop under GUMAP_CSR_SORTED"
                                                                 : "CSR is not symmetric");
    }
    return GUMAP_OK;
}

int check_graph_args(const gumap_graph *g)
{
    if (!g) return set_error(GUMAP_EINVAL, "graph is NULL");
    if (g->n < 0 || g->nnz < 0) return set_error(GUMAP_EINVAL, "negative n or nnz");
    if (g->n > 0 && !g->row_ptr) return set_error(GUMAP_EINVAL, "row_ptr is NULL");
    if (g->nnz > 0 && !g->col_idx) return set_error(GUMAP_EINVAL, "col_idx is NULL");
    if (g->flags & ~(GUMAP_CSR_SORTED | GUMAP_VALIDATE)) return set_error(GUMAP_EINVAL, "unknown flags");
    return GUMAP_OK;
}

int check_k(int32_t k)
{
    if (k < 1 || k > GUMAP_MAX_K) return set_error(GUMAP_EINVAL, "k = %d outside [1, %d]", k, GUMAP_MAX_K);
    return GUMAP_OK;
}

// On failure, let work already enqueued drain so the call stays host-synchronous.
int settle(int status, hipStream_t s)
{
    if (status != GUMAP_OK && status != GUMAP_EINVAL) {
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
    }
    return status;
}

int finish(hipStream_t s, const char *what)
{
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (prof_on()) prof_resolve();
    return hip_status(e, what);
}

// Launch `call` between profiler marks (no-op marks when profiling is off).
#define GM_PROF(name, bytes, call)                 \
    do {                                          \
        const int mark_ = prof_begin((name), s);  \
        e = (call);                               \
        prof_end(mark_, s, (double)(bytes));      \
    } while (0)

// ----------------------------------------------------- all-source BFS --
namespace {

int bit_length(int x)
{
    int b = 0;
    while (x > 0) { ++b; x >>= 1; }
    return b;
}

int choose_words(int32_t n_uniq, const BuildKnobs *kb)
{
    size_t forced = knob("GUMAP_FORCE_WORDS", kb ? kb->words : -1, 0);
    if (forced == 1 || forced == 2 || forced == 4 || forced == 8) return (int)forced;
    int need = (n_uniq + 63) / 64;
    int w = 1;
    while (w < need && w < 8) w <<= 1;
    return w;
}

}  // namespace

// The all-source BFS in rounds of source groups, each round's hop rows going
// to the kNN selection (and the hop matrix), or, with so, only into the
// stress sums of a drawing.
struct StressOut {
    const float *xy = nullptr;
    double sum = 0.0;
    int64_t pairs = 0;
};

int knn_build(const gumap_graph *g, int32_t k, const int32_t *sources, int32_t n_sources,
              int32_t *ids, uint8_t *hops, uint8_t *hop_matrix, hipStream_t s, StressOut *so = nullptr,
              const BuildKnobs *kb = nullptr)
{
    const BuildKnobs none;
    if (!kb) kb = &none;
    const int32_t heavy_forced = (int32_t)knob("GUMAP_HEAVY_DEGREE", kb->heavy, 0);
    int st;
    if ((st = check_graph_args(g))) return st;
    if ((st = check_k(k))) return st;
    if (sources && n_sources < 0) return set_error(GUMAP_EINVAL, "n_sources < 0");
    const int32_t n = g->n;
    const int64_t rows = sources ? n_sources : n;
    if (!so && rows > 0 && (!ids || !hops)) return set_error(GUMAP_EINVAL, "output pointer is NULL");
    if (so && n > 0 && !so->xy) return set_error(GUMAP_EINVAL, "coordinates pointer is NULL");
    if (rows == 0) return GUMAP_OK;
    if (n == 0) return set_error(GUMAP_EINVAL, "source id outside [0, 0)");

    // sources -> sorted unique slots, on the device; one synchronisation below
    // reads the number of unique sources, a range flag and the heavy-vertex
    // list size together
    const bool all_sources = sources == nullptr;
    CanonCsr c;
    if ((st = prepare_graph(g, s, &c))) return st;
    int32_t *usrc = nullptr, *slot_of = nullptr, *first_row = nullptr, *info = nullptr, *mult = nullptr;
    int32_t *heavy = nullptr;
    int64_t *slot_row = nullptr;
    if ((st = scratch_get(kSlotUsrc, (size_t)n * sizeof(int32_t), (void **)&usrc))) return st;
    if ((st = scratch_get(kSlotSlotOf, (size_t)n * sizeof(int32_t), (void **)&slot_of))) return st;
    if ((st = scratch_get(kSlotSlotRow, (size_t)n * sizeof(int64_t), (void **)&slot_row))) return st;
    if ((st = scratch_get(kSlotInfo, 256, (void **)&info))) return st;
    if ((st = scratch_get(kSlotHeavy, (size_t)(n + 1) * sizeof(int32_t), (void **)&heavy))) return st;
    hipError_t e = hipSuccess;
    if (all_sources) {
        e = all_sources_setup(n, usrc, slot_of, slot_row, info, s);
    } else {
        e = hipMemsetAsync(info, 0, 8 * sizeof(int32_t), s);
        if (e != hipSuccess) return hip_status(e, "source setup");
        int32_t *count = nullptr, *marks = nullptr, *pos = nullptr;
        void *scan_tmp = nullptr;
        if ((st = scratch_get(kSlotFirst, (size_t)n * sizeof(int32_t), (void **)&first_row))) return st;
        if ((st = scratch_get(kSlotMarks, (size_t)n * sizeof(int32_t), (void **)&marks))) return st;
        if ((st = scratch_get(kSlotPos, (size_t)(n + 1) * sizeof(int32_t), (void **)&pos))) return st;
        if ((st = scratch_get(kSlotScanTmp, exclusive_scan_scratch_bytes(n), &scan_tmp))) return st;
        if (so) {
            if ((st = scratch_get(kSlotCount, (size_t)n * sizeof(int32_t), (void **)&count))) return st;
            if ((st = scratch_get(kSlotMult, (size_t)n * sizeof(int32_t), (void **)&mult))) return st;
        }
        if (sources_ranked_small(rows, n)) {
            // the ranking kernel stores the final info words into pinned host
            // memory itself (taken now: the read below gets the same buffer)
            void *hv = nullptr;
            if ((st = host_scratch_get(256, &hv))) return st;
            e = prepare_sources_small(sources, rows, n, c.row_ptr, heavy_forced, heavy,
                                      first_row, count, usrc, slot_row, slot_of, mult, info, s, (int32_t *)hv);
        } else
            e = prepare_sources(sources, rows, n, first_row, count, marks, pos, scan_tmp, usrc, slot_row, slot_of,
                                mult, info, s);
    }
    // small graphs: every level of a group in one workgroup with its state in
    // LDS (one 64-source word per vertex), instead of one launch per level
    const bool fused = knob("GUMAP_FUSED", kb->fused, 1) != 0 && env_size("GUMAP_FORCE_WORDS", 0) == 0 &&
                       msbfs_fused_lds_bytes(n) <= 144 * 1024;
    // with every vertex a source the one-workgroup form needs neither the
    // heavy-vertex list nor the source count: no read-back before the search
    const bool setup_known = all_sources && fused;
    // vertices of high degree get a whole wave per level
    if (e == hipSuccess && !setup_known && (all_sources || !sources_ranked_small(rows, n)))
        e = launch_heavy_list(n, c.row_ptr, heavy_forced, heavy, info, s);
    if (e != hipSuccess) return hip_status(e, "source setup");
    int32_t hinfo[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (!setup_known) {
        void *hv = nullptr;
        if ((st = host_scratch_get(256, &hv))) return st;
        const bool published = !all_sources && sources_ranked_small(rows, n);
        if (!published) e = hipMemcpyAsync(hv, info, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e, "source setup");
        std::memcpy(hinfo, hv, sizeof(hinfo));
    }
    if (hinfo[0] & 1) return set_error(GUMAP_EINVAL, "a source id is outside [0, %d)", n);
    const int32_t n_uniq = all_sources ? n : hinfo[3];
    const int32_t n_heavy = hinfo[1], heavy_deg = hinfo[2];
    std::vector<int32_t> h_mult;     // times each unique source is listed (stress only)
    if (mult && n_uniq > 0) {
        h_mult.resize((size_t)n_uniq);
        e = hipMemcpyAsync(h_mult.data(), mult, (size_t)n_uniq * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e, "source multiplicities");
    }

    const int words = fused ? 1 : choose_words(n_uniq, kb);
    const int W = 64 * words;
    const int32_t groups_total = (n_uniq + W - 1) / W;
    const bool full_hops = hop_matrix != nullptr || so != nullptr;   // every finite hop <= 254 is needed
    const int L_cap = full_hops ? 255 : k;
    const int planes_alloc = full_hops ? 8 : bit_length(k);
    // history mode (not for the fused small-graph kernel): the frontiers of
    // hops 1..H are kept, so those hops need no bit-plane commits
    const int hist_levels = fused ? 0 : (int)std::min<size_t>(knob("GUMAP_HIST_LEVELS", kb->hist, 15), 64);
    const size_t state_arrays = hist_levels > 0 ? 1 + (size_t)(hist_levels + 3) + (size_t)planes_alloc
                                                : 3 + (size_t)planes_alloc;
    const size_t arr_per_group = (size_t)n * words;  // uint64 per array per group
    const size_t bytes_per_group = state_arrays * arr_per_group * 8 +
                                   (full_hops ? 0 : (size_t)W * n) + (size_t)W * msbfs_hop_chunks(n, 1) * 16 * 4 +
                                   (size_t)(L_cap + 2) * msbfs_stat_spread() * msbfs_stat_fields() * 8;
    const size_t budget = env_size("GUMAP_BFS_BUDGET_MB", 8192) << 20;
    int32_t groups_round = (int32_t)std::max<size_t>(1, std::min<size_t>(groups_total, budget / std::max<size_t>(1, bytes_per_group)));

    uint64_t *state = nullptr;
    uint8_t *hop_scratch = nullptr;
    unsigned long long *stats = nullptr;
    unsigned int *lvl_cnt = nullptr;
    int64_t *local_rows = nullptr;
    const int SF = msbfs_stat_fields(), SP = msbfs_stat_spread();
    const size_t stats_per_level = (size_t)groups_round * SP * SF;   // u64 per level
    const size_t arr_round = arr_per_group * groups_round;
    if ((st = scratch_get(kSlotBfsState, state_arrays * arr_round * 8, (void **)&state))) return st;
    if ((st = scratch_get(kSlotStats, (size_t)(L_cap + 2) * stats_per_level * 8, (void **)&stats))) return st;
    // hop counts per (slot, transpose block); rounds with fewer groups use more blocks per group
    const size_t lvl_cnt_bytes = std::max((size_t)groups_round * msbfs_hop_chunks(n, groups_round),
                                          (size_t)((groups_total - 1) % groups_round + 1) *
                                              msbfs_hop_chunks(n, (groups_total - 1) % groups_round + 1)) *
                                 W * 16 * 4;
    if ((st = scratch_get(kSlotLvlCnt, lvl_cnt_bytes, (void **)&lvl_cnt))) return st;
    if (!full_hops) {
        if ((st = scratch_get(kSlotHopRows, (size_t)groups_round * W * n, (void **)&hop_scratch))) return st;
        if ((st = scratch_get(kSlotLocalRows, (size_t)groups_round * W * sizeof(int64_t), (void **)&local_rows))) return st;
        if ((e = iota_i64(local_rows, (int64_t)groups_round * W, 0, s)) != hipSuccess) return hip_status(e, "iota");
    }
    void *hstats_v = nullptr;
    if ((st = host_scratch_get((size_t)(L_cap + 2) * stats_per_level * 8 + 256, &hstats_v))) return st;
    unsigned long long *hstats = (unsigned long long *)hstats_v;
    // the level counters are copied back on a side stream, beside the
    // transpose and selection that follow the levels on `s`
    hipStream_t side = nullptr;
    hipEvent_t ev_ready = nullptr, ev_copied = nullptr;
    if ((st = side_stream_get(&side, &ev_ready, &ev_copied))) return st;
    for (int32_t gs = 0; gs < groups_total; gs += groups_round) {
        MsbfsArgs a;
        a.planes_dev = nullptr;
        a.n = n;
        a.row_ptr = c.row_ptr;
        a.col = c.col;
        a.words = words;
        a.groups = std::min(groups_round, groups_total - gs);
        a.slot0 = gs * W;
        a.n_slots = std::min<int32_t>(a.groups * W, n_uniq - a.slot0);
        a.usrc = usrc;
        a.n_usrc = n_uniq;
        a.slot_of = slot_of;
        a.heavy = heavy;
        a.n_heavy = n_heavy;
        a.heavy_deg = heavy_deg;
        a.heavy_maxdeg = hinfo[4];
        a.xcd_map = (int32_t)env_size("GUMAP_XCD_MAP", 1);
        a.hops_variant = (int32_t)env_size("GUMAP_HOPS_VARIANT", 0);
        a.level_verts = (int32_t)knob("GUMAP_LEVEL_VERTS", kb->verts, 4);
        // Level 1 as a fill plus a top-down scatter from the sources (about
        // n_slots * mean degree atomic ORs) on sparse graphs, else by the level
        // kernel's range scan (n * words items per group); GUMAP_FIRST_LEVEL
        // = 0 / 1 forces either.
        const size_t first_env = knob("GUMAP_FIRST_LEVEL", kb->first, 2);
        const bool first_split = first_env == 2 ? (double)g->nnz * 256.0 <= (double)n * (double)n : first_env != 0;
        // Levels 2..push_levels may run top-down per group (see level_pushes):
        // needs the first fill, which clears their next-frontier arrays, and
        // in plane mode only level 2 has an array of its own to clear.
        a.nnz = g->nnz;
        a.push_ratio = (int32_t)std::min<size_t>(env_size("GUMAP_PUSH_RATIO", 4), 1 << 20);
        a.push_levels = first_split ? (int32_t)std::min<size_t>(knob("GUMAP_PUSH_LEVELS", kb->push, 0), hist_levels > 0 ? 3 : 2)
                                    : 0;
        a.push_levels = std::min(a.push_levels, L_cap);
        const size_t arr = arr_per_group * a.groups;
        a.hist_levels = hist_levels;
        a.levels_run = 0;
        if (hist_levels > 0) {
            a.front[0] = a.front[1] = nullptr;
            a.visited = state;
            a.hist = state + arr;
            a.planes = state + (size_t)(1 + hist_levels + 3) * arr;
        } else {
            a.hist = nullptr;
            a.front[0] = state;
            a.front[1] = state + arr;
            a.visited = state + 2 * arr;
            a.planes = state + 3 * arr;
        }
        a.plane_stride = arr;
        bool planes_cleared = false;   // history mode: planes cleared before the first hop above H
        a.stats = stats;
        a.stats_groups = a.groups;
        const size_t spl = (size_t)a.groups * SP * SF;   // u64 per level this round
        int last_level = 0;
        bool range_error = false;
        uint8_t *hop_out = hop_matrix ? hop_matrix : hop_scratch;
        const int64_t *hop_rows_of = hop_matrix ? slot_row + a.slot0 : local_rows;
        bool spec_valid = false;    // hop rows and selection already launched for the complete BFS
        int spec_hops_mark = -1;
        std::vector<int> depth_of(a.groups, 0);   // per group: last hop with vertices (per-level path)
        bool rows_done = false;   // hop rows and their counts written by the search itself
        if (fused) {
            int32_t *gout = nullptr;
            void *hg = nullptr;
            if ((st = scratch_get(kSlotGroupOut, (size_t)a.groups * 2 * sizeof(int32_t), (void **)&gout))) return st;
            if ((st = host_scratch_get((size_t)a.groups * 2 * sizeof(int32_t) + 256, &hg))) return st;
            // with hop rows wanted and the CSR small enough, the search keeps
            // everything in LDS and writes the rows itself
            rows_done = !so && n <= 2048 && msbfs_fused_rows_lds_bytes(n, g->nnz) <= 150 * 1024;
            const int mark = prof_begin("msbfs_level", s);
            if (rows_done) {
                // the selection follows at once: the levels found are read
                // back afterwards, only for the hop-range check
                e = launch_msbfs_fused_rows(a, L_cap, full_hops, g->nnz, hop_out,
                                            hop_rows_of, n, lvl_cnt, gout, s);
                prof_end(mark, s, 0.0);
                if (e == hipSuccess)
                    GM_PROF("knn_select", (double)a.n_slots * n + (double)a.n_slots * k * 5.0,
                            launch_knn_select_counted(n, k, a.n_slots, hop_out, hop_rows_of, n, usrc + a.slot0,
                                                      slot_row + a.slot0, lvl_cnt, 1, c.row_ptr, c.col, ids, hops, s));
                if (e == hipSuccess)
                    e = hipMemcpyAsync(hg, gout, (size_t)a.groups * 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return hip_status(e, "bfs (fused) / selection");
                const int32_t *hgo = (const int32_t *)hg;
                for (int32_t q = 0; q < a.groups; ++q) range_error |= hgo[2 * q + 1] != 0;
                if (range_error)
                    return set_error(GUMAP_ERANGE, "a finite hop exceeds 254; it does not fit the uint8 hop matrix");
                // the CSR read once per group and the hop rows written
                prof_set_bytes(mark, (double)a.groups * (4.0 * (n + 1) + 4.0 * g->nnz) + (double)a.n_slots * n);
                continue;
            } else {
                e = hipMemsetAsync(a.planes, 0, (size_t)planes_alloc * arr * 8, s);
                if (e == hipSuccess) e = launch_msbfs_fused(a, L_cap, full_hops, gout, s);
            }
            prof_end(mark, s, 0.0);
            if (e == hipSuccess) e = hipMemcpyAsync(hg, gout, (size_t)a.groups * 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_status(e, "bfs (fused)");
            const int32_t *hgo = (const int32_t *)hg;
            for (int32_t q = 0; q < a.groups; ++q) {
                last_level = std::max(last_level, (int)hgo[2 * q]);
                range_error |= hgo[2 * q + 1] != 0;
            }
            // per level and group: row pointers and adjacency (read at most
            // once each) and the three LDS state words per vertex
            prof_set_bytes(mark, (double)(last_level + 1) * a.groups * (8.0 * n + 4.0 * g->nnz + 24.0 * n));
        } else {
        // Level 1 sets the source bits and stores every visited word, so the
        // frontier and visited words need no clearing; each bit-plane is
        // cleared before its first hop and the counters of each batch of
        // levels with the batch.

        // sum over spread slots of one field for (level, group)
        auto level_sum = [&](int lv, int q, int field) {
            unsigned long long t = 0;
            const unsigned long long *p = hstats + (size_t)lv * spl + (size_t)q * SP * SF;
            for (int i = 0; i < SP; ++i) t += p[(size_t)i * SF + field];
            return t;
        };
        std::vector<int> marks(L_cap + 3, -1);
        std::vector<char> ran(L_cap + 3, 0);
        // algorithmic bytes of one level launch, from its counters: per
        // group the row pointers (8 per vertex scanned), the frontier,
        // visited and next-frontier rows (3 W/8 per vertex), the neighbour
        // frontier words gathered (W/8 per adjacency entry checked) and the
        // adjacency entries read (4 each).  The lazy commit of the previous
        // level (visited word written back, bit-plane read-modify-writes)
        // is counted apart, in commit_bytes.
        // whether group q ran level lv top-down (the kernels' own test)
        auto pushes = [&](int lv, int q) {
            return lv >= 2 && lv <= a.push_levels &&
                   level_sum(lv - 1, q, 4) * (unsigned long long)a.push_ratio < (unsigned long long)g->nnz * words;
        };
        auto commit_bytes = [&](int lv) {
            double b = 0.0;
            if (lv == 1 && first_split) return b;
            const int hop = lv - 1;
            // history mode keeps hops 1..H as frontiers: no plane writes for them
            const bool to_planes = hist_levels <= 0 || hop > hist_levels;
            const int pc = to_planes ? __builtin_popcount((unsigned)(hop > 0 ? hop : 0)) : 0;
            for (int q = 0; q < a.groups; ++q) {
                if (!(lv == 1 || level_sum(lv - 1, q, 0) != 0) || pushes(lv, q)) continue;
                const double commits = (double)level_sum(lv, q, 3);
                b += 8.0 * commits + 16.0 * commits * pc;
            }
            return b;
        };
        auto level_bytes = [&](int lv, bool commit_only) {
            double b = 0.0;
            if (lv == 1 && first_split) {
                // fill: slot ids read, visited and next-frontier words stored;
                // scatter: adjacency of the sources, one 8-byte atomic OR each
                for (int q = 0; q < a.groups; ++q) b += 4.0 * n + 16.0 * (double)n * words + 20.0 * level_sum(1, q, 2);
                return b;
            }
            for (int q = 0; q < a.groups; ++q) {
                const bool active = lv == 1 || level_sum(lv - 1, q, 0) != 0;
                if (!active || pushes(lv, q)) continue;
                // row pointers, frontier + visited reads, next-frontier writes (none when
                // the launch only committed: no search and nothing found)
                const bool searched = !commit_only && (level_sum(lv, q, 0) != 0 || level_sum(lv, q, 1) != 0);
                b += 8.0 * n + (searched ? 24.0 : 16.0) * (double)n * words;
                // neighbour frontier words gathered and adjacency entries read
                b += 8.0 * (double)level_sum(lv, q, 1) + 4.0 * (double)level_sum(lv, q, 2);
            }
            return b;
        };
        // a top-down level: the frontier words scanned, each frontier item's
        // visited word read and written back (with its plane updates), the
        // adjacency entries read, and per push the neighbour's visited and
        // frontier words read and its next-frontier word ORed
        auto push_bytes = [&](int lv) {
            double b = 0.0;
            const int hop = lv - 1;
            const bool to_planes = hist_levels <= 0 || hop > hist_levels;
            const int pc = to_planes ? __builtin_popcount((unsigned)hop) : 0;
            for (int q = 0; q < a.groups; ++q) {
                if (!pushes(lv, q) || level_sum(lv - 1, q, 0) == 0) continue;
                const double commits = (double)level_sum(lv, q, 3);
                b += 8.0 * (double)n * words + (16.0 + 16.0 * pc) * commits + 4.0 * (double)level_sum(lv, q, 2) +
                     24.0 * (double)level_sum(lv, q, 1);
            }
            return b;
        };
        std::vector<int> push_marks(L_cap + 3, -1);

        // levels launched between reads of the counters: the first batch covers
        // about 1.5x the depth a graph of this mean degree reaches (a level
        // launched past the end returns at once); later batches grow
        const double mean_deg = std::max(2.0, (double)g->nnz / std::max(1, n));
        int L = 1;
        int chunk = (int)std::min(16.0, std::max(4.0, std::ceil(1.5 * std::log((double)n) / std::log(mean_deg)) + 2));
        bool done = false;
        // The transpose and the selection are launched right after each batch
        // of levels, before the host has read the counters, with the plane
        // count computed on the device; they stand when that batch completed
        // the BFS (the usual case), and run again after further levels
        // otherwise.  The host then waits once per round instead of twice.
        int32_t *depth = info + 16;
        while (!done) {
            const int first = L;
            const int batch = std::min(chunk, L_cap + 1 - first);
            e = hipMemsetAsync(stats + (size_t)first * spl, 0, (size_t)batch * spl * 8, s);
            if (e != hipSuccess) return hip_status(e, "level counters");
            for (int c2 = 0; c2 < chunk && L <= L_cap; ++c2, ++L) {
                const int hop = L - 1;   // committed by this launch
                if (hist_levels > 0) {
                    if (hop > hist_levels && !planes_cleared) {
                        e = hipMemsetAsync(a.planes, 0, (size_t)planes_alloc * arr * 8, s);
                        if (e != hipSuccess) return hip_status(e, "plane clear");
                        planes_cleared = true;
                    }
                } else if (hop >= 1 && (hop & (hop - 1)) == 0) {
                    int b = bit_length(hop) - 1;
                    if (b < planes_alloc) e = hipMemsetAsync(a.planes + (size_t)b * arr, 0, arr * 8, s);
                    if (e != hipSuccess) return hip_status(e, "plane clear");
                }
                if (L == 1 && first_split) {
                    marks[L] = prof_begin("msbfs_first", s);
                    e = launch_msbfs_first(a, s);
                } else {
                    if (L <= a.push_levels) {
                        push_marks[L] = prof_begin("msbfs_push", s);
                        e = launch_msbfs_push(a, L, s);
                        prof_end(push_marks[L], s, 0.0);
                        if (e != hipSuccess) return hip_status(e, "bfs level (top-down)");
                    }
                    marks[L] = prof_begin("msbfs_level", s);
                    e = launch_msbfs_level(a, L, false, s);
                }
                prof_end(marks[L], s, 0.0);
                ran[L] = 1;
                if (e != hipSuccess) return hip_status(e, "bfs level");
            }
            e = hipEventRecord(ev_ready, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(side, ev_ready, 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(hstats + (size_t)first * spl, stats + (size_t)first * spl,
                                   (size_t)(L - first) * spl * 8, hipMemcpyDeviceToHost, side);
            if (e == hipSuccess) e = hipEventRecord(ev_copied, side);
            bool spec = false;
            a.levels_run = L - 1;
            if (e == hipSuccess && !so) {
                e = launch_msbfs_depth(a, first, L, depth, s);
                a.planes_dev = depth;
                spec_hops_mark = prof_begin("msbfs_hops", s);
                // if this batch completed the search, no hop exceeds L - 1
                if (e == hipSuccess)
                    e = launch_msbfs_hops_counted(a, std::min(8, bit_length(L - 1)), hop_out, hop_rows_of, n, lvl_cnt, s);
                prof_end(spec_hops_mark, s, 0.0);
                a.planes_dev = nullptr;
                if (e == hipSuccess)
                    GM_PROF("knn_select", (double)a.n_slots * n + (double)a.n_slots * k * 5.0,
                            launch_knn_select_counted(n, k, a.n_slots, hop_out, hop_rows_of, n, usrc + a.slot0,
                                                      slot_row + a.slot0, lvl_cnt, msbfs_hop_chunks(n, a.groups),
                                                      c.row_ptr, c.col, ids, hops, s));
                spec = true;
            }
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            {
                // always waited for: the copy writes host memory this call owns
                const hipError_t ec = hipEventSynchronize(ev_copied);
                if (e == hipSuccess) e = ec;
            }
            if (e != hipSuccess) return hip_status(e, "bfs stats");
            for (int lv = first; lv < L; ++lv) {
                prof_set_bytes(marks[lv], level_bytes(lv, false));
                prof_set_extra(marks[lv], commit_bytes(lv));
                if (push_marks[lv] >= 0) prof_set_bytes(push_marks[lv], push_bytes(lv));
            }
            for (int lv = first; lv < L && !done; ++lv) {
                bool any = false;
                for (int q = 0; q < a.groups; ++q) any |= level_sum(lv, q, 0) != 0;
                if (!any) {
                    done = true;
                    last_level = lv - 1;
                } else if (full_hops && lv == 255) {
                    range_error = true;
                    done = true;
                }
            }
            spec_valid = spec && done && !range_error;
            if (!done && L > L_cap) {
                // level L_cap found vertices; commit them without searching further
                const int hop = L_cap;
                if (hist_levels > 0) {
                    if (hop > hist_levels && !planes_cleared) {
                        e = hipMemsetAsync(a.planes, 0, (size_t)planes_alloc * arr * 8, s);
                        planes_cleared = true;
                    }
                } else if ((hop & (hop - 1)) == 0) {
                    int b = bit_length(hop) - 1;
                    if (b < planes_alloc) e = hipMemsetAsync(a.planes + (size_t)b * arr, 0, arr * 8, s);
                }
                if (e == hipSuccess) e = hipMemsetAsync(stats + (size_t)(L_cap + 1) * spl, 0, spl * 8, s);
                if (e != hipSuccess) return hip_status(e, "plane clear / level counters");
                const int mk = prof_begin("msbfs_level", s);
                e = launch_msbfs_level(a, L_cap + 1, true, s);
                a.levels_run = L_cap + 1;
                // commit-only: reads front + visited, writes the committed words
                prof_end(mk, s, (double)a.groups * (8.0 * n + 16.0 * (double)n * words));
                if (e != hipSuccess) return hip_status(e, "bfs commit");
                last_level = L_cap;
                done = true;
                spec_valid = false;
            }
            chunk = std::max(8, L / 2);
        }
        for (int q = 0; q < a.groups; ++q)
            for (int lv = 1; lv <= last_level; ++lv)
                if (level_sum(lv, q, 0) != 0) depth_of[q] = lv;
        }   // per-level launches
        if (range_error)
            return set_error(GUMAP_ERANGE, "a finite hop exceeds 254; it does not fit the uint8 hop matrix");
        const int planes_used = bit_length(last_level);
        if (so) {
            // stress terms of this round's rows, fused into the transpose
            const int32_t chunks = msbfs_hop_chunks(n, a.groups);
            const size_t parts = (size_t)a.n_slots * chunks;
            StressArgs sa;
            sa.xy = (const float2 *)so->xy;
            if ((st = scratch_get(kSlotStressSum, parts * sizeof(double), (void **)&sa.part_sum))) return st;
            if ((st = scratch_get(kSlotStressPairs, parts * sizeof(unsigned int), (void **)&sa.part_pairs))) return st;
            // profiled by its FP64 work: about 10 operations per reachable pair
            // (two differences, a sum of squares, the square root, the scaling
            // by 1/h, 1 - x and the squared term added), set once the pair
            // counts are read back
            const int stress_mark = prof_begin("msbfs_stress", s);
            e = launch_msbfs_stress(a, planes_used, sa, s);
            prof_end(stress_mark, s, 0.0);
            if (e != hipSuccess) return hip_status(e, "stress");
            std::vector<double> hsum(parts);
            std::vector<unsigned int> hpairs(parts);
            e = hipMemcpyAsync(hsum.data(), sa.part_sum, parts * sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(hpairs.data(), sa.part_pairs, parts * sizeof(unsigned int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_status(e, "stress sums");
            double round_pairs = 0.0;
            for (int32_t ls = 0; ls < a.n_slots; ++ls) {
                double rs = 0.0;
                int64_t rp = 0;
                for (int32_t c2 = 0; c2 < chunks; ++c2) {
                    rs += hsum[(size_t)ls * chunks + c2];
                    rp += hpairs[(size_t)ls * chunks + c2];
                }
                const int64_t m = all_sources ? 1 : h_mult[(size_t)a.slot0 + ls];
                so->sum += rs * (double)m;
                so->pairs += rp * m;
                round_pairs += (double)rp;
            }
            prof_set_bytes(stress_mark, 10.0 * round_pairs);
            continue;
        }
        // bytes of the transpose: the state words it reads per group (visited
        // and the planes in use; in history mode the source slots and the
        // frontiers up to the group's depth, plus the planes of hops above H)
        // and the hop rows it writes
        double hop_bytes = (double)a.n_slots * n;
        for (int q = 0; q < a.groups; ++q) {
            if (hist_levels <= 0) {
                hop_bytes += (double)(planes_used + 1) * (double)arr_per_group * 8.0;
                continue;
            }
            const int dq = depth_of[q];
            const int read = std::min(dq, hist_levels) + (dq > hist_levels ? planes_used : 0);
            hop_bytes += 4.0 * n + (double)read * (double)arr_per_group * 8.0;
        }
        if (spec_valid) {
            prof_set_bytes(spec_hops_mark, hop_bytes);
            continue;
        }
        GM_PROF("msbfs_hops", hop_bytes,
                launch_msbfs_hops_counted(a, planes_used, hop_out, hop_rows_of, n, lvl_cnt, s));
        if (e == hipSuccess)
            GM_PROF("knn_select", (double)a.n_slots * n + (double)a.n_slots * k * 5.0,
                    launch_knn_select_counted(n, k, a.n_slots, hop_out, hop_rows_of, n, usrc + a.slot0,
                                              slot_row + a.slot0, lvl_cnt, msbfs_hop_chunks(n, a.groups),
                                              c.row_ptr, c.col, ids, hops, s));
        if (e != hipSuccess) return hip_status(e, "hop rows / selection");
    }
    if (!so && !all_sources && n_uniq < rows) {
        e = copy_dup_rows(sources, rows, first_row, k, n, ids, hops, hop_matrix, s);
        if (e != hipSuccess) return hip_status(e, "repeated sources");
    }
    return finish(s, "gumap_knn_build");
}

int knn_build_tuned(const gumap_graph *g, int32_t k, const int32_t *sources, int32_t n_sources, int32_t *ids,
                    uint8_t *hops, uint8_t *hop_matrix, hipStream_t s, const BuildKnobs *kb)
{
    return knn_build(g, k, sources, n_sources, ids, hops, hop_matrix, s, nullptr, kb);
}

int stress(const gumap_graph *g, const float *xy, const int32_t *sources, int32_t n_sources, double *sum,
           int64_t *pairs, hipStream_t s)
{
    if (!sum || !pairs) return set_error(GUMAP_EINVAL, "output pointer is NULL");
    StressOut so;
    so.xy = xy;
    BuildKnobs kb;
    const bool tuned = tuned_knobs(g->n, g->nnz, sources ? n_sources : g->n, 1, true, &kb);
    int st = knn_build(g, 1, sources, n_sources, nullptr, nullptr, nullptr, s, &so, tuned ? &kb : nullptr);
    if (st) return st;
    *sum = so.sum;
    *pairs = so.pairs;
    return GUMAP_OK;
}

int neighborhood(const gumap_graph *g, const float *xy, int32_t r, const int32_t *verts, int32_t n_verts,
                 double *score, int32_t *ball, hipStream_t s)
{
    int st;
    if ((st = check_graph_args(g))) return st;
    if (r != 1 && r != 2) return set_error(GUMAP_EINVAL, "r = %d: only 1 and 2 are supported", r);
    if (verts && n_verts < 0) return set_error(GUMAP_EINVAL, "n_vertices < 0");
    const int32_t n = g->n;
    const int64_t rows = verts ? n_verts : n;
    if (rows == 0) return GUMAP_OK;
    if (!xy || !score) return set_error(GUMAP_EINVAL, "NULL coordinates or output pointer");
    if (neighborhood_lds_bytes(n) > 144 * 1024)
        return set_error(GUMAP_EINVAL, "n = %d exceeds the ball set the kernel keeps in LDS", n);
    if (verts) {
        std::vector<int32_t> h((size_t)rows);
        hipError_t e = hipMemcpyAsync(h.data(), verts, (size_t)rows * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e, "reading vertices");
        for (int64_t i = 0; i < rows; ++i)
            if (h[i] < 0 || h[i] >= n) return set_error(GUMAP_EINVAL, "vertex %d outside [0, %d)", h[i], n);
    }
    CanonCsr c;
    if ((st = prepare_graph(g, s, &c))) return st;
    // when launches are timed, count the work: 5 FP64 operations per squared
    // distance (2 differences, 2 products, 1 sum); the kernel is ALU-bound
    unsigned long long *evals = nullptr;
    hipError_t e = hipSuccess;
    if (prof_on()) {
        if ((st = scratch_get(kSlotEvals, 256, (void **)&evals))) return st;
        e = hipMemsetAsync(evals, 0, sizeof(unsigned long long), s);
        if (e != hipSuccess) return hip_status(e, "counter");
    }
    const int mark = prof_begin("neighborhood", s);
    e = launch_neighborhood(n, c.row_ptr, c.col, xy, r, verts, (int32_t)rows, score, ball, evals, s);
    prof_end(mark, s, 0.0);
    if (e != hipSuccess) return hip_status(e, "neighbourhood preservation");
    if (evals) {
        unsigned long long h = 0;
        e = hipMemcpyAsync(&h, evals, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e, "counter");
        prof_set_bytes(mark, 5.0 * (double)h);
    }
    return finish(s, "gumap_neighborhood");
}

// ------------------------------------------------------- canonical CSR --
int csr_canonicalize(const gumap_graph *g, int32_t *out_rp, int32_t *out_col, int32_t *out_nnz, hipStream_t s)
{
    int st;
    if ((st = check_graph_args(g))) return st;
    if (!out_nnz || !out_rp || (g->nnz > 0 && !out_col)) return set_error(GUMAP_EINVAL, "output pointer is NULL");
    if (g->n == 0) {
        *out_nnz = 0;
        hipError_t e = hipMemsetAsync(out_rp, 0, sizeof(int32_t), s);
        if (e != hipSuccess) return hip_status(e, "canonicalize");
        return finish(s, "gumap_csr_canonicalize");
    }
    if (g->flags & GUMAP_VALIDATE) {
        gumap_graph v = *g;
        v.flags = GUMAP_VALIDATE | GUMAP_CSR_SORTED;   // structural checks only here
        int *err = nullptr;
        if ((st = scratch_get(kSlotFlags, 256, (void **)&err))) return st;
        hipError_t e = hipMemsetAsync(err, 0, sizeof(int), s);
        if (e == hipSuccess) e = launch_validate_structure(g->n, g->nnz, g->row_ptr, g->col_idx, err, s);
        if (e != hipSuccess) return hip_status(e, "validate");
        int bad = 0;
        if ((st = read_flag(err, &bad, s))) return st;
        if (bad) return set_error(GUMAP_EGRAPH, "malformed CSR (check bits 0x%x)", bad);
        (void)v;
    }
    void *tmp = nullptr;
    if ((st = scratch_get(kSlotCanonTmp, canon_scratch_bytes(g->n, g->nnz), &tmp))) return st;
    // the scan stores the kept-entry count straight into pinned host memory
    // (at byte 32: read_flag below uses the first bytes of the same buffer)
    void *h = nullptr;
    if ((st = host_scratch_get(64, &h))) return st;
    int32_t *h_total = (int32_t *)h + 8;
    hipError_t e;
    GM_PROF("canonicalize", 2.0 * ((double)g->n * 4 + (double)g->nnz * 4),
            launch_canonicalize(g->n, g->nnz, g->row_ptr, g->col_idx, out_rp, out_col, tmp, s, h_total));
    if (e != hipSuccess) return hip_status(e, "canonicalize");
    if (g->flags & GUMAP_VALIDATE) {
        int *err = nullptr;
        if ((st = scratch_get(kSlotFlags, 256, (void **)&err))) return st;
        e = hipMemsetAsync(err, 0, sizeof(int), s);
        if (e == hipSuccess) e = launch_check_symmetric(g->n, out_rp, out_col, err, s);
        if (e != hipSuccess) return hip_status(e, "validate");
        int bad = 0;
        if ((st = read_flag(err, &bad, s))) return st;
        if (bad) return set_error(GUMAP_EGRAPH, "CSR is not symmetric");
    }
    if ((st = finish(s, "gumap_csr_canonicalize"))) return st;
    *out_nnz = *(volatile int32_t *)h_total;
    if (*out_nnz < 0) return set_error(GUMAP_EDEVICE, "canonicalisation scan did not complete");
    return GUMAP_OK;
}

// --------------------------------------------------------- partial BFS --
int knn_partial(const gumap_graph *g, int32_t k, int32_t *ids, uint8_t *hops, hipStream_t s)
{
    int st;
    if ((st = check_graph_args(g))) return st;
    if ((st = check_k(k))) return st;
    if (g->n > 0 && (!ids || !hops)) return set_error(GUMAP_EINVAL, "output pointer is NULL");
    if (g->n == 0) return GUMAP_OK;
    CanonCsr c;
    if ((st = prepare_graph(g, s, &c))) return st;
    PartialArgs a{};
    a.k = k;
    a.n = c.n;
    a.row_ptr = c.row_ptr;
    a.col = c.col;
    a.ids = ids;
    a.hops = hops;
    hipError_t e;
    GM_PROF("partial_bfs", (double)c.n * (8.0 + 5.0 * k), launch_partial_bfs(a, s));
    if (e != hipSuccess) return hip_status(e, "partial bfs");
    return finish(s, "gumap_knn_partial");
}

int membership(int32_t rows, int32_t k, const uint8_t *hops, float *w, float *rho, float *sigma,
               hipStream_t s)
{
    int st;
    if (rows < 0) return set_error(GUMAP_EINVAL, "rows < 0");
    if ((st = check_k(k))) return st;
    if (rows == 0) return GUMAP_OK;
    if (!hops || !w) return set_error(GUMAP_EINVAL, "hops or weights is NULL");
    hipError_t e;
    GM_PROF("membership", (double)rows * k * 5.0 + (double)rows * 8.0 * (rho && sigma ? 1 : 0),
            launch_membership(rows, k, hops, w, rho, sigma, s));
    if (e != hipSuccess) return hip_status(e, "membership");
    return finish(s, "gumap_membership");
}

// ------------------------------------------------------------ batches --
int check_batch_args(const gumap_batch *b, int32_t k)
{
    if (!b) return set_error(GUMAP_EINVAL, "batch is NULL");
    if (b->n_graphs < 0 || b->total_vertices < 0 || b->total_nnz < 0)
        return set_error(GUMAP_EINVAL, "negative batch sizes");
    if (b->total_vertices >= (int64_t)INT32_MAX || b->total_nnz >= (int64_t)INT32_MAX)
        return set_error(GUMAP_EINVAL, "batch exceeds int32 vertex or edge positions");
    if (b->n_graphs > 0 && (!b->vtx_offset || !b->edge_offset || !b->row_ptr))
        return set_error(GUMAP_EINVAL, "batch array is NULL");
    if (b->total_nnz > 0 && !b->col_idx) return set_error(GUMAP_EINVAL, "col_idx is NULL");
    if (b->flags & ~(GUMAP_CSR_SORTED | GUMAP_VALIDATE)) return set_error(GUMAP_EINVAL, "unknown flags");
    return check_k(k);
}

// Brings a batch to canonical packed form (validating if asked).  out may
// alias the caller's arrays when nothing had to change.
int prepare_batch(const gumap_batch *b, hipStream_t s, gumap_batch *out)
{
    *out = *b;
    int st;
    if (b->n_graphs == 0 || b->total_vertices == 0) return GUMAP_OK;
    const bool validate = (b->flags & GUMAP_VALIDATE) != 0;
    if (validate) {
        std::vector<int64_t> hv(b->n_graphs + 1), he(b->n_graphs + 1);
        hipError_t e = hipMemcpyAsync(hv.data(), b->vtx_offset, hv.size() * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(he.data(), b->edge_offset, he.size() * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e, "reading batch offsets");
        if (hv[0] != 0 || he[0] != 0 || hv.back() != b->total_vertices || he.back() != b->total_nnz)
            return set_error(GUMAP_EGRAPH, "batch offsets inconsistent with the totals");
        for (int32_t i = 0; i < b->n_graphs; ++i)
            if (hv[i] > hv[i + 1] || he[i] > he[i + 1]) return set_error(GUMAP_EGRAPH, "batch offsets not monotone");
        int *err = nullptr;
        if ((st = scratch_get(kSlotFlags, 256, (void **)&err))) return st;
        e = hipMemsetAsync(err, 0, sizeof(int), s);
        if (e == hipSuccess)
            e = validate_batch(b->n_graphs, b->vtx_offset, b->edge_offset, b->row_ptr, b->col_idx,
                               b->total_vertices, b->total_nnz, err, s);
        if (e != hipSuccess) return hip_status(e, "batch validate");
        int bad = 0;
        if ((st = read_flag(err, &bad, s))) return st;
        if (bad) return set_error(GUMAP_EGRAPH, "malformed batch CSR (check bits 0x%x)", bad);
    }
    if ((b->flags & GUMAP_CSR_SORTED) && !validate) return GUMAP_OK;
    // Disjoint-union CSR, canonicalised (or checked), and back to packed form.
    const int32_t nv = (int32_t)b->total_vertices, ne = (int32_t)b->total_nnz;
    int32_t *urp = nullptr, *ucol = nullptr;
    if ((st = scratch_get(kSlotUnionRp, (size_t)(nv + 1) * 4, (void **)&urp))) return st;
    if ((st = scratch_get(kSlotUnionCol, (size_t)(ne > 0 ? ne : 1) * 4, (void **)&ucol))) return st;
    hipError_t e = batch_to_union(b->n_graphs, b->vtx_offset, b->edge_offset, b->row_ptr, b->col_idx,
                                  b->total_vertices, b->total_nnz, urp, ucol, s);
    if (e != hipSuccess) return hip_status(e, "batch union");
    gumap_graph ug{nv, ne, urp, ucol, b->flags & GUMAP_CSR_SORTED};
    CanonCsr c;
    if ((st = prepare_graph(&ug, s, &c))) return st;
    if (validate) {
        int *err = nullptr;
        if ((st = scratch_get(kSlotFlags, 256, (void **)&err))) return st;
        e = hipMemsetAsync(err, 0, sizeof(int), s);
        if (e == hipSuccess && (b->flags & GUMAP_CSR_SORTED)) e = check_sorted(nv, c.row_ptr, c.col, err, s);
        if (e == hipSuccess) e = launch_check_symmetric(nv, c.row_ptr, c.col, err, s);
        if (e != hipSuccess) return hip_status(e, "batch validate");
        int bad = 0;
        if ((st = read_flag(err, &bad, s))) return st;
        if (bad) return set_error(GUMAP_EGRAPH, "batch graph not sorted/symmetric (check bits 0x%x)", bad);
        if (b->flags & GUMAP_CSR_SORTED) return GUMAP_OK;
    }
    // canonical union -> packed
    int32_t total_canon = 0;
    e = hipMemcpyAsync(&total_canon, c.row_ptr + nv, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "batch canonical size");
    int64_t *eoff = nullptr;
    int32_t *rp = nullptr, *col = nullptr;
    if ((st = scratch_get(kSlotBatchEoff, (size_t)(b->n_graphs + 1) * 8, (void **)&eoff))) return st;
    if ((st = scratch_get(kSlotBatchRp, (size_t)(nv + b->n_graphs) * 4, (void **)&rp))) return st;
    if ((st = scratch_get(kSlotBatchCol, (size_t)(total_canon > 0 ? total_canon : 1) * 4, (void **)&col))) return st;
    e = union_to_batch(b->n_graphs, b->vtx_offset, c.row_ptr, c.col, nv, total_canon, eoff, rp, col, s);
    if (e != hipSuccess) return hip_status(e, "batch repack");
    out->edge_offset = eoff;
    out->row_ptr = rp;
    out->col_idx = col;
    out->total_nnz = total_canon;
    out->flags = GUMAP_CSR_SORTED;
    return GUMAP_OK;
}

int batch_enqueue(const gumap_batch *b, int32_t k, int32_t *ids, uint8_t *hops, float *w, float *rho,
                  float *sigma, hipStream_t s, const BatchTune *t)
{
    unsigned long long *counter = nullptr;
    int st;
    if ((st = scratch_get(kSlotCounter, 256, (void **)&counter))) return st;
    BatchArgs a{};
    a.k = k;
    a.n_graphs = b->n_graphs;
    a.total_vertices = b->total_vertices;
    a.vtx_offset = b->vtx_offset;
    a.edge_offset = b->edge_offset;
    a.row_ptr = b->row_ptr;
    a.col = b->col_idx;
    a.ids = ids;
    a.hops = hops;
    a.weights = w;
    a.rho = rho;
    a.sigma = sigma;
    a.work_counter = counter;
    a.chunk = (int32_t)std::min<size_t>(batch_chunk_rows(k), std::max<size_t>(1, env_size("GUMAP_BATCH_CHUNK", 64)));
    if (t && t->chunk > 0) a.chunk = std::min(t->chunk, batch_chunk_rows(k));
    a.lanes = t ? t->lanes : 0;
    a.waves_per_block = 4;
    int64_t maxb = t && t->blocks > 0 ? t->blocks : partial_batch_max_blocks();
    int64_t want = (b->total_vertices + 4 * a.chunk - 1) / (4 * a.chunk);
    a.blocks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(maxb, want));
    hipError_t e = launch_batch_reset(counter, s);
    if (e == hipSuccess)
        GM_PROF("partial_batch", (double)b->total_vertices * (8.0 + 5.0 * k + (w ? 4.0 * k + 8.0 : 0.0)),
                launch_partial_batch(a, s));
    return hip_status(e, "batch launch");
}

int knn_partial_batch(const gumap_batch *b, int32_t k, int32_t *ids, uint8_t *hops, float *w, float *rho,
                      float *sigma, hipStream_t s)
{
    int st;
    if ((st = check_batch_args(b, k))) return st;
    if (b->total_vertices > 0 && (!ids || !hops)) return set_error(GUMAP_EINVAL, "output pointer is NULL");
    if (b->total_vertices == 0) return GUMAP_OK;
    gumap_batch cb;
    if ((st = prepare_batch(b, s, &cb))) return st;
    if ((st = batch_enqueue(&cb, k, ids, hops, w, rho, sigma, s))) return st;
    return finish(s, "gumap_knn_partial_batch");
}

// Autotuner of the batch launch: times every (lanes per source, rows per
// grab, grid size) candidate on the batch itself -- one warm-up launch, then
// the mean of two -- and keeps the fastest.  Every candidate computes the same
// rows, so the pick changes only the time.
int tune_batch(const gumap_batch *b, int32_t k, int32_t *ids, uint8_t *hops, float *w, float *rho, float *sigma,
               hipStream_t s, BatchTune *best, gumap_batch_tuning *info)
{
    *best = BatchTune{};
    info->lanes = 0;
    info->chunk = 0;
    info->blocks = 0;
    info->candidates = 0;
    info->best_ms = info->default_ms = 0.0f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_status(e, "tuning events");
    auto time_one = [&](const BatchTune *t, float *ms) -> int {
        int st = batch_enqueue(b, k, ids, hops, w, rho, sigma, s, t);
        if (st) return st;
        hipError_t x = hipEventRecord(e0, s);
        for (int r = 0; r < 2 && x == hipSuccess && st == GUMAP_OK; ++r)
            st = batch_enqueue(b, k, ids, hops, w, rho, sigma, s, t);
        if (st) return st;
        if (x == hipSuccess) x = hipEventRecord(e1, s);
        if (x == hipSuccess) x = hipEventSynchronize(e1);
        if (x == hipSuccess) x = hipEventElapsedTime(ms, e0, e1);
        if (x != hipSuccess) return hip_status(x, "tuning launch");
        *ms *= 0.5f;
        return GUMAP_OK;
    };
    int st = time_one(nullptr, &info->default_ms);
    float best_ms = info->default_ms;
    int32_t lane_opts[4];
    const int nl = partial_lane_options(k, lane_opts);
    const int32_t maxb = partial_batch_max_blocks();
    const int32_t chunk_max = batch_chunk_rows(k);
    for (int li = 0; li < nl && st == GUMAP_OK; ++li) {
        for (int32_t chunk : {16, 32, 64}) {
            if (chunk > chunk_max && chunk != 16) continue;
            for (int32_t blocks : {maxb / 2, maxb}) {
                BatchTune t;
                t.lanes = lane_opts[li];
                t.chunk = std::min(chunk, chunk_max);
                t.blocks = std::max(1, blocks);
                float ms = 0.0f;
                if ((st = time_one(&t, &ms))) break;
                ++info->candidates;
                if (ms < best_ms) {
                    best_ms = ms;
                    *best = t;
                }
            }
            if (st) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    info->best_ms = best_ms;
    info->lanes = best->lanes;
    info->chunk = best->chunk;
    info->blocks = best->blocks;
    return GUMAP_OK;
}

// ---------------------------------------------------- layout step (C2) --
int fuzzy_union(int32_t rows, int32_t k, const int32_t *ids, const float *w, int32_t *row_ptr, int32_t *col,
                float *val, int64_t cap, int64_t *nnz, hipStream_t s)
{
    int st;
    if (!nnz) return set_error(GUMAP_EINVAL, "nnz is NULL");
    *nnz = 0;
    if (rows < 0) return set_error(GUMAP_EINVAL, "rows < 0");
    if ((st = check_k(k))) return st;
    if (!row_ptr) return set_error(GUMAP_EINVAL, "row_ptr is NULL");
    if (rows == 0) {
        hipError_t e = hipMemsetAsync(row_ptr, 0, sizeof(int32_t), s);
        if (e != hipSuccess) return hip_status(e, "fuzzy union");
        return finish(s, "gumap_fuzzy_union");
    }
    if (!ids || !w) return set_error(GUMAP_EINVAL, "ids or weights is NULL");
    if (cap < 0 || (cap > 0 && (!col || !val))) return set_error(GUMAP_EINVAL, "col or val is NULL");
    if (2 * (int64_t)rows * k >= (int64_t)INT32_MAX) return set_error(GUMAP_EINVAL, "2 * rows * k >= 2^31");
    size_t tmp = 0;
    void *scratch = nullptr;
    char *flags = nullptr;
    if ((st = scratch_get(kSlotUnion, union_scratch_bytes(rows, k, &tmp), &scratch))) return st;
    if ((st = scratch_get(kSlotFlags, 256, (void **)&flags))) return st;
    int *err = (int *)flags;
    int64_t *dnnz = (int64_t *)(flags + 8);
    hipError_t e = hipMemsetAsync(flags, 0, 16, s);
    if (e != hipSuccess) return hip_status(e, "fuzzy union");
    GM_PROF("fuzzy_union", (double)rows * k * (4.0 + 4.0 + 4.0 * k) + 2.0 * rows * k * 8.0,
            launch_fuzzy_union(rows, k, ids, w, row_ptr, col, val, cap, dnnz, err, scratch, s));
    if (e != hipSuccess) return hip_status(e, "fuzzy union");
    void *h = nullptr;
    if ((st = host_scratch_get(64, &h))) return st;
    e = hipMemcpyAsync(h, flags, 16, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_status(e, "fuzzy union");
    if ((st = finish(s, "gumap_fuzzy_union"))) return st;
    const int bad = *(int *)h;
    const int64_t count = *(int64_t *)((char *)h + 8);
    if (bad) return set_error(GUMAP_EINVAL, "a neighbour id is outside [-1, rows) or equals its row");
    *nnz = count;
    if (count == 0) {
        e = hipMemsetAsync(row_ptr, 0, (size_t)(rows + 1) * sizeof(int32_t), s);
        if (e != hipSuccess) return hip_status(e, "fuzzy union");
        if ((st = finish(s, "gumap_fuzzy_union"))) return st;
    }
    if (count > cap) return set_error(GUMAP_ERANGE, "fuzzy union has %lld entries, capacity %lld",
                                      (long long)count, (long long)cap);
    return GUMAP_OK;
}

int edge_shuffle(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val, int64_t m, uint64_t seed,
                 int32_t *head, int32_t *tail, float *w, hipStream_t s)
{
    int st;
    if (n < 0 || m < 0) return set_error(GUMAP_EINVAL, "n < 0 or m < 0");
    if (m >= (int64_t)INT32_MAX) return set_error(GUMAP_EINVAL, "m >= 2^31");
    if (!row_ptr) return set_error(GUMAP_EINVAL, "row_ptr is NULL");
    if (m > 0 && (!col || !val || !head || !tail || !w)) return set_error(GUMAP_EINVAL, "NULL array");
    void *h = nullptr;
    if ((st = host_scratch_get(64, &h))) return st;
    hipError_t e = hipMemcpyAsync(h, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_status(e, "edge shuffle");
    if ((st = finish(s, "gumap_edge_shuffle"))) return st;
    if ((int64_t)*(int32_t *)h != m) return set_error(GUMAP_EINVAL, "m (%lld) != row_ptr[n] (%d)", (long long)m,
                                                       *(int32_t *)h);
    if (m == 0) return GUMAP_OK;
    size_t tmp = 0;
    void *scratch = nullptr;
    if ((st = scratch_get(kSlotShuffle, shuffle_scratch_bytes(m, &tmp), &scratch))) return st;
    GM_PROF("edge_shuffle", (double)m * (4.0 + 4.0 + 4.0 + 12.0) + (double)m * 12.0 * 2.0,
            launch_edge_shuffle(n, m, row_ptr, col, val, seed, head, tail, w, scratch, s));
    if (e != hipSuccess) return hip_status(e, "edge shuffle");
    return finish(s, "gumap_edge_shuffle");
}

int grad_sample(int32_t n, float *xy, int64_t m, const int32_t *head, const int32_t *tail, const float *w,
                const gumap_layout_params *p, int32_t it_begin, int32_t it_end, hipStream_t s)
{
    int st;
    if (!p) return set_error(GUMAP_EINVAL, "params is NULL");
    if (n < 0 || m < 0) return set_error(GUMAP_EINVAL, "n < 0 or m < 0");
    if (m > 0 && n == 0) return set_error(GUMAP_EINVAL, "edges without vertices");
    if (m >= ((int64_t)1 << 30)) return set_error(GUMAP_EINVAL, "m >= 2^30");
    if (p->neg < 0 || p->t < 1) return set_error(GUMAP_EINVAL, "neg < 0 or t < 1");
    if (it_begin < 0 || it_end > p->t || it_begin > it_end)
        return set_error(GUMAP_EINVAL, "iteration range [%d, %d) outside [0, %d]", it_begin, it_end, p->t);
    if (!(p->beta > 0.0) || !(p->alpha > 0.0) || !(p->samp > 0.0 || p->window > 0))
        return set_error(GUMAP_EINVAL, "alpha, beta must be positive; samp or window must be set");
    if (p->parts < 0) return set_error(GUMAP_EINVAL, "parts < 0");
    if (n == 0 || m == 0 || it_begin == it_end) return GUMAP_OK;
    if (!xy || !head || !tail || !w) return set_error(GUMAP_EINVAL, "NULL array");
    int64_t win = p->window;
    if (win == 0) win = (int64_t)floor(pow((double)m, p->samp));
    if (win < 1 || win > m) return set_error(GUMAP_EINVAL, "window %lld outside [1, m = %lld]", (long long)win,
                                             (long long)m);
    long long *pos = nullptr;
    int *err = nullptr;
    void *sort_scratch = nullptr;
    char *inc = nullptr;
    size_t sort_tmp = 0;
    const size_t rec_bytes = (((size_t)(2 * m) * sizeof(uint32_t)) + 255) & ~(size_t)255;
    void *moves = nullptr;
    if ((st = scratch_get(kSlotLayoutMoves, (size_t)m * 32, &moves))) return st;
    const size_t off_bytes = ((size_t)(n + 1) * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t heavy_bytes = ((size_t)n * sizeof(int32_t) + 255) & ~(size_t)255;
    if ((st = scratch_get(kSlotLayoutPos, (size_t)n * 4 * sizeof(long long), (void **)&pos))) return st;
    if ((st = scratch_get(kSlotLayoutSort, incidence_scratch_bytes(n, m, &sort_tmp), &sort_scratch))) return st;
    if ((st = scratch_get(kSlotLayoutRec, rec_bytes + off_bytes + heavy_bytes + 256, (void **)&inc))) return st;
    if ((st = scratch_get(kSlotFlags, 256, (void **)&err))) return st;
    long long *B[2] = {pos, pos + 2 * (size_t)n};
    hipError_t e = hipMemsetAsync(err, 0, sizeof(int), s);
    if (e == hipSuccess) e = launch_edge_check(n, m, head, tail, err, s);
    if (e == hipSuccess) e = launch_layout_init(n, xy, B[0], B[1], err, s);
    if (e != hipSuccess) return hip_status(e, "grad sample");
    int bad = 0;
    if ((st = read_flag(err, &bad, s))) return st;
    if (bad & 1) return set_error(GUMAP_EINVAL, "an edge endpoint is outside [0, n)");
    if (bad & 2) return set_error(GUMAP_EINVAL, "a coordinate is not finite or not below 2^20 in magnitude");
    LayoutArgs g{};
    g.n = n;
    g.m = m;
    g.s = win;
    g.head = head;
    g.tail = tail;
    g.w = w;
    g.alpha = p->alpha;
    g.beta = p->beta;
    g.att_num = (-2.0 * p->alpha) * p->beta;
    g.rep_num = (2.0 * p->gamma) * p->beta;
    g.neg = p->neg;
    g.seed = p->seed;
    GM_PROF("layout_incidence", (double)m * 2.0 * (4.0 + 4.0) * 4.0 + (double)m * 2.0 * 16.0,
            launch_layout_incidence(g, sort_scratch, (int32_t *)(inc + rec_bytes),
                                    (uint32_t *)inc, (int32_t *)(inc + rec_bytes + off_bytes),
                                    (int32_t *)(inc + rec_bytes + off_bytes + heavy_bytes), s));
    if (e != hipSuccess) return hip_status(e, "grad sample");
    int n_heavy = 0;   // one block per heavy vertex in every window
    if ((st = read_flag((const int *)(inc + rec_bytes + off_bytes + heavy_bytes), &n_heavy, s))) return st;
    g.heavy_blocks = n_heavy;
    const int64_t parts = std::min<int64_t>(p->parts > 0 ? p->parts : GUMAP_LAYOUT_DEFAULT_PARTS, win);
    int cur = 0;
    for (int32_t it = it_begin; it < it_end; ++it) {
        const double lr = p->alpha0 * (1.0 - (double)it / (double)p->t);
        for (int64_t c = 0; c < parts; ++c) {
            const int64_t l0 = win * c / parts, l1 = win * (c + 1) / parts;
            // moves: the part's entries (12 B) and the positions of their
            // endpoints and negative samples, 32 B of moves stored; gather:
            // every incidence code and offset, the stored moves read back,
            // positions in and out
            GM_PROF("grad_window", (double)(l1 - l0) * (12.0 + 32.0 + 16.0 * p->neg + 32.0) + (double)m * 2.0 * 4.0 +
                                       (double)n * (8.0 + 32.0) + (double)(l1 - l0) * 32.0,
                    launch_grad_window(g, it, l0, l1, lr, B[cur], B[cur ^ 1], moves, s));
            if (e != hipSuccess) return hip_status(e, "grad sample");
            cur ^= 1;
        }
    }
    e = launch_layout_out(n, B[cur], xy, s);
    if (e != hipSuccess) return hip_status(e, "grad sample");
    return finish(s, "gumap_grad_sample");
}

// -------------------------------------------- spectral initial drawing --
namespace {

// One Lanczos run behind c0 deflated columns: steps until the largest Ritz
// value's residual |beta_m z_m| is at most tol (or the Krylov space is
// exhausted); then that Ritz vector into X[:, k].  *lambda = 1 - the Ritz value.
int lanczos_run(const SpectralArgs &a, int64_t nnz, int c0, int jmax, double tol, uint64_t seed, double *svec,
                int k, double *lambda, int *steps, hipStream_t s)
{
    hipError_t e = launch_lanczos_start(a, c0, seed, s);
    if (e != hipSuccess) return hip_status(e, "lanczos start");
    // Every ten steps the coefficients so far are copied to one of two pinned
    // buffers; a block is checked on the host only after the next block's
    // steps are enqueued, so the GPU keeps working during the check.  Steps
    // past the converged one only write basis columns and coefficients beyond
    // it, which the Ritz vector does not read.
    const size_t per = (size_t)jmax + 2;
    void *hv = nullptr;
    int st = host_scratch_get(4 * per * sizeof(double), &hv);
    if (st) return st;
    double *hbuf[2][2] = {{(double *)hv, (double *)hv + per}, {(double *)hv + 2 * per, (double *)hv + 3 * per}};
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (int i = 0; i < 2; ++i)
        if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess) {
            if (ev[0]) (void)hipEventDestroy(ev[0]);
            return hip_status(e, "lanczos events");
        }
    std::vector<double> ha(per), hb(per), zv(per);
    int m = 0;
    double theta = 0.0;
    bool converged = false;
    // check of the coefficients of steps 1..jc: 1 converged, 0 not, -1 solver
    // failure; leaves the top Ritz value theta and its coefficients zv[0..m)
    auto check = [&](int jc, const double *ca, const double *cb) {
        std::copy(ca, ca + jc + 1, ha.begin());
        std::copy(cb, cb + jc + 1, hb.begin());
        // the recurrence stops at the first zero beta (the Krylov space is exhausted)
        m = jc;
        bool exhausted = false;
        for (int q = 1; q <= jc; ++q)
            if (hb[q] == 0.0) {
                m = q;
                exhausted = true;
                break;
            }
        // the largest eigenvalue of the recurrence matrix and its eigenvector
        // (bisection and inverse iteration, O(m)); its residual in A is
        // |beta_m| times the eigenvector's last component
        if (!tridiag_top(m, ha.data() + 1, hb.data() + 1, &theta, zv.data())) return -1;
        return (exhausted || fabs(hb[m] * zv[m - 1]) <= tol) ? 1 : 0;
    };
    int pend_j = 0, pend = 0, cur = 0, r = 0;
    for (int j = 1; j <= jmax && !converged && r >= 0; ++j) {
        // the sparse product (CSR, degree scales, the vector gathered), the
        // local recurrence and one pass over the basis (projections, update)
        GM_PROF("lanczos_step", (double)nnz * 24.0 + (double)a.n * 120.0 + 2.0 * (double)(c0 + j) * (double)a.n * 8.0,
                launch_lanczos_step(a, c0, j, s));
        if (e != hipSuccess) break;
        if (j % 10 != 0 && j != jmax) continue;
        e = hipMemcpyAsync(hbuf[cur][0], a.alpha, (size_t)(j + 1) * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hbuf[cur][1], a.beta, (size_t)(j + 1) * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(ev[cur], s);
        if (e != hipSuccess) break;
        if (pend_j) {
            if ((e = hipEventSynchronize(ev[pend])) != hipSuccess) break;
            r = check(pend_j, hbuf[pend][0], hbuf[pend][1]);
            converged = r > 0;
        }
        pend_j = j;
        pend = cur;
        cur ^= 1;
    }
    if (e == hipSuccess && !converged && r >= 0 && pend_j) {
        e = hipEventSynchronize(ev[pend]);
        if (e == hipSuccess) {
            r = check(pend_j, hbuf[pend][0], hbuf[pend][1]);
            converged = r > 0;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // no copy into the pinned buffers outlives this call
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (e != hipSuccess) return hip_status(e, "lanczos step");
    if (r < 0) return set_error(GUMAP_EDEVICE, "tridiagonal eigenvector solve failed");
    if (!converged)
        return set_error(GUMAP_ERANGE, "the Lanczos iteration did not reach residual %g in %d steps", tol, jmax);
    // the converged check's eigenvector gives the Ritz vector's coefficients
    e = hipMemcpyAsync(svec, zv.data(), (size_t)m * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // zv lives in this frame
    if (e == hipSuccess) e = launch_ritz_vector(a, c0, m, svec, k, s);
    if (e != hipSuccess) return hip_status(e, "ritz vector");
    *lambda = 1.0 - theta;
    *steps += m;
    return GUMAP_OK;
}

}  // namespace

int spectral_layout(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                    const gumap_spectral_params *p, float *xy, double *eigenvalues, int32_t *steps, hipStream_t s)
{
    int st;
    if (n < 3) return set_error(GUMAP_EINVAL, "n < 3 (two eigenvectors beyond the first need three vertices)");
    if (!row_ptr || !col || !val || !xy) return set_error(GUMAP_EINVAL, "NULL array");
    const int32_t max_steps = p && p->max_steps > 0 ? p->max_steps : 600;
    const double tol = p && p->tol > 0.0 ? p->tol : 1e-5;
    const uint64_t seed = p ? p->seed : 0;
    // run 1 works in the complement of one column, run 2 of two
    const int jmax = (int)std::min<int64_t>(max_steps, (int64_t)n - 1);
    const int tiles = spectral_tiles(n);
    const size_t cols = (size_t)jmax + 3;
    const size_t ld = ((size_t)n + 31) & ~(size_t)31;
    SpectralArgs a{};
    a.n = n;
    a.row_ptr = row_ptr;
    a.col = col;
    a.val = val;
    a.ld = ld;
    a.tiny = 1e-12;
    double *base = nullptr;
    const size_t doubles = cols * ld + 4 * ld + (size_t)tiles * (cols + 4) * 2 + 4 * cols + 16;
    if ((st = scratch_get(kSlotSpectral, doubles * sizeof(double), (void **)&base))) return st;
    double *q = base;
    a.Q = q;            q += cols * ld;
    a.sinv = q;         q += ld;
    a.w = q;            q += ld;
    a.X = q;            q += 2 * ld;
    a.part = q;         q += (size_t)tiles * (cols + 4) * 2;
    a.h = q;            q += cols;
    a.hacc = q;         q += cols;
    a.alpha = q;        q += cols;
    a.beta = q;         q += cols;
    a.scal = q;
    double *svec = nullptr;
    if ((st = scratch_get(kSlotSpectralVec, (size_t)cols * sizeof(double) + 256 + (size_t)n * sizeof(int32_t),
                          (void **)&svec)))
        return st;
    a.heavy = (int32_t *)(svec + cols + 32);
    int *err = nullptr;
    if ((st = scratch_get(kSlotFlags, 256, (void **)&err))) return st;
    int *first = err + 16;
    // err[0]: flags, err[1]: entries (row_ptr[n]), err[2]: long rows
    hipError_t e = hipMemsetAsync(err, 0, 3 * sizeof(int), s);
    if (e == hipSuccess) e = hipMemsetAsync(first, 0x7f, 2 * sizeof(int), s);
    if (e == hipSuccess) e = hipMemcpyAsync(err + 1, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_spectral_setup(a, err, err + 2, s);
    if (e != hipSuccess) return hip_status(e, "spectral setup");
    int hflags[3];
    {
        void *hv = nullptr;
        if ((st = host_scratch_get(64, &hv))) return st;
        e = hipMemcpyAsync(hv, err, 3 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e, "spectral setup");
        std::memcpy(hflags, hv, sizeof(hflags));
    }
    if (hflags[0] & 2) return set_error(GUMAP_EINVAL, "a weight is negative or not finite");
    if (hflags[0] & 1) return set_error(GUMAP_EGRAPH, "a vertex has zero degree (the graph is not connected)");
    const int32_t nnz = hflags[1];   // for the profiler's byte counts
    a.heavy_rows = hflags[2];
    double lam[2] = {0.0, 0.0};
    int total_steps = 0;
    if ((st = lanczos_run(a, nnz, 1, std::min(jmax, n - 1), tol, seed, svec, 0, &lam[0], &total_steps, s)))
        return st;
    if (lam[0] < 1e-10) return set_error(GUMAP_EGRAPH, "second eigenvalue %g: the graph is not connected", lam[0]);
    e = launch_ritz_deflate(a, 0, 1, s);
    if (e != hipSuccess) return hip_status(e, "deflation");
    if ((st = lanczos_run(a, nnz, 2, std::min(jmax, n - 2), tol, seed + 1, svec, 1, &lam[1], &total_steps, s)))
        return st;
    e = launch_spectral_finish(a, first, xy, s);
    if (e != hipSuccess) return hip_status(e, "spectral finish");
    if ((st = finish(s, "gumap_spectral_layout"))) return st;
    if (eigenvalues) {
        eigenvalues[0] = lam[0];
        eigenvalues[1] = lam[1];
    }
    if (steps) *steps = total_steps;
    return GUMAP_OK;
}

// ------------------------------------------------ spectral sparsification --
namespace {

// Scratch of the sparsifier for a canonical graph (n, nnz) and q columns.
int sparsify_args(const CanonCsr &c, int32_t nnz, int32_t q, SparsifyArgs *a, void **scan_tmp)
{
    int st;
    const int32_t n = c.n;
    const int64_t m_max = (int64_t)nnz + 1;   // upper entries, whatever the input
    const int tiles = sparsify_tiles(n);
    const size_t nq = (size_t)n * (size_t)(q > 0 ? q : 1);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t bytes = 2 * al((size_t)(n + 1) * 4) + al((size_t)nnz * 4) + 2 * al((size_t)m_max * 4) +
                   (q > 0 ? 6 * al(nq * 8) + al((size_t)tiles * q * 3 * 8) + al((size_t)q * 3 * 8) +
                                al((size_t)q * 8 * 8) + al((size_t)q * 4) : 0) +
                   al(256) + 4 * al((size_t)n * 4) + 2 * al((size_t)n * 8) + al((size_t)m_max) +
                   al(exclusive_scan_scratch_bytes(n > 0 ? n : 1));
    char *p = nullptr;
    if ((st = scratch_get(kSlotSparsify, bytes, (void **)&p))) return st;
    *a = SparsifyArgs{};
    a->n = n;
    a->row_ptr = c.row_ptr;
    a->col = c.col;
    a->upper = (int32_t *)p;            p += al((size_t)(n + 1) * 4);
    a->eoff = (int32_t *)p;             p += al((size_t)(n + 1) * 4);
    a->eid = (int32_t *)p;              p += al((size_t)nnz * 4);
    a->eu = (int32_t *)p;               p += al((size_t)m_max * 4);
    a->ev = (int32_t *)p;               p += al((size_t)m_max * 4);
    if (q > 0) {
        double **vecs[6] = {&a->B, &a->X, &a->Rv, &a->Z, &a->P, &a->AP};
        for (double **v : vecs) {
            *v = (double *)p;
            p += al(nq * 8);
        }
        a->part = (double *)p;          p += al((size_t)tiles * q * 3 * 8);
        a->sums = (double *)p;          p += al((size_t)q * 3 * 8);
        a->st = (double *)p;            p += al((size_t)q * 8 * 8);
        a->active = (int *)p;           p += al((size_t)q * 4);
    }
    a->n_active = (int *)p;             p += al(256);
    a->comp = (int32_t *)p;             p += al((size_t)n * 4);
    a->parent = (int32_t *)p;           p += al((size_t)n * 4);
    a->bestE = (int32_t *)p;            p += al((size_t)n * 4);
    a->bestR = (unsigned long long *)p; p += al((size_t)n * 8);
    a->vkey = (unsigned long long *)p;  p += al((size_t)n * 8);
    a->ve = (int32_t *)p;               p += al((size_t)n * 4);
    a->keep = (uint8_t *)p;             p += al((size_t)m_max);
    *scan_tmp = p;
    return GUMAP_OK;
}

// Canonical graph, its entry count and the edge ids; a->m read back.
int sparsify_prepare(const gumap_graph *g, int32_t q, hipStream_t s, CanonCsr *c, SparsifyArgs *a, void **scan_tmp)
{
    int st;
    if ((st = prepare_graph(g, s, c))) return st;
    int32_t nnz = g->nnz;
    void *h = nullptr;
    if ((st = host_scratch_get(64, &h))) return st;
    hipError_t e = hipMemcpyAsync(h, c->row_ptr + c->n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "sparsify setup");
    nnz = *(int32_t *)h;
    if ((st = sparsify_args(*c, nnz, q, a, scan_tmp))) return st;
    // row pointers and columns, the binary searches of the lower entries, the ids and edges written
    GM_PROF("edge_ids", (double)(c->n + 1) * 12.0 + (double)nnz * 4.0 * 12.0 + (double)nnz * 8.0,
            launch_edge_ids(*a, *scan_tmp, s));
    if (e == hipSuccess) e = hipMemcpyAsync(h, a->eoff + c->n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "edge ids");
    a->m = *(int32_t *)h;
    // a symmetric graph without self-loops has exactly nnz / 2 edges
    if (2 * a->m != (int64_t)nnz) return set_error(GUMAP_EGRAPH, "the graph is not symmetric or has self-loops");
    return GUMAP_OK;
}

}  // namespace

int effective_resistance(const gumap_graph *g, int32_t q, uint64_t seed, double tol, int32_t max_iters, double *R,
                         int64_t *m_out, int32_t *iters_out, hipStream_t s)
{
    int st;
    if ((st = check_graph_args(g))) return st;
    if (q < 1 || q > 1024) return set_error(GUMAP_EINVAL, "q outside [1, 1024]");
    if (!(tol > 0.0) || max_iters < 1) return set_error(GUMAP_EINVAL, "tol must be positive, max_iters >= 1");
    if (m_out) *m_out = 0;
    if (iters_out) *iters_out = 0;
    if (g->n == 0 || g->nnz == 0) return GUMAP_OK;
    if (!R) return set_error(GUMAP_EINVAL, "R is NULL");
    if ((int64_t)g->n * q >= ((int64_t)1 << 31)) return set_error(GUMAP_EINVAL, "n * q >= 2^31");
    CanonCsr c;
    SparsifyArgs a;
    void *scan_tmp = nullptr;
    if ((st = sparsify_prepare(g, q, s, &c, &a, &scan_tmp))) return st;
    if (m_out) *m_out = a.m;
    if (a.m == 0) return GUMAP_OK;
    hipError_t e;
    GM_PROF("resistance_setup", (double)g->nnz * (4.0 + 4.0) * q + (double)g->n * q * 8.0 * 5.0,
            launch_resistance_setup(a, q, seed, tol, s));
    if (e != hipSuccess) return hip_status(e, "resistance setup");
    int its = 0;
    void *h = nullptr;
    if ((st = host_scratch_get(64, &h))) return st;
    while (its < max_iters) {
        const int batch = std::min(8, max_iters - its);
        for (int b = 0; b < batch; ++b) {
            // per iteration: the Laplacian product (row pointers, adjacency and
            // each vertex's row of q values once: the neighbour-row gathers
            // repeat rows already read), two passes of dot products, the updates
            GM_PROF("cg_iteration", (double)(c.n + 1) * 4.0 + (double)g->nnz * 4.0 + (double)c.n * q * 8.0 * 13.0,
                    launch_cg_iteration(a, q, tol, max_iters, s));
            if (e != hipSuccess) return hip_status(e, "cg iteration");
        }
        its += batch;
        e = hipMemcpyAsync(h, a.n_active, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e, "cg state");
        if (*(int *)h == 0) break;
    }
    GM_PROF("resistance_out", (double)a.m * (8.0 + 16.0 * q + 8.0), launch_resistance_out(a, q, R, s));
    if (e != hipSuccess) return hip_status(e, "resistances");
    std::vector<double> hst((size_t)q * 8);   // per column: iterations at [3]
    e = hipMemcpyAsync(hst.data(), a.st, hst.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_status(e, "cg state");
    if ((st = finish(s, "gumap_effective_resistance"))) return st;
    int most = 0;
    for (int k = 0; k < q; ++k) most = std::max(most, (int)hst[(size_t)k * 8 + 3]);
    if (iters_out) *iters_out = most;
    return GUMAP_OK;
}

int sparsify_select(const gumap_graph *g, const double *R, int64_t target, int32_t *out_row_ptr, int32_t *out_col,
                    int32_t *out_nnz, hipStream_t s)
{
    int st;
    if ((st = check_graph_args(g))) return st;
    if (!out_nnz) return set_error(GUMAP_EINVAL, "out_nnz is NULL");
    *out_nnz = 0;
    if (g->n == 0) return GUMAP_OK;
    if (!out_row_ptr || (g->nnz > 0 && (!R || !out_col))) return set_error(GUMAP_EINVAL, "NULL array");
    CanonCsr c;
    SparsifyArgs a;
    void *scan_tmp = nullptr;
    if ((st = sparsify_prepare(g, 0, s, &c, &a, &scan_tmp))) return st;
    const int32_t n = c.n;
    if (target <= 0) target = n > 1 ? (int64_t)ceil((double)n * log((double)n)) : 0;
    if (target > a.m) target = a.m;
    hipError_t e = launch_forest_init(a, s);
    if (e != hipSuccess) return hip_status(e, "forest");
    int64_t forest = 0;
    void *h = nullptr;
    if ((st = host_scratch_get(64, &h))) return st;
    for (int round = 0; round < 64 && a.m > 0; ++round) {
        e = hipMemsetAsync(a.n_active, 0, sizeof(int), s);
        if (e == hipSuccess) {
            // every entry's edge id, neighbour label and resistance; per vertex its label, best and state
            GM_PROF("forest_round", (double)(2 * a.m) * (4.0 + 4.0 + 4.0 + 8.0) + (double)n * 60.0,
                    launch_forest_round(a, R, a.n_active, s));
        }
        if (e == hipSuccess) e = hipMemcpyAsync(h, a.n_active, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e, "forest round");
        const int added = *(int *)h;
        forest += added;
        if (added == 0) break;
    }
    const int64_t need = target - forest;
    if (need > 0) {
        size_t tmp = 0;
        void *rank = nullptr;
        if ((st = scratch_get(kSlotSparsifyRank, rank_scratch_bytes(a.m, &tmp), &rank))) return st;
        GM_PROF("top_edges", (double)a.m * (8.0 + 12.0) * 8.0, launch_take_top(a, R, need, rank, s));
        if (e != hipSuccess) return hip_status(e, "top edges");
    }
    e = launch_sparsified_csr(a, out_row_ptr, out_col, scan_tmp, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h, out_row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_status(e, "sparsified csr");
    if ((st = finish(s, "gumap_sparsify_select"))) return st;
    *out_nnz = *(int32_t *)h;
    return GUMAP_OK;
}

}  // namespace gm

// ================================================================ C-ABI ===

struct gumap_batch_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t rows = 0;
    gumap_batch_tuning tuning{};
};

extern "C" {

const char *gumap_last_error(void) { return gm::last_error(); }

int gumap_csr_canonicalize(const gumap_graph *g, int32_t *out_row_ptr, int32_t *out_col_idx,
                           int32_t *out_nnz, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::csr_canonicalize(g, out_row_ptr, out_col_idx, out_nnz, stream), stream);
}

int gumap_knn_build(const gumap_graph *g, int32_t k, const int32_t *sources, int32_t n_sources,
                    int32_t *nbr_ids, uint8_t *nbr_hops, uint8_t *hop_matrix, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    gm::BuildKnobs kb;
    const bool tuned = g && gm::tuned_knobs(g->n, g->nnz, sources ? n_sources : g->n, k, hop_matrix != nullptr, &kb);
    return gm::settle(gm::knn_build(g, k, sources, n_sources, nbr_ids, nbr_hops, hop_matrix, stream, nullptr,
                                    tuned ? &kb : nullptr),
                      stream);
}

int gumap_neighborhood(const gumap_graph *g, const float *xy, int32_t r, const int32_t *vertices,
                       int32_t n_vertices, double *score, int32_t *ball, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::neighborhood(g, xy, r, vertices, n_vertices, score, ball, stream), stream);
}

int gumap_stress(const gumap_graph *g, const float *xy, const int32_t *sources, int32_t n_sources, double *sum,
                 int64_t *pairs, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::stress(g, xy, sources, n_sources, sum, pairs, stream), stream);
}

int gumap_knn_partial(const gumap_graph *g, int32_t k, int32_t *nbr_ids, uint8_t *nbr_hops,
                      hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::knn_partial(g, k, nbr_ids, nbr_hops, stream), stream);
}

int gumap_fuzzy_union(int32_t rows, int32_t k, const int32_t *ids, const float *weights, int32_t *row_ptr,
                      int32_t *col, float *val, int64_t cap, int64_t *nnz, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::fuzzy_union(rows, k, ids, weights, row_ptr, col, val, cap, nnz, stream), stream);
}

int gumap_edge_shuffle(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val, int64_t m,
                       uint64_t seed, int32_t *head, int32_t *tail, float *w, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::edge_shuffle(n, row_ptr, col, val, m, seed, head, tail, w, stream), stream);
}

int gumap_grad_sample(int32_t n, float *xy, int64_t m, const int32_t *head, const int32_t *tail, const float *w,
                      const gumap_layout_params *p, int32_t it_begin, int32_t it_end, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::grad_sample(n, xy, m, head, tail, w, p, it_begin, it_end, stream), stream);
}

int gumap_spectral_layout(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                          const gumap_spectral_params *params, float *xy, double *eigenvalues, int32_t *steps,
                          hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::spectral_layout(n, row_ptr, col, val, params, xy, eigenvalues, steps, stream), stream);
}

int gumap_effective_resistance(const gumap_graph *g, int32_t q, uint64_t seed, double tol, int32_t max_iters,
                               double *resistance, int64_t *edges, int32_t *iterations, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::effective_resistance(g, q, seed, tol, max_iters, resistance, edges, iterations, stream),
                      stream);
}

int gumap_sparsify_select(const gumap_graph *g, const double *resistance, int64_t target, int32_t *out_row_ptr,
                          int32_t *out_col_idx, int32_t *out_nnz, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::sparsify_select(g, resistance, target, out_row_ptr, out_col_idx, out_nnz, stream), stream);
}

int gumap_membership(int32_t rows, int32_t k, const uint8_t *nbr_hops, float *weights, float *rho,
                     float *sigma, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::membership(rows, k, nbr_hops, weights, rho, sigma, stream), stream);
}

int gumap_knn_partial_batch(const gumap_batch *b, int32_t k, int32_t *nbr_ids, uint8_t *nbr_hops,
                            float *weights, float *rho, float *sigma, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    return gm::settle(gm::knn_partial_batch(b, k, nbr_ids, nbr_hops, weights, rho, sigma, stream), stream);
}

int gumap_batch_plan_create(const gumap_batch *b, int32_t k, int32_t *nbr_ids, uint8_t *nbr_hops,
                            float *weights, float *rho, float *sigma, hipStream_t stream,
                            gumap_batch_plan **plan)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    int st;
    if (!plan) return gm::set_error(GUMAP_EINVAL, "plan is NULL");
    *plan = nullptr;
    if ((st = gm::check_batch_args(b, k))) return st;
    if (!(b->flags & GUMAP_CSR_SORTED))
        return gm::set_error(GUMAP_EINVAL, "a captured plan needs a canonical batch (GUMAP_CSR_SORTED)");
    if (b->total_vertices > 0 && (!nbr_ids || !nbr_hops)) return gm::set_error(GUMAP_EINVAL, "output pointer is NULL");
    gumap_batch cb;
    if ((st = gm::prepare_batch(b, stream, &cb))) return st;  // validation only
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return gm::hip_status(e, "plan");
    // make sure the scratch the launches use exists before capture
    unsigned long long *counter = nullptr;
    if ((st = gm::scratch_get(gm::kSlotCounter, 256, (void **)&counter))) return st;
    gumap_batch_plan *p = new gumap_batch_plan();
    p->rows = b->total_vertices;
    gm::BatchTune tune;
    if (b->total_vertices > 0 && gm::env_size("GUMAP_PLAN_TUNE", 1) != 0) {
        if ((st = gm::tune_batch(&cb, k, nbr_ids, nbr_hops, weights, rho, sigma, stream, &tune, &p->tuning))) {
            delete p;
            return st;
        }
    }
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete p;
        return gm::hip_status(e, "capture stream");
    }
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = gm::batch_enqueue(&cb, k, nbr_ids, nbr_hops, weights, rho, sigma, cap, &tune);
        hipError_t e2 = hipStreamEndCapture(cap, &p->graph);
        if (st == GUMAP_OK && e2 != hipSuccess) st = gm::hip_status(e2, "end capture");
    } else {
        st = gm::hip_status(e, "begin capture");
    }
    if (st == GUMAP_OK) {
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = gm::hip_status(e, "graph instantiate");
    }
    (void)hipStreamDestroy(cap);
    if (st != GUMAP_OK) {
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        delete p;
        return st;
    }
    *plan = p;
    return GUMAP_OK;
}

int gumap_batch_plan_launch(gumap_batch_plan *plan, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    if (!plan) return gm::set_error(GUMAP_EINVAL, "plan is NULL");
    if (plan->rows == 0) return GUMAP_OK;
    hipError_t e = hipGraphLaunch(plan->exec, stream);
    if (e != hipSuccess) return gm::hip_status(e, "graph launch");
    return gm::finish(stream, "gumap_batch_plan_launch");
}

int gumap_batch_plan_tuning(const gumap_batch_plan *plan, gumap_batch_tuning *out)
{
    gm::clear_error();
    if (!plan || !out) return gm::set_error(GUMAP_EINVAL, "NULL argument");
    *out = plan->tuning;
    return GUMAP_OK;
}

void gumap_batch_plan_destroy(gumap_batch_plan *plan)
{
    if (!plan) return;
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
}

}  // extern "C"
