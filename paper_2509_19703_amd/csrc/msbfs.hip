// All-source BFS hop distances (GUMAP step C0, Sec. 3.1, Alg. 1) as a
// multi-source bit-parallel BFS.
//
// Sources are ranked in ascending id order ("slots") and packed into groups of
// W = 64 * words slots.  For each group every vertex owns `words` uint64 of
// each state array, laid out [group][vertex][word]:
//   front[L & 1]   bits of the sources that reached the vertex at hop L - 1
//   visited        bits of the sources that reached it at any earlier hop
//   planes[b]      bit b of the hop at which each source reached it
// One launch per level.  Level L first commits the previous level's frontier
// into `visited` and the bit-planes (the commit is lazy so one launch per
// level suffices), then finds the level-L bits bottom-up: a vertex ORs the
// frontier words of its neighbours, stopping as soon as every source that has
// not reached it yet is covered.  Level 1 needs no frontier read: on sparse
// graphs a fill stores each vertex's own source bits as visited and a wave
// per source ORs its bit into its neighbours' frontier words; on dense ones
// a vertex scans the part of its sorted adjacency that falls in the id range
// of each 64-source word and sets the bits of the sources it finds.  Either
// way level 1 stores every visited word, so no state is cleared first.
// After the last level a transpose kernel turns the vertex-major bit-planes
// into source-major uint8 hop rows, 64 x 64 bits per wave through shuffle
// butterflies, and counts how many vertices each source reached at hops
// 1..16 (used by the kNN selection to find its last level without a
// separate pass).
#include <algorithm>
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace gm {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kLevelBlock = 256;
constexpr int kFusedBlock = 1024;
#ifndef GM_GATHER_BATCH
#define GM_GATHER_BATCH 4
#endif
constexpr int kGatherBatch = GM_GATHER_BATCH;   // neighbour loads in flight per thread
#ifndef GM_HEAVY_BATCH
#define GM_HEAVY_BATCH 4
#endif
constexpr int kHeavyBatch = GM_HEAVY_BATCH;     // neighbour loads in flight per heavy-wave lane
constexpr int kFullCheckLevels = 32;  // levels up to which a finished group is detected
constexpr int kCountLevels = 16;
constexpr int kSpread = 64;        // level counters are spread over 64 slots per group
constexpr int kStatFields = 5;
// per level: bits found, neighbour words read (pull) or pushed (push),
// adjacency entries read, frontier words committed, and the frontier's
// edge-words (sum over (vertex, word) items found of the vertex degree,
// which prices a top-down next level)
enum { kFieldNewBits = 0, kFieldGathers = 1, kFieldCols = 2, kFieldCommits = 3, kFieldFrontEdges = 4 };

__device__ __forceinline__ uint64_t word_valid_mask(int32_t n_slots, int32_t local_slot0)
{
    int32_t c = n_slots - local_slot0;
    if (c <= 0) return 0ull;
    if (c >= 64) return ~0ull;
    return (1ull << c) - 1ull;
}

struct Counters {
    unsigned long long v[kStatFields];
};

// The array holding the frontier found at hop h (h >= 1).
__device__ __forceinline__ uint64_t *front_of(const MsbfsArgs &a, int h)
{
    if (a.hist_levels > 0) {
        const int slot = h <= a.hist_levels + 1 ? h - 1 : a.hist_levels + 1 + (h & 1);
        return a.hist + (size_t)slot * a.plane_stride;
    }
    return a.front[(h + 1) & 1];
}

// Whether level `level` of group g runs top-down (msbfs_push_kernel) instead
// of bottom-up: only levels 2..push_levels, whose next-frontier arrays the
// first fill clears, and only when the edge-words of the group's frontier
// (the pushes a top-down level makes), weighted by push_ratio, stay below
// nnz * WORDS (what a bottom-up level scans while few vertices are reached).
// Whole-wave call; every block of the group gets the same answer.
template <int WORDS>
__device__ __forceinline__ unsigned long long front_edges(const MsbfsArgs &a, int level, int32_t g)
{
    return wave_sum_u64(
        a.stats[(((size_t)(level - 1) * a.stats_groups + g) * kSpread + lane()) * kStatFields + kFieldFrontEdges]);
}

template <int WORDS>
__device__ __forceinline__ bool level_pushes(const MsbfsArgs &a, int level, int32_t g)
{
    if (level < 2 || level > a.push_levels) return false;
    return front_edges<WORDS>(a, level, g) * (unsigned long long)a.push_ratio < (unsigned long long)a.nnz * WORDS;
}

// Depth of group g (the last hop at which it found vertices) among the
// levels launched so far, capped at hist_levels + 1: whole-block call.
__device__ __forceinline__ int group_depth(const MsbfsArgs &a, int32_t g, int *s_depth)
{
    if (a.hist_levels <= 0) return 0;
    if (threadIdx.x == 0) *s_depth = 0;
    __syncthreads();
    const int levels = min(a.levels_run, a.hist_levels + 1);
    for (int i = threadIdx.x; i < levels * kSpread; i += blockDim.x) {
        const int h = 1 + i / kSpread, sl = i % kSpread;
        if (a.stats[(((size_t)h * a.stats_groups + g) * kSpread + sl) * kStatFields + kFieldNewBits]) atomicMax(s_depth, h);
    }
    __syncthreads();
    return *s_depth;
}

// Visited and first PL bit-plane words of lane l's vertex in each of TILES
// consecutive 64-vertex tiles from `tile` (word w of group g; items past the
// graph or past t_end read as 0).  Plane mode reads the stored arrays.  In
// history mode the visited word is the vertex's own source bit (hop 0) ORed
// with the frontiers of hops 1..min(depth, H) and the stored planes of the
// hops above H, and plane bit b is the OR of the frontiers of the hops with
// bit b set: the frontier loads go out four hops at a time for all tiles
// before any is used, so that they overlap.
constexpr int kHistBatch = 2;   // frontier hops loaded together per tile

template <int WORDS, int PL, int TILES>
__device__ __forceinline__ void load_tile_state(const MsbfsArgs &a, int32_t g, int w, int32_t tile, int32_t t_end,
                                                int planes_used, int depth, uint64_t (&wv)[TILES],
                                                uint64_t (&wp)[TILES][PL], bool want_vis = true)
{
    constexpr int LW = WORDS == 1 ? 0 : (WORDS == 2 ? 1 : (WORDS == 4 ? 2 : 3));
    const size_t gbase = (size_t)g * a.n * WORDS + w;
    size_t me[TILES];
    bool in[TILES];
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
        const int32_t v = (tile + t) * 64 + lane();
        in[t] = v < a.n && tile + t < t_end;
        me[t] = gbase + ((size_t)(in[t] ? v : 0) << LW);
#pragma unroll
        for (int b = 0; b < PL; ++b) wp[t][b] = 0ull;
    }
    if (a.hist_levels <= 0) {
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            wv[t] = in[t] ? a.visited[me[t]] : 0ull;
#pragma unroll
            for (int b = 0; b < PL; ++b)
                if (b < planes_used && in[t]) wp[t][b] = a.planes[(size_t)b * a.plane_stride + me[t]];
        }
        return;
    }
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
        wv[t] = 0ull;
        if (!want_vis) continue;   // the caller rebuilds it from the planes
        const int32_t v = (tile + t) * 64 + lane();
        const int32_t ls = (in[t] ? a.slot_of[v] : -1) - a.slot0;
        const int32_t bit = ls - (g * 64 * WORDS + 64 * w);
        wv[t] = (in[t] && ls >= 0 && ls < a.n_slots && bit >= 0 && bit < 64) ? 1ull << bit : 0ull;
    }
    const int hmax = min(depth, a.hist_levels);
    for (int h0 = 1; h0 <= hmax; h0 += kHistBatch) {
        uint64_t f[TILES][kHistBatch];
#pragma unroll
        for (int u = 0; u < kHistBatch; ++u)
#pragma unroll
            for (int t = 0; t < TILES; ++t)
                f[t][u] = (in[t] && h0 + u <= hmax) ? a.hist[(size_t)(h0 + u - 1) * a.plane_stride + me[t]] : 0ull;
#pragma unroll
        for (int u = 0; u < kHistBatch; ++u) {
            const int h = h0 + u;
#pragma unroll
            for (int t = 0; t < TILES; ++t) {
                if (want_vis) wv[t] |= f[t][u];
#pragma unroll
                for (int b = 0; b < PL; ++b)
                    if ((h >> b) & 1) wp[t][b] |= f[t][u];
            }
        }
    }
    if (depth > a.hist_levels) {
#pragma unroll
        for (int t = 0; t < TILES; ++t)
#pragma unroll
            for (int b = 0; b < PL; ++b)
                if (b < planes_used && in[t]) {
                    const uint64_t x = a.planes[(size_t)b * a.plane_stride + me[t]];
                    wp[t][b] |= x;
                    if (want_vis) wv[t] |= x;
                }
    }
}

// Commit of the previous level's frontier word f of (vertex, word) at `me`,
// whose visited word is vis; returns the new visited word.  Level 1 (hop 0)
// stores visited = f for every word, so visited needs no clearing; the
// bit-planes (every hop in plane mode, hops above H in history mode) are
// cleared by the host before their first use.
__device__ __forceinline__ uint64_t commit_word(const MsbfsArgs &a, int level, size_t me, uint64_t f, uint64_t vis,
                                                Counters &c)
{
    if (level == 1) {
        a.visited[me] = f;
        if (f) c.v[kFieldCommits] += 1;
        return f;
    }
    if (f) {
        vis |= f;
        a.visited[me] = vis;
        const int hop = level - 1;
        if (a.hist_levels <= 0 || hop > a.hist_levels)
            for (int b = 0; b < 8; ++b)
                if ((hop >> b) & 1) a.planes[(size_t)b * a.plane_stride + me] |= f;
        c.v[kFieldCommits] += 1;
    }
    return vis;
}

template <int WORDS, int VERTS>
__global__ void __launch_bounds__(kLevelBlock)
msbfs_level_kernel(MsbfsArgs a, int level, int commit_only, int light_blocks, int per_group, int xcd_map)
{
    constexpr int LW = WORDS == 1 ? 0 : (WORDS == 2 ? 1 : (WORDS == 4 ? 2 : 3));
    constexpr int G = GM_WAVE / WORDS;            // neighbour lanes per word in a heavy wave
    __shared__ unsigned long long red[kLevelBlock / GM_WAVE][kStatFields];
    // Workgroups are handed to the 8 XCDs round-robin by linear id.  With
    // xcd_map, group g runs only on XCD g % 8, so its frontier stays in that
    // XCD's L2 instead of being cached by all of them.
    int32_t g, vb;
    if (xcd_map) {
        const int32_t xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
        g = xcd + 8 * (j / per_group);
        vb = j % per_group;
    } else {
        g = blockIdx.x / per_group;
        vb = blockIdx.x % per_group;
    }
    const int l = lane(), wid = threadIdx.x / GM_WAVE;
    const int heavy_blocks = per_group - light_blocks;
    const size_t gbase = (size_t)g * a.n * WORDS;
    if (!commit_only && level_pushes<WORDS>(a, level, g)) return;   // run top-down by msbfs_push_kernel
    if (level >= 2) {
        // previous level found nothing for this group: nothing to commit or search
        const unsigned long long x =
            a.stats[(((size_t)(level - 1) * a.stats_groups + g) * kSpread + l) * kStatFields + kFieldNewBits];
        if (__ballot(x != 0ull) == 0ull) return;
    }
    if (level >= 2 && level <= kFullCheckLevels) {
        // every source of the group has reached every other vertex by level - 1
        // (counts of finished launches only): only the commit is left
        unsigned long long got = 0;
        for (int lv = 1; lv < level; ++lv)
            got += a.stats[(((size_t)lv * a.stats_groups + g) * kSpread + l) * kStatFields + kFieldNewBits];
        got = wave_sum_u64(got);
        const int32_t in_group = min(64 * WORDS, a.n_slots - g * 64 * WORDS);
        if (got == (unsigned long long)(a.n - 1) * (unsigned long long)in_group) commit_only = 1;
    }
    Counters c{};
    const uint64_t *__restrict__ fr = level >= 2 ? front_of(a, level - 1) : nullptr;
    uint64_t *__restrict__ nx = front_of(a, level);
    // heavy-vertex waves come first in launch order: the longest rows start
    // early instead of forming the tail of the level
    if (vb >= heavy_blocks) {
        const int32_t lb = vb - heavy_blocks;
        // VERTS (vertex, word) items per thread, kLevelBlock apart: the row
        // pointers, frontier and visited words of all of them are loaded
        // before any is used, so that each wave keeps several loads in
        // flight.  Every vertex is committed; the search of vertices of
        // degree > heavy_deg is left to the heavy waves (except at level 1,
        // where all are searched here).
        const int64_t idx0 = (int64_t)lb * kLevelBlock * VERTS + threadIdx.x;
        const int w = (int)(idx0 & (WORDS - 1));
        int32_t e0[VERTS], e1[VERTS];
        uint64_t f[VERTS], vis[VERTS];
#pragma unroll
        for (int j = 0; j < VERTS; ++j) {
            const int32_t v = (int32_t)((idx0 + (int64_t)j * kLevelBlock) >> LW);
            const bool in = v < a.n;
            const size_t me = gbase + ((size_t)v << LW) + w;
            e0[j] = in ? a.row_ptr[v] : 0;
            e1[j] = in ? a.row_ptr[v + 1] : 0;
            if (level == 1) {
                // hop 0: the vertex's own bit if it is a source of this word
                const int32_t ls = (in ? a.slot_of[v] : -1) - a.slot0;
                const int32_t bit = ls - (g * 64 * WORDS + 64 * w);
                f[j] = (in && ls >= 0 && ls < a.n_slots && bit >= 0 && bit < 64) ? 1ull << bit : 0ull;
                vis[j] = 0ull;
            } else {
                f[j] = in ? fr[me] : 0ull;
                vis[j] = in ? a.visited[me] : 0ull;
            }
        }
#pragma unroll
        for (int j = 0; j < VERTS; ++j) {
            const int32_t v = (int32_t)((idx0 + (int64_t)j * kLevelBlock) >> LW);
            if (v < a.n) vis[j] = commit_word(a, level, gbase + ((size_t)v << LW) + w, f[j], vis[j], c);
        }
#pragma unroll
        for (int j = 0; j < VERTS; ++j) {
            const int32_t v = (int32_t)((idx0 + (int64_t)j * kLevelBlock) >> LW);
            const size_t me = gbase + ((size_t)v << LW) + w;
            int cols = 0;
            if (v < a.n && !commit_only && (level == 1 || e1[j] - e0[j] <= a.heavy_deg)) {
                const int32_t ls0 = g * 64 * WORDS + 64 * w;
                const uint64_t unv = ~vis[j] & word_valid_mask(a.n_slots, ls0);
                uint64_t acc = 0;
                if (unv) {
                    if (level == 1) {
                        const int32_t gs0 = a.slot0 + ls0;
                        const int32_t gl = min(gs0 + 63, a.slot0 + a.n_slots - 1);
                        const int32_t lo = a.usrc[gs0], hi = a.usrc[gl];
                        int32_t lo_e = e0[j], hi_e = e1[j];
                        while (lo_e < hi_e) {
                            const int32_t mid = (lo_e + hi_e) >> 1;
                            ++cols;
                            if (a.col[mid] < lo) lo_e = mid + 1;
                            else hi_e = mid;
                        }
                        for (int32_t e = lo_e; e < e1[j]; ++e) {
                            const int32_t u = a.col[e];
                            ++cols;
                            if (u > hi) break;
                            const int32_t s = a.slot_of[u];
                            if (s >= 0) acc |= 1ull << (s - gs0);
                        }
                    } else {
                        for (int32_t e = e0[j]; e < e1[j]; e += kGatherBatch) {
                            // kGatherBatch independent neighbour loads in flight
                            int32_t u[kGatherBatch];
#pragma unroll
                            for (int i = 0; i < kGatherBatch; ++i) u[i] = e + i < e1[j] ? a.col[e + i] : -1;
                            uint64_t x = 0;
#pragma unroll
                            for (int i = 0; i < kGatherBatch; ++i)
                                if (u[i] >= 0) x |= fr[gbase + ((size_t)u[i] << LW) + w];
                            const int got = min(kGatherBatch, e1[j] - e);
                            cols += got;
                            c.v[kFieldGathers] += got;
                            acc |= x;
                            if ((acc & unv) == unv) break;
                        }
                    }
                }
                const uint64_t nw = acc & unv;
                nx[me] = nw;
                c.v[kFieldNewBits] += __popcll(nw);
                if (nw) c.v[kFieldFrontEdges] += (unsigned long long)(e1[j] - e0[j]);
            }
            // adjacency entries are shared by the word threads of a vertex: count the longest scan once
#pragma unroll
            for (int o = 1; o < WORDS; o <<= 1) cols = max(cols, __shfl_xor(cols, o, GM_WAVE));
            if (w == 0) c.v[kFieldCols] += cols;
        }
    } else if (level >= 2) {
        // one wave per heavy vertex: lane = (neighbour group, word)
        const int32_t hidx = vb * (kLevelBlock / GM_WAVE) + wid;
        if (hidx < a.n_heavy) {
            const int32_t v = a.heavy[hidx];
            const int w = l & (WORDS - 1), grp = l >> LW;
            const size_t me = gbase + ((size_t)v << LW) + w;
            // the light threads commit this vertex in the same launch; visited
            // | frontier is the committed value whichever of the two is read
            uint64_t vis = 0;
            if (grp == 0) vis = a.visited[me] | fr[me];
            vis = __shfl(vis, w, GM_WAVE);
            if (!commit_only) {
                const int32_t ls0 = g * 64 * WORDS + 64 * w;
                const uint64_t unv = ~vis & word_valid_mask(a.n_slots, ls0);
                uint64_t redv = 0;
                if (__ballot(unv != 0ull)) {
                    const int32_t e0 = a.row_ptr[v], e1 = a.row_ptr[v + 1];
                    uint64_t acc = 0;
                    for (int32_t base = e0; base < e1; base += kHeavyBatch * G) {
                        int got = 0;
#pragma unroll
                        for (int i = 0; i < kHeavyBatch; ++i) {
                            const int32_t e = base + grp + G * i;
                            if (e < e1) {
                                acc |= fr[gbase + ((size_t)a.col[e] << LW) + w];
                                ++got;
                            }
                        }
                        c.v[kFieldGathers] += got;
                        if (w == 0) c.v[kFieldCols] += got;
                        redv = acc;
#pragma unroll
                        for (int o = WORDS; o < GM_WAVE; o <<= 1) redv |= __shfl_xor(redv, o, GM_WAVE);
                        if (__ballot((redv & unv) != unv) == 0ull) break;
                    }
                }
                const uint64_t nw = redv & unv;
                if (grp == 0) {
                    nx[me] = nw;
                    c.v[kFieldNewBits] += __popcll(nw);
                    if (nw) c.v[kFieldFrontEdges] += (unsigned long long)(a.row_ptr[v + 1] - a.row_ptr[v]);
                }
            }
        }
    }
    // block totals -> one atomic per field into a spread slot
#pragma unroll
    for (int f = 0; f < kStatFields; ++f) {
        const unsigned long long t = wave_sum_u64(c.v[f]);
        if (l == 0) red[wid][f] = t;
    }
    __syncthreads();
    if (threadIdx.x < kStatFields) {
        unsigned long long t = 0;
        for (int q = 0; q < kLevelBlock / GM_WAVE; ++q) t += red[q][threadIdx.x];
        if (t)
            atomicAdd(&a.stats[(((size_t)level * a.stats_groups + g) * kSpread + (vb & (kSpread - 1))) *
                                   kStatFields + threadIdx.x],
                      t);
    }
}

// Level 1 in two launches (the default; the level kernel can run it too, by
// a range scan of every vertex's sorted adjacency).  The fill stores, for
// every (vertex, word) item, visited = the vertex's own bit if it is a
// source of that word (hop 0) and clears the item's next-frontier word.
template <int WORDS>
__global__ void __launch_bounds__(256) msbfs_first_fill_kernel(MsbfsArgs a)
{
    constexpr int LW = WORDS == 1 ? 0 : (WORDS == 2 ? 1 : (WORDS == 4 ? 2 : 3));
    const int32_t g = blockIdx.y;
    const int64_t items = (int64_t)a.n * WORDS;
    const size_t gbase = (size_t)g * items;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < items;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(idx >> LW);
        const int w = (int)(idx & (WORDS - 1));
        const int32_t ls = a.slot_of[v] - a.slot0;
        const int32_t bit = ls - (g * 64 * WORDS + 64 * w);
        a.visited[gbase + idx] = (ls >= 0 && ls < a.n_slots && bit >= 0 && bit < 64) ? 1ull << bit : 0ull;
        front_of(a, 1)[gbase + idx] = 0ull;
        for (int h = 2; h <= a.push_levels; ++h) front_of(a, h)[gbase + idx] = 0ull;
    }
}

// Then one wave per source ORs the source's bit into the hop-1 frontier word
// of each of its neighbours (top-down: a source's neighbours are exactly the
// vertices at hop 1 from it) and counts the bits it newly set.
template <int WORDS>
__global__ void __launch_bounds__(256) msbfs_first_scatter_kernel(MsbfsArgs a)
{
    constexpr int LW = WORDS == 1 ? 0 : (WORDS == 2 ? 1 : (WORDS == 4 ? 2 : 3));
    const int l = lane();
    const int32_t slot = blockIdx.x * (256 / GM_WAVE) + (int32_t)(threadIdx.x / GM_WAVE);   // local slot
    if (slot >= a.n_slots) return;
    const int32_t g = slot / (64 * WORDS), w = (slot % (64 * WORDS)) >> 6;
    const unsigned long long bit = 1ull << (slot & 63);
    const int32_t v = a.usrc[a.slot0 + slot];
    const int32_t e0 = a.row_ptr[v], e1 = a.row_ptr[v + 1];
    unsigned long long *fr = (unsigned long long *)front_of(a, 1) + (size_t)g * a.n * WORDS + w;
    unsigned long long nb = 0, fe = 0;
    if (a.push_levels >= 2) {
        // level 2 may run top-down: it needs the edges of the items newly in
        // the frontier, so each OR returns the word it found
        for (int32_t e = e0 + l; e < e1; e += GM_WAVE) {
            const int32_t u = a.col[e];
            const unsigned long long old = atomicOr(fr + ((size_t)u << LW), bit);
            nb += (old & bit) ? 0ull : 1ull;
            if (old == 0ull) fe += (unsigned long long)(a.row_ptr[u + 1] - a.row_ptr[u]);   // item newly in the frontier
        }
        nb = wave_sum_u64(nb);
        fe = wave_sum_u64(fe);
    } else {
        // the ORs return nothing (no wait per batch of 64 neighbours): on the
        // canonical CSR each neighbour gets this source's bit exactly once,
        // so the new bits are the degree
        for (int32_t e = e0 + l; e < e1; e += GM_WAVE)
            (void)__hip_atomic_fetch_or(fr + ((size_t)a.col[e] << LW), bit, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        nb = (unsigned long long)(e1 - e0);
    }
    if (l == 0) {
        unsigned long long *st = a.stats + ((size_t)(1 * a.stats_groups + g) * kSpread + (slot & (kSpread - 1))) * kStatFields;
        if (nb) atomicAdd(st + kFieldNewBits, nb);
        if (e1 > e0) atomicAdd(st + kFieldCols, (unsigned long long)(e1 - e0));
        if (fe) atomicAdd(st + kFieldFrontEdges, fe);
    }
}

// A level run top-down, for the groups level_pushes picks (small frontiers,
// the levels right after the sources): every frontier item (u, w), f = its
// word of hop level - 1, is committed, and f less what each neighbour v has
// reached by hop level - 1 (v's visited word ORed with its frontier word,
// the same whether or not v's own commit has landed) and not yet in v's
// next-frontier word (cleared by the first fill) is ORed into it.  A bit that several
// frontier vertices reach is counted once, by the OR that set it.  One
// thread per item for vertices of degree <= heavy_deg; a heavy vertex's
// adjacency is cut into chunks of (64 / WORDS) * kHeavyBatch entries, one
// wave per chunk (lane = entry, word; all its loads in flight at once),
// heavy waves first.
template <int WORDS>
__global__ void __launch_bounds__(kLevelBlock)
msbfs_push_kernel(MsbfsArgs a, int level, int light_blocks, int per_group, int chunks)
{
    constexpr int LW = WORDS == 1 ? 0 : (WORDS == 2 ? 1 : (WORDS == 4 ? 2 : 3));
    constexpr int G = GM_WAVE / WORDS;
    __shared__ unsigned long long red[kLevelBlock / GM_WAVE][kStatFields];
    const int32_t g = blockIdx.x / per_group, vb = blockIdx.x % per_group;
    if (!level_pushes<WORDS>(a, level, g)) return;
    const int l = lane(), wid = threadIdx.x / GM_WAVE;
    const int heavy_blocks = per_group - light_blocks;
    const size_t gbase = (size_t)g * a.n * WORDS;
    const uint64_t *__restrict__ fr = front_of(a, level - 1);
    unsigned long long *nx = (unsigned long long *)front_of(a, level);
    Counters c{};
    auto push = [&](int32_t u, int w, uint64_t f) {
        const size_t mu = gbase + ((size_t)u << LW) + w;
        // bits already in the next-frontier word need no atomic: a hub that
        // many frontier vertices reach then takes a few ORs, not one each (a
        // stale read only costs an OR; bits are never cleared)
        const uint64_t x = f & ~(a.visited[mu] | fr[mu] | nx[mu]);
        if (x) {
            const uint64_t old = atomicOr(nx + mu, (unsigned long long)x);
            c.v[kFieldNewBits] += __popcll(x & ~old);
            if (old == 0ull) c.v[kFieldFrontEdges] += (unsigned long long)(a.row_ptr[u + 1] - a.row_ptr[u]);
        }
    };
    if (vb >= heavy_blocks) {
        const int64_t idx = (int64_t)(vb - heavy_blocks) * kLevelBlock + threadIdx.x;
        const int32_t v = (int32_t)(idx >> LW);
        const int w = (int)(idx & (WORDS - 1));
        if (v < a.n) {
            const size_t me = gbase + (size_t)idx;
            const uint64_t f = fr[me];
            if (f) {
                commit_word(a, level, me, f, a.visited[me], c);
                const int32_t e0 = a.row_ptr[v], e1 = a.row_ptr[v + 1];
                if (e1 - e0 <= a.heavy_deg) {
                    for (int32_t e = e0; e < e1; e += kGatherBatch) {
                        int32_t u[kGatherBatch];
#pragma unroll
                        for (int i = 0; i < kGatherBatch; ++i) u[i] = e + i < e1 ? a.col[e + i] : -1;
#pragma unroll
                        for (int i = 0; i < kGatherBatch; ++i)
                            if (u[i] >= 0) push(u[i], w, f);
                    }
                    c.v[kFieldGathers] += (unsigned long long)(e1 - e0);
                    if (w == 0) c.v[kFieldCols] += (unsigned long long)(e1 - e0);
                }
            }
        }
    } else {
        const int64_t hw = (int64_t)vb * (kLevelBlock / GM_WAVE) + wid;
        const int32_t hidx = (int32_t)(hw / chunks), ch = (int32_t)(hw % chunks);
        if (hidx < a.n_heavy) {
            const int32_t v = a.heavy[hidx];
            const int w = l & (WORDS - 1), grp = l >> LW;
            const uint64_t f = fr[gbase + ((size_t)v << LW) + w];
            const int32_t e1 = a.row_ptr[v + 1];
            const int32_t cb = a.row_ptr[v] + ch * (G * kHeavyBatch);
            if (__ballot(f != 0ull) && cb < e1) {
                int32_t u[kHeavyBatch];
#pragma unroll
                for (int i = 0; i < kHeavyBatch; ++i) {
                    const int32_t e = cb + grp + G * i;
                    u[i] = f && e < e1 ? a.col[e] : -1;
                }
#pragma unroll
                for (int i = 0; i < kHeavyBatch; ++i)
                    if (u[i] >= 0) {
                        push(u[i], w, f);
                        c.v[kFieldGathers] += 1;
                    }
                if (l == 0) c.v[kFieldCols] += (unsigned long long)min(G * kHeavyBatch, e1 - cb);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < kStatFields; ++f) {
        const unsigned long long t = wave_sum_u64(c.v[f]);
        if (l == 0) red[wid][f] = t;
    }
    __syncthreads();
    if (threadIdx.x < kStatFields) {
        unsigned long long t = 0;
        for (int q = 0; q < kLevelBlock / GM_WAVE; ++q) t += red[q][threadIdx.x];
        if (t)
            atomicAdd(&a.stats[(((size_t)level * a.stats_groups + g) * kSpread + (vb & (kSpread - 1))) *
                                   kStatFields + threadIdx.x],
                      t);
    }
}

// Small graphs: all levels of one group in one workgroup, the frontier and
// visited words (one 64-source word per vertex) in LDS, the bit-planes in
// global memory for the hop-row transpose.  Same levels, commits and stop
// rules as the one-launch-per-level path; per group, group_out[2g] = last
// level that found vertices and group_out[2g + 1] = 1 if a hop above 254
// was found while every finite hop is needed.
__global__ void __launch_bounds__(kFusedBlock)
msbfs_fused_kernel(MsbfsArgs a, int L_cap, int full_hops, int32_t *group_out)
{
    extern __shared__ uint64_t fsm[];
    const int32_t n = a.n, g = blockIdx.x;
    uint64_t *front0 = fsm, *front1 = fsm + n, *vis = fsm + 2 * (size_t)n;
    __shared__ unsigned long long red[kFusedBlock / GM_WAVE];
    const uint64_t valid = word_valid_mask(a.n_slots, g * 64);
    for (int32_t v = threadIdx.x; v < n; v += kFusedBlock) {
        const int32_t sl = a.slot_of[v];
        front1[v] = (sl >= a.slot0 + g * 64 && sl < a.slot0 + g * 64 + 64) ? 1ull << (sl - a.slot0 - g * 64) : 0ull;
        front0[v] = 0ull;
        vis[v] = 0ull;
    }
    __syncthreads();
    const size_t gbase = (size_t)g * n;
    int last = 0, range = 0;
    for (int L = 1;; ++L) {
        uint64_t *cur = (L & 1) ? front1 : front0, *nxt = (L & 1) ? front0 : front1;
        const bool search = L <= L_cap;
        unsigned long long found = 0;
        for (int32_t v = threadIdx.x; v < n; v += kFusedBlock) {
            const uint64_t f = cur[v];
            uint64_t vv = vis[v];
            if (f) {
                vv |= f;
                vis[v] = vv;
                const int hop = L - 1;
                for (int b = 0; b < 8; ++b)
                    if ((hop >> b) & 1) a.planes[(size_t)b * a.plane_stride + gbase + v] |= f;
            }
            if (!search) continue;
            const uint64_t unv = ~vv & valid;
            uint64_t acc = 0;
            if (unv) {
                for (int32_t e = a.row_ptr[v]; e < a.row_ptr[v + 1]; ++e) {
                    acc |= cur[a.col[e]];
                    if ((acc & unv) == unv) break;
                }
            }
            const uint64_t nw = acc & unv;
            nxt[v] = nw;
            found += __popcll(nw);
        }
        found = wave_sum_u64(found);
        if (lane() == 0) red[threadIdx.x / GM_WAVE] = found;
        __syncthreads();
        unsigned long long tot = 0;
#pragma unroll
        for (int q = 0; q < kFusedBlock / GM_WAVE; ++q) tot += red[q];
        __syncthreads();
        if (!search) break;                  // the commit-only step after the hop cap
        if (tot == 0) break;                 // level L found nothing: hop L-1 was the last
        last = L;
        if (full_hops && L == 255) {
            range = 1;
            break;
        }
    }
    for (int32_t v = threadIdx.x; v < n; v += kFusedBlock) a.visited[gbase + v] = vis[v];
    if (threadIdx.x == 0) {
        group_out[2 * g] = last;
        group_out[2 * g + 1] = range;
    }
}

// Small graphs, hop rows wanted (no stress): as msbfs_fused_kernel, with
// the whole search in LDS -- the CSR, the frontier and visited words, and a
// 64 x n tile of hop bytes in which each commit records, for every source
// bit of the committed word, the hop at which that source reached the
// vertex (255 stays for unreached) and counts hops 1..16 per source.  The
// block then writes its 64 hop rows (to row hop_row[slot] of hop_out, n
// bytes each) and the counts (part[slot * 16 + h - 1]) itself, so no
// bit-planes, transpose or plane clears are needed.  One barrier per level.
constexpr int kRowsVerts = 2;   // vertices per thread of msbfs_fused_rows_kernel (n <= 2 * kFusedBlock)
constexpr int kRowsNbrs = 8;    // neighbour ids of a vertex held in registers

__global__ void __launch_bounds__(kFusedBlock)
msbfs_fused_rows_kernel(MsbfsArgs a, int L_cap, int full_hops, int32_t nnz, uint8_t *__restrict__ hop_out,
                        const int64_t *__restrict__ hop_row, int64_t row_stride, unsigned int *__restrict__ part,
                        int32_t *group_out)
{
    extern __shared__ uint64_t fsm[];
    const int32_t n = a.n, g = blockIdx.x;
    uint64_t *front0 = fsm, *front1 = fsm + n;
    unsigned int *cnt = (unsigned int *)(fsm + 3 * (size_t)n);            // [64][16]
    int32_t *rp = (int32_t *)(cnt + 64 * kCountLevels);                   // [n + 1]
    int32_t *col = rp + (n + 1);                                          // [nnz]
    const size_t tile_off = ((3 * (size_t)n * 8 + 64 * kCountLevels * 4 + ((size_t)n + 1 + nnz) * 4) + 15) & ~(size_t)15;
    uint8_t *tile = (uint8_t *)fsm + tile_off;                            // [64][n], 16-byte aligned
    __shared__ int found[3];
    const uint64_t valid = word_valid_mask(a.n_slots, g * 64);
    for (int32_t i = threadIdx.x; i <= n; i += kFusedBlock) rp[i] = a.row_ptr[i];
    for (int32_t i = threadIdx.x; i < nnz; i += kFusedBlock) col[i] = a.col[i];
    for (int32_t i = threadIdx.x; i < 64 * kCountLevels; i += kFusedBlock) cnt[i] = 0u;
    {
        uint32_t *t4 = (uint32_t *)tile;
        const int32_t words = 16 * n;   // 64 * n bytes
        for (int32_t i = threadIdx.x; i < words; i += kFusedBlock) t4[i] = 0xFFFFFFFFu;
    }
    if (threadIdx.x < 3) found[threadIdx.x] = 0;
    __syncthreads();
    // a thread's own vertices: their frontier and visited words (only this
    // thread writes them) and their first kRowsNbrs neighbours in registers
    uint64_t fw[kRowsVerts], vw[kRowsVerts];
    int32_t e0[kRowsVerts], e1[kRowsVerts], nb[kRowsVerts][kRowsNbrs];
#pragma unroll
    for (int j = 0; j < kRowsVerts; ++j) {
        const int32_t v = threadIdx.x + j * kFusedBlock;
        const bool in = v < n;
        const int32_t sl = in ? a.slot_of[v] : -1;
        fw[j] = (in && sl >= a.slot0 + g * 64 && sl < a.slot0 + g * 64 + 64) ? 1ull << (sl - a.slot0 - g * 64) : 0ull;
        vw[j] = 0ull;
        e0[j] = in ? rp[v] : 0;
        e1[j] = in ? rp[v + 1] : 0;
#pragma unroll
        for (int i = 0; i < kRowsNbrs; ++i) nb[j][i] = e0[j] + i < e1[j] ? col[e0[j] + i] : -1;
        if (in) front1[v] = fw[j];
    }
    __syncthreads();
    int last = 0, range = 0;
    for (int L = 1;; ++L) {
        const uint64_t *cur = (L & 1) ? front1 : front0;
        uint64_t *nxt = (L & 1) ? front0 : front1;
        const bool search = L <= L_cap;
        const int hop = L - 1;
        // found[L % 3] is written in this level; found[(L + 1) % 3] was last
        // read two levels ago (before the previous barrier): clear it for the next
        if (threadIdx.x == 0) found[(L + 1) % 3] = 0;
#pragma unroll
        for (int j = 0; j < kRowsVerts; ++j) {
            const int32_t v = threadIdx.x + j * kFusedBlock;
            const uint64_t f = fw[j];
            if (f) {
                vw[j] |= f;
                const uint8_t hb = (uint8_t)min(hop, 255);
                for (uint64_t m = f; m; m &= m - 1) {
                    const int sbit = __ffsll((unsigned long long)m) - 1;
                    tile[(size_t)sbit * n + v] = hb;
                    if (hop >= 1 && hop <= kCountLevels) atomicAdd(&cnt[sbit * kCountLevels + hop - 1], 1u);
                }
            }
            if (!search || v >= n) continue;
            const uint64_t unv = ~vw[j] & valid;
            uint64_t acc = 0;
            if (unv) {
#pragma unroll
                for (int i = 0; i < kRowsNbrs; ++i)
                    if (nb[j][i] >= 0) acc |= cur[nb[j][i]];
                for (int32_t e = e0[j] + kRowsNbrs; e < e1[j] && (acc & unv) != unv; ++e) acc |= cur[col[e]];
            }
            const uint64_t nw = acc & unv;
            nxt[v] = nw;
            fw[j] = nw;
            if (nw) found[L % 3] = 1;
        }
        __syncthreads();
        const bool any = found[L % 3] != 0;
        if (!search) break;                  // the commit-only step after the hop cap
        if (!any) break;                     // level L found nothing: hop L-1 was the last
        last = L;
        if (full_hops && L == 255) {
            range = 1;
            break;
        }
    }
    __syncthreads();
    // the group's rows: 16-byte pieces when rows are 16-byte aligned
    const int32_t in_group = min(64, a.n_slots - g * 64);
    const bool a16 = (n & 15) == 0 && (row_stride & 15) == 0 && (((uintptr_t)hop_out) & 15) == 0;
    if (a16) {
        const int32_t per_row = n / 16;
        for (int32_t i = threadIdx.x; i < in_group * per_row; i += kFusedBlock) {
            const int32_t sb = i / per_row, c = i % per_row;
            const uint4 q = *(const uint4 *)(tile + (size_t)sb * n + 16 * c);
            *(uint4 *)(hop_out + hop_row[g * 64 + sb] * row_stride + 16 * c) = q;
        }
    } else {
        for (int32_t i = threadIdx.x; i < in_group * n; i += kFusedBlock) {
            const int32_t sb = i / n, v = i % n;
            hop_out[hop_row[g * 64 + sb] * row_stride + v] = tile[(size_t)sb * n + v];
        }
    }
    for (int32_t i = threadIdx.x; i < in_group * kCountLevels; i += kFusedBlock)
        part[(size_t)(g * 64) * kCountLevels + i] = cnt[i];
    if (threadIdx.x == 0) {
        group_out[2 * g] = last;
        group_out[2 * g + 1] = range;
    }
}

// Degree above which a vertex is searched by a whole wave: hubs well above
// the mean degree (a lone thread would walk their rows serially while the
// rest of its wave waits); dense graphs with an even degree keep one thread
// per vertex word, which stops early.  info[1] = count, info[2] = threshold.
// Plane count of the levels run so far: one block looks at the new-vertex
// field of every (level, group, spread slot) counter of levels [first, last),
// each thread kDepthLoads counters of the flat (level, slot) range at a time
// with all of its loads in flight (the levels are independent).
constexpr int kDepthThreads = 1024;
constexpr int kDepthLoads = 4;

__global__ void __launch_bounds__(kDepthThreads)
msbfs_depth_kernel(const unsigned long long *__restrict__ stats, int32_t groups, int first, int last,
                   int32_t *__restrict__ out)
{
    __shared__ int found[256];
    const int per_level = groups * kSpread;
    const int nlev = min(last, first + 256) - first;
    for (int i = threadIdx.x; i < nlev; i += blockDim.x) found[i] = 0;
    __syncthreads();
    const int64_t total = (int64_t)max(nlev, 0) * per_level;
    for (int64_t b = 0; b < total; b += (int64_t)kDepthThreads * kDepthLoads) {
        unsigned long long x[kDepthLoads];
#pragma unroll
        for (int j = 0; j < kDepthLoads; ++j) {
            const int64_t idx = b + threadIdx.x + (int64_t)j * kDepthThreads;
            x[j] = idx < total ? stats[((size_t)first * per_level + idx) * kStatFields + 0] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < kDepthLoads; ++j) {
            const int64_t idx = b + threadIdx.x + (int64_t)j * kDepthThreads;
            if (x[j]) found[idx / per_level] = 1;   // every writer stores 1
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int last_found = first - 1;   // the level before the batch found vertices
        bool more = true;
        for (int lv = first; lv < last && lv < first + 256; ++lv) {
            if (!found[lv - first]) {
                more = false;
                break;
            }
            last_found = lv;
        }
        int bits = 0;
        while (bits < 31 && (1 << bits) <= last_found) ++bits;
        out[0] = bits;
        out[1] = more ? 1 : 0;
    }
}

__global__ void heavy_list_kernel(int32_t n, const int32_t *__restrict__ rp, int32_t forced, int32_t *heavy,
                                  int32_t *info)
{
    const int32_t thr = heavy_threshold(n, rp, forced);
    if (blockIdx.x == 0 && threadIdx.x == 0) info[2] = thr;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (rp[v + 1] - rp[v] > thr) {
            heavy[atomicAdd(&info[1], 1)] = (int32_t)v;
            atomicMax(&info[4], rp[v + 1] - rp[v]);
        }
}

// x from lane (this lane) ^ S.  Strides 1 and 2 are quad permutations and 8
// a rotation of the 16-lane row by 8, done by DPP moves on the VALU; 4, 16
// and 32 go through ds_bpermute.
template <int S>
__device__ __forceinline__ uint64_t xor_lane(uint64_t x)
{
    if constexpr (S == 1 || S == 2 || S == 8) {
        constexpr int ctrl = S == 1 ? 0xB1 : (S == 2 ? 0x4E : 0x128);   // quad_perm [1,0,3,2], [2,3,0,1]; row_ror:8
        const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)x, ctrl, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), ctrl, 0xF, 0xF, false);
        return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
    } else {
        return __shfl_xor(x, S, GM_WAVE);
    }
}

template <int K>
__device__ __forceinline__ void transpose_stage(uint64_t &x, int l)
{
    constexpr int s = 32 >> K;
    constexpr uint64_t M = K == 0 ? 0x00000000FFFFFFFFull
                         : K == 1 ? 0x0000FFFF0000FFFFull
                         : K == 2 ? 0x00FF00FF00FF00FFull
                         : K == 3 ? 0x0F0F0F0F0F0F0F0Full
                         : K == 4 ? 0x3333333333333333ull
                                  : 0x5555555555555555ull;
    const uint64_t y = xor_lane<s>(x);
    if ((l & s) == 0) x = (x & M) | ((y & M) << s);
    else x = (x & ~M) | ((y & ~M) >> s);
}

// Transpose of a 64 x 64 bit matrix held one row per lane: afterwards lane j
// holds column j (bit i = old bit j of lane i).  Six butterfly stages; in
// stage K lanes l and l ^ (32 >> K) swap blocks of 32 >> K bits.
__device__ __forceinline__ uint64_t transpose64(uint64_t x)
{
    const int l = lane();
    transpose_stage<0>(x, l);
    transpose_stage<1>(x, l);
    transpose_stage<2>(x, l);
    transpose_stage<3>(x, l);
    transpose_stage<4>(x, l);
    transpose_stage<5>(x, l);
    return x;
}

// Adds to cnt[h - 1] the vertices at hop h (1 <= h <= 16) among the 64 of a
// transposed tile (bit i of pl[b] is bit b of vertex i's hop; planes 5..7
// must be clear for a vertex to count), through a decision tree over the
// planes: 29 ANDs for the 16 classes instead of 5 per class.
__device__ __forceinline__ void count_hops(uint64_t vis, const uint64_t *pl, unsigned int *cnt)
{
    static_assert(kCountLevels == 16, "hops 1..16 are four planes plus the fifth");
    const uint64_t low_ok = vis & ~(pl[5] | pl[6] | pl[7]);
    const uint64_t base = low_ok & ~pl[4];   // hops 0..15
    uint64_t t1[2], t2[4], t3[8];
    t1[0] = base & ~pl[0];
    t1[1] = base & pl[0];
#pragma unroll
    for (int i = 0; i < 4; ++i) t2[i] = t1[i & 1] & (((i >> 1) & 1) ? pl[1] : ~pl[1]);
#pragma unroll
    for (int i = 0; i < 8; ++i) t3[i] = t2[i & 3] & (((i >> 2) & 1) ? pl[2] : ~pl[2]);
#pragma unroll
    for (int h = 1; h < 16; ++h) cnt[h - 1] += __popcll(t3[h & 7] & (((h >> 3) & 1) ? pl[3] : ~pl[3]));
    cnt[15] += __popcll(low_ok & pl[4] & ~(pl[0] | pl[1] | pl[2] | pl[3]));
}

// 4 bits -> 4 bytes holding 0 or 1, bit i in byte i (one 24-bit multiply:
// the four shifted copies n, n << 7, n << 14, n << 21 do not overlap).
__device__ __forceinline__ uint32_t spread4(uint32_t nib)
{
    return __umul24(nib & 0xFu, 0x00204081u) & 0x01010101u;
}

// Hop bytes of vertices 8c .. 8c + 7 of a transposed tile: byte i is 0xFF
// where the vertex is not visited, else the hop whose bit b is plane b
// (planes past the ones in use are zero).
template <int PL>
__device__ __forceinline__ uint64_t hop_bytes8(uint64_t vis, const uint64_t *pl, int c)
{
    uint32_t half[2];
#pragma unroll
    for (int nib = 0; nib < 2; ++nib) {
        const int sh = 8 * c + 4 * nib;
        const uint32_t nv = spread4((uint32_t)(~vis >> sh));
        uint32_t r = (nv << 8) - nv;   // 0xFF in the bytes of unvisited vertices
#pragma unroll
        for (int b = 0; b < PL; ++b) r |= spread4((uint32_t)(pl[b] >> sh)) << b;
        half[nib] = r;
    }
    return (uint64_t)half[0] | ((uint64_t)half[1] << 32);
}


// Block: one wave per word of a group, all on the same vertex tiles, so the
// waves of a block together read whole 64-byte state rows.  Wave w walks
// the block's share of the 64-vertex tiles; lane j ends with the hop bytes of
// slot (group, w, j) for the tile and writes them (64 bytes) to its row.
// Per-slot counts of vertices at hops 1..16 are written per block (no
// atomics) to part[(slot * chunks + block) * 16 + h - 1].
template <int WORDS, int STEP, bool NT>
__global__ void __launch_bounds__(WORDS * GM_WAVE)
msbfs_hops_kernel(MsbfsArgs a, int planes_arg, uint8_t *__restrict__ hop_out,
                  const int64_t *__restrict__ slot_row, int64_t row_stride, unsigned int *__restrict__ part)
{
    const int planes_used = a.planes_dev ? *a.planes_dev : planes_arg;
    const int w = threadIdx.x / GM_WAVE, l = lane();
    const int32_t g = blockIdx.y;
    __shared__ int s_depth;
    const int depth = group_depth(a, g, &s_depth);
    const int32_t local_slot = g * 64 * WORDS + 64 * w + l;
    const bool slot_ok = local_slot < a.n_slots;
    const int64_t row = slot_ok ? slot_row[local_slot] : 0;
    const int32_t ntiles = (a.n + 63) / 64;
    unsigned int cnt[kCountLevels];
#pragma unroll
    for (int h = 0; h < kCountLevels; ++h) cnt[h] = 0;

    // tiles of 64 vertices, STEP at a time: each lane then writes 64 * STEP
    // contiguous bytes of its row per step; block x of a group takes tiles [x * ntiles / chunks, (x + 1) * ntiles / chunks)
    const int32_t t_begin = (int32_t)((int64_t)blockIdx.x * ntiles / gridDim.x);
    const int32_t t_end = (int32_t)((int64_t)(blockIdx.x + 1) * ntiles / gridDim.x);
    for (int32_t tile = t_begin; tile < t_end; tile += STEP) {
        uint64_t outw[STEP][8];
        uint64_t sv[STEP], sp[STEP][8];
        load_tile_state<WORDS, 8, STEP>(a, g, w, tile, t_end, planes_used, depth, sv, sp);
#pragma unroll
        for (int half = 0; half < STEP; ++half) {
            uint64_t vis = transpose64(sv[half]);
            uint64_t pl[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) pl[b] = sp[half][b];
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b < planes_used) pl[b] = transpose64(pl[b]);
            // counts of vertices at hops 1..16 (planes 5.. must be clear)
            count_hops(vis, pl, cnt);
#pragma unroll
            for (int c = 0; c < 8; ++c) outw[half][c] = hop_bytes8<8>(vis, pl, c);
        }
        if (slot_ok) {
            const int32_t v0 = tile * 64;
            uint8_t *dst = hop_out + row * row_stride + v0;
            const int valid = min(min(64 * STEP, a.n - v0), (t_end - tile) * 64);
            if (valid == 64 * STEP && (((uintptr_t)dst) & 15) == 0) {
                u32x4 *d4 = (u32x4 *)dst;
#pragma unroll
                for (int c = 0; c < 4 * STEP; ++c) {
                    const uint64_t lo = outw[c >> 2][(2 * c) & 7], hi = outw[c >> 2][(2 * c + 1) & 7];
                    u32x4 q = {(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
                    if (NT) __builtin_nontemporal_store(q, d4 + c);
                    else d4[c] = q;
                }
            } else {
                for (int i = 0; i < valid; ++i) dst[i] = (uint8_t)(outw[i >> 6][(i >> 3) & 7] >> (8 * (i & 7)));
            }
        }
    }
    if (part && slot_ok) {
        uint4 *p = (uint4 *)(part + ((size_t)local_slot * gridDim.x + blockIdx.x) * kCountLevels);
#pragma unroll
        for (int q = 0; q < kCountLevels / 4; ++q) p[q] = make_uint4(cnt[4 * q], cnt[4 * q + 1], cnt[4 * q + 2], cnt[4 * q + 3]);
    }
}

// The same transpose with the stores staged in LDS: each wave leaves the hop
// bytes of its 64 sources for TILES 64-vertex tiles (64 * TILES bytes per
// source) in LDS, and the whole block then writes the rows out as whole
// segments (8 * TILES threads per row), instead of 16 bytes into 64
// different rows per store.  Needs rows aligned to 8 * TILES bytes.
// With STRESS the staged bytes are not stored: each row's stress terms
// ((h - |X_s - X_v|) / h)^2 over reachable v != s (Sec. 4.1.3) are summed in
// FP64 instead, one partial sum and pair count per (slot, block).
constexpr int kStressIts = 8;   // rows per thread in the store / stress phase of the staged transpose

// Body of the staged transpose for at most PL bit-planes.  With PL = 4 (every
// hop <= 15, the usual depth) the visited and plane words of the next tiles
// are loaded before the current tiles' rows are stored, so that the loads
// overlap the stores; the 8-plane form would need too many registers for that.
template <int WORDS, int TILES, bool STRESS, int PL>
__device__ __forceinline__ void hops_staged_body(const MsbfsArgs &a, int planes_used, int depth,
                                                 uint8_t *__restrict__ hop_out, unsigned int *__restrict__ part,
                                                 const StressArgs &sa, uint8_t *stage, const int64_t *row_base,
                                                 const double *rinv, double *st_sum, unsigned int *st_cnt,
                                                 const float2 *st_xy)
{
    constexpr int ROWS = WORDS * GM_WAVE;        // sources of the group = rows staged
    constexpr int SEG = 64 * TILES;              // bytes per row per step
    constexpr int UNIT = 8 * TILES;              // bytes per store: 8 or 16
    constexpr int PITCH = SEG + UNIT;            // padded against bank conflicts, UNIT-aligned
    constexpr bool PREFETCH = PL <= 4;
    typedef typename std::conditional<TILES == 2, u32x4, uint64_t>::type unit_t;
    const int w = threadIdx.x / GM_WAVE, l = lane();
    const int32_t g = blockIdx.y;
    const int32_t local_slot = g * ROWS + 64 * w + l;
    const bool slot_ok = local_slot < a.n_slots;
    const int32_t ntiles = (a.n + 63) / 64;
    unsigned int cnt[kCountLevels];
#pragma unroll
    for (int h = 0; h < kCountLevels; ++h) cnt[h] = 0;
    // block x of a group takes tiles [x * ntiles / chunks, (x + 1) * ntiles / chunks)
    const int32_t t_begin = (int32_t)((int64_t)blockIdx.x * ntiles / gridDim.x);
    const int32_t t_end = (int32_t)((int64_t)(blockIdx.x + 1) * ntiles / gridDim.x);
    uint64_t wv[TILES], wp[TILES][PL];   // visited and plane words of the tiles being (or next to be) transposed
    // With the frontier history and every hop <= 15 a vertex is visited iff it
    // is the row's own source or one of the four planes holds it: the visited
    // word is then rebuilt after the transpose instead of loaded and
    // transposed (the source's vertex is read once per lane).
    constexpr bool kPlanesGiveVis = PL <= 4;
    const bool derive_vis = kPlanesGiveVis && a.hist_levels > 0;
    const int32_t self_v = (derive_vis && slot_ok) ? a.usrc[a.slot0 + local_slot] : -1;
    auto load_tiles = [&](int32_t tile) {
        load_tile_state<WORDS, PL, TILES>(a, g, w, tile, t_end, planes_used, depth, wv, wp, !derive_vis);
    };
    if (PREFETCH && t_begin < t_end) load_tiles(t_begin);
    for (int32_t tile = t_begin; tile < t_end; tile += TILES) {
        if (!PREFETCH) load_tiles(tile);
#pragma unroll
        for (int half = 0; half < TILES; ++half) {
            uint64_t pl[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) pl[b] = (b < PL && b < planes_used) ? transpose64(wp[half][b < PL ? b : 0]) : 0ull;
            uint64_t vis;
            if (kPlanesGiveVis && derive_vis) {
                const int32_t tt = tile + half;
                vis = pl[0] | pl[1] | pl[2] | pl[3] |
                      ((self_v >= 0 && (self_v >> 6) == tt) ? 1ull << (self_v & 63) : 0ull);
            } else {
                vis = transpose64(wv[half]);
            }
            count_hops(vis, pl, cnt);
            uint64_t *dst = (uint64_t *)(stage + (size_t)(64 * w + l) * PITCH + 64 * half);
#pragma unroll
            for (int c = 0; c < 8; ++c) dst[c] = hop_bytes8<PL>(vis, pl, c);
        }
        __syncthreads();
        if (PREFETCH && tile + TILES < t_end) load_tiles(tile + TILES);
        // rows out: 8 threads per row, UNIT bytes each
        const int32_t v0 = tile * 64;
        const int valid = min(SEG, min(a.n - v0, (t_end - tile) * 64));
        // a thread's UNIT vertices (offset (threadIdx.x & 7) * UNIT) are the
        // same for all its rows: their coordinates are loaded once
        float2 pv[STRESS ? UNIT : 1];
        if (STRESS) {
            const int off = (threadIdx.x & 7) * UNIT;
#pragma unroll
            for (int i = 0; i < UNIT; ++i) pv[i] = off + i < valid ? sa.xy[v0 + off + i] : make_float2(0.0f, 0.0f);
        }
#pragma unroll
        for (int it = 0; it < kStressIts; ++it) {
            const int q = threadIdx.x + it * ROWS;
            const int r = q >> 3, off = (q & 7) * UNIT;
            const uint8_t *src = stage + (size_t)r * PITCH + off;
            if (STRESS) {
                if (g * ROWS + r >= a.n_slots) continue;
                const double xs = (double)st_xy[it].x, ys = (double)st_xy[it].y;
#pragma unroll
                for (int i = 0; i < UNIT; ++i) {
                    const int h = src[i];
                    if (off + i >= valid || h == 0 || h == 255) continue;
                    const double dx = xs - (double)pv[i].x, dy = ys - (double)pv[i].y;
                    // (h - e) / h = 1 - e / h
                    const double t = 1.0 - sqrt(dx * dx + dy * dy) * rinv[h];
                    st_sum[it] += t * t;
                    st_cnt[it] += 1;
                }
            } else {
                const int64_t base = row_base[r];
                if (base < 0 || off >= valid) continue;
                uint8_t *dstp = hop_out + base + v0 + off;
                if (off + UNIT <= valid) {
                    *(unit_t *)dstp = *(const unit_t *)src;
                } else {
                    for (int i = 0; off + i < valid; ++i) dstp[i] = src[i];
                }
            }
        }
        __syncthreads();
    }
    if (!STRESS && part && slot_ok) {
        uint4 *p = (uint4 *)(part + ((size_t)local_slot * gridDim.x + blockIdx.x) * kCountLevels);
#pragma unroll
        for (int q = 0; q < kCountLevels / 4; ++q) p[q] = make_uint4(cnt[4 * q], cnt[4 * q + 1], cnt[4 * q + 2], cnt[4 * q + 3]);
    }
}

// The same transpose with the stores staged in LDS: each wave leaves the hop
// bytes of its 64 sources for TILES 64-vertex tiles (64 * TILES bytes per
// source) in LDS, and the whole block then writes the rows out as whole
// segments (8 * TILES threads per row), instead of 16 bytes into 64
// different rows per store.  Needs rows aligned to 8 * TILES bytes.
// With STRESS the staged bytes are not stored: each row's stress terms
// ((h - |X_s - X_v|) / h)^2 over reachable v != s (Sec. 4.1.3) are summed in
// FP64 instead, one partial sum and pair count per (slot, block).
// PL (4 or 8) bounds the planes in use; the launcher picks it from
// planes_arg, an upper bound of the count read from planes_dev when that is
// set, so that each form gets its own register budget.
template <int WORDS, int TILES, bool STRESS, int PL>
__global__ void __launch_bounds__(WORDS * GM_WAVE) __attribute__((amdgpu_waves_per_eu(STRESS || PL > 4 ? 1 : 4)))
msbfs_hops_staged_kernel(MsbfsArgs a, int planes_arg, uint8_t *__restrict__ hop_out,
                         const int64_t *__restrict__ slot_row, int64_t row_stride, unsigned int *__restrict__ part,
                         StressArgs sa)
{
    const int planes_used = min(a.planes_dev ? *a.planes_dev : planes_arg, PL);
    constexpr int ROWS = WORDS * GM_WAVE;
    constexpr int PITCH = 64 * TILES + 8 * TILES;
    __shared__ __align__(16) uint8_t stage[ROWS * PITCH];
    __shared__ int64_t row_base[ROWS];
    __shared__ int s_depth;
    __shared__ double rinv[STRESS ? 256 : 1];   // 1 / h for the stress terms
    const int32_t g = blockIdx.y;
    const int32_t local_slot = g * ROWS + threadIdx.x;
    // store / stress rows of this thread: r = threadIdx.x / 8 + it * ROWS / 8
    double st_sum[kStressIts];
    unsigned int st_cnt[kStressIts];
    float2 st_xy[kStressIts];
    if (STRESS) {
        for (int h = threadIdx.x; h < 256; h += blockDim.x) rinv[h] = h ? 1.0 / (double)h : 0.0;
#pragma unroll
        for (int it = 0; it < kStressIts; ++it) {
            st_sum[it] = 0.0;
            st_cnt[it] = 0;
            const int32_t ls = g * ROWS + (threadIdx.x >> 3) + it * (ROWS >> 3);
            st_xy[it] = ls < a.n_slots ? sa.xy[a.usrc[a.slot0 + ls]] : make_float2(0.0f, 0.0f);
        }
    } else {
        row_base[threadIdx.x] = local_slot < a.n_slots ? slot_row[local_slot] * row_stride : -1;
    }
    const int depth = group_depth(a, g, &s_depth);
    hops_staged_body<WORDS, TILES, STRESS, PL>(a, planes_used, depth, hop_out, part, sa, stage, row_base, rinv, st_sum,
                                               st_cnt, st_xy);
    if (STRESS) {
        // the 8 threads of a row are adjacent lanes: reduce, then one writes
#pragma unroll
        for (int it = 0; it < kStressIts; ++it) {
            double v = st_sum[it];
            unsigned int c = st_cnt[it];
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                v += __shfl_xor(v, o, GM_WAVE);
                c += __shfl_xor(c, o, GM_WAVE);
            }
            const int32_t ls = g * ROWS + (threadIdx.x >> 3) + it * (ROWS >> 3);
            if ((threadIdx.x & 7) == 0 && ls < a.n_slots) {
                sa.part_sum[(size_t)ls * gridDim.x + blockIdx.x] = v;
                sa.part_pairs[(size_t)ls * gridDim.x + blockIdx.x] = c;
            }
        }
    }
}

template <int WORDS>
hipError_t launch_hops_words(dim3 grid, int variant, const MsbfsArgs &a, int planes_used, uint8_t *hop_out,
                             const int64_t *slot_row, int64_t row_stride, unsigned int *part, hipStream_t s)
{
    dim3 block(WORDS * GM_WAVE);
    const bool a16 = (row_stride % 16) == 0 && (((uintptr_t)hop_out) & 15) == 0;
    const bool a8 = (row_stride % 8) == 0 && (((uintptr_t)hop_out) & 7) == 0;
    const StressArgs none{};
    const bool pl4 = planes_used <= 4;
    if (variant == 0 && a16) {
        if (pl4)
            hipLaunchKernelGGL((msbfs_hops_staged_kernel<WORDS, 2, false, 4>), grid, block, 0, s, a, planes_used, hop_out, slot_row, row_stride, part, none);
        else
            hipLaunchKernelGGL((msbfs_hops_staged_kernel<WORDS, 2, false, 8>), grid, block, 0, s, a, planes_used, hop_out, slot_row, row_stride, part, none);
    } else if ((variant == 0 || variant == 3) && a8) {
        if (pl4)
            hipLaunchKernelGGL((msbfs_hops_staged_kernel<WORDS, 1, false, 4>), grid, block, 0, s, a, planes_used, hop_out, slot_row, row_stride, part, none);
        else
            hipLaunchKernelGGL((msbfs_hops_staged_kernel<WORDS, 1, false, 8>), grid, block, 0, s, a, planes_used, hop_out, slot_row, row_stride, part, none);
    }
    else if (variant == 2)
        hipLaunchKernelGGL((msbfs_hops_kernel<WORDS, 2, false>), grid, block, 0, s, a, planes_used, hop_out, slot_row, row_stride, part);
    else
        hipLaunchKernelGGL((msbfs_hops_kernel<WORDS, 1, false>), grid, block, 0, s, a, planes_used, hop_out, slot_row, row_stride, part);
    return hipGetLastError();
}

template <int WORDS>
void launch_stress_words(dim3 grid, const MsbfsArgs &a, int planes_used, const StressArgs &sa, hipStream_t s)
{
    if (planes_used <= 4)
        hipLaunchKernelGGL((msbfs_hops_staged_kernel<WORDS, 2, true, 4>), grid, dim3(WORDS * GM_WAVE), 0, s, a, planes_used, nullptr, nullptr, 0, nullptr, sa);
    else
        hipLaunchKernelGGL((msbfs_hops_staged_kernel<WORDS, 2, true, 8>), grid, dim3(WORDS * GM_WAVE), 0, s, a, planes_used, nullptr, nullptr, 0, nullptr, sa);
}

}  // namespace

template <int WORDS>
void launch_level_words(int verts, dim3 grid, hipStream_t s, const MsbfsArgs &a, int level, int co, int light,
                        int per_group, int xcd)
{
    if (verts == 8)
        hipLaunchKernelGGL((msbfs_level_kernel<WORDS, 8>), grid, dim3(kLevelBlock), 0, s, a, level, co, light, per_group, xcd);
    else if (verts == 4)
        hipLaunchKernelGGL((msbfs_level_kernel<WORDS, 4>), grid, dim3(kLevelBlock), 0, s, a, level, co, light, per_group, xcd);
    else if (verts == 2)
        hipLaunchKernelGGL((msbfs_level_kernel<WORDS, 2>), grid, dim3(kLevelBlock), 0, s, a, level, co, light, per_group, xcd);
    else
        hipLaunchKernelGGL((msbfs_level_kernel<WORDS, 1>), grid, dim3(kLevelBlock), 0, s, a, level, co, light, per_group, xcd);
}

template <int WORDS>
void launch_first_words(const MsbfsArgs &a, hipStream_t s)
{
    const int64_t items = (int64_t)a.n * WORDS;
    const unsigned fill_blocks = (unsigned)std::min<int64_t>((items + 255) / 256, 65535);
    hipLaunchKernelGGL(msbfs_first_fill_kernel<WORDS>, dim3(fill_blocks, (unsigned)a.groups), dim3(256), 0, s, a);
    hipLaunchKernelGGL(msbfs_first_scatter_kernel<WORDS>, dim3((unsigned)((a.n_slots + 3) / 4)), dim3(256), 0, s, a);
}

hipError_t launch_msbfs_first(const MsbfsArgs &a, hipStream_t s)
{
    if (a.n <= 0 || a.n_slots <= 0) return hipSuccess;
    switch (a.words) {
    case 1: launch_first_words<1>(a, s); break;
    case 2: launch_first_words<2>(a, s); break;
    case 4: launch_first_words<4>(a, s); break;
    case 8: launch_first_words<8>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_msbfs_level(const MsbfsArgs &a, int level, bool commit_only, hipStream_t s)
{
    const int64_t items = (int64_t)a.n * a.words;
    const int verts = a.level_verts == 2 || a.level_verts == 4 || a.level_verts == 8 ? a.level_verts : 1;
    const int light = (int)((items + (int64_t)kLevelBlock * verts - 1) / ((int64_t)kLevelBlock * verts));
    const int heavy = level >= 2 ? (a.n_heavy + kLevelBlock / GM_WAVE - 1) / (kLevelBlock / GM_WAVE) : 0;
    const int per_group = light + heavy;
    const int xcd = (a.xcd_map && a.groups % 8 == 0) ? 1 : 0;
    dim3 grid((unsigned)((int64_t)per_group * a.groups));
    const int co = commit_only ? 1 : 0;
    switch (a.words) {
    case 1: launch_level_words<1>(verts, grid, s, a, level, co, light, per_group, xcd); break;
    case 2: launch_level_words<2>(verts, grid, s, a, level, co, light, per_group, xcd); break;
    case 4: launch_level_words<4>(verts, grid, s, a, level, co, light, per_group, xcd); break;
    case 8: launch_level_words<8>(verts, grid, s, a, level, co, light, per_group, xcd); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_msbfs_push(const MsbfsArgs &a, int level, hipStream_t s)
{
    const int64_t items = (int64_t)a.n * a.words;
    const int light = (int)((items + kLevelBlock - 1) / kLevelBlock);
    const int chunk = (GM_WAVE / std::max(1, a.words)) * kHeavyBatch;   // adjacency entries per heavy wave
    const int chunks = std::max(1, (a.heavy_maxdeg + chunk - 1) / chunk);
    const int64_t heavy_waves = (int64_t)a.n_heavy * chunks;
    const int heavy = (int)((heavy_waves + kLevelBlock / GM_WAVE - 1) / (kLevelBlock / GM_WAVE));
    const int per_group = light + heavy;
    dim3 grid((unsigned)((int64_t)per_group * a.groups));
    switch (a.words) {
    case 1: hipLaunchKernelGGL(msbfs_push_kernel<1>, grid, dim3(kLevelBlock), 0, s, a, level, light, per_group, chunks); break;
    case 2: hipLaunchKernelGGL(msbfs_push_kernel<2>, grid, dim3(kLevelBlock), 0, s, a, level, light, per_group, chunks); break;
    case 4: hipLaunchKernelGGL(msbfs_push_kernel<4>, grid, dim3(kLevelBlock), 0, s, a, level, light, per_group, chunks); break;
    case 8: hipLaunchKernelGGL(msbfs_push_kernel<8>, grid, dim3(kLevelBlock), 0, s, a, level, light, per_group, chunks); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t msbfs_fused_lds_bytes(int32_t n) { return 3 * (size_t)n * sizeof(uint64_t); }

hipError_t launch_msbfs_fused(const MsbfsArgs &a, int L_cap, bool full_hops, int32_t *group_out, hipStream_t s)
{
    if (a.words != 1 || a.groups <= 0) return hipErrorInvalidValue;
    const size_t lds = msbfs_fused_lds_bytes(a.n);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static size_t lds_set[64] = {};   // the LDS limit is an attribute of the kernel on each device
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (lds > 48 * 1024 && lds > lds_set[dev]) {
        e = hipFuncSetAttribute((const void *)msbfs_fused_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set[dev] = lds;
    }
    hipLaunchKernelGGL(msbfs_fused_kernel, dim3(a.groups), dim3(kFusedBlock), lds, s, a, L_cap, full_hops ? 1 : 0,
                       group_out);
    return hipGetLastError();
}

size_t msbfs_fused_rows_lds_bytes(int32_t n, int32_t nnz)
{
    return 3 * (size_t)n * sizeof(uint64_t) + 64 * kCountLevels * sizeof(unsigned int) +
           ((size_t)n + 1 + (size_t)nnz) * sizeof(int32_t) + 64 * (size_t)n + 16;
}

hipError_t launch_msbfs_fused_rows(const MsbfsArgs &a, int L_cap, bool full_hops, int32_t nnz, uint8_t *hop_out,
                                   const int64_t *hop_row, int64_t row_stride, unsigned int *part,
                                   int32_t *group_out, hipStream_t s)
{
    if (a.words != 1 || a.groups <= 0 || a.n > kRowsVerts * kFusedBlock) return hipErrorInvalidValue;
    const size_t lds = msbfs_fused_rows_lds_bytes(a.n, nnz);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static size_t lds_set[64] = {};
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (lds > 48 * 1024 && lds > lds_set[dev]) {
        e = hipFuncSetAttribute((const void *)msbfs_fused_rows_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        if (e != hipSuccess) return e;
        lds_set[dev] = lds;
    }
    hipLaunchKernelGGL(msbfs_fused_rows_kernel, dim3(a.groups), dim3(kFusedBlock), lds, s, a, L_cap,
                       full_hops ? 1 : 0, nnz, hop_out, hop_row, row_stride, part, group_out);
    return hipGetLastError();
}

hipError_t launch_heavy_list(int32_t n, const int32_t *row_ptr, int32_t forced, int32_t *heavy, int32_t *info,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<int64_t>(4096, ((int64_t)n + 255) / 256);
    hipLaunchKernelGGL(heavy_list_kernel, dim3(blocks), dim3(256), 0, s, n, row_ptr, forced, heavy, info);
    return hipGetLastError();
}

hipError_t launch_msbfs_depth(const MsbfsArgs &a, int first, int last, int32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(msbfs_depth_kernel, dim3(1), dim3(kDepthThreads), 0, s, (const unsigned long long *)a.stats,
                       a.stats_groups, first, last, out);
    return hipGetLastError();
}

int msbfs_stat_fields() { return kStatFields; }
int msbfs_stat_spread() { return kSpread; }

// Blocks per group of the hop-row transpose: about two resident blocks per
// compute unit over all groups, each taking an equal share of the tiles (at
// least two).
int msbfs_hop_chunks(int32_t n, int32_t groups)
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
            (void)hipGetLastError();
            cus = 256;
        }
    }
    const int32_t ntiles = (n + 63) / 64;
    const int32_t per_group = std::max(1, 2 * cus / std::max(1, groups));
    return std::max(1, std::min(per_group, (ntiles + 1) / 2));
}

hipError_t launch_msbfs_hops_counted(const MsbfsArgs &a, int planes_used, uint8_t *hop_out,
                                     const int64_t *slot_row, int64_t row_stride,
                                     unsigned int *part, hipStream_t s)
{
    dim3 grid((unsigned)msbfs_hop_chunks(a.n, a.groups), (unsigned)a.groups);
    const int variant = a.hops_variant;
    switch (a.words) {
    case 1: return launch_hops_words<1>(grid, variant, a, planes_used, hop_out, slot_row, row_stride, part, s);
    case 2: return launch_hops_words<2>(grid, variant, a, planes_used, hop_out, slot_row, row_stride, part, s);
    case 4: return launch_hops_words<4>(grid, variant, a, planes_used, hop_out, slot_row, row_stride, part, s);
    case 8: return launch_hops_words<8>(grid, variant, a, planes_used, hop_out, slot_row, row_stride, part, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_msbfs_stress(const MsbfsArgs &a, int planes_used, const StressArgs &sa, hipStream_t s)
{
    dim3 grid((unsigned)msbfs_hop_chunks(a.n, a.groups), (unsigned)a.groups);
    switch (a.words) {
    case 1: launch_stress_words<1>(grid, a, planes_used, sa, s); break;
    case 2: launch_stress_words<2>(grid, a, planes_used, sa, s); break;
    case 4: launch_stress_words<4>(grid, a, planes_used, sa, s); break;
    case 8: launch_stress_words<8>(grid, a, planes_used, sa, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_msbfs_hops(const MsbfsArgs &a, int planes_used, uint8_t *hop_out,
                             const int64_t *slot_row, int64_t row_stride, hipStream_t s)
{
    return launch_msbfs_hops_counted(a, planes_used, hop_out, slot_row, row_stride, nullptr, s);
}

}  // namespace gm
