// Truncated partial BFS (SL-/SSSL-GUMAP steps C0 + C1, Sec. 3.3.1, Alg. 4)
// and the UMAP membership kernels (Sec. 2.1).
//
// One wavefront per source v.  Level h+1 of the BFS consists of the
// neighbours of level h not seen before.  Adjacency rows are sorted, so the
// level can be produced in ascending id order by a k-way merge of the sorted
// rows of level h (one row head per lane, wave-wide minimum per step): every
// value comes out once, values already seen (v and the earlier levels, at
// most k + 1 of them, held one per lane) are skipped, and the merge stops the
// moment the k-th neighbour is taken.  Levels before the last therefore come
// out complete and in id order, and the last one contributes exactly its
// smallest ids -- the (hop, id) order -- while each neighbour row is read at
// most (needed + seen) entries deep, however large its degree.
#include <algorithm>
#include <cstdlib>

#include "device.h"
#include "kernels.h"
#include "membership.h"

namespace gm {

namespace {

constexpr int kPartialWaves = 4;
constexpr int kMaxRow = 256;     // k <= 254 picks; frontier and seen sets < 256
constexpr int kStashBytes = 2048; // hops of one chunk kept for the fused membership

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct WaveLds {
    int32_t fa[kMaxRow];      // current level (frontier)
    int32_t fb[kMaxRow];      // level being built
    int32_t seen[kMaxRow];    // v and all completed levels
    int32_t row_ids[kMaxRow];
    uint8_t row_hops[kMaxRow];
};

// NQ: 64-entry chunks needed for k + 1 seen vertices (1, 2 or 4).
// Leaves the row (ids, hops, padded) in s.row_ids / s.row_hops.
template <int NQ>
__device__ void partial_row(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                            int32_t v, int k, WaveLds &s)
{
    const int l = lane();
    // level 1: the first min(deg, k) entries of v's sorted row
    const int32_t e0 = rp[v], e1 = rp[v + 1];
    const int t1 = min(e1 - e0, k);
    if (l == 0) s.seen[0] = v;
    for (int i = l; i < t1; i += 64) {
        const int32_t u = col[e0 + i];
        s.fa[i] = u;
        s.seen[1 + i] = u;
        s.row_ids[i] = u;
        s.row_hops[i] = 1;
    }
    wave_sync();
    int nf = t1, nseen = 1 + t1, taken = t1, h = 1;
    int32_t *fa = s.fa, *fb = s.fb;
    while (taken < k && nf > 0) {
        ++h;
        int32_t p[NQ], e[NQ], hv[NQ], sv[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = l + 64 * q;
            hv[q] = GM_INF_ID;
            p[q] = 0;
            e[q] = 0;
            if (j < nf) {
                const int32_t u = fa[j];
                p[q] = rp[u];
                e[q] = rp[u + 1];
                if (p[q] < e[q]) hv[q] = col[p[q]];
            }
            sv[q] = j < nseen ? s.seen[j] : -1;
        }
        int nnew = 0;
        for (;;) {
            int mine = hv[0];
#pragma unroll
            for (int q = 1; q < NQ; ++q) mine = min(mine, hv[q]);
            const int m = wave_min(mine);
            if (m == GM_INF_ID) break;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (hv[q] == m) {
                    ++p[q];
                    hv[q] = p[q] < e[q] ? col[p[q]] : GM_INF_ID;
                }
            }
            bool hit = false;
#pragma unroll
            for (int q = 0; q < NQ; ++q) hit |= (sv[q] == m);
            if (__ballot(hit) == 0ull) {
                if (l == 0) {
                    fb[nnew] = m;
                    s.row_ids[taken] = m;
                    s.row_hops[taken] = (uint8_t)h;
                }
                ++nnew;
                ++taken;
                if (taken == k) break;
            }
        }
        wave_sync();
        for (int j = l; j < nnew; j += 64) s.seen[nseen + j] = fb[j];
        nseen += nnew;
        int32_t *t = fa;
        fa = fb;
        fb = t;
        nf = nnew;
        wave_sync();
    }
    for (int i = taken + l; i < k; i += 64) {
        s.row_ids[i] = -1;
        s.row_hops[i] = 255;
    }
    wave_sync();
}

// Minimum over each group of ROW lanes (ROW = 16, 32 or 64): DPP inside a
// 16-lane row (mirror, half-mirror and two quad permutations reach all 16),
// shuffles across rows.
template <int ROW>
__device__ __forceinline__ int group_min(int x)
{
    x = min(x, __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false));   // row_mirror
    x = min(x, __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false));   // row_half_mirror
    x = min(x, __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
    x = min(x, __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
    if (ROW >= 32) x = min(x, __shfl_xor(x, 16, GM_WAVE));
    if (ROW >= 64) x = min(x, __shfl_xor(x, 32, GM_WAVE));
    return x;
}

// The same search with one group of ROW lanes per source (64 / ROW sources
// per wave) and all state in registers: lane j of a group holds the j-th
// vertex of the seen set, the j-th frontier vertex with a window of the next
// four entries of its sorted row, and entry j of the output row.  Needs
// k + 1 <= ROW.  v < 0 marks an idle group.  On return lane j of the group
// holds (id, hop) of entry j (padding -1 / 255 past the last neighbour).
template <int ROW>
__device__ void partial_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t v,
                             int k, int32_t &my_id, int &my_hop)
{
    const int l = lane();
    const int rl = l & (ROW - 1);
    const int rb = l & ~(ROW - 1);
    const unsigned long long gmask = ROW == 64 ? ~0ull : (((1ull << ROW) - 1ull) << rb);
    // Level 1 is the sorted row of v itself: its first min(deg, k) entries,
    // read in one coalesced load (rows hold no self-loop).
    int32_t e0 = 0, e1 = 0;
    if (v >= 0) {
        e0 = rp[v];
        e1 = rp[v + 1];
    }
    const int t1 = min(e1 - e0, k);
    const int32_t x = rl < t1 ? col[e0 + rl] : -1;
    my_id = rl < t1 ? x : -1;
    my_hop = rl < t1 ? 1 : 255;
    // seen set: v in lane 0, level 1 in lanes 1..t1; the frontier is level 1
    const int32_t up = __shfl(x, rb + (rl > 0 ? rl - 1 : 0), GM_WAVE);
    int32_t sv = rl == 0 ? v : (rl - 1 < t1 ? up : -1);
    int32_t fr = x;
    int taken = t1, nf = t1, nseen = 1 + t1, h = 1;
    for (;;) {
        const bool go = taken < k && nf > 0;
        if (__ballot(go) == 0ull) break;
        ++h;
        int32_t p = 0, e = 0, w0 = GM_INF_ID, w1 = GM_INF_ID, w2 = GM_INF_ID, w3 = GM_INF_ID;
        if (go && rl < nf) {
            p = rp[fr];
            e = rp[fr + 1];
            if (p < e) w0 = col[p];
            if (p + 1 < e) w1 = col[p + 1];
            if (p + 2 < e) w2 = col[p + 2];
            if (p + 3 < e) w3 = col[p + 3];
            p += 4;
        }
        int nnew = 0;
        int32_t nfr = -1;
        bool open = go;
        for (;;) {
            const int m = group_min<ROW>(open ? w0 : GM_INF_ID);
            const bool live = open && m != GM_INF_ID;
            if (__ballot(live) == 0ull) break;
            if (live && w0 == m) {
                w0 = w1;
                w1 = w2;
                w2 = w3;
                w3 = GM_INF_ID;
                if (w0 == GM_INF_ID && p < e) {
                    w0 = col[p];
                    if (p + 1 < e) w1 = col[p + 1];
                    if (p + 2 < e) w2 = col[p + 2];
                    if (p + 3 < e) w3 = col[p + 3];
                    p += 4;
                }
            }
            const bool hit = (__ballot(live && sv == m) & gmask) != 0ull;
            if (live && !hit) {
                if (rl == taken) {
                    my_id = m;
                    my_hop = h;
                }
                if (rl == nnew) nfr = m;
                ++taken;
                ++nnew;
                if (taken == k) open = false;
            }
            if (!live) open = false;
        }
        // the finished level joins the seen set: lane nseen + j takes the j-th new vertex
        const int src = rl - nseen;
        const int32_t moved = __shfl(nfr, rb + (src >= 0 && src < ROW ? src : 0), GM_WAVE);
        if (go) {
            if (src >= 0 && src < nnew) sv = moved;
            nseen += nnew;
            fr = nfr;
            nf = nnew;
        }
    }
}

template <int NQ>
__global__ void __launch_bounds__(kPartialWaves * GM_WAVE)
partial_bfs_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int k,
                   int32_t *__restrict__ ids, uint8_t *__restrict__ hops)
{
    __shared__ WaveLds lds[kPartialWaves];
    const int wid = threadIdx.x / GM_WAVE, l = lane();
    WaveLds &s = lds[wid];
    for (int64_t v = (int64_t)blockIdx.x * kPartialWaves + wid; v < n;
         v += (int64_t)gridDim.x * kPartialWaves) {
        partial_row<NQ>(rp, col, (int32_t)v, k, s);
        const int64_t o = v * k;
        for (int i = l; i < k; i += 64) {
            ids[o + i] = s.row_ids[i];
            hops[o + i] = s.row_hops[i];
        }
        wave_sync();
    }
}

template <int ROW>
__global__ void __launch_bounds__(kPartialWaves * GM_WAVE)
partial_rows_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int k,
                    int32_t *__restrict__ ids, uint8_t *__restrict__ hops)
{
    constexpr int PER_WAVE = GM_WAVE / ROW;
    const int wid = threadIdx.x / GM_WAVE, l = lane(), rl = l & (ROW - 1);
    const int64_t step = (int64_t)gridDim.x * kPartialWaves * PER_WAVE;
    for (int64_t base = ((int64_t)blockIdx.x * kPartialWaves + wid) * PER_WAVE; base < n; base += step) {
        const int64_t v = base + l / ROW;
        int32_t my_id;
        int my_hop;
        partial_rows<ROW>(rp, col, v < n ? (int32_t)v : -1, k, my_id, my_hop);
        if (v < n && rl < k) {
            ids[v * k + rl] = my_id;
            hops[v * k + rl] = (uint8_t)my_hop;
        }
    }
}

// Rows [begin, end) of one graph (begin..end at most kStashBytes / k rows):
// partial BFS per row, rows written out, and, when weights are wanted, the
// membership of the chunk's rows computed one row per lane from the hops
// kept in LDS.  Output row of local vertex v is out_row0 + (v - begin).
template <int NQ, int ROW>
__device__ void chunk_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int k,
                           int32_t begin, int32_t end, int64_t out_row0, int32_t *ids, uint8_t *hops,
                           float *weights, float *rho, float *sigma, WaveLds &s, uint8_t *stash)
{
    const int l = lane();
    if (ROW > 0) {
        constexpr int R = ROW > 0 ? ROW : 64;
        constexpr int PER_WAVE = GM_WAVE / R;
        const int rl = l & (R - 1);
        for (int32_t v0 = begin; v0 < end; v0 += PER_WAVE) {
            const int32_t v = v0 + l / R;
            int32_t my_id;
            int my_hop;
            partial_rows<R>(rp, col, v < end ? v : -1, k, my_id, my_hop);
            if (v < end && rl < k) {
                const int slot = v - begin;
                const int64_t o = (out_row0 + slot) * k;
                ids[o + rl] = my_id;
                hops[o + rl] = (uint8_t)my_hop;
                stash[slot * k + rl] = (uint8_t)my_hop;
            }
        }
        wave_sync();
    } else {
        for (int32_t v = begin; v < end; ++v) {
            partial_row<NQ>(rp, col, v, k, s);
            const int slot = v - begin;
            const int64_t o = (out_row0 + slot) * k;
            for (int i = l; i < k; i += 64) {
                ids[o + i] = s.row_ids[i];
                hops[o + i] = s.row_hops[i];
                stash[slot * k + i] = s.row_hops[i];
            }
            wave_sync();
        }
    }
    if (weights && l < end - begin) {
        const uint8_t *hrow = stash + l * k;
        const int64_t r = out_row0 + l;
        membership_row([&](int j) { return (int)hrow[j]; }, k, weights + r * k, rho ? rho + r : nullptr,
                       sigma ? sigma + r : nullptr);
    }
    wave_sync();
}

// Batched persistent form: waves take chunks of packed vertices from a device
// counter (a chunk may span several graphs).
template <int NQ, int ROW>
__global__ void __launch_bounds__(kPartialWaves * GM_WAVE)
partial_batch_kernel(BatchArgs a)
{
    __shared__ WaveLds lds[kPartialWaves];
    __shared__ uint8_t stash[kPartialWaves][kStashBytes];
    const int wid = threadIdx.x / GM_WAVE, l = lane();
    WaveLds &s = lds[wid];
    for (;;) {
        unsigned long long start = 0;
        if (l == 0) start = atomicAdd(a.work_counter, (unsigned long long)a.chunk);
        start = __shfl(start, 0, GM_WAVE);
        if ((int64_t)start >= a.total_vertices) break;
        const int64_t end = min((int64_t)start + a.chunk, a.total_vertices);
        // graph of the first vertex: last g with vtx_offset[g] <= start
        int lo = 0, hi = a.n_graphs;   // vtx_offset[lo] <= start < vtx_offset[hi]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (a.vtx_offset[mid] <= (int64_t)start) lo = mid;
            else hi = mid;
        }
        int64_t gi = (int64_t)start;
        for (int g = lo; gi < end; ++g) {
            const int64_t voff = a.vtx_offset[g], vend = a.vtx_offset[g + 1];
            if (vend <= gi) continue;
            const int64_t stop = min(end, vend);
            chunk_rows<NQ, ROW>(a.row_ptr + voff + g, a.col + a.edge_offset[g], a.k, (int32_t)(gi - voff),
                           (int32_t)(stop - voff), gi, a.ids, a.hops, a.weights, a.rho, a.sigma, s,
                           stash[wid]);
            gi = stop;
        }
    }
}

// Served form: an explicit list of (job, first row, end row) chunks over a
// table of resident jobs.
template <int NQ, int ROW>
__global__ void __launch_bounds__(kPartialWaves * GM_WAVE)
partial_jobs_kernel(const DevJob *__restrict__ jobs, const JobChunk *__restrict__ chunks, int32_t n_chunks,
                    unsigned long long *counter)
{
    __shared__ WaveLds lds[kPartialWaves];
    __shared__ uint8_t stash[kPartialWaves][kStashBytes];
    const int wid = threadIdx.x / GM_WAVE, l = lane();
    WaveLds &s = lds[wid];
    for (;;) {
        unsigned long long c = 0;
        if (l == 0) c = atomicAdd(counter, 1ull);
        c = __shfl(c, 0, GM_WAVE);
        if ((int64_t)c >= n_chunks) break;
        const JobChunk ch = chunks[c];
        const DevJob &j = jobs[ch.job];
        chunk_rows<NQ, ROW>(j.row_ptr, j.col, j.k, ch.begin, ch.end, ch.begin, j.ids, j.hops, j.weights, j.rho,
                       j.sigma, s, stash[wid]);
    }
}

__global__ void batch_reset_kernel(unsigned long long *counter) { *counter = 0ull; }

// Rows of k <= kMembStageK: a block of kMembRows threads, one row each,
// with its rows' hop bytes and weights staged in LDS so that the global
// reads and writes are contiguous runs instead of k-strided ones.
constexpr int kMembRows = 256;
constexpr int kMembStageK = 32;

__global__ void __launch_bounds__(kMembRows)
membership_staged_kernel(int32_t rows, int32_t k, const uint8_t *__restrict__ hops, float *__restrict__ weights,
                         float *__restrict__ rho, float *__restrict__ sigma)
{
    __shared__ uint8_t hs[kMembRows * kMembStageK];
    __shared__ float ws[kMembRows * kMembStageK];
    const int64_t r0 = (int64_t)blockIdx.x * kMembRows;
    const int nr = (int)min((int64_t)kMembRows, (int64_t)rows - r0);
    const int cells = nr * k;
    const uint8_t *src = hops + r0 * k;
    for (int i = threadIdx.x; i < cells; i += kMembRows) hs[i] = src[i];
    __syncthreads();
    if ((int)threadIdx.x < nr) {
        const uint8_t *h = hs + threadIdx.x * k;
        membership_row([&](int j) { return (int)h[j]; }, k, ws + threadIdx.x * k,
                       rho ? rho + r0 + threadIdx.x : nullptr, sigma ? sigma + r0 + threadIdx.x : nullptr);
    }
    __syncthreads();
    float *dst = weights + r0 * k;
    for (int i = threadIdx.x; i < cells; i += kMembRows) dst[i] = ws[i];
}

__global__ void membership_kernel(int32_t rows, int32_t k, const uint8_t *__restrict__ hops,
                                  float *__restrict__ weights, float *__restrict__ rho,
                                  float *__restrict__ sigma)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t *h = hops + r * k;
        membership_row([&](int j) { return (int)h[j]; }, k, weights + r * k, rho ? rho + r : nullptr,
                       sigma ? sigma + r : nullptr);
    }
}

int nq_for(int k) { return k + 1 <= 64 ? 1 : (k + 1 <= 128 ? 2 : 4); }

// Lanes per source of the register-resident search (0: one wave per source
// with LDS state, the only form for k >= 64).  GUMAP_PARTIAL_LANES forces a
// width (0, 16, 32, 64) when k fits it; the result does not depend on it.
int lanes_for(int k)
{
    int auto_lanes = k + 1 <= 16 ? 16 : (k + 1 <= 32 ? 32 : (k + 1 <= 64 ? 64 : 0));
    const char *env = getenv("GUMAP_PARTIAL_LANES");
    if (env && *env) {
        int f = atoi(env);
        if (f == 0) return 0;
        if ((f == 16 || f == 32 || f == 64) && k + 1 <= f) return f;
    }
    return auto_lanes;
}

}  // namespace

hipError_t launch_partial_bfs(const PartialArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const dim3 block(kPartialWaves * GM_WAVE);
    const int lanes = lanes_for(a.k);
    if (lanes > 0) {
        const int64_t per_block = (int64_t)kPartialWaves * (GM_WAVE / lanes);
        const int blocks = (int)std::min<int64_t>(1048576, ((int64_t)a.n + per_block - 1) / per_block);
        if (lanes == 16)
            hipLaunchKernelGGL(partial_rows_kernel<16>, dim3(blocks), block, 0, s, a.n, a.row_ptr, a.col, a.k, a.ids, a.hops);
        else if (lanes == 32)
            hipLaunchKernelGGL(partial_rows_kernel<32>, dim3(blocks), block, 0, s, a.n, a.row_ptr, a.col, a.k, a.ids, a.hops);
        else
            hipLaunchKernelGGL(partial_rows_kernel<64>, dim3(blocks), block, 0, s, a.n, a.row_ptr, a.col, a.k, a.ids, a.hops);
        return hipGetLastError();
    }
    int64_t blocks64 = ((int64_t)a.n + kPartialWaves - 1) / kPartialWaves;
    int blocks = (int)(blocks64 > 1048576 ? 1048576 : blocks64);
    switch (nq_for(a.k)) {
    case 1: hipLaunchKernelGGL(partial_bfs_kernel<1>, dim3(blocks), block, 0, s, a.n, a.row_ptr, a.col, a.k, a.ids, a.hops); break;
    case 2: hipLaunchKernelGGL(partial_bfs_kernel<2>, dim3(blocks), block, 0, s, a.n, a.row_ptr, a.col, a.k, a.ids, a.hops); break;
    default: hipLaunchKernelGGL(partial_bfs_kernel<4>, dim3(blocks), block, 0, s, a.n, a.row_ptr, a.col, a.k, a.ids, a.hops); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_reset(unsigned long long *counter, hipStream_t s)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, counter);
    return hipGetLastError();
}

int batch_chunk_rows(int k)
{
    int c = kStashBytes / k;
    return c > 64 ? 64 : (c < 1 ? 1 : c);
}

#define GM_BATCH_LAUNCH(NQ_, ROW_) \
    hipLaunchKernelGGL((partial_batch_kernel<NQ_, ROW_>), dim3(a.blocks), dim3(kPartialWaves * GM_WAVE), 0, s, a)

int partial_lane_options(int k, int32_t *out)
{
    int c = 0;
    for (int l : {16, 32, 64})
        if (k + 1 <= l) out[c++] = l;
    out[c++] = -1;
    return c;
}

hipError_t launch_partial_batch(const BatchArgs &a, hipStream_t s)
{
    if (a.total_vertices <= 0) return hipSuccess;
    if (a.chunk < 1 || a.chunk > batch_chunk_rows(a.k)) return hipErrorInvalidValue;
    if (a.lanes > 0 && (a.k + 1 > a.lanes || (a.lanes != 16 && a.lanes != 32 && a.lanes != 64)))
        return hipErrorInvalidValue;
    const int lanes = a.lanes == 0 ? lanes_for(a.k) : (a.lanes < 0 ? 0 : a.lanes);
    if (lanes == 16) GM_BATCH_LAUNCH(1, 16);
    else if (lanes == 32) GM_BATCH_LAUNCH(1, 32);
    else if (lanes == 64) GM_BATCH_LAUNCH(1, 64);
    else if (nq_for(a.k) == 1) GM_BATCH_LAUNCH(1, 0);
    else if (nq_for(a.k) == 2) GM_BATCH_LAUNCH(2, 0);
    else GM_BATCH_LAUNCH(4, 0);
    return hipGetLastError();
}

#define GM_JOBS_LAUNCH(NQ_, ROW_)                                                                              \
    hipLaunchKernelGGL((partial_jobs_kernel<NQ_, ROW_>), dim3(blocks), dim3(kPartialWaves * GM_WAVE), 0, s, jobs, \
                       chunks, n_chunks, counter)

hipError_t launch_partial_jobs(const DevJob *jobs, const JobChunk *chunks, int32_t n_chunks, int max_k,
                               unsigned long long *counter, int blocks, hipStream_t s)
{
    if (n_chunks <= 0) return hipSuccess;
    const int lanes = lanes_for(max_k);
    if (lanes == 16) GM_JOBS_LAUNCH(1, 16);
    else if (lanes == 32) GM_JOBS_LAUNCH(1, 32);
    else if (lanes == 64) GM_JOBS_LAUNCH(1, 64);
    else if (nq_for(max_k) == 1) GM_JOBS_LAUNCH(1, 0);
    else if (nq_for(max_k) == 2) GM_JOBS_LAUNCH(2, 0);
    else GM_JOBS_LAUNCH(4, 0);
    return hipGetLastError();
}

int partial_batch_max_blocks()
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, partial_batch_kernel<1, 16>,
                                                     kPartialWaves * GM_WAVE, 0) != hipSuccess || per < 1)
        per = 4;
    return cus * per;
}

hipError_t launch_membership(int32_t rows, int32_t k, const uint8_t *hops, float *weights,
                             float *rho, float *sigma, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    if (k <= kMembStageK) {
        const int64_t blocks = ((int64_t)rows + kMembRows - 1) / kMembRows;
        hipLaunchKernelGGL(membership_staged_kernel, dim3((unsigned)blocks), dim3(kMembRows), 0, s, rows, k, hops,
                           weights, rho, sigma);
        return hipGetLastError();
    }
    int blocks = (rows + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(membership_kernel, dim3(blocks), dim3(256), 0, s, rows, k, hops, weights, rho, sigma);
    return hipGetLastError();
}

}  // namespace gm
