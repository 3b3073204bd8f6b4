// Small helper kernels of the host orchestration: fills, slot maps, checks
// of sorted input, and the conversions between the packed per-graph batch
// layout and one disjoint-union CSR.
#include "device.h"
#include "util.h"
#include "kernels.h"

#include <algorithm>
#include <climits>

namespace gm {

namespace {

int blocks_for(int64_t items, int threads = 256, int cap = 65536)
{
    int64_t b = (items + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

#define GRID_STRIDE(i, count)                                                              \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (count);         \
         i += (int64_t)gridDim.x * blockDim.x)

__global__ void fill_i32_k(int32_t *p, int64_t count, int32_t v) { GRID_STRIDE(i, count) p[i] = v; }
__global__ void iota_i32_k(int32_t *p, int64_t count) { GRID_STRIDE(i, count) p[i] = (int32_t)i; }
__global__ void iota_i64_k(int64_t *p, int64_t count, int64_t start) { GRID_STRIDE(i, count) p[i] = start + i; }
// Every vertex a source: slot = vertex = row, and the eight info words cleared.
__global__ void all_sources_setup_k(int32_t n, int32_t *usrc, int32_t *slot_of, int64_t *slot_row, int32_t *info)
{
    if (blockIdx.x == 0 && threadIdx.x < 8) info[threadIdx.x] = 0;
    GRID_STRIDE(i, (int64_t)n)
    {
        usrc[i] = (int32_t)i;
        slot_of[i] = (int32_t)i;
        slot_row[i] = i;
    }
}
__global__ void scatter_slots_k(const int32_t *usrc, int32_t count, int32_t *slot_of)
{
    GRID_STRIDE(i, count) slot_of[usrc[i]] = (int32_t)i;
}

// Listed sources: first row of each vertex (atomic minimum), times listed,
// bit 1 of info[0] for an id outside [0, n).
__global__ void source_first_k(const int32_t *src, int64_t rows, int32_t n, int32_t *first, int32_t *count,
                               int32_t *info)
{
    GRID_STRIDE(r, rows)
    {
        const int32_t v = src[r];
        if (v < 0 || v >= n) {
            atomicOr(&info[0], 1);
            continue;
        }
        atomicMin(&first[v], (int32_t)r);
        if (count) atomicAdd(&count[v], 1);
    }
}

__global__ void source_marks_k(int32_t n, const int32_t *first, int32_t *marks)
{
    GRID_STRIDE(v, (int64_t)n) marks[v] = first[v] != INT32_MAX ? 1 : 0;
}

// Unique sources in ascending id order: slot = exclusive prefix of the marks.
__global__ void source_slots_k(int32_t n, const int32_t *first, const int32_t *pos, const int32_t *count,
                               int32_t *usrc, int64_t *slot_row, int32_t *slot_of, int32_t *mult, int32_t *info)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) info[3] = pos[n];
    GRID_STRIDE(v, (int64_t)n)
    {
        if (first[v] != INT32_MAX) {
            const int32_t s = pos[v];
            usrc[s] = (int32_t)v;
            slot_row[s] = first[v];
            slot_of[v] = s;
            if (mult) mult[s] = count[v];
        } else {
            slot_of[v] = -1;
        }
    }
}

// Few listed sources on a small graph (at most kRankMax rows, kRankMaxN vertices).  First a pass over the
// vertices: not a source yet (first = INT32_MAX, slot -1, count 0), and the
// heavy-vertex list of the level kernel (info[1] entries, threshold info[2],
// largest degree among them info[4]).
constexpr int kRankThreads = 1024;
constexpr int kRankMax = 4096;
static_assert(kRankMax % kRankThreads == 0, "rows are read kRankMax / kRankThreads per thread");

__global__ void source_vertex_prep_k(int32_t n, const int32_t *__restrict__ rp, int32_t forced, int32_t *first,
                                     int32_t *count, int32_t *slot_of, int32_t *heavy, int32_t *info)
{
    const int32_t thr = heavy_threshold(n, rp, forced);
    if (blockIdx.x == 0 && threadIdx.x == 0) info[2] = thr;
    GRID_STRIDE(v, (int64_t)n)
    {
        first[v] = INT32_MAX;
        slot_of[v] = -1;
        if (count) count[v] = 0;
        if (rp[v + 1] - rp[v] > thr) {
            heavy[atomicAdd(&info[1], 1)] = (int32_t)v;
            atomicMax(&info[4], rp[v + 1] - rp[v]);
        }
    }
}

// Then one workgroup ranks the rows with an n-bit set of the listed vertices
// in LDS: the slot of a listed vertex is the number of listed vertices with
// a smaller id (word popcounts, prefix-summed); the first row and the times
// listed of each slot are LDS atomics over the rows.  Same outputs as the
// scan-based path for larger inputs.
constexpr int kRankMaxN = 131072;
constexpr int kRankWords = kRankMaxN / 64;

__device__ __forceinline__ int32_t rank_of(const uint64_t *bits, const int32_t *prefix, int32_t v)
{
    const int w = v >> 6, b = v & 63;
    return prefix[w] + __popcll(bits[w] & ((1ull << b) - 1ull));
}

__global__ void __launch_bounds__(kRankThreads)
source_rank_small_k(const int32_t *__restrict__ src, int32_t rows, int32_t n, int32_t *first, int32_t *count,
                    int32_t *usrc, int64_t *slot_row, int32_t *slot_of, int32_t *mult, int32_t *info,
                    int32_t *host_info)
{
    __shared__ uint64_t bits[kRankWords];
    __shared__ int32_t prefix[kRankWords];
    __shared__ int32_t first_row[kRankMax];
    __shared__ int32_t times[kRankMax];
    __shared__ int32_t wsum[kRankThreads / GM_WAVE];
    const int t = threadIdx.x;
    const int W = (n + 63) / 64;
    // this thread's rows t, t + kRankThreads, ... (rows <= kRankMax), read once
    constexpr int kPer = kRankMax / kRankThreads;
    int32_t sv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int r = t + j * kRankThreads;
        sv[j] = r < rows ? src[r] : 0;
    }
    for (int w = t; w < W; w += kRankThreads) bits[w] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int r = t + j * kRankThreads;
        if (r >= rows) continue;
        const int32_t v = sv[j];
        if (v < 0 || v >= n) atomicOr(&info[0], 1);
        else atomicOr(&bits[v >> 6], 1ull << (v & 63));
    }
    __syncthreads();
    // exclusive prefix of the word popcounts: thread t takes words [t * per, (t + 1) * per)
    const int per = (W + kRankThreads - 1) / kRankThreads;
    int local = 0;
    for (int w = t * per; w < min(W, (t + 1) * per); ++w) local += __popcll(bits[w]);
    int x = local;
    for (int o = 1; o < GM_WAVE; o <<= 1) {
        const int y = __shfl_up(x, o, GM_WAVE);
        if (lane() >= o) x += y;
    }
    if (lane() == GM_WAVE - 1) wsum[t / GM_WAVE] = x;
    __syncthreads();
    if (t == 0)
        for (int w = 1; w < kRankThreads / GM_WAVE; ++w) wsum[w] += wsum[w - 1];
    __syncthreads();
    int run = x - local + (t >= GM_WAVE ? wsum[t / GM_WAVE - 1] : 0);
    for (int w = t * per; w < min(W, (t + 1) * per); ++w) {
        prefix[w] = run;
        run += __popcll(bits[w]);
    }
    const int total = wsum[kRankThreads / GM_WAVE - 1];
    for (int q = t; q < total; q += kRankThreads) {
        first_row[q] = INT32_MAX;
        times[q] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int r = t + j * kRankThreads;
        const int32_t v = sv[j];
        if (r >= rows || v < 0 || v >= n) continue;
        const int32_t q = rank_of(bits, prefix, v);
        atomicMin(&first_row[q], r);
        atomicAdd(&times[q], 1);
    }
    __syncthreads();
    for (int w = t; w < W; w += kRankThreads) {
        uint64_t m = bits[w];
        int32_t q = prefix[w];
        while (m) {
            const int b = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int32_t v = 64 * w + b;
            usrc[q] = v;
            slot_of[v] = q;
            slot_row[q] = first_row[q];
            first[v] = first_row[q];
            if (mult) mult[q] = times[q];
            if (count) count[v] = times[q];
            ++q;
        }
    }
    if (t == 0) info[3] = total;
    if (host_info) {
        // the info words are final here (the vertex pass ran before this
        // launch, this block's atomics before its barriers): publish them to
        // pinned host memory, so that no copy follows
        __syncthreads();
        if (t == 0) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                host_info[i] = i == 3 ? total : __hip_atomic_load(&info[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Rows naming a source listed earlier copy that row's results.
__global__ void copy_dup_rows_k(const int32_t *src, int64_t rows, const int32_t *first, int32_t k, int32_t n,
                                int32_t *ids, uint8_t *hops, uint8_t *hop_matrix)
{
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t f = first[src[r]];
        if (f == r) continue;
        for (int i = threadIdx.x; i < k; i += blockDim.x) {
            ids[r * k + i] = ids[f * k + i];
            hops[r * k + i] = hops[f * k + i];
        }
        if (hop_matrix)
            for (int64_t i = threadIdx.x; i < n; i += blockDim.x) hop_matrix[r * (int64_t)n + i] = hop_matrix[f * (int64_t)n + i];
    }
}

// Rows strictly increasing, no self-loops (bit 32 of *err otherwise).
__global__ void check_sorted_k(int32_t n, const int32_t *rp, const int32_t *col, int *err)
{
    int bad = 0;
    GRID_STRIDE(v, (int64_t)n)
    {
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            if (col[e] == v) bad = 32;
            if (e > rp[v] && col[e] <= col[e - 1]) bad = 32;
        }
    }
    if (bad) atomicOr(err, bad);
}

__device__ __forceinline__ int graph_of(const int64_t *off, int32_t n_graphs, int64_t x)
{
    // last g with off[g] <= x (off[0] = 0 <= x < off[n_graphs])
    int lo = 0, hi = n_graphs;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Packed batch structure (offsets already checked on the host): local row
// pointers consistent and local ids in range.  Bits: 128 row pointers, 256 ids.
__global__ void validate_batch_k(int32_t n_graphs, const int64_t *voff, const int64_t *eoff,
                                 const int32_t *rp, const int32_t *col, int64_t total_v,
                                 int64_t total_e, int *err)
{
    int bad = 0;
    GRID_STRIDE(i, total_v + n_graphs)
    {
        // entry i of the packed row pointers belongs to graph g with
        // voff[g] + g <= i <= voff[g + 1] + g
        int lo = 0, hi = n_graphs;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (voff[mid] + mid <= i) lo = mid;
            else hi = mid;
        }
        const int g = lo;
        const int64_t local = i - (voff[g] + g);
        const int64_t ng = voff[g + 1] - voff[g], ne = eoff[g + 1] - eoff[g];
        const int32_t x = rp[i];
        if (local == 0 && x != 0) bad |= 128;
        if (local == ng && x != ne) bad |= 128;
        if (x < 0 || x > ne) bad |= 128;
        if (local < ng && rp[i + 1] < x) bad |= 128;
    }
    GRID_STRIDE(e, total_e)
    {
        const int g = graph_of(eoff, n_graphs, e);
        const int64_t ng = voff[g + 1] - voff[g];
        if (col[e] < 0 || col[e] >= ng) bad |= 256;
    }
    if (bad) atomicOr(err, bad);
}

__global__ void batch_to_union_rp_k(int32_t n_graphs, const int64_t *voff, const int64_t *eoff,
                                    const int32_t *rp, int64_t total_v, int64_t total_e, int32_t *urp)
{
    GRID_STRIDE(i, total_v + 1)
    {
        if (i == total_v) {
            urp[i] = (int32_t)total_e;
        } else {
            const int g = graph_of(voff, n_graphs, i);
            urp[i] = (int32_t)(eoff[g] + rp[i + g]);
        }
    }
}

__global__ void batch_to_union_col_k(int32_t n_graphs, const int64_t *voff, const int64_t *eoff,
                                     const int32_t *col, int64_t total_e, int32_t *ucol)
{
    GRID_STRIDE(e, total_e)
    {
        const int g = graph_of(eoff, n_graphs, e);
        ucol[e] = (int32_t)(col[e] + voff[g]);
    }
}

__global__ void union_edge_offsets_k(int32_t n_graphs, const int64_t *voff, const int32_t *urp,
                                     int64_t *eoff_out)
{
    GRID_STRIDE(g, (int64_t)n_graphs + 1) eoff_out[g] = urp[voff[g]];
}

__global__ void union_to_batch_rp_k(int32_t n_graphs, const int64_t *voff, const int64_t *eoff,
                                    const int32_t *urp, int64_t total_v, int32_t *rp)
{
    GRID_STRIDE(i, total_v + n_graphs)
    {
        int lo = 0, hi = n_graphs;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (voff[mid] + mid <= i) lo = mid;
            else hi = mid;
        }
        const int g = lo;
        const int64_t uv = i - g;   // union row index (the terminal entry maps to voff[g+1])
        rp[i] = (int32_t)(urp[uv] - eoff[g]);
    }
}

__global__ void union_to_batch_col_k(int32_t n_graphs, const int64_t *voff, const int64_t *eoff,
                                     const int32_t *ucol, int64_t total_e, int32_t *col)
{
    GRID_STRIDE(e, total_e)
    {
        const int g = graph_of(eoff, n_graphs, e);
        col[e] = (int32_t)(ucol[e] - voff[g]);
    }
}

}  // namespace

hipError_t fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_k, dim3(blocks_for(count)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t iota_i32(int32_t *p, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_i32_k, dim3(blocks_for(count)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t all_sources_setup(int32_t n, int32_t *usrc, int32_t *slot_of, int64_t *slot_row, int32_t *info,
                             hipStream_t s)
{
    hipLaunchKernelGGL(all_sources_setup_k, dim3(blocks_for(n > 0 ? n : 1)), dim3(256), 0, s, n, usrc, slot_of,
                       slot_row, info);
    return hipGetLastError();
}

hipError_t iota_i64(int64_t *p, int64_t count, int64_t start, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_i64_k, dim3(blocks_for(count)), dim3(256), 0, s, p, count, start);
    return hipGetLastError();
}

hipError_t scatter_slots(const int32_t *usrc, int32_t count, int32_t *slot_of, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_slots_k, dim3(blocks_for(count)), dim3(256), 0, s, usrc, count, slot_of);
    return hipGetLastError();
}

hipError_t check_sorted(int32_t n, const int32_t *rp, const int32_t *col, int *err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(check_sorted_k, dim3(blocks_for(n)), dim3(256), 0, s, n, rp, col, err);
    return hipGetLastError();
}

hipError_t validate_batch(int32_t n_graphs, const int64_t *voff, const int64_t *eoff, const int32_t *rp,
                          const int32_t *col, int64_t total_v, int64_t total_e, int *err, hipStream_t s)
{
    int64_t items = total_v + n_graphs > total_e ? total_v + n_graphs : total_e;
    hipLaunchKernelGGL(validate_batch_k, dim3(blocks_for(items, 256, 16384)), dim3(256), 0, s,
                       n_graphs, voff, eoff, rp, col, total_v, total_e, err);
    return hipGetLastError();
}

hipError_t batch_to_union(int32_t n_graphs, const int64_t *voff, const int64_t *eoff, const int32_t *rp,
                          const int32_t *col, int64_t total_v, int64_t total_e, int32_t *urp,
                          int32_t *ucol, hipStream_t s)
{
    hipLaunchKernelGGL(batch_to_union_rp_k, dim3(blocks_for(total_v + 1)), dim3(256), 0, s, n_graphs,
                       voff, eoff, rp, total_v, total_e, urp);
    if (total_e > 0)
        hipLaunchKernelGGL(batch_to_union_col_k, dim3(blocks_for(total_e)), dim3(256), 0, s, n_graphs,
                           voff, eoff, col, total_e, ucol);
    return hipGetLastError();
}

hipError_t union_to_batch(int32_t n_graphs, const int64_t *voff, const int32_t *urp, const int32_t *ucol,
                          int64_t total_v, int64_t total_e_canon, int64_t *eoff_out, int32_t *rp_out,
                          int32_t *col_out, hipStream_t s)
{
    hipLaunchKernelGGL(union_edge_offsets_k, dim3(blocks_for((int64_t)n_graphs + 1)), dim3(256), 0, s,
                       n_graphs, voff, urp, eoff_out);
    hipLaunchKernelGGL(union_to_batch_rp_k, dim3(blocks_for(total_v + n_graphs)), dim3(256), 0, s,
                       n_graphs, voff, eoff_out, urp, total_v, rp_out);
    if (total_e_canon > 0)
        hipLaunchKernelGGL(union_to_batch_col_k, dim3(blocks_for(total_e_canon)), dim3(256), 0, s,
                           n_graphs, voff, eoff_out, ucol, total_e_canon, col_out);
    return hipGetLastError();
}

bool sources_ranked_small(int64_t rows, int32_t n) { return rows <= kRankMax && n <= kRankMaxN; }

hipError_t prepare_sources_small(const int32_t *src, int64_t rows, int32_t n, const int32_t *row_ptr,
                                 int32_t heavy_forced, int32_t *heavy, int32_t *first, int32_t *count,
                                 int32_t *usrc, int64_t *slot_row, int32_t *slot_of, int32_t *mult, int32_t *info,
                                 hipStream_t s, int32_t *host_info)
{
    if (!sources_ranked_small(rows, n)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(source_vertex_prep_k, dim3(blocks_for(n)), dim3(256), 0, s, n, row_ptr, heavy_forced, first,
                       count, slot_of, heavy, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || rows <= 0) return e;
    hipLaunchKernelGGL(source_rank_small_k, dim3(1), dim3(kRankThreads), 0, s, src, (int32_t)rows, n, first, count,
                       usrc, slot_row, slot_of, mult, info, host_info);
    return hipGetLastError();
}

hipError_t prepare_sources(const int32_t *src, int64_t rows, int32_t n, int32_t *first, int32_t *count,
                           int32_t *marks, int32_t *pos, void *scan_tmp, int32_t *usrc, int64_t *slot_row,
                           int32_t *slot_of, int32_t *mult, int32_t *info, hipStream_t s)
{
    hipError_t e = fill_i32(first, n, INT32_MAX, s);
    if (e == hipSuccess && count) e = fill_i32(count, n, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(source_first_k, dim3(blocks_for(rows)), dim3(256), 0, s, src, rows, n, first, count, info);
    hipLaunchKernelGGL(source_marks_k, dim3(blocks_for(n)), dim3(256), 0, s, n, first, marks);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_exclusive_scan(marks, pos, n, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(source_slots_k, dim3(blocks_for(n)), dim3(256), 0, s, n, first, pos, count, usrc, slot_row,
                       slot_of, mult, info);
    return hipGetLastError();
}

hipError_t copy_dup_rows(const int32_t *src, int64_t rows, const int32_t *first, int32_t k, int32_t n, int32_t *ids,
                         uint8_t *hops, uint8_t *hop_matrix, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_dup_rows_k, dim3((unsigned)std::min<int64_t>(rows, 4096)), dim3(256), 0, s, src, rows,
                       first, k, n, ids, hops, hop_matrix);
    return hipGetLastError();
}

}  // namespace gm
