// CSR ingest: structural validation, symmetry check, canonicalisation
// (rows sorted ascending, repeats and self-loops removed) and the exclusive
// scan used to rebuild row pointers.  The kNN results depend only on the
// undirected edge set; a canonical adjacency is what lets the partial BFS
// merge sorted neighbour lists and stop early.
#include "device.h"
#include "kernels.h"

namespace gm {

namespace {

constexpr int kSmallRow = 64;      // one wave, registers
constexpr int kMidRow = 1024;      // one wave, registers
constexpr int kBigRow = 32768;     // one workgroup, LDS
constexpr int kCanonBlock = 256;   // 4 waves
constexpr int kBigBlock = 1024;
constexpr int kHugeBlocks = 32;

__global__ void validate_structure_kernel(int32_t n, int32_t nnz, const int32_t *__restrict__ row_ptr,
                                          const int32_t *__restrict__ col, int *err)
{
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    if (tid == 0) {
        if (row_ptr[0] != 0) bad |= 1;
        if (row_ptr[n] != nnz) bad |= 4;
    }
    for (int64_t v = tid; v < n; v += stride) {
        int32_t a = row_ptr[v], b = row_ptr[v + 1];
        if (a > b || a < 0 || b > nnz) bad |= 2;
    }
    for (int64_t e = tid; e < nnz; e += stride) {
        int32_t w = col[e];
        if (w < 0 || w >= n) bad |= 8;
    }
    if (bad) atomicOr(err, bad);
}

// One wave per row u: every neighbour w must list u (canonical rows).
__global__ void check_symmetric_kernel(int32_t n, const int32_t *__restrict__ row_ptr,
                                       const int32_t *__restrict__ col, int *err)
{
    const int waves = blockDim.x / GM_WAVE;
    int64_t u = (int64_t)blockIdx.x * waves + threadIdx.x / GM_WAVE;
    int64_t wstride = (int64_t)gridDim.x * waves;
    for (; u < n; u += wstride) {
        int32_t a = row_ptr[u], b = row_ptr[u + 1];
        int bad = 0;
        for (int32_t e = a + lane(); e < b; e += GM_WAVE) {
            int32_t w = col[e];
            int32_t wa = row_ptr[w], wb = row_ptr[w + 1];
            int32_t p = lower_bound(col, wa, wb, (int)u);
            if (p >= wb || col[p] != u) bad = 16;
        }
        if (__ballot(bad != 0)) {
            if (lane() == 0) atomicOr(err, 16);
        }
    }
}

constexpr int kTinyRow = 16;       // four rows per wave, 16 lanes each

// Bitonic sort of one row of 64 * R entries (padding GM_INF_ID) held in
// registers: element i = lane + 64 * r sits in register r of lane i % 64.
// Compare-exchange distances below 64 cross lanes (shuffles), larger ones
// stay within a lane.  Unique entries other than v go to tmp[a, ...) in
// order and their count to cnt[v].
template <int R>
__device__ __forceinline__ void wave_sort_row(int64_t v, int32_t a, int32_t d, const int32_t *__restrict__ col,
                                              int32_t *__restrict__ tmp, int32_t *__restrict__ cnt)
{
    constexpr int P = GM_WAVE * R;
    const int l = lane();
    int x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = l + GM_WAVE * r;
        x[r] = i < d ? col[a + i] : GM_INF_ID;
    }
#pragma unroll
    for (int kk = 2; kk <= P; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= GM_WAVE) {
                const int q = j / GM_WAVE;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if ((r & q) == 0) {
                        const int i = l + GM_WAVE * r;
                        const bool up = (i & kk) == 0;
                        const int lo = min(x[r], x[r | q]), hi = max(x[r], x[r | q]);
                        x[r] = up ? lo : hi;
                        x[r | q] = up ? hi : lo;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = l + GM_WAVE * r;
                    const int p = __shfl_xor(x[r], j, GM_WAVE);
                    const bool up = (i & kk) == 0;
                    const bool low = (i & j) == 0;
                    x[r] = (low == up) ? min(x[r], p) : max(x[r], p);
                }
            }
        }
    }
    int base = 0, carry = GM_INF_ID;   // carry: last element of the previous register
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int prev = __shfl_up(x[r], 1, GM_WAVE);
        if (l == 0) prev = carry;
        const bool keep = x[r] != GM_INF_ID && x[r] != (int)v && (r + l == 0 || x[r] != prev);
        const unsigned long long m = __ballot(keep);
        if (keep) tmp[a + base + lanes_below(m)] = x[r];
        base += __popcll(m);
        carry = __shfl(x[r], GM_WAVE - 1, GM_WAVE);
    }
    if (l == 0) cnt[v] = base;
}

// Sorts row v (a = its first entry, d its length, kTinyRow < d) into
// tmp[a, a + unique) and records the count; rows longer than kMidRow are
// queued for the workgroup kernels.
__device__ __forceinline__ void canon_one_row(int64_t v, int32_t a, int32_t d, const int32_t *__restrict__ col,
                              int32_t *__restrict__ tmp, int32_t *__restrict__ cnt, int32_t *big_list,
                              int32_t *big_count, int32_t *huge_list, int32_t *huge_count)
{
    const int l = lane();
    if (d > kMidRow) {
        if (l == 0) {
            if (d > kBigRow) huge_list[atomicAdd(huge_count, 1)] = (int32_t)v;
            else big_list[atomicAdd(big_count, 1)] = (int32_t)v;
        }
        return;
    }
    if (d <= kSmallRow) {
        int x = l < d ? col[a + l] : GM_INF_ID;
        // bitonic sort across the 64 lanes, ascending
#pragma unroll
        for (int kk = 2; kk <= GM_WAVE; kk <<= 1) {
#pragma unroll
            for (int j = kk >> 1; j > 0; j >>= 1) {
                int p = __shfl_xor(x, j, GM_WAVE);
                bool up = (l & kk) == 0;
                bool low = (l & j) == 0;
                x = (low == up) ? min(x, p) : max(x, p);
            }
        }
        int prev = __shfl_up(x, 1, GM_WAVE);
        bool keep = x != GM_INF_ID && x != (int)v && (l == 0 || x != prev);
        unsigned long long m = __ballot(keep);
        if (keep) tmp[a + lanes_below(m)] = x;
        if (l == 0) cnt[v] = __popcll(m);
        return;
    }
    // 64 < d <= 1024: bitonic sort in registers, R = 2..16 per lane
    if (d <= 128) wave_sort_row<2>(v, a, d, col, tmp, cnt);
    else if (d <= 256) wave_sort_row<4>(v, a, d, col, tmp, cnt);
    else if (d <= 512) wave_sort_row<8>(v, a, d, col, tmp, cnt);
    else wave_sort_row<16>(v, a, d, col, tmp, cnt);
}

// Rows of length <= 16, four per wave: one 16-lane segment each, bitonic
// sort within the segment.  Longer rows are left to canon_rows_kernel.
__global__ void __launch_bounds__(kCanonBlock)
canon_tiny_kernel(int32_t n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                  int32_t *__restrict__ tmp, int32_t *__restrict__ cnt)
{
    const int l = lane();
    const int seg = l >> 4, sl = l & (kTinyRow - 1);
    const int64_t waves = blockDim.x / GM_WAVE;
    for (int64_t v0 = ((int64_t)blockIdx.x * waves + threadIdx.x / GM_WAVE) * 4; v0 < n;
         v0 += (int64_t)gridDim.x * waves * 4) {
        const int64_t v = v0 + seg;
        int32_t a = 0, d = 0;
        if (v < n) {
            a = row_ptr[v];
            d = row_ptr[v + 1] - a;
        }
        const bool tiny = v < n && d <= kTinyRow;
        int x = (tiny && sl < d) ? col[a + sl] : GM_INF_ID;
#pragma unroll
        for (int kk = 2; kk <= kTinyRow; kk <<= 1) {
#pragma unroll
            for (int j = kk >> 1; j > 0; j >>= 1) {
                int p = __shfl_xor(x, j, GM_WAVE);
                bool up = (sl & kk) == 0;
                bool low = (sl & j) == 0;
                x = (low == up) ? min(x, p) : max(x, p);
            }
        }
        const int prev = __shfl_up(x, 1, GM_WAVE);
        const bool keep = tiny && x != GM_INF_ID && x != (int)v && (sl == 0 || x != prev);
        const unsigned long long m = __ballot(keep);
        const unsigned long long segm = 0xFFFFull << (16 * seg);
        if (keep) tmp[a + __popcll(m & segm & ((1ull << l) - 1ull))] = x;
        if (tiny && sl == 0) cnt[v] = __popcll(m & segm);
    }
}

// Rows longer than 16, one wave each (see canon_one_row); rows longer than
// kMidRow are queued for the workgroup kernels.
__global__ void __launch_bounds__(kCanonBlock)
canon_rows_kernel(int32_t n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                  int32_t *__restrict__ tmp, int32_t *__restrict__ cnt, int32_t *big_list,
                  int32_t *big_count, int32_t *huge_list, int32_t *huge_count)
{
    const int wid = threadIdx.x / GM_WAVE;
    const int waves = blockDim.x / GM_WAVE;
    for (int64_t v = (int64_t)blockIdx.x * waves + wid; v < n; v += (int64_t)gridDim.x * waves) {
        const int32_t a = row_ptr[v], d = row_ptr[v + 1] - a;
        if (d <= kTinyRow) continue;
        canon_one_row(v, a, d, col, tmp, cnt, big_list, big_count, huge_list, huge_count);
    }
}

// One workgroup per queued row of length (kMidRow, kBigRow].
__global__ void __launch_bounds__(kBigBlock)
canon_big_kernel(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                 int32_t *__restrict__ tmp, int32_t *__restrict__ cnt, const int32_t *big_list,
                 const int32_t *big_count)
{
    extern __shared__ int32_t sbuf[];  // kBigRow ints + 32 ints of wave counts
    int32_t *wcnt = sbuf + kBigRow;
    const int nbig = *big_count;
    const int t = threadIdx.x, l = lane(), wid = t / GM_WAVE;
    for (int r = blockIdx.x; r < nbig; r += gridDim.x) {
        const int32_t v = big_list[r];
        const int32_t a = row_ptr[v], d = row_ptr[v + 1] - a;
        int P = 2048;
        while (P < d) P <<= 1;
        for (int i = t; i < P; i += blockDim.x) sbuf[i] = i < d ? col[a + i] : GM_INF_ID;
        __syncthreads();
        for (int kk = 2; kk <= P; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int i = t; i < P; i += blockDim.x) {
                    int q = i ^ j;
                    if (q > i) {
                        int x = sbuf[i], y = sbuf[q];
                        bool up = (i & kk) == 0;
                        if ((x > y) == up) { sbuf[i] = y; sbuf[q] = x; }
                    }
                }
                __syncthreads();
            }
        }
        int base = 0;
        for (int c = 0; c < P; c += blockDim.x) {
            int i = c + t;
            int x = sbuf[i];
            bool keep = x != GM_INF_ID && x != v && (i == 0 || x != sbuf[i - 1]);
            unsigned long long m = __ballot(keep);
            if (l == 0) wcnt[wid] = __popcll(m);
            __syncthreads();
            int before = 0, total = 0;
            for (int w = 0; w < (int)(blockDim.x / GM_WAVE); ++w) {
                int cw = wcnt[w];
                if (w < wid) before += cw;
                total += cw;
            }
            if (keep) tmp[a + base + before + lanes_below(m)] = x;
            base += total;
            __syncthreads();
        }
        if (t == 0) cnt[v] = base;
        __syncthreads();
    }
}

// Rows longer than kBigRow: mark neighbours in a bitmap of n bits (one bitmap
// per workgroup, in scratch), then emit the set bits in order.
__global__ void __launch_bounds__(kBigBlock)
canon_huge_kernel(int32_t n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                  int32_t *__restrict__ tmp, int32_t *__restrict__ cnt, const int32_t *huge_list,
                  const int32_t *huge_count, uint32_t *bitmaps)
{
    __shared__ int32_t part[kBigBlock];
    const int nhuge = *huge_count;
    const int64_t words = ((int64_t)n + 31) / 32;
    uint32_t *bm = bitmaps + (int64_t)blockIdx.x * words;
    const int t = threadIdx.x;
    for (int r = blockIdx.x; r < nhuge; r += gridDim.x) {
        const int32_t v = huge_list[r];
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        for (int64_t i = t; i < words; i += blockDim.x) bm[i] = 0u;
        __threadfence();
        __syncthreads();
        for (int32_t e = a + t; e < b; e += blockDim.x) {
            int32_t w = col[e];
            if (w != v) atomicOr(&bm[w >> 5], 1u << (w & 31));
        }
        __threadfence();
        __syncthreads();
        // contiguous word range per thread
        const int64_t per = (words + blockDim.x - 1) / blockDim.x;
        const int64_t w0 = min(words, (int64_t)t * per), w1 = min(words, w0 + per);
        int mine = 0;
        for (int64_t i = w0; i < w1; ++i)
            mine += __popc(__hip_atomic_load(&bm[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        part[t] = mine;
        __syncthreads();
        for (int o = 1; o < (int)blockDim.x; o <<= 1) {
            int x = t >= o ? part[t - o] : 0;
            __syncthreads();
            part[t] += x;
            __syncthreads();
        }
        int pos = part[t] - mine;
        for (int64_t i = w0; i < w1; ++i) {
            uint32_t bits = __hip_atomic_load(&bm[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (bits) {
                int bit = __ffs(bits) - 1;
                bits &= bits - 1;
                tmp[a + pos++] = (int32_t)(i * 32 + bit);
            }
        }
        if (t == blockDim.x - 1) cnt[v] = part[t];
        __syncthreads();
    }
}

// The sorted rows are written to col_out at the input offsets.  When every
// entry was kept (the scanned total equals nnz) that already is the output;
// otherwise they are staged to tmp and compacted back into col_out.
__global__ void canon_stage_kernel(int32_t nnz, const int32_t *__restrict__ row_ptr_out, int32_t n,
                                   const int32_t *__restrict__ col_out, int32_t *__restrict__ tmp)
{
    if (row_ptr_out[n] == nnz) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x)
        tmp[i] = col_out[i];
}

__global__ void canon_copy_kernel(int32_t n, int32_t nnz, const int32_t *__restrict__ row_ptr_in,
                                  const int32_t *__restrict__ tmp, const int32_t *__restrict__ row_ptr_out,
                                  int32_t *__restrict__ col_out)
{
    if (row_ptr_out[n] == nnz) return;
    const int waves = blockDim.x / GM_WAVE;
    for (int64_t v = (int64_t)blockIdx.x * waves + threadIdx.x / GM_WAVE; v < n;
         v += (int64_t)gridDim.x * waves) {
        const int32_t a = row_ptr_in[v], o = row_ptr_out[v], c = row_ptr_out[v + 1] - o;
        for (int32_t i = lane(); i < c; i += GM_WAVE) col_out[o + i] = tmp[a + i];
    }
}

// ------------------------------------------------------ exclusive scan ---
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ int block_excl_scan(int x, int *sh, int *total)
{
    // sh: kScanBlock / 64 ints
    const int l = lane(), wid = threadIdx.x / GM_WAVE;
    int inc = wave_incl_scan(x);
    if (l == GM_WAVE - 1) sh[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < kScanBlock / GM_WAVE; ++w) {
        int s = sh[w];
        if (w < wid) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

__global__ void __launch_bounds__(kScanBlock)
scan_tile_sums_kernel(const int32_t *__restrict__ in, int64_t len, int32_t *__restrict__ sums)
{
    __shared__ int sh[kScanBlock / GM_WAVE];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < len) s += in[base + i];
    int total;
    block_excl_scan(s, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the tile sums in place, carrying across chunks.
__global__ void __launch_bounds__(kScanBlock)
scan_sums_kernel(int32_t *sums, int64_t ntiles)
{
    __shared__ int sh[kScanBlock / GM_WAVE];
    int carry = 0;
    for (int64_t c = 0; c < ntiles; c += kScanBlock) {
        int64_t i = c + threadIdx.x;
        int x = i < ntiles ? sums[i] : 0;
        int total;
        int ex = block_excl_scan(x, sh, &total);
        if (i < ntiles) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(kScanBlock)
scan_apply_kernel(const int32_t *__restrict__ in, int64_t len, const int32_t *__restrict__ sums,
                  int32_t *__restrict__ out)
{
    __shared__ int sh[kScanBlock / GM_WAVE];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int vals[kScanItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        vals[i] = base + i < len ? in[base + i] : 0;
        s += vals[i];
    }
    int total;
    int ex = block_excl_scan(s, sh, &total) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < len) out[base + i] = ex;
        ex += vals[i];
    }
    if (base < len && base + kScanItems >= len) out[len] = ex;  // thread holding the last item
}

__global__ void fill_i32_kernel(int32_t *p, int64_t count, int32_t value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

int grid_for(int64_t items, int per_block, int cap = 65536)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

hipError_t launch_validate_structure(int32_t n, int32_t nnz, const int32_t *row_ptr,
                                     const int32_t *col_idx, int *err, hipStream_t s)
{
    int64_t items = (int64_t)n > nnz ? n : nnz;
    hipLaunchKernelGGL(validate_structure_kernel, dim3(grid_for(items, 256, 8192)), dim3(256), 0, s,
                       n, nnz, row_ptr, col_idx, err);
    return hipGetLastError();
}

hipError_t launch_check_symmetric(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                  int *err, hipStream_t s)
{
    hipLaunchKernelGGL(check_symmetric_kernel, dim3(grid_for(n, 4, 16384)), dim3(256), 0, s, n,
                       row_ptr, col_idx, err);
    return hipGetLastError();
}

size_t exclusive_scan_scratch_bytes(int64_t len)
{
    int64_t tiles = (len + kScanTile - 1) / kScanTile;
    return align256((size_t)(tiles + 1) * sizeof(int32_t));
}

hipError_t launch_exclusive_scan(const int32_t *in, int32_t *out, int64_t len, void *scratch,
                                 hipStream_t s)
{
    if (len <= 0) {
        hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, out, (int64_t)1, 0);
        return hipGetLastError();
    }
    int64_t tiles = (len + kScanTile - 1) / kScanTile;
    int32_t *sums = (int32_t *)scratch;
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, len, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, s, sums, tiles);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, len, sums, out);
    return hipGetLastError();
}

size_t canon_scratch_bytes(int32_t n, int32_t nnz)
{
    size_t b = 0;
    b += align256((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));  // tmp
    b += align256((size_t)(n + 1) * sizeof(int32_t));              // cnt
    b += align256((size_t)(n + 1) * sizeof(int32_t));              // big list
    b += align256((size_t)(n + 1) * sizeof(int32_t));              // huge list
    b += align256(2 * sizeof(int32_t));                            // counters
    b += align256((size_t)kHugeBlocks * (((size_t)n + 31) / 32) * sizeof(uint32_t));
    b += exclusive_scan_scratch_bytes(n);
    return b;
}

hipError_t launch_canonicalize(int32_t n, int32_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, int32_t *out_row_ptr, int32_t *out_col,
                               void *scratch, hipStream_t s)
{
    char *p = (char *)scratch;
    int32_t *tmp = (int32_t *)p;      p += align256((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int32_t *cnt = (int32_t *)p;      p += align256((size_t)(n + 1) * sizeof(int32_t));
    int32_t *big = (int32_t *)p;      p += align256((size_t)(n + 1) * sizeof(int32_t));
    int32_t *huge = (int32_t *)p;     p += align256((size_t)(n + 1) * sizeof(int32_t));
    int32_t *counters = (int32_t *)p; p += align256(2 * sizeof(int32_t));
    uint32_t *bitmaps = (uint32_t *)p; p += align256((size_t)kHugeBlocks * (((size_t)n + 31) / 32) * sizeof(uint32_t));
    void *scan_scratch = p;
    if (n <= 0) {
        hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, out_row_ptr, (int64_t)1, 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, counters, (int64_t)2, 0);
    // rows are sorted straight into out_col at the input offsets
    hipLaunchKernelGGL(canon_tiny_kernel, dim3(grid_for((n + 3) / 4, kCanonBlock / GM_WAVE, 32768)),
                       dim3(kCanonBlock), 0, s, n, row_ptr, col_idx, out_col, cnt);
    hipLaunchKernelGGL(canon_rows_kernel, dim3(grid_for(n, kCanonBlock / GM_WAVE, 32768)),
                       dim3(kCanonBlock), 0, s, n, row_ptr, col_idx, out_col, cnt, big, counters, huge,
                       counters + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t big_lds = (kBigRow + 32) * sizeof(int32_t);
    // the LDS limit is an attribute of the kernel on each device
    static bool lds_set[64] = {};
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64 || !lds_set[dev]) {
        e = hipFuncSetAttribute((const void *)canon_big_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)big_lds);
        if (e != hipSuccess) return e;
        if (dev >= 0 && dev < 64) lds_set[dev] = true;
    }
    hipLaunchKernelGGL(canon_big_kernel, dim3(512), dim3(kBigBlock), big_lds, s, row_ptr, col_idx,
                       out_col, cnt, big, counters);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(canon_huge_kernel, dim3(kHugeBlocks), dim3(kBigBlock), 0, s, n, row_ptr,
                       col_idx, out_col, cnt, huge, counters + 1, bitmaps);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan(cnt, out_row_ptr, n, scan_scratch, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(canon_stage_kernel, dim3(grid_for(nnz, 256, 8192)), dim3(256), 0, s, nnz, out_row_ptr, n,
                       out_col, tmp);
    hipLaunchKernelGGL(canon_copy_kernel, dim3(grid_for(n, 4, 32768)), dim3(256), 0, s, n, nnz, row_ptr,
                       tmp, out_row_ptr, out_col);
    return hipGetLastError();
}

}  // namespace gm
