// CSR ingest: structural validation, symmetry check, canonicalisation
// (rows sorted ascending, repeats and self-loops removed) and the exclusive
// scan used elsewhere to rebuild offsets.  The kNN results depend only on the
// undirected edge set; a canonical adjacency is what lets the partial BFS
// merge sorted neighbour lists and stop early.
//
// Canonicalisation is two launches, three on graphs of more than 262,144
// vertices.  The row kernel sorts a thread per row of at most 32 entries,
// workgroup b taking rows [256 b, 256 b + 256) (neighbouring threads read
// neighbouring rows); longer rows are dealt with a stride (rows b,
// b + blocks, ...), so that the long rows, which a preferential-attachment
// graph puts at its lowest ids, land in different workgroups: a wave per row
// of at most 256 entries (registers), the whole workgroup above that (an
// n-bit set in LDS, whatever the row's length, when n <= 262,144; else a
// bitonic sort in LDS up to 4,096 entries).  On larger graphs the rows past
// 4,096 entries are listed and sorted by a 1,024-thread workgroup each (LDS,
// or an n-bit bitmap past 32,768 entries), reached through a slot
// permutation that spreads them.  Then a single-pass scan with decoupled
// look-back writes the row pointers and moves the rows that an earlier
// dropped repeat or self-loop shifted (rows are sorted in place at their
// input offsets, with a staged copy for that case).
#include "device.h"
#include "kernels.h"

namespace gm {

namespace {

constexpr int kSmallRow = 64;      // one wave, registers
constexpr int kMidRow = 256;       // one wave, registers (longer: the workgroup, LDS)
constexpr int kBigRow = 32768;     // one workgroup, LDS
constexpr int kCanonBlock = 256;   // 4 waves
constexpr int kBigBlock = 1024;

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


// Bitonic sort of one row of 64 * R entries (padding GM_INF_ID) held in
// registers: element i = lane + 64 * r sits in register r of lane i % 64.
// Compare-exchange distances below 64 cross lanes (shuffles), larger ones
// stay within a lane.  Unique entries other than v go to out[a, ...) and
// stg[a, ...) in order and their count to cnt[v].
template <int R>
__device__ __forceinline__ void wave_sort_row(int64_t v, int32_t a, int32_t d, const int32_t *__restrict__ col,
                                              int32_t *__restrict__ out, int32_t *__restrict__ stg,
                                              int32_t *__restrict__ cnt)
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
        if (keep) {
            out[a + base + lanes_below(m)] = x[r];
            stg[a + base + lanes_below(m)] = x[r];
        }
        base += __popcll(m);
        carry = __shfl(x[r], GM_WAVE - 1, GM_WAVE);
    }
    if (l == 0) cnt[v] = base;
}

// Sorts row v (a = its first entry, kThreadRow < d <= kMidRow) with one wave
// into out and stg at [a, a + unique) and records the count.
__device__ __forceinline__ void canon_one_row(int64_t v, int32_t a, int32_t d, const int32_t *__restrict__ col,
                                             int32_t *__restrict__ out, int32_t *__restrict__ stg,
                                             int32_t *__restrict__ cnt)
{
    const int l = lane();
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
        if (keep) {
            out[a + lanes_below(m)] = x;
            stg[a + lanes_below(m)] = x;
        }
        if (l == 0) cnt[v] = __popcll(m);
        return;
    }
    // 64 < d <= 1024: bitonic sort in registers, R = 2..16 per lane
    if (d <= 128) wave_sort_row<2>(v, a, d, col, out, stg, cnt);
    else if (d <= 256) wave_sort_row<4>(v, a, d, col, out, stg, cnt);
    else if (d <= 512) wave_sort_row<8>(v, a, d, col, out, stg, cnt);
    else wave_sort_row<16>(v, a, d, col, out, stg, cnt);
}

// Short rows (at most kThreadRow entries) are sorted by one thread each,
// with a bitonic network over N registers (compile-time indices, so the row
// stays in registers); repeats and the row's own vertex are dropped as the
// row is written.
constexpr int kThreadRow = 32;
constexpr int kListRows = 256;   // rows per block of canon_sort_kernel

template <int N>
__device__ __forceinline__ void thread_sort_row(int64_t v, int32_t a, int32_t d, const int32_t *__restrict__ src,
                                                int32_t *__restrict__ out, int32_t *__restrict__ stg,
                                                int32_t *__restrict__ cnt)
{
    int x[N];   // src: the row's first entry (in global memory or in LDS)
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = i < d ? src[i] : GM_INF_ID;
#pragma unroll
    for (int kk = 2; kk <= N; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int o = i ^ j;
                if (o > i) {
                    const int lo = min(x[i], x[o]), hi = max(x[i], x[o]);
                    const bool up = (i & kk) == 0;
                    x[i] = up ? lo : hi;
                    x[o] = up ? hi : lo;
                }
            }
        }
    }
    int c = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const bool keep = x[i] != GM_INF_ID && x[i] != (int)v && (i == 0 || x[i] != x[i > 0 ? i - 1 : 0]);
        if (keep) {
            out[a + c] = x[i];
            stg[a + c] = x[i];
        }
        c += keep;
    }
    cnt[v] = c;
}

// Exclusive prefix of `mine` over a workgroup of kListRows threads, and the
// total, through per-wave sums in wsum[kListRows / 64].  The caller passes a
// barrier before wsum is written again.
__device__ __forceinline__ int row_block_scan(int mine, int32_t *wsum, int *total)
{
    const int l = lane(), wid = threadIdx.x / GM_WAVE;
    const int inc = wave_incl_scan(mine);
    if (l == GM_WAVE - 1) wsum[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kListRows / GM_WAVE; ++w) {
        const int x = wsum[w];
        if (w < wid) before += x;
        tot += x;
    }
    *total = tot;
    return before + inc - mine;
}

// Rows of kMidRow + 1 .. kBlockSortMax entries are sorted by the whole
// workgroup of canon_rows_kernel in LDS (bitonic over the next power of two
// >= max(d, 256) entries), then written without repeats and without v.
constexpr int kBlockSortMax = 4096;

__device__ void block_sort_row(int32_t v, int32_t a, int32_t d, const int32_t *__restrict__ col, int32_t *sbuf,
                               int32_t *part, int32_t *__restrict__ out, int32_t *__restrict__ stg,
                               int32_t *__restrict__ cnt)
{
    const int t = threadIdx.x, nt = blockDim.x;
    int P = nt;
    while (P < d) P <<= 1;
    for (int i = t; i < P; i += nt) sbuf[i] = i < d ? col[a + i] : GM_INF_ID;
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = t; i < P; i += nt) {
                const int o = i ^ j;
                if (o > i) {
                    const int x = sbuf[i], y = sbuf[o];
                    const bool up = (i & kk) == 0;
                    if ((x > y) == up) {
                        sbuf[i] = y;
                        sbuf[o] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    // kept entries: per-thread counts of a contiguous range, a block scan, the writes
    const int chunk = P / nt;
    const int i0 = t * chunk;
    int mine = 0;
    for (int i = i0; i < i0 + chunk; ++i) {
        const int x = sbuf[i];
        mine += x != GM_INF_ID && x != v && (i == 0 || x != sbuf[i - 1]);
    }
    int total = 0;
    int pos = row_block_scan(mine, part, &total);
    for (int i = i0; i < i0 + chunk; ++i) {
        const int x = sbuf[i];
        if (x != GM_INF_ID && x != v && (i == 0 || x != sbuf[i - 1])) {
            out[a + pos] = x;
            stg[a + pos] = x;
            ++pos;
        }
    }
    if (t == 0) cnt[v] = total;
    __syncthreads();
}

// A row of any length above kMidRow through an n-bit set in LDS when
// n <= 32 * kRowBitmapWords: the entries other than v set their bits
// (repeats collapse), then each thread counts the set bits of a contiguous
// range of words, a block scan gives its first output position, and it
// writes its bits' ids in order.  The cost is n / 32 words plus d / 256
// entries per thread.
constexpr int kRowBitmapWords = 8192;   // 32 KB: graphs of up to 262,144 vertices

__device__ void block_bitmap_row(int32_t v, int32_t a, int32_t d, int32_t n, const int32_t *__restrict__ col,
                                 uint32_t *bm, int32_t *part, int32_t *__restrict__ out, int32_t *__restrict__ stg,
                                 int32_t *__restrict__ cnt)
{
    const int t = threadIdx.x, nt = blockDim.x;
    const int32_t words = (n + 31) / 32;
    for (int32_t i = t; i < words; i += nt) bm[i] = 0u;
    __syncthreads();
    for (int32_t e = t; e < d; e += nt) {
        const int32_t u = col[a + e];
        if (u != v) atomicOr(&bm[u >> 5], 1u << (u & 31));
    }
    __syncthreads();
    const int32_t wper = (words + nt - 1) / nt;
    const int32_t w0 = min(words, t * wper), w1 = min(words, w0 + wper);
    int mine = 0;
    for (int32_t i = w0; i < w1; ++i) mine += __popc(bm[i]);
    int total = 0;
    int pos = row_block_scan(mine, part, &total);
    for (int32_t i = w0; i < w1; ++i) {
        uint32_t bits = bm[i];
        while (bits) {
            const int32_t u = i * 32 + __ffs(bits) - 1;
            bits &= bits - 1;
            out[a + pos] = u;
            stg[a + pos] = u;
            ++pos;
        }
    }
    if (t == 0) cnt[v] = total;
    __syncthreads();
}

// The row kernel, 2 * blocks workgroups of kListRows threads.
//   b < blocks (launched first) takes share b, the rows b, b + blocks,
//     b + 2 blocks, ... (the long rows of a preferential-attachment graph sit
//     at the lowest ids; striding puts them in different workgroups), and
//     sorts those of more than kThreadRow entries: up to kMidRow a wave each
//     in registers, longer ones the whole workgroup, through the n-bit set
//     when n <= 32 * kRowBitmapWords (any length), else by the LDS bitonic
//     sort up to kBlockSortMax; rows left over (n above that bound and more
//     than kBlockSortMax entries) are listed (kListRows slots per workgroup,
//     list_big[b * kListRows ...], count in n_big[b]) for canon_big_kernel.  Workgroup 0
//     also clears the look-back flags of canon_scan_kernel.
//   b >= blocks, c = b - blocks, sorts the rows of at most kThreadRow entries
//     among [c * kListRows, (c + 1) * kListRows), a thread each in registers;
//     when the range's entries fit in LDS they are first loaded there with
//     contiguous reads.
// The long rows thus run beside the short ones instead of after them.
static_assert(kRowBitmapWords >= kBlockSortMax, "the LDS row buffer serves both workgroup sorts");

__global__ void __launch_bounds__(kListRows)
canon_rows_kernel(int32_t n, int32_t blocks, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                  int32_t *__restrict__ out, int32_t *__restrict__ stg, int32_t *__restrict__ cnt,
                  int32_t *__restrict__ list_big, int32_t *__restrict__ n_big,
                  unsigned long long *__restrict__ flags, int32_t n_flags)
{
    // s_n: wave rows kept (listed from the front of s_rows), workgroup rows
    // kept (from the back), rows listed for canon_big_kernel; in a short-row
    // workgroup, its range's first entry and end
    __shared__ int32_t s_n[3];
    __shared__ int32_t s_rows[kListRows], s_a[kListRows], s_d[kListRows];   // row, first entry, length
    __shared__ int32_t lbuf[kRowBitmapWords];  // the n-bit set, the bitonic sort's entries, or staged short rows
    __shared__ int32_t part[kListRows / GM_WAVE];
    const int t = threadIdx.x, wid = t / GM_WAVE;
    if ((int32_t)blockIdx.x < blocks) {
        const int32_t share = (int32_t)blockIdx.x;
        if (share == 0)
            for (int32_t i = t; i < n_flags; i += blockDim.x) flags[i] = 0ull;
        if (t < 3) s_n[t] = 0;
        __syncthreads();
        const bool bitmap_rows = n <= 32 * kRowBitmapWords;
        const int64_t vs = (int64_t)share + (int64_t)t * blocks;
        if (vs < n) {
            const int32_t a = row_ptr[vs], d = row_ptr[vs + 1] - a;
            int slot = -1;
            if (d > kMidRow) {
                if (bitmap_rows || d <= kBlockSortMax) slot = kListRows - 1 - atomicAdd(&s_n[1], 1);
                else list_big[(int64_t)share * kListRows + atomicAdd(&s_n[2], 1)] = (int32_t)vs;
            } else if (d > kThreadRow) {
                slot = atomicAdd(&s_n[0], 1);
            }
            if (slot >= 0) {
                s_rows[slot] = (int32_t)vs;
                s_a[slot] = a;
                s_d[slot] = d;
            }
        }
        __syncthreads();
        const int nm = s_n[0], nb = s_n[1];
        for (int i = wid; i < nm; i += kListRows / GM_WAVE)
            canon_one_row(s_rows[i], s_a[i], s_d[i], col, out, stg, cnt);
        for (int i = 0; i < nb; ++i) {
            const int32_t rv = s_rows[kListRows - 1 - i];
            const int32_t a = s_a[kListRows - 1 - i], d = s_d[kListRows - 1 - i];
            if (bitmap_rows) block_bitmap_row(rv, a, d, n, col, (uint32_t *)lbuf, part, out, stg, cnt);
            else block_sort_row(rv, a, d, col, lbuf, part, out, stg, cnt);
        }
        if (t == 0) n_big[share] = s_n[2];
        return;
    }
    const int64_t v0 = ((int64_t)blockIdx.x - blocks) * kListRows;
    const int32_t rows_here = (int32_t)min((int64_t)kListRows, (int64_t)n - v0);
    int32_t a = 0, d = 0;
    if (t < rows_here) {
        a = row_ptr[v0 + t];
        d = row_ptr[v0 + t + 1] - a;
        if (t == 0) s_n[0] = a;                       // the range's first entry
        if (t == rows_here - 1) s_n[1] = a + d;       // and its end
    }
    __syncthreads();
    const int32_t base = s_n[0], span = s_n[1] - base;
    const bool staged = span <= kRowBitmapWords;   // the same for the whole workgroup
    if (staged) {
        for (int32_t j = t; j < span; j += kListRows) lbuf[j] = col[base + j];
        __syncthreads();
    }
    if (t < rows_here) {
        const int64_t v = v0 + t;
        if (staged) {
            if (d <= 16) thread_sort_row<16>(v, a, d, lbuf + (a - base), out, stg, cnt);
            else if (d <= kThreadRow) thread_sort_row<kThreadRow>(v, a, d, lbuf + (a - base), out, stg, cnt);
        } else {
            if (d <= 16) thread_sort_row<16>(v, a, d, col + a, out, stg, cnt);
            else if (d <= kThreadRow) thread_sort_row<kThreadRow>(v, a, d, col + a, out, stg, cnt);
        }
    }
}

// The listed rows are addressed by slots s in [0, S), S the power of two at
// or above blocks * kListRows: slot s stands for entry f % kListRows of
// block f / kListRows's list, f = s * kSlotMul mod S (kSlotMul odd, so this
// is a permutation), when f is inside the lists.  Long rows cluster in a few
// blocks (the low ids of a preferential-attachment graph); scattering the
// slots spreads them over many waves instead of leaving a block's list to
// one.
constexpr uint64_t kSlotMul = 2654435761ull;

__device__ __forceinline__ bool list_slot(int64_t s, int64_t slots_pow2, int64_t slots,
                                          const int32_t *__restrict__ counts, int64_t &entry)
{
    if (s >= slots_pow2) return false;
    const int64_t f = (int64_t)(((uint64_t)s * kSlotMul) & (uint64_t)(slots_pow2 - 1));
    if (f >= slots) return false;
    entry = f;
    return (f % kListRows) < counts[f / kListRows];
}

// Rows longer than kBlockSortMax, each sorted by a whole 1,024-thread workgroup:
// up to kBigRow entries by a bitonic sort in LDS, longer ones by marking the
// neighbours in an n-bit bitmap (this workgroup's own, in scratch) and
// emitting the set bits in order.  Workgroup c looks at big-list slots
// [1024 c', 1024 c' + 1024) for c' = c, c + gridDim.x, ...
__global__ void __launch_bounds__(kBigBlock)
canon_big_kernel(int32_t n, int32_t blocks, int64_t slots_pow2, const int32_t *__restrict__ row_ptr,
                 const int32_t *__restrict__ col, int32_t *__restrict__ out, int32_t *__restrict__ stg,
                 int32_t *__restrict__ cnt, const int32_t *__restrict__ list_big, const int32_t *__restrict__ n_big,
                 uint32_t *__restrict__ bitmaps)
{
    extern __shared__ int32_t sbuf[];  // kBigRow ints, then kBigBlock ints of per-thread counts
    int32_t *part = sbuf + kBigRow;
    __shared__ int32_t found[kBigBlock];
    __shared__ int32_t n_found;
    const int t = threadIdx.x;
    const int64_t words = ((int64_t)n + 31) / 32;
    uint32_t *bm = bitmaps + (int64_t)blockIdx.x * words;
    const int64_t slots = (int64_t)blocks * kListRows;
    for (int64_t c0 = (int64_t)blockIdx.x * kBigBlock; c0 < slots_pow2; c0 += (int64_t)gridDim.x * kBigBlock) {
        if (t == 0) n_found = 0;
        __syncthreads();
        {
            int64_t entry = 0;
            if (list_slot(c0 + t, slots_pow2, slots, n_big, entry)) found[atomicAdd(&n_found, 1)] = list_big[entry];
        }
        __syncthreads();
        const int nf = n_found;
        for (int q = 0; q < nf; ++q) {
            const int32_t rv = found[q];
            const int32_t a = row_ptr[rv], d = row_ptr[rv + 1] - a;
            if (d <= kBigRow) {
                int P = kBigBlock;
                while (P < d) P <<= 1;
                for (int i = t; i < P; i += blockDim.x) sbuf[i] = i < d ? col[a + i] : GM_INF_ID;
                __syncthreads();
                for (int kk = 2; kk <= P; kk <<= 1) {
                    for (int j = kk >> 1; j > 0; j >>= 1) {
                        for (int i = t; i < P; i += blockDim.x) {
                            const int o = i ^ j;
                            if (o > i) {
                                const int x = sbuf[i], y = sbuf[o];
                                const bool up = (i & kk) == 0;
                                if ((x > y) == up) {
                                    sbuf[i] = y;
                                    sbuf[o] = x;
                                }
                            }
                        }
                        __syncthreads();
                    }
                }
                // unique entries other than rv, in order: per-thread counts of
                // a contiguous range, a block scan, then the writes
                const int chunk = P / (int)blockDim.x;
                const int i0 = t * chunk;
                int mine = 0;
                for (int i = i0; i < i0 + chunk; ++i) {
                    const int x = sbuf[i];
                    mine += x != GM_INF_ID && x != rv && (i == 0 || x != sbuf[i - 1]);
                }
                part[t] = mine;
                __syncthreads();
                for (int o = 1; o < (int)blockDim.x; o <<= 1) {
                    const int y = t >= o ? part[t - o] : 0;
                    __syncthreads();
                    part[t] += y;
                    __syncthreads();
                }
                int pos = part[t] - mine;
                for (int i = i0; i < i0 + chunk; ++i) {
                    const int x = sbuf[i];
                    if (x != GM_INF_ID && x != rv && (i == 0 || x != sbuf[i - 1])) {
                        out[a + pos] = x;
                        stg[a + pos] = x;
                        ++pos;
                    }
                }
                if (t == (int)blockDim.x - 1) cnt[rv] = part[t];
                __syncthreads();
            } else {
                for (int64_t i = t; i < words; i += blockDim.x) bm[i] = 0u;
                __threadfence_block();
                __syncthreads();
                for (int32_t e = a + t; e < a + d; e += blockDim.x) {
                    const int32_t w = col[e];
                    if (w != rv) atomicOr(&bm[w >> 5], 1u << (w & 31));
                }
                __threadfence_block();
                __syncthreads();
                const int64_t wper = (words + blockDim.x - 1) / blockDim.x;
                const int64_t w0 = min(words, (int64_t)t * wper), w1 = min(words, w0 + wper);
                int mine = 0;
                for (int64_t i = w0; i < w1; ++i)
                    mine += __popc(__hip_atomic_load(&bm[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                part[t] = mine;
                __syncthreads();
                for (int o = 1; o < (int)blockDim.x; o <<= 1) {
                    const int y = t >= o ? part[t - o] : 0;
                    __syncthreads();
                    part[t] += y;
                    __syncthreads();
                }
                int pos = part[t] - mine;
                for (int64_t i = w0; i < w1; ++i) {
                    uint32_t bits = __hip_atomic_load(&bm[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    while (bits) {
                        const int bit = __ffs(bits) - 1;
                        bits &= bits - 1;
                        out[a + pos] = (int32_t)(i * 32 + bit);
                        stg[a + pos] = (int32_t)(i * 32 + bit);
                        ++pos;
                    }
                }
                if (t == (int)blockDim.x - 1) cnt[rv] = part[t];
                __syncthreads();
            }
        }
    }
}

// Single-pass scan of the row counts with decoupled look-back.  Tile b =
// rows [b * kScanRows, ...): its count total is published as an aggregate,
// the exclusive prefix is found by walking back over earlier tiles' flags
// (a published inclusive prefix ends the walk), and the tile's inclusive
// prefix is published; then it writes its output row pointers.  A flag is 0
// (not ready), or (status << 62 | value) with status 1 = aggregate, 2 =
// inclusive prefix; canon_rows_kernel cleared them for this call.  A wait on
// a flag is bounded: past kSpinLimit polls the tile writes
// out_row_ptr[n] = -1 and stops (the host reports it).
constexpr int kScanRows = 1024;
constexpr int kScanThreads = 256;
constexpr int kScanPer = kScanRows / kScanThreads;
constexpr unsigned long long kFlagAgg = 1ull << 62, kFlagPrefix = 2ull << 62;
constexpr unsigned long long kFlagValue = (1ull << 62) - 1ull;
constexpr int kSpinLimit = 1 << 22;

__global__ void __launch_bounds__(kScanThreads)
canon_scan_kernel(int32_t n, const int32_t *__restrict__ cnt, int32_t *__restrict__ out_row_ptr,
                  unsigned long long *flags, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ stg,
                  int32_t *__restrict__ out_col, int32_t *host_total)
{
    __shared__ int32_t s_wave[kScanThreads / GM_WAVE];
    __shared__ int64_t s_excl;
    __shared__ int s_fail;
    __shared__ int32_t s_long[kScanRows];   // rows of more than 64 kept entries to move
    __shared__ int s_nlong;
    const int t = threadIdx.x, l = lane(), wid = t / GM_WAVE;
    const int64_t v0 = (int64_t)blockIdx.x * kScanRows;
    const int rows = (int)min((int64_t)kScanRows, (int64_t)n - v0);
    int c[kScanPer];
    int mine = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int r = t * kScanPer + q;
        c[q] = r < rows ? cnt[v0 + r] : 0;
        mine += c[q];
    }
    const int inc = wave_incl_scan(mine);
    if (l == GM_WAVE - 1) s_wave[wid] = inc;
    if (t == 0) s_fail = 0;
    __syncthreads();
    int before = 0, agg = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / GM_WAVE; ++w) {
        if (w < wid) before += s_wave[w];
        agg += s_wave[w];
    }
    if (wid == 0) {
        // look-back by the first wave, 64 earlier tiles per window: lane q
        // reads tile j - q; the window is summed up to the nearest published
        // inclusive prefix once every flag before it is ready
        int64_t excl = 0;
        if (blockIdx.x == 0) {
            if (l == 0)
                __hip_atomic_store(&flags[0], kFlagPrefix | (unsigned long long)agg, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (l == 0)
                __hip_atomic_store(&flags[blockIdx.x], kFlagAgg | (unsigned long long)agg, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            int64_t j = (int64_t)blockIdx.x - 1;
            int spins = 0;
            bool fail = false;
            while (j >= 0) {
                const int64_t tile = j - l;
                const unsigned long long f = tile >= 0
                    ? __hip_atomic_load(&flags[tile], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    : kFlagPrefix;   // before tile 0: an empty prefix
                const unsigned long long pre = __ballot((f & ~kFlagValue) == kFlagPrefix);
                const int stop = pre ? __ffsll((long long)pre) - 1 : GM_WAVE - 1;   // nearest prefix lane
                const unsigned long long need = stop == GM_WAVE - 1 ? ~0ull : ((2ull << stop) - 1ull);
                if ((__ballot(f != 0ull) & need) != need) {
                    if (++spins > kSpinLimit) {
                        fail = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                const unsigned long long mine_v = (l <= stop && tile >= 0) ? (f & kFlagValue) : 0ull;
                excl += (int64_t)wave_sum_u64(mine_v);
                if (pre) break;
                j -= GM_WAVE;
            }
            if (l == 0)
                __hip_atomic_store(&flags[blockIdx.x], kFlagPrefix | (unsigned long long)(excl + agg),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (l == 0 && fail) s_fail = 1;
        }
        if (l == 0) s_excl = excl;
    }
    __syncthreads();
    if (s_fail) {
        if (t == 0) {
            out_row_ptr[n] = -1;
            if (host_total) *host_total = -1;
        }
        return;
    }
    const int off0 = (int)s_excl + before + inc - mine;
    int off = off0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int r = t * kScanPer + q;
        if (r < rows) out_row_ptr[v0 + r] = off;
        off += c[q];
    }
    if (v0 + rows == n && t == kScanThreads - 1) {
        out_row_ptr[n] = off;
        if (host_total) *host_total = off;
    }
    // The sorted rows sit at their input offsets (kept entries first, also
    // in the staged copy).  A row moves to its output offset when an entry
    // was dropped before it: nothing moves in a tile that starts where its
    // input starts and keeps every entry.
    const int32_t in0 = row_ptr[v0], in1 = row_ptr[v0 + rows];
    if ((int64_t)s_excl == (int64_t)in0 && (int64_t)agg == (int64_t)in1 - in0) return;
    if (t == 0) s_nlong = 0;
    __syncthreads();
    off = off0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int r = t * kScanPer + q;
        if (r < rows) {
            const int32_t a = row_ptr[v0 + r];
            if (off != a) {
                if (c[q] <= GM_WAVE) {
                    for (int i = 0; i < c[q]; ++i) out_col[off + i] = stg[a + i];
                } else {
                    s_long[atomicAdd(&s_nlong, 1)] = r;
                }
            }
        }
        off += c[q];
    }
    __syncthreads();
    const int nl = s_nlong;
    for (int i = wid; i < nl; i += kScanThreads / GM_WAVE) {
        const int64_t v = v0 + s_long[i];
        const int32_t a = row_ptr[v], o = out_row_ptr[v], cv = cnt[v];
        for (int32_t e = l; e < cv; e += GM_WAVE) out_col[o + e] = stg[a + e];
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

constexpr int kLongBlocks = 64;

int64_t pow2_at_least(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

size_t canon_scratch_bytes(int32_t n, int32_t nnz)
{
    const size_t blocks = ((size_t)n + kListRows - 1) / kListRows;
    size_t b = 0;
    b += align256((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));                               // staged rows
    b += align256((size_t)(n + 1) * sizeof(int32_t));                                           // cnt
    b += align256(blocks * kListRows * sizeof(int32_t));                                        // long-row lists
    b += align256((blocks + 1) * sizeof(int32_t));                                              // list counts
    b += align256((size_t)((n + kScanRows - 1) / kScanRows + 1) * sizeof(unsigned long long));   // flags
    b += align256((size_t)kLongBlocks * (((size_t)n + 31) / 32) * sizeof(uint32_t));             // bitmaps
    return b;
}

hipError_t launch_canonicalize(int32_t n, int32_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, int32_t *out_row_ptr, int32_t *out_col,
                               void *scratch, hipStream_t s, int32_t *host_total)
{
    if (n <= 0) {
        hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, out_row_ptr, (int64_t)1, 0);
        return hipGetLastError();
    }
    const int32_t blocks = (int32_t)(((int64_t)n + kListRows - 1) / kListRows);
    const int32_t tiles = (int32_t)(((int64_t)n + kScanRows - 1) / kScanRows);
    const int64_t slots_pow2 = pow2_at_least((int64_t)blocks * kListRows);
    char *p = (char *)scratch;
    int32_t *stg = (int32_t *)p;       p += align256((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int32_t *cnt = (int32_t *)p;       p += align256((size_t)(n + 1) * sizeof(int32_t));
    // rows past kBlockSortMax on graphs above the n-bit set's bound: kListRows
    // slots per workgroup and a count per workgroup
    int32_t *list_big = (int32_t *)p;  p += align256((size_t)blocks * kListRows * sizeof(int32_t));
    int32_t *n_big = (int32_t *)p;     p += align256(((size_t)blocks + 1) * sizeof(int32_t));
    unsigned long long *flags = (unsigned long long *)p;
    p += align256((size_t)(tiles + 1) * sizeof(unsigned long long));
    uint32_t *bitmaps = (uint32_t *)p;
    hipLaunchKernelGGL(canon_rows_kernel, dim3(2 * (unsigned)blocks), dim3(kListRows), 0, s, n, blocks, row_ptr, col_idx,
                       out_col, stg, cnt, list_big, n_big, flags, tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n <= 32 * kRowBitmapWords) {   // the row kernel sorted every row
        hipLaunchKernelGGL(canon_scan_kernel, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, n, (const int32_t *)cnt,
                           out_row_ptr, flags, row_ptr, (const int32_t *)stg, out_col, host_total);
        return hipGetLastError();
    }
    const size_t big_lds = (kBigRow + kBigBlock) * sizeof(int32_t);
    static bool lds_set[64] = {};   // the LDS limit is an attribute of the kernel on each device
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64 || !lds_set[dev]) {
        e = hipFuncSetAttribute((const void *)canon_big_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)big_lds);
        if (e != hipSuccess) return e;
        if (dev >= 0 && dev < 64) lds_set[dev] = true;
    }
    hipLaunchKernelGGL(canon_big_kernel, dim3(kLongBlocks), dim3(kBigBlock), big_lds, s, n, blocks, slots_pow2, row_ptr,
                       col_idx, out_col, stg, cnt, list_big, n_big, bitmaps);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(canon_scan_kernel, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, n, (const int32_t *)cnt,
                       out_row_ptr, flags, row_ptr, (const int32_t *)stg, out_col, host_total);
    return hipGetLastError();
}

}  // namespace gm
