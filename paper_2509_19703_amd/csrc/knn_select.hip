// kNN selection from hop rows (GUMAP step C1, Sec. 3.1, Alg. 1): per source
// row of n hop bytes, the k smallest (hop, id) pairs with 1 <= hop <= 254
// (hop 0 is the source itself, 255 unreachable).
//
// With c(h) = number of vertices at hop h, the last hop taken is the smallest
// h* with c(1) + ... + c(h*) >= k.  Every vertex with hop < h* is taken and
// the first k - (c(1) + ... + c(h*-1)) vertices at hop h* in id order.  The
// counts come either from the BFS transpose (hops 1..16, per chunk of the row)
// or from a histogram pass of this kernel.  One streaming pass over the row in
// id order then writes the taken entries straight to their (hop, id) position
// and stops as soon as all of them are found.  With per-chunk counts the pass
// visits only the chunks that hold a vertex with hop < h* or one of the
// needed vertices at hop h*.  Bytes are classified four at a time with SWAR
// compares; only lanes holding a taken entry walk their bytes.  On the
// canonical CSR the vertices at hop 1 are exactly the source's adjacency row,
// already in id order: the counted kernel copies them from there (all of
// them, or the first k when hop 1 alone reaches k) and scans the hop row
// only for hops 2..h*, unless the row's length disagrees with the count of
// hop 1 (then it scans for every hop).
#include "device.h"
#include "kernels.h"

namespace gm {

namespace {

constexpr int kCountLevels = 16;
constexpr int kSelWaves = 4;
constexpr int kMaxK = 254;
constexpr int kMaxChunks = 512;   // chunk list capacity per wave of the counted kernel

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __noinline__ uint4 load16_slow(const uint8_t *row, int32_t n, int32_t v)
{
    uint32_t q[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
#pragma unroll 1
    for (int i = 0; i < 16; ++i) {
        const int32_t id = v + i;
        if (id < n) {
            const uint32_t b = row[id];
            const int sh = 8 * (i & 3);
            const uint32_t m = ~(0xFFu << sh);
            if ((i >> 2) == 0) q[0] = (q[0] & m) | (b << sh);
            else if ((i >> 2) == 1) q[1] = (q[1] & m) | (b << sh);
            else if ((i >> 2) == 2) q[2] = (q[2] & m) | (b << sh);
            else q[3] = (q[3] & m) | (b << sh);
        }
    }
    return make_uint4(q[0], q[1], q[2], q[3]);
}

// Loads the 16 hop bytes starting at vertex `v` (bytes past n read as 255).
__device__ __forceinline__ uint4 load16(const uint8_t *row, int32_t n, int32_t v, bool aligned)
{
    if (aligned && v + 16 <= n) return *(const uint4 *)(row + v);
    return load16_slow(row, n, v);
}

// High bit of each byte set where the byte is zero.
__device__ __forceinline__ uint32_t zero_hi(uint32_t y)
{
    const uint32_t t = (y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    return ~(t | y | 0x7F7F7F7Fu);
}

// High bit of each byte set where the byte is >= c (1 <= c <= 128).
__device__ __forceinline__ uint32_t ge_hi(uint32_t x, uint32_t c)
{
    return (x | ((x | 0x80808080u) - c * 0x01010101u)) & 0x80808080u;
}

struct Classes {
    uint32_t lt[4], eq[4];   // high-bit masks: 1 <= b < h*, b == h*
};

// lt: lo <= b < h* (lo = 1, or 2 when hop 1 is taken from the CSR row).
__device__ __forceinline__ Classes classify(uint4 q, int hstar, int lo, bool swar)
{
    Classes c;
    const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t x = qq[i];
        if (swar) {
            c.eq[i] = zero_hi(x ^ ((uint32_t)hstar * 0x01010101u));
            c.lt[i] = ~ge_hi(x, (uint32_t)hstar) & ge_hi(x, (uint32_t)lo);
        } else {
            uint32_t lt = 0, eq = 0;
#pragma unroll 1
            for (int j = 0; j < 4; ++j) {
                const int b = (x >> (8 * j)) & 0xFF;
                if (b >= lo && b < hstar && b <= 254) lt |= 0x80u << (8 * j);
                if (b == hstar) eq |= 0x80u << (8 * j);
            }
            c.lt[i] = lt;
            c.eq[i] = eq;
        }
    }
    return c;
}

// Vertex range [b, e) of chunk c when the row's 64-vertex tiles are split
// into `chunks` equal shares (the partition of the BFS transpose).
__device__ __forceinline__ void chunk_range(int32_t c, int32_t chunks, int32_t n, int32_t &b, int32_t &e)
{
    const int64_t ntiles = (n + 63) / 64;
    b = (int32_t)(64 * ((int64_t)c * ntiles / chunks));
    e = (int32_t)min<int64_t>(n, 64 * (((int64_t)c + 1) * ntiles / chunks));
}

// Selection pass.  cnt[h] (h = 1..hmax) holds the per-hop counts; got/base
// are per-wave LDS scratch of 256 ints each.  The pass scans the chunks
// list[0..nlist) in that (ascending) order, or the whole row if list is null.
// With lo = 2 the entries at hop 1 (positions 0 .. cnt[1] - 1, h* > 1) are
// written by the caller and the pass takes hops 2 and up.
__device__ __forceinline__ void select_row(const uint8_t *row, int32_t n, int32_t k, const unsigned int *cnt,
                                           int hmax, const int32_t *list, int nlist, int32_t chunks, int *got,
                                           int *base, int32_t *ids_out, uint8_t *hops_out, int lo)
{
    const int l = lane();
    int c = 0, hstar = hmax + 1, need = 0;
    for (int h = 1; h <= hmax; ++h) {
        const int ch = (int)cnt[h];
        if (c + ch >= k) {
            hstar = h;
            need = k - c;
            break;
        }
        c += ch;
    }
    const int c_less = c;
    const int c_scan = lo == 2 ? c_less - (int)cnt[1] : c_less;   // hop < h* entries the pass writes
    if (l == 0) {
        int acc = 0;
        for (int h = 1; h < hstar && h <= hmax; ++h) {
            base[h] = acc;
            got[h] = 0;
            acc += (int)cnt[h];
        }
    }
    wave_sync();
    const bool aligned = (((uintptr_t)row) & 15) == 0;
    const bool swar = hstar <= 128;
    if (!list) nlist = 1;
    int found_lt = 0, found_eq = 0;
    if ((c_scan > 0 || need > 0) && nlist > 0) {
        // lanes at or past the end of the current chunk read all-255 bytes
        auto load = [&](int32_t v, int32_t e) {
            return v < e ? load16(row, n, v, aligned) : make_uint4(~0u, ~0u, ~0u, ~0u);
        };
        int li = 0;
        int32_t vb = 0, ce = n;
        if (list) chunk_range(list[0], chunks, n, vb, ce);
        uint4 q = load(vb + 16 * l, ce);
        for (;;) {
            // next position: the following 16 * 64 bytes of this chunk, else the next listed chunk
            int nli = li;
            int32_t nvb = vb + 16 * GM_WAVE, nce = ce;
            if (nvb >= ce) {
                ++nli;
                if (nli < nlist) chunk_range(list[nli], chunks, n, nvb, nce);
            }
            const bool more = nli < nlist;
            const uint4 qn = more ? load(nvb + 16 * l, nce) : make_uint4(~0u, ~0u, ~0u, ~0u);   // in flight
            const int32_t v = vb + 16 * l;
            const Classes cl = classify(q, hstar, lo, swar);
            const int n_lt = __popc(cl.lt[0]) + __popc(cl.lt[1]) + __popc(cl.lt[2]) + __popc(cl.lt[3]);
            const int n_eq = __popc(cl.eq[0]) + __popc(cl.eq[1]) + __popc(cl.eq[2]) + __popc(cl.eq[3]);
            const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
            unsigned long long lt_mask = __ballot(n_lt > 0);
            if (lt_mask) {
                found_lt += wave_sum(n_lt);
                while (lt_mask) {
                    const int L = __ffsll((long long)lt_mask) - 1;
                    lt_mask &= lt_mask - 1;
                    if (l == L) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            uint32_t mk = cl.lt[i];
                            while (mk) {
                                const int bit = __ffs(mk) - 1;
                                mk &= mk - 1;
                                const int j = bit >> 3;
                                const int b = (qq[i] >> (8 * j)) & 0xFF;
                                const int pos = base[b] + got[b];
                                got[b] = got[b] + 1;
                                if (pos < c_less) {
                                    ids_out[pos] = v + 4 * i + j;
                                    hops_out[pos] = (uint8_t)b;
                                }
                            }
                        }
                    }
                    wave_sync();
                }
            }
            if (found_eq < need) {
                const int incl = wave_incl_scan(n_eq);
                int rank = found_eq + incl - n_eq;
                if (n_eq > 0 && rank < need) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        uint32_t mk = cl.eq[i];
                        while (mk && rank < need) {
                            const int bit = __ffs(mk) - 1;
                            mk &= mk - 1;
                            ids_out[c_less + rank] = v + 4 * i + (bit >> 3);
                            hops_out[c_less + rank] = (uint8_t)hstar;
                            ++rank;
                        }
                    }
                }
                found_eq += __shfl(incl, GM_WAVE - 1, GM_WAVE);
            }
            if ((found_lt >= c_scan && found_eq >= need) || !more) break;
            li = nli;
            vb = nvb;
            ce = nce;
            q = qn;
        }
    }
    const int K = c_less + (need < found_eq ? need : found_eq);
    for (int i = K + l; i < k; i += GM_WAVE) {
        ids_out[i] = -1;
        hops_out[i] = 255;
    }
}

// Counts from the BFS transpose (k <= 16).  One wave per row.
__global__ void __launch_bounds__(kSelWaves * GM_WAVE)
knn_select_counted_kernel(int32_t n, int32_t k, int32_t rows, const uint8_t *__restrict__ hop_rows,
                          const int64_t *__restrict__ row_of, int64_t row_stride,
                          const int64_t *__restrict__ out_row, const unsigned int *__restrict__ part,
                          int32_t chunks, const int32_t *__restrict__ csr_row_ptr,
                          const int32_t *__restrict__ csr_col, const int32_t *__restrict__ src_of,
                          int32_t *__restrict__ ids, uint8_t *__restrict__ hops)
{
    __shared__ unsigned int cnt[kSelWaves][kCountLevels + 2];
    __shared__ int got[kSelWaves][kCountLevels + 2];
    __shared__ int base[kSelWaves][kCountLevels + 2];
    __shared__ int32_t list[kSelWaves][kMaxChunks];
    const int wid = threadIdx.x / GM_WAVE, l = lane();
    for (int32_t r = blockIdx.x * kSelWaves + wid; r < rows; r += gridDim.x * kSelWaves) {
        // the source's adjacency row and its first k entries (the candidates
        // at hop 1) are loaded first, beside the counts; they are stored once
        // the row's other entries are placed
        int32_t ca = 0, cdeg = -1, h1 = 0;
        if (csr_row_ptr) {
            const int32_t sv = src_of[r];
            ca = csr_row_ptr[sv];
            cdeg = csr_row_ptr[sv + 1] - ca;
            if (l < min(cdeg, k)) h1 = csr_col[ca + l];
        }
        // each lane loads the 16 per-level counts of its chunks (l, l + 64,
        // ...) once, summing them per level; its first chunk's stay in registers
        unsigned int my[kCountLevels], lsum[kCountLevels];
#pragma unroll
        for (int h = 0; h < kCountLevels; ++h) my[h] = lsum[h] = 0;
        for (int32_t cc = l; cc < chunks; cc += GM_WAVE) {
            const uint4 *p = (const uint4 *)(part + ((size_t)r * chunks + cc) * kCountLevels);
#pragma unroll
            for (int i = 0; i < kCountLevels / 4; ++i) {
                const uint4 x = p[i];
                const unsigned int xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    lsum[4 * i + j] += xs[j];
                    if (cc == l) my[4 * i + j] = xs[j];
                }
            }
        }
        // per-level totals, level by level until the k-th vertex is reached:
        // the last level h* and the number of its vertices taken (cnt[1..h*]
        // for select_row, which stops at the same level)
        int c = 0, hstar = kCountLevels + 1, need = 0, c1 = 0;
        bool found = false;
#pragma unroll
        for (int hh = 1; hh <= kCountLevels; ++hh) {
            if (!found) {
                const int ch = wave_sum((int)lsum[hh - 1]);
                if (hh == 1) c1 = ch;
                if (l == 0) cnt[wid][hh] = (unsigned int)ch;
                if (c + ch >= k) {
                    hstar = hh;
                    need = k - c;
                    found = true;
                } else {
                    c += ch;
                }
            }
        }
        // hop 1 from the source's canonical adjacency row when its length
        // matches the count: the first `need` entries when h* = 1, else all
        const int64_t o = out_row[r] * (int64_t)k;
        const int lo = cdeg == c1 ? 2 : 1;
        const int take1 = lo == 2 ? (hstar == 1 ? need : c1) : 0;   // at most k - 1 <= 63, or need = k <= 16
        if (lo == 2 && hstar == 1) {   // row complete: k entries at hop 1
            if (l < take1) {
                ids[o + l] = h1;
                hops[o + l] = 1;
            }
            continue;
        }
        // chunks holding a vertex with lo <= hop < h*, or one of the first
        // `need` vertices at hop h* (eq counts scanned in chunk order), in order
        int nlist = 0, eq_carry = 0;
        for (int32_t c0 = 0; c0 < chunks; c0 += GM_WAVE) {
            const int32_t cc = c0 + l;
            unsigned int v[kCountLevels];
            if (c0 == 0) {
#pragma unroll
                for (int h = 0; h < kCountLevels; ++h) v[h] = my[h];
            } else {
#pragma unroll
                for (int h = 0; h < kCountLevels; ++h) v[h] = 0;
                if (cc < chunks) {
                    const uint4 *p = (const uint4 *)(part + ((size_t)r * chunks + cc) * kCountLevels);
#pragma unroll
                    for (int i = 0; i < kCountLevels / 4; ++i) {
                        const uint4 x = p[i];
                        v[4 * i] = x.x;
                        v[4 * i + 1] = x.y;
                        v[4 * i + 2] = x.z;
                        v[4 * i + 3] = x.w;
                    }
                }
            }
            int lt_c = 0, eq_c = 0;
#pragma unroll
            for (int h = 0; h < kCountLevels; ++h) {
                if (h + 1 >= lo && h + 1 < hstar) lt_c += (int)v[h];
                else if (h + 1 == hstar) eq_c = (int)v[h];
            }
            const int incl = wave_incl_scan(eq_c);
            const bool needed = cc < chunks && (lt_c > 0 || (eq_c > 0 && eq_carry + incl - eq_c < need));
            const unsigned long long mk = __ballot(needed);
            if (needed) list[wid][nlist + lanes_below(mk)] = cc;
            nlist += __popcll(mk);
            eq_carry += __shfl(incl, GM_WAVE - 1, GM_WAVE);
        }
        wave_sync();
        const uint8_t *row = hop_rows + row_of[r] * row_stride;
        select_row(row, n, k, cnt[wid], kCountLevels, list[wid], nlist, chunks, got[wid], base[wid], ids + o,
                   hops + o, lo);
        if (l < take1) {
            ids[o + l] = h1;
            hops[o + l] = 1;
        }
        wave_sync();
    }
}

// Histogram in this kernel (any k).  One wave per block, per-lane bins.
__global__ void __launch_bounds__(GM_WAVE)
knn_select_hist_kernel(int32_t n, int32_t k, int32_t rows, const uint8_t *__restrict__ hop_rows,
                       const int64_t *__restrict__ row_of, int64_t row_stride,
                       const int64_t *__restrict__ out_row, int32_t *__restrict__ ids,
                       uint8_t *__restrict__ hops)
{
    extern __shared__ unsigned int bins[];  // [(k + 1)][64] then cnt[256]
    unsigned int *cnt = bins + (size_t)(k + 1) * GM_WAVE;
    __shared__ int got[256];
    __shared__ int base[256];
    const int l = lane();
    for (int32_t r = blockIdx.x; r < rows; r += gridDim.x) {
        for (int h = 0; h <= k; ++h) bins[h * GM_WAVE + l] = 0;
        wave_sync();
        const uint8_t *row = hop_rows + row_of[r] * row_stride;
        const bool aligned = (((uintptr_t)row) & 15) == 0;
        for (int32_t vb = 0; vb < n; vb += 16 * GM_WAVE) {
            const uint4 q = load16(row, n, vb + 16 * l, aligned);
            const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll 1
            for (int i = 0; i < 16; ++i) {
                const int b = (qq[i >> 2] >> (8 * (i & 3))) & 0xFF;
                if (b >= 1 && b <= k) bins[b * GM_WAVE + l] += 1;
            }
        }
        wave_sync();
        for (int h = 1 + l; h <= k; h += GM_WAVE) {
            unsigned int s = 0;
            for (int j = 0; j < GM_WAVE; ++j) s += bins[h * GM_WAVE + j];
            cnt[h] = s;
        }
        wave_sync();
        const int64_t o = out_row[r] * (int64_t)k;
        select_row(row, n, k, cnt, k, nullptr, 0, 1, got, base, ids + o, hops + o, 1);
        wave_sync();
    }
}

__global__ void copy_rows_kernel(int32_t pairs, const int64_t *__restrict__ dst_src, int32_t k, int32_t n,
                                 int32_t *ids, uint8_t *hops, uint8_t *hop_matrix)
{
    for (int32_t p = blockIdx.x; p < pairs; p += gridDim.x) {
        const int64_t d = dst_src[2 * p], s = dst_src[2 * p + 1];
        for (int i = threadIdx.x; i < k; i += blockDim.x) {
            ids[d * k + i] = ids[s * k + i];
            hops[d * k + i] = hops[s * k + i];
        }
        if (hop_matrix)
            for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
                hop_matrix[d * (int64_t)n + i] = hop_matrix[s * (int64_t)n + i];
    }
}

}  // namespace

hipError_t launch_knn_select_counted(int32_t n, int32_t k, int32_t rows, const uint8_t *hop_rows,
                                     const int64_t *row_of, int64_t row_stride, const int32_t *src_of,
                                     const int64_t *out_row, const unsigned int *part, int32_t chunks,
                                     const int32_t *csr_row_ptr, const int32_t *csr_col,
                                     int32_t *ids, uint8_t *hops, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    if (!src_of) csr_row_ptr = nullptr;
    if (part && k <= kCountLevels && chunks >= 1 && chunks <= kMaxChunks) {
        int blocks = (rows + kSelWaves - 1) / kSelWaves;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(knn_select_counted_kernel, dim3(blocks), dim3(kSelWaves * GM_WAVE), 0, s, n, k,
                           rows, hop_rows, row_of, row_stride, out_row, part, chunks, csr_row_ptr, csr_col,
                           src_of, ids, hops);
    } else {
        const size_t lds = ((size_t)(k + 1) * GM_WAVE + 256) * sizeof(unsigned int);
        static bool lds_set[64] = {};   // the LDS limit is an attribute of the kernel on each device
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev < 0 || dev >= 64 || !lds_set[dev]) {
            e = hipFuncSetAttribute((const void *)knn_select_hist_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(((size_t)(kMaxK + 1) * GM_WAVE + 256) * sizeof(unsigned int)));
            if (e != hipSuccess) return e;
            if (dev >= 0 && dev < 64) lds_set[dev] = true;
        }
        const int blocks = rows > 65536 ? 65536 : rows;
        hipLaunchKernelGGL(knn_select_hist_kernel, dim3(blocks), dim3(GM_WAVE), lds, s, n, k, rows, hop_rows,
                           row_of, row_stride, out_row, ids, hops);
    }
    return hipGetLastError();
}

hipError_t launch_knn_select(int32_t n, int32_t k, int32_t rows, const uint8_t *hop_rows,
                             const int64_t *row_of, int64_t row_stride, const int32_t *src_of,
                             const int64_t *out_row, int32_t *ids, uint8_t *hops, hipStream_t s)
{
    return launch_knn_select_counted(n, k, rows, hop_rows, row_of, row_stride, src_of, out_row, nullptr, 0,
                                     nullptr, nullptr, ids, hops, s);
}

hipError_t launch_copy_rows(int32_t pairs, const int64_t *dst_src, int32_t k, int32_t n,
                            int32_t *ids, uint8_t *hops, uint8_t *hop_matrix, hipStream_t s)
{
    if (pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_rows_kernel, dim3(pairs > 4096 ? 4096 : pairs), dim3(256), 0, s, pairs,
                       dst_src, k, n, ids, hops, hop_matrix);
    return hipGetLastError();
}

}  // namespace gm
