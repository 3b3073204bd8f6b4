// kNN selection from hop rows (GUMAP step C1, Sec. 3.1, Alg. 1): per source
// row of n hop bytes, the k smallest (hop, id) pairs with 1 <= hop <= 254
// (hop 0 is the source itself, 255 unreachable).
//
// With c(h) = number of vertices at hop h, the last hop taken is the smallest
// h* with c(1) + ... + c(h*) >= k.  Every vertex with hop < h* is taken and
// the first k - (c(1) + ... + c(h*-1)) vertices at hop h* in id order.  The
// counts come either from the BFS transpose (hops 1..16) or from a histogram
// pass of this kernel.  One streaming pass over the row in id order then
// writes the taken entries straight to their (hop, id) position and stops as
// soon as all of them are found.
#include "device.h"
#include "kernels.h"

namespace gm {

namespace {

constexpr int kCountLevels = 16;
constexpr int kSelWaves = 4;
#define GUMAP_MAX_K_INTERNAL 254

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Loads the 16 hop bytes of lane-chunk starting at vertex `v` (bytes past n
// read as 255, i.e. skipped).
__device__ __forceinline__ void load16(const uint8_t *row, int32_t n, int32_t v, bool aligned,
                                       uint32_t q[4])
{
    if (aligned && v + 16 <= n) {
        uint4 x = *(const uint4 *)(row + v);
        q[0] = x.x; q[1] = x.y; q[2] = x.z; q[3] = x.w;
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t w = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int32_t id = v + 4 * i + j;
                uint32_t b = id < n ? row[id] : 255u;
                w |= b << (8 * j);
            }
            q[i] = w;
        }
    }
}

// Selection pass shared by both kernels.  cnt_lds[h] (h = 1..hmax) holds the
// per-hop counts; got/base are per-wave LDS scratch of 256 ints each.
__device__ void select_row(const uint8_t *row, int32_t n, int32_t k, int32_t src,
                           const unsigned int *cnt_lds, int hmax, int *got, int *base,
                           int32_t *ids_out, uint8_t *hops_out)
{
    const int l = lane();
    // last hop and how many to take at it
    int c = 0, hstar = hmax + 1, need = 0;
    for (int h = 1; h <= hmax; ++h) {
        int ch = (int)cnt_lds[h];
        if (c + ch >= k) { hstar = h; need = k - c; break; }
        c += ch;
    }
    const int c_less = c;
    // output offset of each hop below h*
    if (l == 0) {
        int acc = 0;
        for (int h = 1; h < hstar && h <= hmax; ++h) {
            base[h] = acc;
            got[h] = 0;
            acc += (int)cnt_lds[h];
        }
    }
    wave_sync();
    const bool aligned = (((uintptr_t)row) & 15) == 0;
    int found_lt = 0, found_eq = 0;
    if (c_less > 0 || need > 0) {
        for (int32_t vb = 0; vb < n; vb += 16 * GM_WAVE) {
            const int32_t v = vb + 16 * l;
            uint32_t q[4];
            load16(row, n, v, aligned, q);
            int n_lt = 0, n_eq = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                int b = (q[i >> 2] >> (8 * (i & 3))) & 0xFF;
                n_lt += (b >= 1 && b < hstar && b <= 254);
                n_eq += (b == hstar);
            }
            unsigned long long lt_mask = __ballot(n_lt > 0);
            while (lt_mask) {
                const int L = __ffsll((long long)lt_mask) - 1;
                lt_mask &= lt_mask - 1;
                if (l == L) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        int b = (q[i >> 2] >> (8 * (i & 3))) & 0xFF;
                        if (b >= 1 && b < hstar && b <= 254) {
                            int pos = base[b] + got[b];
                            got[b] = got[b] + 1;
                            if (pos < c_less) {
                                ids_out[pos] = v + i;
                                hops_out[pos] = (uint8_t)b;
                            }
                        }
                    }
                }
                wave_sync();
            }
            if (need > 0) {
                const int incl = wave_incl_scan(n_eq);
                int rank = found_eq + incl - n_eq;
                if (n_eq > 0 && rank < need) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        int b = (q[i >> 2] >> (8 * (i & 3))) & 0xFF;
                        if (b == hstar) {
                            if (rank < need) {
                                ids_out[c_less + rank] = v + i;
                                hops_out[c_less + rank] = (uint8_t)b;
                            }
                            ++rank;
                        }
                    }
                }
                found_eq += __shfl(incl, GM_WAVE - 1, GM_WAVE);
            }
            found_lt += wave_sum(n_lt);
            if (found_lt >= c_less && found_eq >= need) break;
        }
    }
    (void)src;
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
                          const int32_t *__restrict__ src_of, const int64_t *__restrict__ out_row,
                          const unsigned int *__restrict__ lvl_cnt, int32_t *__restrict__ ids,
                          uint8_t *__restrict__ hops)
{
    __shared__ unsigned int cnt[kSelWaves][kCountLevels + 2];
    __shared__ int got[kSelWaves][256];
    __shared__ int base[kSelWaves][256];
    const int wid = threadIdx.x / GM_WAVE, l = lane();
    for (int32_t r = blockIdx.x * kSelWaves + wid; r < rows; r += gridDim.x * kSelWaves) {
        if (l < kCountLevels) cnt[wid][l + 1] = lvl_cnt[(size_t)r * kCountLevels + l];
        wave_sync();
        const uint8_t *row = hop_rows + row_of[r] * row_stride;
        const int64_t o = out_row[r] * (int64_t)k;
        select_row(row, n, k, src_of[r], cnt[wid], kCountLevels, got[wid], base[wid], ids + o, hops + o);
        wave_sync();
    }
}

// Histogram in this kernel (any k).  One wave per block, per-lane bins.
__global__ void __launch_bounds__(GM_WAVE)
knn_select_hist_kernel(int32_t n, int32_t k, int32_t rows, const uint8_t *__restrict__ hop_rows,
                       const int64_t *__restrict__ row_of, int64_t row_stride,
                       const int32_t *__restrict__ src_of, const int64_t *__restrict__ out_row,
                       int32_t *__restrict__ ids, uint8_t *__restrict__ hops)
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
            uint32_t q[4];
            load16(row, n, vb + 16 * l, aligned, q);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                int b = (q[i >> 2] >> (8 * (i & 3))) & 0xFF;
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
        select_row(row, n, k, src_of[r], cnt, k, got, base, ids + o, hops + o);
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
                                     const int64_t *out_row, const unsigned int *lvl_cnt,
                                     int32_t *ids, uint8_t *hops, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    if (lvl_cnt && k <= kCountLevels) {
        int blocks = (rows + kSelWaves - 1) / kSelWaves;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(knn_select_counted_kernel, dim3(blocks), dim3(kSelWaves * GM_WAVE), 0, s,
                           n, k, rows, hop_rows, row_of, row_stride, src_of, out_row, lvl_cnt, ids, hops);
    } else {
        size_t lds = ((size_t)(k + 1) * GM_WAVE + 256) * sizeof(unsigned int);
        static bool lds_set = false;
        if (!lds_set) {
            hipError_t e = hipFuncSetAttribute((const void *)knn_select_hist_kernel,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)(((size_t)(GUMAP_MAX_K_INTERNAL + 1) * GM_WAVE + 256) * sizeof(unsigned int)));
            if (e != hipSuccess) return e;
            lds_set = true;
        }
        int blocks = rows > 65536 ? 65536 : rows;
        hipLaunchKernelGGL(knn_select_hist_kernel, dim3(blocks), dim3(GM_WAVE), lds, s, n, k, rows,
                           hop_rows, row_of, row_stride, src_of, out_row, ids, hops);
    }
    return hipGetLastError();
}

hipError_t launch_knn_select(int32_t n, int32_t k, int32_t rows, const uint8_t *hop_rows,
                             const int64_t *row_of, int64_t row_stride, const int32_t *src_of,
                             const int64_t *out_row, int32_t *ids, uint8_t *hops, hipStream_t s)
{
    return launch_knn_select_counted(n, k, rows, hop_rows, row_of, row_stride, src_of, out_row,
                                     nullptr, ids, hops, s);
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
