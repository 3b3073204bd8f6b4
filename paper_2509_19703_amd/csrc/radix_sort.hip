// Stable least-significant-digit radix sort of (key, 32-bit value) pairs,
// used by the layout step (fuzzy-union keys, the keyed shuffle of E_k that
// opens Alg. 5, the incidence lists of GradSample) and by the sparsifier's
// ranking of edges by effective resistance (Alg. 2).
//
// One pass per 8-bit digit of the requested key bits, each in three steps:
//   histogram  a workgroup per tile counts the tile's digits in LDS
//              (one sub-histogram per wave, then summed) and writes them
//              digit-major, counts[digit * tiles + tile];
//   scan       a device-wide exclusive scan of that array gives every
//              (digit, tile) its first output position: digits in order, and
//              within a digit the tiles in order;
//   scatter    a workgroup walks its tile in rounds of 256 items (one per
//              thread, in input order) and ranks each item among the equal
//              digits before it: inside a wave by eight ballots (one per
//              digit bit) that leave the lanes holding the same digit, a
//              popcount of those below the lane; across the round's waves by
//              the per-wave digit counts in LDS; across rounds by a running
//              count per digit.
// Every item keeps its order among equal digits, so the sort is stable and
// equal keys keep their input order.  Tiles are 256 x rounds items, rounds
// chosen so that a launch has at least ~1,024 workgroups when the input is
// large enough.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "kernels.h"

namespace gm {
namespace {

constexpr int kRsBlock = 256;
constexpr int kRsWaves = kRsBlock / 64;
constexpr int kRsMaxRounds = 16;

template <typename K>
__global__ void __launch_bounds__(kRsBlock)
rs_hist_kernel(const K *__restrict__ keys, int64_t count, int shift, int rounds, int64_t tiles,
               int32_t *__restrict__ counts)
{
    __shared__ int32_t h[kRsWaves][256];
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) h[q][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * rounds * kRsBlock + t;
    for (int r0 = 0; r0 < rounds; r0 += 4) {
        K k[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = base + (int64_t)(r0 + u) * kRsBlock;
            ok[u] = r0 + u < rounds && i < count;
            k[u] = ok[u] ? keys[i] : (K)0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (ok[u]) atomicAdd(&h[w][(int)((k[u] >> shift) & 255u)], 1);
    }
    __syncthreads();
    int32_t c = 0;
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) c += h[q][t];
    counts[(int64_t)t * tiles + blockIdx.x] = c;
}

template <typename K>
__global__ void __launch_bounds__(kRsBlock)
rs_scatter_kernel(const K *__restrict__ keys, const uint32_t *__restrict__ vals, K *__restrict__ okeys,
                  uint32_t *__restrict__ ovals, int64_t count, int shift, int rounds, int64_t tiles,
                  const int32_t *__restrict__ offsets)
{
    __shared__ int32_t run[256];
    __shared__ int32_t wc[2][kRsWaves][256];   // per-wave digit counts, double-buffered by round
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    run[t] = offsets[(int64_t)t * tiles + blockIdx.x];
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) wc[0][q][t] = 0;
    __syncthreads();
    const uint64_t below_mask = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * rounds * kRsBlock + t;
    for (int r = 0; r < rounds; ++r) {
        const int cur = r & 1;
        const int64_t i = base + (int64_t)r * kRsBlock;
        const bool valid = i < count;
        K k = (K)0;
        uint32_t v = 0;
        if (valid) {
            k = keys[i];
            v = vals[i];
        }
        const int d = (int)((k >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int below = __popcll(peers & below_mask);
        if (valid && (peers >> lane) == 1ull) wc[cur][w][d] = __popcll(peers);   // highest lane of its digit
        // the next round's counts start at zero
#pragma unroll
        for (int q = 0; q < kRsWaves; ++q) wc[cur ^ 1][q][t] = 0;
        __syncthreads();
        if (valid) {
            int32_t pos = run[d] + below;
            for (int q = 0; q < w; ++q) pos += wc[cur][q][d];
            okeys[pos] = k;
            ovals[pos] = v;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int q = 0; q < kRsWaves; ++q) add += wc[cur][q][t];
        run[t] += add;
        // run[] is read again only after the next round's first barrier
    }
}

int rs_rounds(int64_t count)
{
    int rounds = kRsMaxRounds;
    while (rounds > 1 && (count + (int64_t)kRsBlock * rounds - 1) / ((int64_t)kRsBlock * rounds) < 1024) rounds >>= 1;
    return rounds;
}

int64_t rs_tiles(int64_t count, int rounds)
{
    const int64_t per = (int64_t)kRsBlock * rounds;
    return count > 0 ? (count + per - 1) / per : 0;
}

size_t rs_align(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t radix_sort_scratch_bytes(int64_t count)
{
    const int64_t tiles = rs_tiles(count, rs_rounds(count));
    const int64_t cells = 256 * (tiles > 0 ? tiles : 1);
    return 2 * rs_align((size_t)(cells + 1) * sizeof(int32_t)) + exclusive_scan_scratch_bytes(cells);
}

template <typename K>
hipError_t radix_sort_pairs(K *keys, K *keys_alt, uint32_t *vals, uint32_t *vals_alt, int64_t count, int begin_bit,
                            int end_bit, void *scratch, hipStream_t s, bool *in_alt)
{
    *in_alt = false;
    if (count <= 1 || end_bit <= begin_bit) return hipSuccess;
    if (count >= ((int64_t)1 << 31) || begin_bit < 0 || end_bit > (int)(8 * sizeof(K))) return hipErrorInvalidValue;
    const int rounds = rs_rounds(count);
    const int64_t tiles = rs_tiles(count, rounds);
    const int64_t cells = 256 * tiles;
    char *p = (char *)scratch;
    int32_t *counts = (int32_t *)p;
    int32_t *offsets = (int32_t *)(p + rs_align((size_t)(cells + 1) * sizeof(int32_t)));
    void *scan_tmp = p + 2 * rs_align((size_t)(cells + 1) * sizeof(int32_t));
    K *src_k = keys, *dst_k = keys_alt;
    uint32_t *src_v = vals, *dst_v = vals_alt;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL(rs_hist_kernel<K>, dim3((unsigned)tiles), dim3(kRsBlock), 0, s, (const K *)src_k, count,
                           shift, rounds, tiles, counts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_exclusive_scan(counts, offsets, cells, scan_tmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(rs_scatter_kernel<K>, dim3((unsigned)tiles), dim3(kRsBlock), 0, s, (const K *)src_k,
                           (const uint32_t *)src_v, dst_k, dst_v, count, shift, rounds, tiles,
                           (const int32_t *)offsets);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        K *tk = src_k;
        src_k = dst_k;
        dst_k = tk;
        uint32_t *tv = src_v;
        src_v = dst_v;
        dst_v = tv;
        *in_alt = !*in_alt;
    }
    return hipSuccess;
}

template hipError_t radix_sort_pairs<uint32_t>(uint32_t *, uint32_t *, uint32_t *, uint32_t *, int64_t, int, int,
                                               void *, hipStream_t, bool *);
template hipError_t radix_sort_pairs<unsigned long>(unsigned long *, unsigned long *, uint32_t *, uint32_t *,
                                                    int64_t, int, int, void *, hipStream_t, bool *);
template hipError_t radix_sort_pairs<unsigned long long>(unsigned long long *, unsigned long long *, uint32_t *,
                                                         uint32_t *, int64_t, int, int, void *, hipStream_t,
                                                         bool *);

}  // namespace gm
