// Wave64 helpers shared by the gfx950 kernels of this library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GM_WAVE 64
#define GM_INF_ID 0x7fffffff

namespace gm {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Degree above which a vertex gets a whole wave in the BFS level kernel:
// `forced` if positive, else max(64, 8 * mean degree).
__device__ __forceinline__ int32_t heavy_threshold(int32_t n, const int32_t *row_ptr, int32_t forced)
{
    const int32_t mean = n > 0 ? row_ptr[n] / n : 0;
    return forced > 0 ? forced : max(64, 8 * mean);
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, GM_WAVE));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, GM_WAVE));
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, GM_WAVE);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, GM_WAVE);
    return v;
}

// Inclusive prefix sum across the wave (Hillis-Steele with shuffles).
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int l = lane();
#pragma unroll
    for (int o = 1; o < GM_WAVE; o <<= 1) {
        int t = __shfl_up(v, o, GM_WAVE);
        if (l >= o) v += t;
    }
    return v;
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int lanes_below(unsigned long long mask)
{
    return __popcll(mask & ((1ull << lane()) - 1ull));
}

// Lower bound of `key` in the sorted int32 range [lo, hi).
__device__ __forceinline__ int lower_bound(const int32_t *a, int lo, int hi, int key)
{
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace gm
