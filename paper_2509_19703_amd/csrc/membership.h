// UMAP fuzzy membership of one kNN row (Sec. 2.1: h_ij = exp(-(d_ij -
// rho_i)/sigma_i), rho_i the distance to the nearest neighbour, sigma_i set so
// that sum_j h_ij = log2 k).  One thread per row.
//
// Hops are integers, so with x = exp(-1/sigma) the row's sum is the
// polynomial P(x) = sum_j x^(h_j - rho), increasing on (0, 1) from
// c0 = #{h_j = rho} to K (the valid entries).  The root of P(x) = log2 k is
// bisected directly in x in double precision (Horner-free incremental powers
// over the sorted row, no exp per step); sigma = -1/ln x and w_j = x^(h_j-rho).
// Rows without a root take the limits: K = 0 -> all zero; c0 >= log2 k ->
// sigma = 0, weights 1 at rho and 0 beyond; K <= log2 k -> sigma = +inf,
// weights 1.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace gm {

template <typename HopAt>
__device__ __forceinline__ double membership_poly(HopAt hop_at, int K, int rho, double x)
{
    double sum = 0.0, pw = 1.0;
    int cur = 0;
    for (int j = 0; j < K; ++j) {
        const int d = hop_at(j) - rho;
        while (cur < d) { pw *= x; ++cur; }
        sum += pw;
    }
    return sum;
}

// hop_at(j) returns the j-th hop of the row (0 <= j < k), sorted ascending,
// 255 = padding.  Writes k weights and the row's rho and sigma.
template <typename HopAt>
__device__ __forceinline__ void membership_row(HopAt hop_at, int k, float *w, float *rho_out,
                                               float *sigma_out)
{
    int K = 0;
    while (K < k && hop_at(K) != 255) ++K;
    if (K == 0) {
        for (int j = 0; j < k; ++j) w[j] = 0.0f;
        if (rho_out) *rho_out = 0.0f;
        if (sigma_out) *sigma_out = 0.0f;
        return;
    }
    const int rho = hop_at(0);
    const double T = log2((double)k);
    int c0 = 0;
    for (int j = 0; j < K; ++j) c0 += (hop_at(j) == rho);
    float sigma;
    if ((double)c0 >= T) {
        sigma = 0.0f;
        for (int j = 0; j < K; ++j) w[j] = hop_at(j) == rho ? 1.0f : 0.0f;
    } else if ((double)K <= T) {
        sigma = INFINITY;
        for (int j = 0; j < K; ++j) w[j] = 1.0f;
    } else {
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 2000; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid == lo || mid == hi) break;
            if (membership_poly(hop_at, K, rho, mid) < T) lo = mid;
            else hi = mid;
        }
        const double lx = log(hi);
        sigma = (float)(-1.0 / lx);
        for (int j = 0; j < K; ++j) w[j] = (float)exp((double)(hop_at(j) - rho) * lx);
    }
    for (int j = K; j < k; ++j) w[j] = 0.0f;
    if (rho_out) *rho_out = (float)rho;
    if (sigma_out) *sigma_out = sigma;
}

}  // namespace gm
