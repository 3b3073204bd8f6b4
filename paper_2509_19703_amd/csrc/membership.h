// UMAP fuzzy membership of one kNN row (Sec. 2.1: h_ij = exp(-(d_ij -
// rho_i)/sigma_i), rho_i the distance to the nearest neighbour, sigma_i set so
// that sum_j h_ij = log2 k).  One thread per row.
//
// Hops are integers, so with x = exp(-1/sigma) the row's sum is the
// polynomial P(x) = sum_d c_d x^d over the counts c_d of entries at hop
// rho + d, increasing and convex on (0, 1) from c_0 to K (the valid
// entries).  The root of P(x) = log2 k is found in double precision by
// Newton's method started at x = 1: on a convex increasing function the
// iterates decrease monotonically onto the root, and the loop ends when
// rounding stops the decrease.  Rows whose hops span more than kMembLevels
// levels keep the counts implicit and bisect in x instead.  Then
// sigma = -1/ln x and w_j = x^(h_j - rho).  Rows without a root take the
// limits: K = 0 -> all zero; c_0 >= log2 k -> sigma = 0, weights 1 at rho
// and 0 beyond; K <= log2 k -> sigma = +inf, weights 1.  The weights are
// x^(h_j - rho) by repeated products in double, no exponentials.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace gm {

constexpr int kMembLevels = 16;

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
    const int rho = k > 0 ? hop_at(0) : 255;
    if (rho == 255) {
        for (int j = 0; j < k; ++j) w[j] = 0.0f;
        if (rho_out) *rho_out = 0.0f;
        if (sigma_out) *sigma_out = 0.0f;
        return;
    }
    // counts per level above rho (one pass over the row), as 8-bit fields
    // (a count is at most k <= 254) of two words: levels 0..7 and 8..15
    uint64_t lo8 = 0, hi8 = 0;
    int K = 0;
    bool wide = false;
    for (; K < k; ++K) {
        const int h = hop_at(K);
        if (h == 255) break;
        const int d = h - rho;
        if (d < 8) lo8 += 1ull << (8 * d);
        else if (d < kMembLevels) hi8 += 1ull << (8 * (d - 8));
        else wide = true;
    }
    const int c0 = (int)(lo8 & 0xFF);
    const double T = log2((double)k);
    float sigma;
    if ((double)c0 >= T) {
        sigma = 0.0f;
        for (int j = 0; j < K; ++j) w[j] = hop_at(j) == rho ? 1.0f : 0.0f;
    } else if ((double)K <= T) {
        sigma = INFINITY;
        for (int j = 0; j < K; ++j) w[j] = 1.0f;
    } else {
        double x = 1.0;
        if (!wide) {
            // P and P' over the levels the row has (d <= dmax, often 2 or 3),
            // the counts read from their 8-bit fields
            const int dmax = hop_at(K - 1) - rho;
            for (int it = 0; it < 1000; ++it) {
                double p = 0.0, dp = 0.0, pw = 1.0, pwm1 = 0.0;   // x^d, x^(d - 1)
                for (int d = 0; d <= dmax; ++d) {
                    const double c = (double)(((d < 8 ? lo8 : hi8) >> (8 * (d & 7))) & 0xFF);
                    p = fma(c, pw, p);
                    dp = fma(c * (double)d, pwm1, dp);
                    pwm1 = pw;
                    pw *= x;
                }
                const double xn = x - (p - T) / dp;
                if (!(xn < x)) break;
                x = xn > 0.0 ? xn : 0.5 * x;
            }
        } else {
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < 2000; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mid == lo || mid == hi) break;
                if (membership_poly(hop_at, K, rho, mid) < T) lo = mid;
                else hi = mid;
            }
            x = hi;
        }
        sigma = (float)(-1.0 / log(x));
        // w_j = x^(h_j - rho); the hops are sorted, so one running power
        // serves the row (at most 254 products, relative error below 1e-13)
        double pw = 1.0;
        int cur = 0;
        for (int j = 0; j < K; ++j) {
            const int d = hop_at(j) - rho;
            while (cur < d) {
                pw *= x;
                ++cur;
            }
            w[j] = (float)pw;
        }
    }
    for (int j = K; j < k; ++j) w[j] = 0.0f;
    if (rho_out) *rho_out = (float)rho;
    if (sigma_out) *sigma_out = sigma;
}

}  // namespace gm
