// FP64 pair arithmetic shared by the kick, drift, diagnostic and large-group kernels, and the
// Bulirsch-Stoer helpers shared by the one-wave and the grid-wide encounter steps.
#pragma once

#include <hip/hip_runtime.h>

#include "genga_internal.h"

namespace genga {

// separation^2 and squares without contraction: encounter decisions use exactly the rounding
// of the definition ((dx*dx + dy*dy) + dz*dz, then compare with rc*rc)
__device__ __forceinline__ double sep2_rn(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    return (a + b) + c;
}

__device__ __forceinline__ double sq_rn(double a)
{
#pragma clang fp contract(off)
    return a * a;
}

// Changeover weight of Chambers (1999), cited in Sect. 1: K(y) = y^2 / (2y^2 - 2y + 1) on
// [0, 1], 0 below, 1 above.
__device__ __forceinline__ double changeover_k(double y)
{
    if (y <= 0.0) return 0.0;
    if (y >= 1.0) return 1.0;
    double y2 = y * y;
    return y2 / (2.0 * y2 - 2.0 * y + 1.0);
}

// 1/sqrt(q) in FP64: v_rsq_f64 (about 2^-24) and one third-order correction
__device__ __forceinline__ double inv_sqrt64(double q)
{
    const double y0 = __builtin_amdgcn_rsq(q);
    const double t = q * y0;
    const double e = fma(-t, y0, 1.0);
    const double p = fma(0.375, e, 0.5);
    return fma(y0 * e, p, y0);
}

// Step reduction after a rejected step: 0.9 (tol/err)^(1/15) from the last column's error,
// kept within [1/50, 1/2].
__device__ __forceinline__ double shrink_factor(double err, double tol)
{
    const double f = 0.9 * pow(tol / err, 1.0 / (2 * BS_KMAX - 1));
    return fmax(0.02, fmin(0.5, f));
}

// Polynomial extrapolation in h^2 to h = 0 over the nodes n_0..n_k (n_j = 2(j+1)) has the
// Lagrange weights w_j = prod_{m != j} n_j^2 / (n_j^2 - n_m^2); it is the value Neville's
// scheme computes, T(k, k), and the same over the nodes 1..k gives T(k, k-1).  Both sets of
// weights sum to one, so the sums are formed relative to T(0, 0), which keeps their rounding
// at the size of the differences.
struct LagrangeTable {
    double w[BS_KMAX][BS_KMAX]; // w[k][j]: weight of T(j, 0) in T(k, k)
    double d[BS_KMAX][BS_KMAX]; // d[k][j]: weight of T(j, 0) in T(k, k) - T(k, k-1)
    constexpr LagrangeTable() : w(), d()
    {
        for (int k = 0; k < BS_KMAX; ++k)
            for (int j = 0; j <= k; ++j) {
                const double nj2 = 4.0 * (j + 1) * (j + 1);
                double a = 1.0, b = 1.0;
                for (int m = 0; m <= k; ++m) {
                    if (m == j) continue;
                    const double nm2 = 4.0 * (m + 1) * (m + 1);
                    a *= nj2 / (nj2 - nm2);
                    if (m >= 1) b *= nj2 / (nj2 - nm2);
                }
                w[k][j] = a;
                d[k][j] = j >= 1 ? a - b : a;
            }
    }
};
__constant__ constexpr LagrangeTable LAGRANGE{};

// Minimum / maximum over the 64 lanes of a wave.
__device__ __forceinline__ double wave_minv(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_maxv(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Bounding box of the positions held by the lanes with v = true, into
// out[t * 8 + 0..5] = (min x, y, z, max x, y, z).  Every lane of the wave calls it.
__device__ __forceinline__ void tile_box(bool v, double x, double y, double z, double *out, int t)
{
    const int lane = threadIdx.x & 63;
    const double lo[3] = {wave_minv(v ? x : INFINITY), wave_minv(v ? y : INFINITY), wave_minv(v ? z : INFINITY)};
    const double hi[3] = {wave_maxv(v ? x : -INFINITY), wave_maxv(v ? y : -INFINITY), wave_maxv(v ? z : -INFINITY)};
    if (lane < 3) {
        out[t * 8 + lane] = lo[lane];
        out[t * 8 + 3 + lane] = hi[lane];
    }
}


} // namespace genga
