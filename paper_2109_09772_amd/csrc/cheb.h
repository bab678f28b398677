// Chebyshev points of the second kind and barycentric Lagrange interpolation
// (tensor-product proxies of the treecodes).
#pragma once

#include "rism_internal.h"

namespace rism {

constexpr int kMaxDeg = 16;

// Chebyshev points of the second kind on [lo, hi] and their barycentric
// weights: s_k = lo + (hi - lo)(1 + cos(k pi/n))/2, w_k = (-1)^k delta_k with
// delta_0 = delta_n = 1/2, else 1.
__device__ __forceinline__ double cheb_point(double lo, double hi, int k, int n)
{
    return lo + (hi - lo) * 0.5 * (1.0 + cos(kPi * k / n));
}
__device__ __forceinline__ double bary_weight(int k, int n)
{
    double w = (k & 1) ? -1.0 : 1.0;
    return (k == 0 || k == n) ? 0.5 * w : w;
}

// Lagrange basis values L_k(x), k = 0..n, of the Chebyshev points of [lo, hi],
// written to dst[k * stride] (LDS or global memory; a per-thread array with a
// run-time bound would live in scratch memory).
__device__ inline void lagrange_to(double x, double lo, double hi, int n, double *dst, int stride)
{
    double den = 0.0;
    int exact = -1;
    for (int k = 0; k <= n; ++k) {
        double d = x - cheb_point(lo, hi, k, n);
        if (d == 0.0) exact = k;
        double t = bary_weight(k, n) / d;
        dst[k * stride] = t;
        den += t;
    }
    const double inv = 1.0 / den;
    for (int k = 0; k <= n; ++k)
        dst[k * stride] = exact >= 0 ? (k == exact ? 1.0 : 0.0) : dst[k * stride] * inv;
}

// lagrange_to with the cosines cos(k pi / n), k = 0..n, given (the same
// values cheb_point forms): the points are lo + (hi - lo)(1 + c_k)/2.
__device__ inline void lagrange_to_cos(double x, double lo, double hi, int n, const double *cosk,
                                       double *dst, int stride)
{
    double den = 0.0;
    int exact = -1;
    for (int k = 0; k <= n; ++k) {
        double d = x - (lo + (hi - lo) * 0.5 * (1.0 + cosk[k]));
        if (d == 0.0) exact = k;
        double t = bary_weight(k, n) / d;
        dst[k * stride] = t;
        den += t;
    }
    const double inv = 1.0 / den;
    for (int k = 0; k <= n; ++k)
        dst[k * stride] = exact >= 0 ? (k == exact ? 1.0 : 0.0) : dst[k * stride] * inv;
}

// Element ax (0, 1, 2) of a three-vector held in registers (a run-time index
// into a private array would place it in scratch memory).
__device__ __forceinline__ double pick3(const double *v, int ax)
{
    return ax == 0 ? v[0] : (ax == 1 ? v[1] : v[2]);
}

// Proxy box of a node: its tight box, padded so that no axis is degenerate.
__device__ __forceinline__ void proxy_box(const double *box, double *pb)
{
    for (int k = 0; k < 3; ++k) {
        double lo = box[k], hi = box[3 + k];
        double w = hi - lo;
        if (w < 1e-3) {
            double c = 0.5 * (lo + hi);
            lo = c - 5e-4;
            hi = c + 5e-4;
        }
        pb[k] = lo;
        pb[3 + k] = hi;
    }
}

}  // namespace rism
