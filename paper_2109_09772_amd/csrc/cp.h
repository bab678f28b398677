// Implicit octree of the grid targets (cluster-particle treecode and its
// adjoint): level-l clusters are blocks of (B 2^l)^3 grid points clipped to
// the grid; level 0 are the leaves; the top level T is one cluster.
#pragma once

#include "rism_internal.h"

namespace rism {

constexpr int kCpMaxLev = 20;

struct CpLevels {
    int B, T, nx, ny, nz;
    double h[3];
    double theta;
    // > 0: distance condition added to the MAC, |y - c_C| - r_C >= guard (no
    // target of an accepting cluster closer to the atom than guard); 0: none
    double guard;
    int cx[kCpMaxLev + 1], cy[kCpMaxLev + 1], cz[kCpMaxLev + 1];
    int off[kCpMaxLev + 2];   // first id of level l (l = 1..T); off[T + 1] = clusters
};

__host__ __device__ inline void cp_box(const CpLevels &L, int lvl, int I, int J, int K,
                                       double lo[3], double hi[3])
{
    const int e = L.B << lvl;
    const int il = I * e, jl = J * e, kl = K * e;
    const int ih = (il + e < L.nx ? il + e : L.nx) - 1;
    const int jh = (jl + e < L.ny ? jl + e : L.ny) - 1;
    const int kh = (kl + e < L.nz ? kl + e : L.nz) - 1;
    lo[0] = il * L.h[0];
    lo[1] = jl * L.h[1];
    lo[2] = kl * L.h[2];
    hi[0] = ih * L.h[0];
    hi[1] = jh * L.h[1];
    hi[2] = kh * L.h[2];
}

__host__ __device__ inline void cp_centre(const CpLevels &L, int lvl, int I, int J, int K,
                                          double c[3], double &r)
{
    double lo[3], hi[3];
    cp_box(L, lvl, I, J, K, lo, hi);
    double r2 = 0;
    for (int k = 0; k < 3; ++k) {
        c[k] = 0.5 * (lo[k] + hi[k]);
        r2 += 0.25 * (hi[k] - lo[k]) * (hi[k] - lo[k]);
    }
    r = sqrt(r2);
}

// Proxy box of a cluster: its box, widened to half a spacing around a single
// grid plane so that no axis is degenerate.
__device__ inline void cp_proxy_box(const CpLevels &L, int lvl, int I, int J, int K, double pb[6])
{
    double lo[3], hi[3];
    cp_box(L, lvl, I, J, K, lo, hi);
    for (int k = 0; k < 3; ++k) {
        if (hi[k] - lo[k] < 0.25 * L.h[k]) {
            lo[k] -= 0.5 * L.h[k];
            hi[k] += 0.5 * L.h[k];
        }
        pb[k] = lo[k];
        pb[3 + k] = hi[k];
    }
}

// One axis of cp_box, cp_proxy_box and the centre of cp_centre (the same
// values: each axis of those is formed from its own index alone).
__host__ __device__ inline void cp_box_axis(const CpLevels &L, int lvl, int ax, int I, double &lo,
                                            double &hi)
{
    const int e = L.B << lvl;
    const int n = ax == 0 ? L.nx : (ax == 1 ? L.ny : L.nz);
    const double h = ax == 0 ? L.h[0] : (ax == 1 ? L.h[1] : L.h[2]);
    const int il = I * e;
    const int ih = (il + e < n ? il + e : n) - 1;
    lo = il * h;
    hi = ih * h;
}

__device__ inline void cp_proxy_axis(const CpLevels &L, int lvl, int ax, int I, double &lo,
                                     double &hi)
{
    cp_box_axis(L, lvl, ax, I, lo, hi);
    const double h = ax == 0 ? L.h[0] : (ax == 1 ? L.h[1] : L.h[2]);
    if (hi - lo < 0.25 * h) {
        lo -= 0.5 * h;
        hi += 0.5 * h;
    }
}

__device__ inline double cp_centre_axis(const CpLevels &L, int lvl, int ax, int I)
{
    double lo, hi;
    cp_box_axis(L, lvl, ax, I, lo, hi);
    return 0.5 * (lo + hi);
}

__device__ inline void cp_decode(const CpLevels &L, int id, int &lvl, int &I, int &J, int &K)
{
    lvl = 1;
    while (lvl < L.T && id >= L.off[lvl + 1]) ++lvl;
    int r = id - L.off[lvl];
    I = r % L.cx[lvl];
    r /= L.cx[lvl];
    J = r % L.cy[lvl];
    K = r / L.cy[lvl];
}

__device__ inline int cp_id(const CpLevels &L, int lvl, int I, int J, int K)
{
    return L.off[lvl] + (K * L.cy[lvl] + J) * L.cx[lvl] + I;
}

__device__ inline bool cp_mac(const CpLevels &L, int lvl, int I, int J, int K, const double y[3])
{
    double lo[3], hi[3];
    cp_box(L, lvl, I, J, K, lo, hi);
    double r2 = 0, d2 = 0;
    for (int k = 0; k < 3; ++k) {
        const double w = hi[k] - lo[k], d = y[k] - 0.5 * (lo[k] + hi[k]);
        r2 += 0.25 * w * w;
        d2 += d * d;
    }
    return r2 < L.theta * L.theta * d2 && (L.guard <= 0.0 || sqrt(d2) - sqrt(r2) >= L.guard);
}

// Radius around a cluster's centre (half-diagonal r) beyond which every atom
// is well separated from it: r / theta, or r + guard if that is larger.
__host__ __device__ inline double cp_sep_radius(const CpLevels &L, double r)
{
    const double a = r / L.theta, b = r + L.guard;
    return L.guard > 0.0 && b > a ? b : a;
}

// The MAC terms of one cluster, formed as cp_mac forms them: the box centre
// and the squared half-diagonal.  Kept in LDS for a cluster's chain of
// ancestors, they turn each test into a distance and one comparison.
struct CpMac {
    double c[3], r2, r;
};

__device__ inline void cp_mac_terms(const CpLevels &L, int lvl, int I, int J, int K, CpMac &m)
{
    double lo[3], hi[3];
    cp_box(L, lvl, I, J, K, lo, hi);
    double r2 = 0;
    for (int k = 0; k < 3; ++k) {
        const double w = hi[k] - lo[k];
        m.c[k] = 0.5 * (lo[k] + hi[k]);
        r2 += 0.25 * w * w;
    }
    m.r2 = r2;
    m.r = sqrt(r2);
}

// Same result as cp_mac for the cluster whose terms m holds.
__device__ inline bool cp_mac_at(const CpLevels &L, const CpMac &m, const double y[3])
{
    double d2 = 0;
    for (int k = 0; k < 3; ++k) {
        const double d = y[k] - m.c[k];
        d2 += d * d;
    }
    return m.r2 < L.theta * L.theta * d2 && (L.guard <= 0.0 || sqrt(d2) - m.r >= L.guard);
}

// Coarsest level in [stop, T] along the chain of the level-0 block (I0, J0,
// K0) at which y is well separated; 0 if none.
__device__ inline int cp_accept_level(const CpLevels &L, int I0, int J0, int K0, const double y[3],
                                      int stop)
{
    for (int lvl = L.T; lvl >= stop; --lvl)
        if (cp_mac(L, lvl, I0 >> lvl, J0 >> lvl, K0 >> lvl, y)) return lvl;
    return 0;
}

__device__ __forceinline__ double gap2_point_box(const double c[3], const double *box)
{
    double s = 0;
    for (int k = 0; k < 3; ++k) {
        double g = fmax(0.0, fmax(box[k] - c[k], c[k] - box[3 + k]));
        s += g * g;
    }
    return s;
}

__device__ __forceinline__ double gap2_box_box(const double lo[3], const double hi[3],
                                               const double *box)
{
    double s = 0;
    for (int k = 0; k < 3; ++k) {
        double g = fmax(0.0, fmax(box[k] - hi[k], lo[k] - box[3 + k]));
        s += g * g;
    }
    return s;
}

__device__ __forceinline__ void atom_pos(const float4 *rec, int stride_f4, int i, double y[3])
{
    const float4 a = rec[(size_t)i * stride_f4];
    const float4 b = rec[(size_t)i * stride_f4 + 1];
    y[0] = (double)a.x + b.x;
    y[1] = (double)a.y + b.y;
    y[2] = (double)a.z + b.z;
}


// Levels of the target octree of a grid with batch edge B.
inline int cp_levels(const GridParams &g, int B, double theta, CpLevels &L)
{
    L = CpLevels{};
    L.B = B;
    L.nx = g.nx;
    L.ny = g.ny;
    L.nz = g.nz;
    for (int k = 0; k < 3; ++k) L.h[k] = g.h[k];
    L.theta = theta;
    const int maxdim = g.nx > g.ny ? (g.nx > g.nz ? g.nx : g.nz) : (g.ny > g.nz ? g.ny : g.nz);
    L.T = 0;
    while ((B << L.T) < maxdim) ++L.T;
    if (L.T > kCpMaxLev) return RISM_E_UNSUPPORTED;
    for (int l = 0; l <= L.T; ++l) {
        const int e = B << l;
        L.cx[l] = (L.nx + e - 1) / e;
        L.cy[l] = (L.ny + e - 1) / e;
        L.cz[l] = (L.nz + e - 1) / e;
    }
    L.off[1] = 0;
    for (int l = 1; l <= L.T; ++l) L.off[l + 1] = L.off[l] + L.cx[l] * L.cy[l] * L.cz[l];
    return RISM_OK;
}

}  // namespace rism
