// FP32 pair arithmetic shared by the direct kernel and the treecode near field.
#pragma once

#include "rism_internal.h"

namespace rism {

struct PairConst {
    float tinv;     // table intervals per angstrom
    float yk;       // -kappa log2(e)
    float inv_eta;  // 1/eta
    float aa;       // kappa eta / 2
    float rs2;      // R_s^2: radius of the smeared-kernel corrections
    float dcf0;     // erf(d/eta)/d at d = 0
    float tcf0;     // Eq. 6 bracket over d at d = 0
};

__host__ __device__ inline PairConst make_pair_const(const AsymParams &a)
{
    PairConst c;
    c.tinv = (float)a.tab_inv_h;
    c.yk = (float)a.yk;
    c.inv_eta = (float)a.inv_eta;
    c.aa = (float)a.a;
    c.rs2 = (float)a.rs2;
    c.dcf0 = (float)a.dcf0;
    c.tcf0 = (float)a.tcf0;
    return c;
}

// Read-only data in the constant address space: uniform loads through such a
// pointer are always served by the scalar data cache (s_load), also after
// stores or atomics earlier in the kernel that would otherwise make the
// compiler fall back to per-lane vector loads.
template <class T>
using ConstAS = const __attribute__((address_space(4))) T;

template <class T>
__device__ __forceinline__ ConstAS<T> *as_const(const T *p)
{
    return (ConstAS<T> *)p;
}

// Partial sums of one grid point over a block of sources.
// C: Coulomb 1/d of the directly summed atoms, Y: their e^{-kappa d}/d, SC /
// SH: within R_s, the smeared kernels' differences erf(d/eta)/d - 1/d and
// bracket/d - 2 e^{-kappa d}/d (of every atom within R_s, whether its far
// form reaches the point directly or through the clusters).
template <int NS>
struct PairAcc {
    float C, Y, SC, SH;
    float L[NS];
    __device__ __forceinline__ void zero()
    {
        C = Y = SC = SH = 0.f;
#pragma unroll
        for (int s = 0; s < NS; ++s) L[s] = 0.f;
    }
};

// Running sums of one grid point: electrostatic sums in FP64 (they cancel in
// sign across sources), LJ sums as TwoSum-compensated FP32 pairs.
template <int NS>
struct PointAcc {
    double C, Y, SC, SH;
    float ls[NS], lc[NS];
    bool hit;
    __device__ __forceinline__ void zero()
    {
        C = Y = SC = SH = 0.0;
        hit = false;
#pragma unroll
        for (int s = 0; s < NS; ++s) { ls[s] = 0.f; lc[s] = 0.f; }
    }
    template <bool LJ, bool ASYM>
    __device__ __forceinline__ void flush(const PairAcc<NS> &p)
    {
        C += (double)p.C;
        if (ASYM) {
            Y += (double)p.Y;
            SC += (double)p.SC;
            SH += (double)p.SH;
        }
        if (LJ) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                // Knuth's TwoSum
                float t = ls[s] + p.L[s];
                float z = t - ls[s];
                lc[s] += (ls[s] - (t - z)) + (p.L[s] - z);
                ls[s] = t;
            }
        }
    }
};

// Grid point in FP32 hi/lo form, relative to the grid origin.
struct GridPt {
    float xh, yh, zh, xl, yl, zl;
};

__device__ __forceinline__ GridPt grid_pt(const GridParams &g, int i, int j, int k)
{
    GridPt p;
    double x = i * g.h[0], y = j * g.h[1], z = k * g.h[2];
    p.xh = (float)x; p.xl = (float)(x - (double)p.xh);
    p.yh = (float)y; p.yl = (float)(y - (double)p.yh);
    p.zh = (float)z; p.zl = (float)(z - (double)p.zh);
    return p;
}

// Cubic interpolation of both smeared kernels at distance d < R_s.
__device__ __forceinline__ void smear_eval(const float4 *tab, float tinv, float d, float &gc,
                                           float &gh)
{
    const float u = d * tinv;
    int i = (int)u;
    i = i < kSmearIntervals - 1 ? i : kSmearIntervals - 1;
    const float t = u - (float)i;
    const float4 c = tab[2 * i], h = tab[2 * i + 1];
    gc = fmaf(fmaf(fmaf(c.w, t, c.z), t, c.y), t, c.x);
    gh = fmaf(fmaf(fmaf(h.w, t, h.z), t, h.y), t, h.x);
}

// Squared FP32 distance of a pair from the hi/lo coordinates.  EXACT: the
// point's coordinates are exact in FP32 (no lo words).  Every kernel forms d2
// through this function, so a test of d2 == 0 made elsewhere (a coincident
// atom) agrees with the pair loops bit for bit.
template <bool EXACT, class Rec>
__device__ __forceinline__ float pair_d2(const Rec &at, const GridPt &g)
{
    float dx, dy, dz;
    if (EXACT) {
        dx = (g.xh - at.xh) - at.xl;
        dy = (g.yh - at.yh) - at.yl;
        dz = (g.zh - at.zh) - at.zl;
    } else {
        dx = (g.xh - at.xh) + (g.xl - at.xl);
        dy = (g.yh - at.yh) + (g.yl - at.yl);
        dz = (g.zh - at.zh) + (g.zl - at.zl);
    }
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Whether the atom sits on a grid point in the FP32 pair arithmetic: d2 == 0
// for that point, formed as the pair loops form it.  d2 underflows to zero
// only when every coordinate difference is below ~1e-22 A, so only the atom's
// nearest grid point can give it.
template <class Rec>
__device__ __forceinline__ bool on_grid_point(const Rec &at, const GridParams &g)
{
    const double u = rint(((double)at.xh + (double)at.xl) / g.h[0]);
    const double v = rint(((double)at.yh + (double)at.yl) / g.h[1]);
    const double w = rint(((double)at.zh + (double)at.zl) / g.h[2]);
    if (!(u >= 0.0 && u < g.nx && v >= 0.0 && v < g.ny && w >= 0.0 && w < g.nz)) return false;
    const GridPt p = grid_pt(g, (int)u, (int)v, (int)w);
    return (g.exact ? pair_d2<true>(at, p) : pair_d2<false>(at, p)) == 0.f;
}

// One (point, atom) pair.  FULL: every term of the atom: 1/d (into C),
// e^{-kappa d}/d (into Y) and, for d < R_s, the differences
// erf(d/eta)/d - 1/d and bracket/d - 2 e^{-kappa d}/d from the table (into SC,
// SH); beyond R_s those differences are < 1e-12 relative and dropped.  At a
// coincident point (d = 0) only the smeared kernels' limits enter.
// Not FULL (the atom's 1/d and e^{-kappa d}/d reach the point through
// proxies): only LJ within the cut-off and the differences within R_s.
// GUARD false (FULL pairs only): the caller has established that d2 > 0 for
// every pair of the call, so the coincidence handling is left out.
template <int NS, int LJM, bool ASYM, bool EXACT, bool FULL, bool GUARD = true, class Rec>
__device__ __forceinline__ void pair_eval(const Rec &at, const GridPt &g,
                                          const PairConst &k, const float4 *tab, PairAcc<NS> &p,
                                          bool &hit)
{
    constexpr bool G = GUARD || !FULL;
    const float d2 = pair_d2<EXACT>(at, g);
    // raw v_rsq_f32 of d2 clamped to 1e-30: a coincident point (d2 = 0, FULL
    // pairs only: a short-range atom is well separated from the point) gets a
    // large finite 1/d that reaches u alone (set to +inf through `hit`), and
    // d = d2/sqrt(d2) stays ~0, so the smeared kernels take their d = 0
    // values from the table
    const float ri = __builtin_amdgcn_rsqf(G ? fmaxf(d2, 1e-30f) : d2);
    if (FULL && G) hit |= (d2 == 0.f);
    if (LJM != LJ_NONE) {
        // 1/d^2 for the LJ powers: ri^2 carries twice the error of the
        // reciprocal square root, and r^-12 multiplies it by six again,
        // enough to reach ~1.3e-6 at grid points next to an atom (where one
        // pair dominates u).  One Newton step for the reciprocal of d2,
        // r2 += r2 (1 - d2 r2), brings it to about half an ulp whatever the
        // error of ri.
        float r2 = ri * ri;
        r2 = fmaf(r2, fmaf(-d2, r2, 1.0f), r2);
        float r6 = r2 * r2 * r2;
        if (LJM == LJ_CUT1) r6 = d2 < at.rc2[0] ? r6 : 0.f;
        // (A r^-6 - B) r^-6: the difference is formed before the product, so
        // near the zero crossing of the LJ term it carries no cancellation
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            float r6s = r6;
            if (LJM == LJ_CUT) r6s = d2 < at.rc2[s] ? r6 : 0.f;
            p.L[s] = fmaf(fmaf(at.A[s], r6s, -at.B[s]), r6s, p.L[s]);
        }
    }
    const float aq = at.q;
    const float qr = aq * ri;
    if (!ASYM) {
        if (FULL) p.C += qr;
        return;
    }
    const bool nearp = d2 < k.rs2;
    const float d = d2 * ri;
    const float e = __builtin_amdgcn_exp2f(k.yk * d);
    // a FULL atom adds 1/d and e^{-kappa d}/d at every distance (a coincident
    // point excepted: its terms are the d -> 0 limits of the smeared kernels
    // alone), and within R_s the smeared kernels' differences to those far
    // forms, as a short-range atom does
    const float qe = FULL && G && d2 == 0.f ? 0.f : qr;
    if (FULL) {
        p.C += qe;
        p.Y = fmaf(qe, e, p.Y);
    }
    if (nearp) {
        float gc, gh;
        smear_eval(tab, k.tinv, d, gc, gh);
        p.SC = fmaf(aq, gc, p.SC - qe);
        p.SH = fmaf(aq, gh, fmaf(-qe, e + e, p.SH));
    }
}

// Copies the smeared-kernel table into LDS (every thread of the block).
__device__ __forceinline__ void load_smear_table(float4 *dst, const float4 *src, int nthreads)
{
    for (int i = threadIdx.x; i < 2 * kSmearIntervals; i += nthreads) dst[i] = src[i];
    __syncthreads();
}

__device__ __forceinline__ void store_val(void *base, int f64, int64_t idx, double v)
{
    if (f64)
        static_cast<double *>(base)[idx] = v;
    else
        static_cast<float *>(base)[idx] = static_cast<float>(v);
}

// Writes every requested output of one grid point from its running sums.
// far_u / far_c: far-field sums kept apart from acc.C because u and c^lr
// take different far fields (the Taylor treecode's 1/d and erf(d/eta)/d
// expansions); zero elsewhere.
template <int NS, int LJM, bool ASYM>
__device__ __forceinline__ void store_point(const OutParams &o, const GridParams &g, int64_t p,
                                            const PointAcc<NS> &acc, double far_u = 0.0,
                                            double far_c = 0.0)
{
    if (o.want_u) {
        const double coul = acc.C + far_u;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s < o.ns) {
                double lj = LJM != LJ_NONE ? (double)acc.ls[s] + (double)acc.lc[s] : 0.0;
                store_val(o.u, o.f64, s * g.m + p, acc.hit ? INFINITY : o.u_coul[s] * coul + lj);
            }
        }
    }
    if (ASYM) {
        if (o.want_c)
            for (int s = 0; s < o.ns; ++s)
                store_val(o.c, o.f64, s * g.m + p, o.c_scale[s] * (acc.C + acc.SC + far_c));
        if (o.want_h)
            for (int s = 0; s < o.n_ionic; ++s)
                store_val(o.h, o.f64, s * g.m + p, o.h_scale[s] * (2.0 * acc.Y + acc.SH));
    }
}

template <int NS>
inline size_t rec32_size() { return sizeof(AtomF32<NS>); }

inline size_t rec32_bytes_of(int ns_pad)
{
    switch (ns_pad) {
    case 1: return sizeof(AtomF32<1>);
    case 2: return sizeof(AtomF32<2>);
    case 4: return sizeof(AtomF32<4>);
    default: return sizeof(AtomF32<8>);
    }
}

inline size_t rec64_bytes_of(int ns_pad)
{
    switch (ns_pad) {
    case 1: return sizeof(AtomF64<1>);
    case 2: return sizeof(AtomF64<2>);
    case 4: return sizeof(AtomF64<4>);
    default: return sizeof(AtomF64<8>);
    }
}

}  // namespace rism
