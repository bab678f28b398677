// FP32 pair arithmetic shared by the direct kernel and the treecode near field.
#pragma once

#include "rism_internal.h"

namespace rism {

struct PairConst {
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
    c.yk = (float)a.yk;
    c.inv_eta = (float)a.inv_eta;
    c.aa = (float)a.a;
    c.rs2 = (float)a.rs2;
    c.dcf0 = (float)a.dcf0;
    c.tcf0 = (float)a.tcf0;
    return c;
}

// Partial sums of one grid point over a block of sources.
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

// One (point, atom) pair.  FULL: Coulomb and Yukawa for every pair plus the
// short-range terms; otherwise only the short-range terms (LJ within the
// cut-off, smeared-kernel corrections within R_s) of an atom whose far field
// is accounted for elsewhere.
//   c correction: -Q erfc(d/eta)/d                          (d < R_s)
//   h correction: -Q [e^{-kd} erfc(d/eta - a) + e^{kd} erfc(d/eta + a)]/d
// so that 1/d + c-corr = erf(d/eta)/d and 2 e^{-kd}/d + h-corr = the Eq. 6
// bracket over d, exactly for d < R_s and to < 1e-12 beyond.
template <int NS, int LJM, bool ASYM, bool EXACT, bool FULL>
__device__ __forceinline__ void pair_eval(const AtomF32<NS> &at, const GridPt &g,
                                          const PairConst &k, PairAcc<NS> &p, bool &hit)
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
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    // raw v_rsq_f32 (d2 is never denormal unless a point sits within 1e-19 A
    // of an atom); a coincident point gets 1/d = 0 and is handled through
    // `hit` and the d -> 0 limits
    const float ri = d2 > 0.f ? __builtin_amdgcn_rsqf(d2) : 0.f;
    if (FULL) hit |= (d2 == 0.f);
    if (LJM != LJ_NONE) {
        const float r2 = ri * ri;
        const float r6 = r2 * r2 * r2;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            float r6s = r6;
            if (LJM == LJ_CUT) r6s = d2 < at.rc2[s] ? r6 : 0.f;
            p.L[s] = fmaf(fmaf(at.A[s], r6s, -at.B[s]), r6s, p.L[s]);
        }
    }
    const float aq = at.q;
    const float qr = aq * ri;
    if (FULL) p.C += qr;
    if (ASYM) {
        const float d = d2 * ri;
        const float e = __builtin_amdgcn_exp2f(k.yk * d);
        if (FULL) p.Y = fmaf(qr, e, p.Y);
        if (d2 < k.rs2) {
            const float x = d * k.inv_eta;
            p.SC = fmaf(-qr, erfcf(x), p.SC);
            const float ep = __builtin_amdgcn_rcpf(e);
            const float br = fmaf(e, erfcf(x - k.aa), ep * erfcf(x + k.aa));
            p.SH = fmaf(-qr, br, p.SH);
            if (FULL && d2 == 0.f) {
                p.SC = fmaf(aq, k.dcf0, p.SC);
                p.SH = fmaf(aq, k.tcf0, p.SH);
            }
        }
    }
}

__device__ __forceinline__ void store_val(void *base, int f64, int64_t idx, double v)
{
    if (f64)
        static_cast<double *>(base)[idx] = v;
    else
        static_cast<float *>(base)[idx] = static_cast<float>(v);
}

// Writes every requested output of one grid point from its running sums.
template <int NS, int LJM, bool ASYM>
__device__ __forceinline__ void store_point(const OutParams &o, const GridParams &g, int64_t p,
                                            const PointAcc<NS> &acc)
{
    if (o.want_u) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s < o.ns) {
                double lj = LJM != LJ_NONE ? (double)acc.ls[s] + (double)acc.lc[s] : 0.0;
                store_val(o.u, o.f64, s * g.m + p, acc.hit ? INFINITY : o.u_coul[s] * acc.C + lj);
            }
        }
    }
    if (ASYM) {
        if (o.want_c)
            for (int s = 0; s < o.ns; ++s)
                store_val(o.c, o.f64, s * g.m + p, o.c_scale[s] * (acc.C + acc.SC));
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
