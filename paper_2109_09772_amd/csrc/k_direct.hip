// Direct-sum kernels: atom staging, LJ tail constants, the FP64 reference
// direct sum, the FP32 compensated direct sum, and the error report.
//
// Thread mapping of the direct sums: one thread per grid point, a 256-thread
// workgroup covers a 16 x 4 x 4 brick (a wave is a 16 x 4 slab, so its rows
// write 64 contiguous bytes and its points stay within 8 A x 2 A, which keeps
// the divergent short-range branch rare).  Every thread walks the whole atom
// array; atom records are wave-uniform and arrive through scalar loads.
#include <algorithm>
#include <cmath>

#include "pair.h"

namespace rism {

// ------------------------------------------------------------------ helpers

struct BrickIndex {
    int i, j, k;
    bool valid;
};

__device__ __forceinline__ BrickIndex brick_index(const GridParams &g)
{
    const int bx = (g.nx + 15) / 16, by = (g.ny + 3) / 4;
    int b = blockIdx.x;
    int bi = b % bx;
    b /= bx;
    int bj = b % by;
    int bk = b / by;
    int t = threadIdx.x;
    BrickIndex r;
    r.i = bi * 16 + (t & 15);
    r.j = bj * 4 + ((t >> 4) & 3);
    r.k = bk * 4 + (t >> 6);
    r.valid = r.i < g.nx && r.j < g.ny && r.k < g.nz;
    return r;
}

inline int brick_blocks(const GridParams &g)
{
    return ((g.nx + 15) / 16) * ((g.ny + 3) / 4) * ((g.nz + 3) / 4);
}

// ------------------------------------------------------ smeared-kernel table

// erf(d/eta)/d and [e^{-kappa d} erfc(a - d/eta) - e^{kappa d} erfc(a + d/eta)]/d
// (a = kappa eta / 2) in FP64, with their d -> 0 limits.
__device__ inline void smear_f64(const AsymParams &A, double d, double &fc, double &fh)
{
    if (d == 0.0) {
        fc = A.dcf0;
        fh = A.tcf0;
        return;
    }
    const double x = d * A.inv_eta;
    fc = erf(x) / d;
    const double t2 = A.a + x < 27.0 ? exp(A.kappa * d) * erfc(A.a + x) : 0.0;
    fh = (exp(-A.kappa * d) * erfc(A.a - x) - t2) / d;
}

// Four threads per interval, one per Chebyshev node of the interval (the
// kernel values are the costly part); the interval's first thread forms the
// cubic through the four values (Newton form, expanded to monomials in the
// local variable t).
__device__ __forceinline__ void smear_table_block(const AsymParams &A, float4 *tab, int blk)
{
    const int g = blk * kBlock + threadIdx.x;
    const int i = g >> 2, node = g & 3, lane = threadIdx.x & 63, lead = lane & ~3;
    const double h = 1.0 / A.tab_inv_h;
    double t[4];
    for (int j = 0; j < 4; ++j) t[j] = 0.5 * (1.0 - cos((2 * j + 1) * kPi / 8.0));
    double fc = 0.0, fh = 0.0;
    if (i < kSmearIntervals) smear_f64(A, (i + t[node]) * h, fc, fh);
    double vc[4], vh[4];
    for (int j = 0; j < 4; ++j) {
        vc[j] = __shfl(fc, lead + j);
        vh[j] = __shfl(fh, lead + j);
    }
    if (i >= kSmearIntervals || node != 0) return;
    double *v[2] = {vc, vh};
    for (int f = 0; f < 2; ++f) {
        double d0 = v[f][0], d1 = v[f][1], d2 = v[f][2], d3 = v[f][3];
        // divided differences
        const double a1 = (d1 - d0) / (t[1] - t[0]);
        const double b1 = (d2 - d1) / (t[2] - t[1]);
        const double c1 = (d3 - d2) / (t[3] - t[2]);
        const double a2 = (b1 - a1) / (t[2] - t[0]);
        const double b2 = (c1 - b1) / (t[3] - t[1]);
        const double a3 = (b2 - a2) / (t[3] - t[0]);
        const double s3 = t[0] + t[1] + t[2];
        const double p2 = t[0] * t[1] + t[0] * t[2] + t[1] * t[2];
        float4 c;
        c.w = (float)a3;
        c.z = (float)(a2 - a3 * s3);
        c.y = (float)(a1 - a2 * (t[0] + t[1]) + a3 * p2);
        c.x = (float)(d0 - a1 * t[0] + a2 * t[0] * t[1] - a3 * t[0] * t[1] * t[2]);
        tab[2 * i + f] = c;
    }
}

// ------------------------------------------------------------------ staging

// Lorentz-Berthelot mixing and the A, B, r_cut of every (site, atom) pair,
// plus the FP32 hi/lo split of the atom coordinates relative to the grid
// origin.  Padding atoms (a >= n) carry no charge and no LJ and sit far away.
// With a.smear_tab, kSmearBlocks more workgroups form the smeared-kernel
// table in the same launch.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_stage(SiteParams sp, StageArgs a)
{
    const int nstage = (int)((a.npad + kBlock - 1) / kBlock);
    if ((int)blockIdx.x >= nstage) {   // whole workgroup
        smear_table_block(a.smear, a.smear_tab, blockIdx.x - nstage);
        return;
    }
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool live = i < a.npad;   // every lane stays for the wave-wide maximum below
    double x = kFarAway, y = kFarAway, z = kFarAway, q = 0.0, sig = 0.0, eps = 0.0;
    bool real = i < a.n;
    int r2max = 0;   // largest (1 + 1e-6) rc^2 of the atom's sites, as float bits
    bool f_bad = false, f_tol = false;   // this atom's input-check flags
    if (real) {
        x = a.xyz[3 * i] - a.origin[0];
        y = a.xyz[3 * i + 1] - a.origin[1];
        z = a.xyz[3 * i + 2] - a.origin[2];
        q = a.q[i];
        sig = a.sig[i];
        eps = a.eps[i];
        bool bad = !(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(q) &&
                     isfinite(sig) && isfinite(eps)) || sig < 0.0 || eps < 0.0;
        f_bad = bad;
        f_tol = a.check_eps && !(eps > 0.0);
    }
    double A[NS], B[NS], rc[NS];
#pragma unroll
    for (int g = 0; g < NS; ++g) {
        A[g] = 0.0;
        B[g] = 0.0;
        rc[g] = INFINITY;
        if (real && g < sp.ns) {
            double s_ga = 0.5 * (sp.sig[g] + sig);
            double e_ga = sqrt(sp.eps[g] * eps);
            double s2 = s_ga * s_ga, s6 = s2 * s2 * s2;
            A[g] = 4.0 * e_ga * s6 * s6;
            B[g] = 4.0 * e_ga * s6;
            if (a.lj_mode == LJ_CUT) {
                if (a.lj_tol > 0.0 && e_ga == 0.0) {
                    // eps_ga = 0: the pair has no LJ term (A = B = 0), which
                    // is below any tolerance at every distance; radius 0
                    // drops it and adds nothing to the tail
                    rc[g] = 0.0;
                } else if (a.lj_tol > 0.0) {
                    // |u(r)| = tol beyond the minimum: with t = (s_ga/r)^6,
                    // 4 e (t^2 - t) = -tol, smaller root, written without
                    // cancellation: t = (z/2) / (1 + sqrt(1 - z)), z = tol/e.
                    double zz = a.lj_tol / e_ga;
                    if (!(zz < 1.0)) {
                        f_tol = true;
                        rc[g] = 0.0;
                    } else {
                        double t = 0.5 * zz / (1.0 + sqrt(1.0 - zz));
                        rc[g] = s_ga * pow(t, -1.0 / 6.0);
                    }
                } else {
                    rc[g] = a.lj_cutoff;
                }
            }
            if (a.rcut) a.rcut[(int64_t)g * a.n + i] = rc[g];
            if (a.lj_mode == LJ_CUT && rc[g] > 0.0) {
                // positive floats order like their bit patterns
                float r2f = (float)(rc[g] * rc[g]) * (1.0f + 1e-6f);
                r2max = max(r2max, __float_as_int(r2f));
            }
        }
    }
    // the workgroup's flags and largest cut-off radius, and with bbox_part its
    // box of the positions the FP32 records carry, as the tree forms them
    // ((double)hi + lo): wave reductions, then the waves' values through LDS
    {
        __shared__ int wflag[3][kBlock / 64];
        __shared__ double wbox[6][kBlock / 64];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int off = 32; off > 0; off >>= 1) r2max = max(r2max, __shfl_xor(r2max, off));
        const bool any_bad = __ballot(f_bad) != 0, any_tol = __ballot(f_tol) != 0;
        if (lane == 0) {
            wflag[0][wave] = any_bad ? 1 : 0;
            wflag[1][wave] = any_tol ? 1 : 0;
            wflag[2][wave] = r2max;
        }
        if (a.bbox_part) {
            double bl[3], bh[3];
            const double v[3] = {(double)(float)x + (double)(float)(x - (double)(float)x),
                                 (double)(float)y + (double)(float)(y - (double)(float)y),
                                 (double)(float)z + (double)(float)(z - (double)(float)z)};
            for (int k = 0; k < 3; ++k) {
                bl[k] = real ? v[k] : 1e300;
                bh[k] = real ? v[k] : -1e300;
            }
            for (int off = 32; off > 0; off >>= 1)
                for (int k = 0; k < 3; ++k) {
                    bl[k] = fmin(bl[k], __shfl_xor(bl[k], off));
                    bh[k] = fmax(bh[k], __shfl_xor(bh[k], off));
                }
            if (lane == 0)
                for (int k = 0; k < 3; ++k) {
                    wbox[k][wave] = bl[k];
                    wbox[3 + k][wave] = bh[k];
                }
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            const int k = threadIdx.x;
            int r = wflag[k][0];
            for (int w = 1; w < kBlock / 64; ++w) r = k < 2 ? (r | wflag[k][w]) : max(r, wflag[k][w]);
            a.err_part[3 * blockIdx.x + k] = r;
        }
        if (a.bbox_part && threadIdx.x >= 64 && threadIdx.x < 70) {
            const int k = threadIdx.x - 64;
            double r = wbox[k][0];
            for (int w = 1; w < kBlock / 64; ++w)
                r = k < 3 ? fmin(r, wbox[k][w]) : fmax(r, wbox[k][w]);
            a.bbox_part[6 * blockIdx.x + k] = r;
        }
    }
    if (!live) return;
    if (a.rec64) {
        AtomF64<NS> r;
        r.x = x; r.y = y; r.z = z; r.q = q;
#pragma unroll
        for (int g = 0; g < NS; ++g) { r.A[g] = A[g]; r.B[g] = B[g]; r.rc2[g] = rc[g] * rc[g]; }
        static_cast<AtomF64<NS> *>(a.rec64)[i] = r;
    }
    if (a.rec32) {
        AtomF32<NS> r;
        r.xh = (float)x; r.xl = (float)(x - (double)r.xh);
        r.yh = (float)y; r.yl = (float)(y - (double)r.yh);
        r.zh = (float)z; r.zl = (float)(z - (double)r.zh);
        r.q = (float)q;
        r.on_grid = real && on_grid_point(r, a.grid) ? 1.f : 0.f;
#pragma unroll
        for (int g = 0; g < NS; ++g) {
            r.A[g] = (float)A[g];
            r.B[g] = (float)B[g];
            r.rc2[g] = (float)(rc[g] * rc[g]);
        }
        static_cast<AtomF32<NS> *>(a.rec32)[i] = r;
    }
}

// The staging workgroups' flag words [3 * nparts] into flags[0..2]: any
// non-finite input, any tolerance / eps failure, the largest squared cut-off
// radius (float bits).  One workgroup.
__global__ __launch_bounds__(kBlock) void k_stage_flags(const int *part, int nparts, int *flags)
{
    __shared__ int w[3][kBlock / 64];
    int f0 = 0, f1 = 0, f2 = 0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) {
        f0 |= part[3 * i];
        f1 |= part[3 * i + 1];
        f2 = max(f2, part[3 * i + 2]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        f0 |= __shfl_xor(f0, off);
        f1 |= __shfl_xor(f1, off);
        f2 = max(f2, __shfl_xor(f2, off));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        w[0][wave] = f0;
        w[1][wave] = f1;
        w[2][wave] = f2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        int r = w[k][0];
        for (int v = 1; v < kBlock / 64; ++v) r = k < 2 ? (r | w[k][v]) : max(r, w[k][v]);
        flags[k] = r;
    }
}

int launch_stage_flags(const int *part, int nparts, int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_stage_flags, 1, kBlock, 0, s, part, nparts, flags);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

int launch_stage(const SiteParams &sp, const StageArgs &a, hipStream_t s)
{
    int blocks = (int)((a.npad + kBlock - 1) / kBlock);
    if (a.smear_tab) blocks += kSmearBlocks;
    if (blocks == 0) return RISM_OK;
    switch (sp.ns_pad) {
    case 1: hipLaunchKernelGGL(k_stage<1>, blocks, kBlock, 0, s, sp, a); break;
    case 2: hipLaunchKernelGGL(k_stage<2>, blocks, kBlock, 0, s, sp, a); break;
    case 4: hipLaunchKernelGGL(k_stage<4>, blocks, kBlock, 0, s, sp, a); break;
    default: hipLaunchKernelGGL(k_stage<8>, blocks, kBlock, 0, s, sp, a); break;
    }
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

// T_g = (4 pi / 3) sum_a (A/(3 rc^9) - B/rc^3), one workgroup per site,
// fixed-order reduction (bitwise reproducible).
__global__ __launch_bounds__(kBlock) void k_lj_tail(SiteParams sp, const double *rcut,
                                                    const double *sig, const double *eps,
                                                    int64_t n, double *tail)
{
    __shared__ double red[kBlock];
    int g = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        double s_ga = 0.5 * (sp.sig[g] + sig[i]);
        double e_ga = sqrt(sp.eps[g] * eps[i]);
        double s2 = s_ga * s_ga, s6 = s2 * s2 * s2;
        double A = 4.0 * e_ga * s6 * s6, B = 4.0 * e_ga * s6;
        double rc = rcut[(int64_t)g * n + i];
        double rc3 = rc * rc * rc;
        // rc = 0 marks a pair without LJ term (eps_ga = 0 under a tolerance)
        if (rc > 0.0) acc += A / (3.0 * rc3 * rc3 * rc3) - B / rc3;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) tail[g] = 4.0 * kPi / 3.0 * red[0];
}

int launch_lj_tail(const SiteParams &sp, const double *rcut, const double *sig, const double *eps,
                   int64_t n, double *tail_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_lj_tail, sp.ns, kBlock, 0, s, sp, rcut, sig, eps, n, tail_dev);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

// ---------------------------------------------------------- FP64 direct sum

// The definitions term by term in FP64: Coulomb, LJ (all pairs or truncated),
// erf(d/eta)/d and the Eq. 6 bracket over d, each pair evaluated in full.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_direct_f64(SiteParams sp, DirectArgs a)
{
    const GridParams &g = a.g;
    BrickIndex bi = brick_index(g);
    int i = bi.valid ? bi.i : 0, j = bi.valid ? bi.j : 0, k = bi.valid ? bi.k : 0;
    const double gx = i * g.h[0], gy = j * g.h[1], gz = k * g.h[2];
    const AtomF64<NS> *__restrict__ atoms = static_cast<const AtomF64<NS> *>(a.atoms);
    const bool want_u = a.out.want_u, want_c = a.out.want_c && a.asym_on,
               want_h = a.out.want_h && a.asym_on;
    const int ljm = a.lj_mode;
    const double inv_eta = a.asym.inv_eta, kap = a.asym.kappa, aa = a.asym.a;
    double coul = 0.0, sc = 0.0, sh = 0.0;
    double lj[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) lj[s] = 0.0;
    bool hit = false;
    for (int64_t n = 0; n < a.n; ++n) {
        const AtomF64<NS> at = atoms[n];
        double dx = gx - at.x, dy = gy - at.y, dz = gz - at.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 == 0.0) {
            hit = true;
            sc += at.q * a.asym.dcf0;
            sh += at.q * a.asym.tcf0;
            continue;
        }
        double d = sqrt(d2);
        double ri = 1.0 / d;
        if (want_u) {
            coul += at.q * ri;
            if (ljm != LJ_NONE) {
                double r2 = ri * ri, r6 = r2 * r2 * r2;
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (ljm == LJ_ALL || d2 < at.rc2[s]) lj[s] += (at.A[s] * r6 - at.B[s]) * r6;
            }
        }
        if (want_c) sc += at.q * erf(d * inv_eta) * ri;
        if (want_h) {
            double x = d * inv_eta;
            // erfc(aa + x) is exactly 0 in FP64 beyond 26.6; skipping the
            // product there avoids inf * 0 when exp(kappa d) overflows
            double t2 = aa + x < 27.0 ? exp(kap * d) * erfc(aa + x) : 0.0;
            sh += at.q * (exp(-kap * d) * erfc(aa - x) - t2) * ri;
        }
    }
    if (!bi.valid) return;
    const int64_t p = ((int64_t)k * g.ny + j) * g.nx + i;
    const OutParams &o = a.out;
    if (want_u)
        for (int s = 0; s < o.ns; ++s)
            store_val(o.u, o.f64, s * g.m + p, hit ? INFINITY : o.u_coul[s] * coul + lj[s]);
    if (want_c)
        for (int s = 0; s < o.ns; ++s) store_val(o.c, o.f64, s * g.m + p, o.c_scale[s] * sc);
    if (want_h)
        for (int s = 0; s < o.n_ionic; ++s) store_val(o.h, o.f64, s * g.m + p, o.h_scale[s] * sh);
}

int launch_direct_f64(const SiteParams &sp, const DirectArgs &a, hipStream_t s)
{
    int blocks = brick_blocks(a.g);
    switch (sp.ns_pad) {
    case 1: hipLaunchKernelGGL(k_direct_f64<1>, blocks, kBlock, 0, s, sp, a); break;
    case 2: hipLaunchKernelGGL(k_direct_f64<2>, blocks, kBlock, 0, s, sp, a); break;
    case 4: hipLaunchKernelGGL(k_direct_f64<4>, blocks, kBlock, 0, s, sp, a); break;
    default: hipLaunchKernelGGL(k_direct_f64<8>, blocks, kBlock, 0, s, sp, a); break;
    }
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}


// ------------------------------------------------- FP32 compensated direct sum

// Per pair, in FP32: d from hi/lo coordinates, 1/d by rsqrt, Coulomb Q/d,
// LJ (A r^-6 - B) r^-6 per site; beyond R_s the smeared kernels are 1/d and
// 2 e^{-kappa d}/d (exp2) to < 1e-12, within R_s they come from the cubic
// table in LDS.  Partial sums over 8 atoms are flushed into FP64
// (electrostatic sums, which cancel in sign) or into TwoSum-compensated FP32
// (LJ).
template <int NS, int LJM, bool ASYM, bool EXACT>
__global__ __launch_bounds__(kBlock) void k_direct_f32(SiteParams sp, DirectArgs a)
{
    const GridParams &g = a.g;
    BrickIndex bi = brick_index(g);
    const GridPt gp = grid_pt(g, bi.valid ? bi.i : 0, bi.valid ? bi.j : 0, bi.valid ? bi.k : 0);
    ConstAS<AtomF32<NS>> *atoms = as_const(static_cast<const AtomF32<NS> *>(a.atoms));
    const PairConst kc = make_pair_const(a.asym);
    __shared__ float4 tab[ASYM ? 2 * kSmearIntervals : 1];
    if (ASYM) load_smear_table(tab, a.asym.tab, kBlock);
    PointAcc<NS> acc;
    acc.zero();
    for (int64_t n0 = 0; n0 < a.npad; n0 += kAtomPad) {
        PairAcc<NS> p;
        p.zero();
#pragma unroll 2
        for (int t = 0; t < kAtomPad; ++t)
            pair_eval<NS, LJM, ASYM, EXACT, true>(atoms[n0 + t], gp, kc, tab, p, acc.hit);
        acc.template flush<LJM != LJ_NONE, ASYM>(p);
    }
    if (!bi.valid) return;
    const int64_t p = ((int64_t)bi.k * g.ny + bi.j) * g.nx + bi.i;
    store_point<NS, LJM, ASYM>(a.out, g, p, acc);
}

template <int NS, int LJM, bool ASYM>
static void launch_f32_exact(bool exact, int blocks, const SiteParams &sp, const DirectArgs &a,
                             hipStream_t s)
{
    if (exact)
        hipLaunchKernelGGL((k_direct_f32<NS, LJM, ASYM, true>), blocks, kBlock, 0, s, sp, a);
    else
        hipLaunchKernelGGL((k_direct_f32<NS, LJM, ASYM, false>), blocks, kBlock, 0, s, sp, a);
}

template <int NS>
static void launch_f32_ns(int blocks, const SiteParams &sp, const DirectArgs &a, hipStream_t s)
{
    bool ex = a.g.exact != 0;
    if (a.asym_on) {
        if (a.lj_mode == LJ_NONE) launch_f32_exact<NS, LJ_NONE, true>(ex, blocks, sp, a, s);
        else if (a.lj_mode == LJ_ALL) launch_f32_exact<NS, LJ_ALL, true>(ex, blocks, sp, a, s);
        else if (a.lj_uniform) launch_f32_exact<NS, LJ_CUT1, true>(ex, blocks, sp, a, s);
        else launch_f32_exact<NS, LJ_CUT, true>(ex, blocks, sp, a, s);
    } else {
        if (a.lj_mode == LJ_NONE) launch_f32_exact<NS, LJ_NONE, false>(ex, blocks, sp, a, s);
        else if (a.lj_mode == LJ_ALL) launch_f32_exact<NS, LJ_ALL, false>(ex, blocks, sp, a, s);
        else if (a.lj_uniform) launch_f32_exact<NS, LJ_CUT1, false>(ex, blocks, sp, a, s);
        else launch_f32_exact<NS, LJ_CUT, false>(ex, blocks, sp, a, s);
    }
}

int launch_direct_f32(const SiteParams &sp, const DirectArgs &a, hipStream_t s)
{
    int blocks = brick_blocks(a.g);
    switch (sp.ns_pad) {
    case 1: launch_f32_ns<1>(blocks, sp, a, s); break;
    case 2: launch_f32_ns<2>(blocks, sp, a, s); break;
    case 4: launch_f32_ns<4>(blocks, sp, a, s); break;
    default: launch_f32_ns<8>(blocks, sp, a, s); break;
    }
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

// ------------------------------------------------------------- error report

// Partial sums per workgroup (fixed order within the group); the host adds
// the per-group partials in group order.  Points whose mask byte is 0 are
// left out entirely (mask may be null: every point).
__global__ __launch_bounds__(kBlock) void k_compare(const void *x, int f64, const double *ref,
                                                    const uint8_t *mask, int64_t n, double cap,
                                                    double *part)
{
    __shared__ double r0[kBlock], r1[kBlock], r2[kBlock], r3[kBlock], r4[kBlock], r5[kBlock];
    double se = 0.0, sr = 0.0, mx = 0.0, ex = 0.0, mism = 0.0, cnt = 0.0;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += stride) {
        if (mask && mask[i] == 0) continue;
        double v = f64 ? static_cast<const double *>(x)[i] : (double)static_cast<const float *>(x)[i];
        double r = ref[i];
        bool vr = isfinite(v) && (cap <= 0.0 || fabs(v) <= cap);
        bool rr = isfinite(r) && (cap <= 0.0 || fabs(r) <= cap);
        if (vr && rr) {
            double d = v - r;
            se += d * d;
            sr += r * r;
            mx = fmax(mx, fabs(d));
            cnt += 1.0;
        } else {
            ex += 1.0;
            if (vr != rr) mism += 1.0;
        }
    }
    int t = threadIdx.x;
    r0[t] = se; r1[t] = sr; r2[t] = mx; r3[t] = ex; r4[t] = mism; r5[t] = cnt;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
            r0[t] += r0[t + w];
            r1[t] += r1[t + w];
            r2[t] = fmax(r2[t], r2[t + w]);
            r3[t] += r3[t + w];
            r4[t] += r4[t + w];
            r5[t] += r5[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[6 * blockIdx.x + 0] = r0[0];
        part[6 * blockIdx.x + 1] = r1[0];
        part[6 * blockIdx.x + 2] = r2[0];
        part[6 * blockIdx.x + 3] = r3[0];
        part[6 * blockIdx.x + 4] = r4[0];
        part[6 * blockIdx.x + 5] = r5[0];
    }
}

int launch_compare(const void *x, int f64, const double *ref, const uint8_t *mask, int64_t n,
                   double cap, double *partials, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_compare, nblocks, kBlock, 0, s, x, f64, ref, mask, n, cap, partials);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

// ------------------------------------------------------------ near-atom mask

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One wave per atom: the grid points of the box around the atom that lie
// closer than `radius` (FP64, absolute coordinates) get mask 0.  Several
// atoms may clear one point; they all write 0.
__global__ __launch_bounds__(64) void k_near_mask(const double *xyz, int64_t n, GridParams g,
                                                  double radius, uint8_t *mask)
{
    const int64_t a = blockIdx.x;
    if (a >= n) return;
    const double y[3] = {xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2]};
    const int nd[3] = {g.nx, g.ny, g.nz};
    int lo[3], cnt[3];
    for (int k = 0; k < 3; ++k) {
        // candidate indices, one spacing of slack on each side
        double l = floor((y[k] - radius - g.o[k]) / g.h[k]) - 1.0;
        double h = ceil((y[k] + radius - g.o[k]) / g.h[k]) + 1.0;
        l = fmax(l, 0.0);
        h = fmin(h, (double)(nd[k] - 1));
        lo[k] = (int)l;
        cnt[k] = h >= l ? (int)(h - l) + 1 : 0;
    }
    const int64_t tot = (int64_t)cnt[0] * cnt[1] * cnt[2];
    for (int64_t t = threadIdx.x; t < tot; t += 64) {
        const int i = lo[0] + (int)(t % cnt[0]);
        const int j = lo[1] + (int)((t / cnt[0]) % cnt[1]);
        const int k = lo[2] + (int)(t / ((int64_t)cnt[0] * cnt[1]));
        const double dx = g.o[0] + i * g.h[0] - y[0];
        const double dy = g.o[1] + j * g.h[1] - y[1];
        const double dz = g.o[2] + k * g.h[2] - y[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (sqrt(d2) < radius) mask[((int64_t)k * g.ny + j) * g.nx + i] = 0;
    }
}

int launch_near_mask(const double *xyz, int64_t n, const GridParams &g, double radius,
                     uint8_t *mask, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((g.m + kBlock - 1) / kBlock, 16384);
    hipLaunchKernelGGL(k_fill_u8, (int)std::max<int64_t>(blocks, 1), kBlock, 0, s, mask, g.m,
                       (uint8_t)1);
    if (n > 0 && radius > 0.0)
        hipLaunchKernelGGL(k_near_mask, (unsigned)n, 64, 0, s, xyz, n, g, radius, mask);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

}  // namespace rism
