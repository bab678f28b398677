// Treecode evaluation: one workgroup per batch of B^3 grid points.
//
//  far   : proxies of accepted source clusters -> Coulomb 1/d and Yukawa
//          e^{-kappa d}/d.  Proxies are staged in LDS as float4 (position
//          relative to the batch's first point, computed in FP64, and the
//          FP32 proxy charge); every lane reads the same entry (broadcast).
//  near  : atoms of the leaves that were not accepted -> the full pair
//          (Coulomb, Yukawa, LJ within the cut-off, smeared kernels).
//  short : atoms of leaves inside accepted clusters that still come within
//          the short range of the batch -> LJ, and the smeared kernels less
//          1/d and 2 e^{-kappa d}/d within R_s.
// Partial sums over 16 proxies / 8 atoms are flushed into FP64 (electrostatic
// sums) and TwoSum FP32 (LJ), as in the direct kernel.
#include <cmath>

#include "pair.h"
#include "tree.h"

namespace rism {

namespace {

constexpr int kChunk = 1024;   // proxies staged per LDS round

template <int B>
struct EvalShape {
    static constexpr int threads = B == 4 ? 64 : 256;
    static constexpr int ppt = B == 4 ? 1 : 2;   // points per thread per pass
    static constexpr int passes = (B * B * B) / (threads * ppt);
};

__device__ __forceinline__ double cheb_pt(double lo, double hi, int k, int n)
{
    return lo + (hi - lo) * 0.5 * (1.0 + cos(kPi * k / n));
}

}  // namespace

template <int NS, int LJM, bool ASYM, int B>
__global__ __launch_bounds__(EvalShape<B>::threads) void k_tree_eval(SiteParams sp, TreeEvalArgs a)
{
    using S = EvalShape<B>;
    constexpr int PPT = S::ppt;
    __shared__ float4 prox[kChunk];
    __shared__ float4 tab[ASYM ? 2 * kSmearIntervals : 1];
    const GridParams &g = a.g;
    const int b = blockIdx.x;
    const int bi = b % a.l.bx, bj = (b / a.l.bx) % a.l.by, bk = b / (a.l.bx * a.l.by);
    const int i0 = bi * B, j0 = bj * B, k0 = bk * B;
    const double r0[3] = {i0 * g.h[0], j0 * g.h[1], k0 * g.h[2]};
    const PairConst kc = make_pair_const(a.asym);
    if (ASYM) load_smear_table(tab, a.asym.tab, S::threads);
    ConstAS<AtomF32<NS>> *rec = as_const(static_cast<const AtomF32<NS> *>(a.rec));
    ConstAS<int> *begin = as_const(a.begin);
    ConstAS<int> *end = as_const(a.end);
    ConstAS<int> *near_l = as_const(a.l.near);
    ConstAS<int> *short_l = as_const(a.l.shrt);
    const int n1 = a.degree + 1;
    const int f0 = a.l.far_off[b], f1 = a.l.far_off[b + 1];
    const int e0 = a.l.near_off[b], e1 = a.l.near_off[b + 1];
    const int s0 = a.l.short_off[b], s1 = a.l.short_off[b + 1];

    for (int pass = 0; pass < S::passes; ++pass) {
        int gi[PPT], gj[PPT], gk[PPT];
        bool valid[PPT];
        GridPt gp[PPT];
        float fx[PPT], fy[PPT], fz[PPT];   // relative to r0 (far field)
        PointAcc<NS> acc[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int l = (pass * PPT + q) * S::threads + threadIdx.x;
            const int li = l % B, lj = (l / B) % B, lk = l / (B * B);
            gi[q] = i0 + li;
            gj[q] = j0 + lj;
            gk[q] = k0 + lk;
            valid[q] = gi[q] < g.nx && gj[q] < g.ny && gk[q] < g.nz;
            gp[q] = grid_pt(g, valid[q] ? gi[q] : i0, valid[q] ? gj[q] : j0, valid[q] ? gk[q] : k0);
            fx[q] = (float)(li * g.h[0]);
            fy[q] = (float)(lj * g.h[1]);
            fz[q] = (float)(lk * g.h[2]);
            acc[q].zero();
        }

        // ---------------------------------------------------------- far
        for (int f = f0; f < f1; ++f) {
            const int node = a.l.far[f];
            const double *pb = a.pbox + 6 * node;
            const double *pq = a.pq + (size_t)node * a.np;
            for (int c0 = 0; c0 < a.np; c0 += kChunk) {
                const int cnt = min(kChunk, a.np - c0);
                __syncthreads();
                for (int k = threadIdx.x; k < cnt; k += S::threads) {
                    const int kk = c0 + k;
                    const int k1 = kk % n1, k2 = (kk / n1) % n1, k3 = kk / (n1 * n1);
                    float4 v;
                    v.x = (float)(cheb_pt(pb[0], pb[3], k1, a.degree) - r0[0]);
                    v.y = (float)(cheb_pt(pb[1], pb[4], k2, a.degree) - r0[1]);
                    v.z = (float)(cheb_pt(pb[2], pb[5], k3, a.degree) - r0[2]);
                    v.w = (float)pq[kk];
                    prox[k] = v;
                }
                __syncthreads();
                for (int k = 0; k < cnt; k += 16) {
                    PairAcc<NS> p[PPT];
#pragma unroll
                    for (int q = 0; q < PPT; ++q) p[q].zero();
                    const int kend = min(k + 16, cnt);
                    for (int kk = k; kk < kend; ++kk) {
                        const float4 v = prox[kk];
#pragma unroll
                        for (int q = 0; q < PPT; ++q) {
                            const float dx = fx[q] - v.x, dy = fy[q] - v.y, dz = fz[q] - v.z;
                            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                            const float ri = __builtin_amdgcn_rsqf(d2);
                            const float qr = v.w * ri;
                            p[q].C += qr;
                            if (ASYM) {
                                const float e = __builtin_amdgcn_exp2f(kc.yk * (d2 * ri));
                                p[q].Y = fmaf(qr, e, p[q].Y);
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < PPT; ++q) acc[q].template flush<false, ASYM>(p[q]);
                }
            }
        }

        // ---------------------------------------------------------- near
        for (int e = e0; e < e1; ++e) {
            const int leaf = near_l[e];
            const int ab = begin[leaf], ae = end[leaf];
            for (int t0 = ab; t0 < ae; t0 += kAtomPad) {
                PairAcc<NS> p[PPT];
#pragma unroll
                for (int q = 0; q < PPT; ++q) p[q].zero();
                const int tend = min(t0 + kAtomPad, ae);
                for (int t = t0; t < tend; ++t) {
                    ConstAS<AtomF32<NS>> &at = rec[t];
#pragma unroll
                    for (int q = 0; q < PPT; ++q)
                        pair_eval<NS, LJM, ASYM, false, true>(at, gp[q], kc, tab, p[q], acc[q].hit);
                }
#pragma unroll
                for (int q = 0; q < PPT; ++q) acc[q].template flush<LJM != LJ_NONE, ASYM>(p[q]);
            }
        }

        // ---------------------------------------------------------- short
        if (LJM != LJ_NONE || ASYM) {
            for (int e = s0; e < s1; ++e) {
                const int leaf = short_l[e];
                const int ab = begin[leaf], ae = end[leaf];
                for (int t0 = ab; t0 < ae; t0 += kAtomPad) {
                    PairAcc<NS> p[PPT];
#pragma unroll
                    for (int q = 0; q < PPT; ++q) p[q].zero();
                    const int tend = min(t0 + kAtomPad, ae);
                    for (int t = t0; t < tend; ++t) {
                        ConstAS<AtomF32<NS>> &at = rec[t];
#pragma unroll
                        for (int q = 0; q < PPT; ++q)
                            pair_eval<NS, LJM, ASYM, false, false>(at, gp[q], kc, tab, p[q],
                                                                  acc[q].hit);
                    }
#pragma unroll
                    for (int q = 0; q < PPT; ++q)
                        acc[q].template flush<LJM != LJ_NONE, ASYM>(p[q]);
                }
            }
        }

#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            if (!valid[q]) continue;
            const int64_t p = ((int64_t)gk[q] * g.ny + gj[q]) * g.nx + gi[q];
            store_point<NS, LJM, ASYM>(a.out, g, p, acc[q]);
        }
    }
}

namespace {

template <int NS, int LJM, bool ASYM>
void launch_b(int B, const SiteParams &sp, const TreeEvalArgs &a, hipStream_t s)
{
    const int nb = a.l.nb;
    if (B == 4)
        hipLaunchKernelGGL((k_tree_eval<NS, LJM, ASYM, 4>), nb, EvalShape<4>::threads, 0, s, sp, a);
    else if (B == 8)
        hipLaunchKernelGGL((k_tree_eval<NS, LJM, ASYM, 8>), nb, EvalShape<8>::threads, 0, s, sp, a);
    else
        hipLaunchKernelGGL((k_tree_eval<NS, LJM, ASYM, 16>), nb, EvalShape<16>::threads, 0, s, sp, a);
}

template <int NS>
void launch_ns(int lj_mode, bool asym, int B, const SiteParams &sp, const TreeEvalArgs &a,
               hipStream_t s)
{
    if (lj_mode == LJ_CUT) {
        if (asym) launch_b<NS, LJ_CUT, true>(B, sp, a, s);
        else launch_b<NS, LJ_CUT, false>(B, sp, a, s);
    } else {
        if (asym) launch_b<NS, LJ_NONE, true>(B, sp, a, s);
        else launch_b<NS, LJ_NONE, false>(B, sp, a, s);
    }
}

}  // namespace

int launch_tree_eval(const SiteParams &sp, int lj_mode, bool asym, int B, const TreeEvalArgs &a,
                     hipStream_t s)
{
    if (a.l.nb == 0) return RISM_OK;
    switch (sp.ns_pad) {
    case 1: launch_ns<1>(lj_mode, asym, B, sp, a, s); break;
    case 2: launch_ns<2>(lj_mode, asym, B, sp, a, s); break;
    case 4: launch_ns<4>(lj_mode, asym, B, sp, a, s); break;
    default: launch_ns<8>(lj_mode, asym, B, sp, a, s); break;
    }
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

}  // namespace rism
