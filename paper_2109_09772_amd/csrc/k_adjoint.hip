// Adjoint of the potential u_gamma(r) (Coulomb + LJ) with respect to atom
// positions, charges, eps_a and sigma_a.
//
// L = sum_g sum_r w_g(r) u_g(r).  For atom a, d = |r - R_a|, s6 = (sigma_ga/d)^6:
//   dL/dQ_a     = k_C sum_r W(r)/d,            W(r) = sum_g q_g w_g(r)
//   dL/dR_a     = sum_r [k_C Q_a W/d^3 + sum_g 24 eps_ga w_g s6 (2 s6 - 1)/d^2] (r - R_a)
//   dL/deps_a   = sum_g (2 eps_ga/eps_a) sum_r w_g s6 (s6 - 1)
//   dL/dsigma_a = sum_g (12 eps_ga/sigma_ga) sum_r w_g s6 (2 s6 - 1)
// (the last two follow from sigma_ga = (sigma_g + sigma_a)/2 and
// eps_ga = sqrt(eps_g eps_a)).
//
// Direct form: one lane per atom, grid points wave-uniform (their positions
// come from per-axis coordinate tables and their weights w_g(r) through
// scalar loads).  Each workgroup covers 256 atoms x one chunk of grid points
// and writes its per-atom partial gradients; a second kernel adds the chunk
// partials in chunk order, so the result is bitwise reproducible.
#include <cmath>
#include <type_traits>

#include "rism_internal.h"

namespace rism {

namespace {

// Per-site lane constants of one atom.
template <int NS, class T>
struct AtomLane {
    T x, y, z, xl, yl, zl, q;
    T sg6[NS];   // sigma_ga^6
    T e24[NS];   // 24 eps_ga
    T rc2[NS];
};

template <int NS>
__device__ __forceinline__ void load_lane(const AtomF32<NS> &r, AtomLane<NS, float> &l, float kc)
{
    l.x = r.xh; l.y = r.yh; l.z = r.zh;
    l.xl = r.xl; l.yl = r.yl; l.zl = r.zl;
    l.q = r.q * kc;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        // A = 4 e s^12, B = 4 e s^6  =>  s^6 = A/B, 24 e = 6 B^2/A
        float A = r.A[s], B = r.B[s];
        l.sg6[s] = B > 0.f ? A / B : 0.f;
        l.e24[s] = A > 0.f ? 6.f * B * B / A : 0.f;
        l.rc2[s] = r.rc2[s];
    }
}

template <int NS>
__device__ __forceinline__ void load_lane(const AtomF64<NS> &r, AtomLane<NS, double> &l, double kc)
{
    l.x = r.x; l.y = r.y; l.z = r.z;
    l.xl = 0; l.yl = 0; l.zl = 0;
    l.q = r.q * kc;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        double A = r.A[s], B = r.B[s];
        l.sg6[s] = B > 0.0 ? A / B : 0.0;
        l.e24[s] = A > 0.0 ? 6.0 * B * B / A : 0.0;
        l.rc2[s] = r.rc2[s];
    }
}

__device__ __forceinline__ float rsq(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

}  // namespace

struct AdjKernelArgs {
    const void *atoms;
    int64_t npad;
    int ns;
    int nx, ny, nz;
    int64_t m;
    int64_t chunk;           // grid points per chunk
    int nchunks;
    const float *axh[3];     // per-axis coordinates i*h relative to the origin (hi)
    const float *axl[3];     // (lo)
    const double *axd[3];    // FP64 per-axis coordinates
    const void *w;           // [S][M]
    int w_f64;
    double sq[kMaxSites];    // site charges
    double kc;
    int lj_cut;
    double *part;            // [nchunks][6][npad]
};

template <int NS, class T, bool CUT>
__global__ __launch_bounds__(kBlock) void k_adjoint_direct(AdjKernelArgs a)
{
    using Rec = typename std::conditional<std::is_same<T, float>::value, AtomF32<NS>, AtomF64<NS>>::type;
    const int64_t atom = blockIdx.x * (int64_t)kBlock + threadIdx.x;   // < npad (padded to 256)
    const int chunk = blockIdx.y;
    const Rec *recs = static_cast<const Rec *>(a.atoms);
    AtomLane<NS, T> L;
    if (atom < a.npad) load_lane(recs[atom], L, (T)a.kc);
    else load_lane(recs[0], L, (T)0);   // idle lane (never stored)

    const int64_t p0 = chunk * a.chunk;
    const int64_t p1 = p0 + a.chunk < a.m ? p0 + a.chunk : a.m;
    T sq[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) sq[s] = s < a.ns ? (T)a.sq[s] : (T)0;

    double gx = 0, gy = 0, gz = 0, gq = 0, gE[NS], gS[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) { gE[s] = 0; gS[s] = 0; }

    constexpr int BLK = 8;
    // (i, j, k) of the current point, advanced incrementally (uniform).
    int i = (int)(p0 % a.nx);
    int j = (int)((p0 / a.nx) % a.ny);
    int k = (int)(p0 / ((int64_t)a.nx * a.ny));
    for (int64_t pb = p0; pb < p1; pb += BLK) {
        T fx = 0, fy = 0, fz = 0, fq = 0, fE[NS], fS[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) { fE[s] = 0; fS[s] = 0; }
        const int cnt = (int)(p1 - pb < BLK ? p1 - pb : BLK);
        for (int t = 0; t < cnt; ++t) {
            const int64_t p = pb + t;
            T dx, dy, dz;
            if (std::is_same<T, float>::value) {
                dx = (T)((a.axh[0][i] - (float)L.x) + (a.axl[0][i] - (float)L.xl));
                dy = (T)((a.axh[1][j] - (float)L.y) + (a.axl[1][j] - (float)L.yl));
                dz = (T)((a.axh[2][k] - (float)L.z) + (a.axl[2][k] - (float)L.zl));
            } else {
                dx = (T)(a.axd[0][i] - (double)L.x);
                dy = (T)(a.axd[1][j] - (double)L.y);
                dz = (T)(a.axd[2][k] - (double)L.z);
            }
            if (++i == a.nx) {
                i = 0;
                if (++j == a.ny) { j = 0; ++k; }
            }
            T w[NS];
            T W = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                T v = 0;
                if (s < a.ns)
                    v = a.w_f64 ? (T) static_cast<const double *>(a.w)[s * a.m + p]
                                : (T) static_cast<const float *>(a.w)[s * a.m + p];
                w[s] = v;
                W += sq[s] * v;
            }
            T d2 = dx * dx + dy * dy + dz * dz;
            T ri = d2 > (T)0 ? rsq(d2) : (T)0;
            T r2 = ri * ri;
            T r6 = r2 * r2 * r2;
            T tq = W * ri;
            fq += tq;
            T F = L.q * tq * r2;   // k_C Q W / d^3
            T Flj = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                T ws = w[s];
                if (CUT) ws = d2 < L.rc2[s] ? ws : (T)0;
                T s6 = L.sg6[s] * r6;
                T ws6 = ws * s6;
                T v = ws6 * (s6 + s6 - (T)1);      // w s6 (2 s6 - 1)
                fS[s] += v;
                fE[s] += ws6 * (s6 - (T)1);        // w s6 (s6 - 1)
                Flj += L.e24[s] * v;
            }
            F += Flj * r2;
            // d/dR_a of u(|r - R_a|) is F (r - R_a) with F as above
            fx += F * dx;
            fy += F * dy;
            fz += F * dz;
        }
        gx += (double)fx;
        gy += (double)fy;
        gz += (double)fz;
        gq += (double)fq;
#pragma unroll
        for (int s = 0; s < NS; ++s) { gE[s] += (double)fE[s]; gS[s] += (double)fS[s]; }
    }
    if (atom >= a.npad) return;
    // Fold the per-site sums with eps_ga, sigma_ga recovered from the record
    // (eps_ga = B^2/(4A), sigma_ga = (A/B)^(1/6)); 1/eps_a is applied by the
    // reduction kernel.
    double e_sum = 0, s_sum = 0;
    const Rec &rr = recs[atom];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        double A = (double)rr.A[s], B = (double)rr.B[s];
        // eps_ga = B^2/(4A), sigma_ga^6 = A/B
        double e_ga = A > 0 ? B * B / (4.0 * A) : 0.0;
        double sg = B > 0 ? pow(A / B, 1.0 / 6.0) : 0.0;
        e_sum += 2.0 * e_ga * gE[s];          // divided by eps_a in the reduction
        s_sum += sg > 0 ? 12.0 * e_ga / sg * gS[s] : 0.0;
    }
    double *out = a.part + (size_t)chunk * 6 * a.npad;
    out[0 * a.npad + atom] = gx;
    out[1 * a.npad + atom] = gy;
    out[2 * a.npad + atom] = gz;
    out[3 * a.npad + atom] = a.kc * gq;
    out[4 * a.npad + atom] = e_sum;
    out[5 * a.npad + atom] = s_sum;
}

__global__ __launch_bounds__(kBlock) void k_adjoint_reduce(const double *part, int nchunks,
                                                           int64_t n, int64_t npad,
                                                           const double *eps_in,
                                                           const double *sig_in, double *dxyz,
                                                           double *dq, double *deps, double *dsig)
{
    int64_t atom = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (atom >= n) return;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < nchunks; ++c)
        for (int k = 0; k < 6; ++k) v[k] += part[((size_t)c * 6 + k) * npad + atom];
    if (dxyz) {
        dxyz[3 * atom] = v[0];
        dxyz[3 * atom + 1] = v[1];
        dxyz[3 * atom + 2] = v[2];
    }
    if (dq) dq[atom] = v[3];
    if (deps) deps[atom] = v[4] / eps_in[atom];
    if (dsig) dsig[atom] = v[5];
    (void)sig_in;
}

namespace {

__global__ void k_axis_tables(double o_unused, double h, int n, float *hi, float *lo, double *dd)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = i * h;
    float xh = (float)x;
    hi[i] = xh;
    lo[i] = (float)(x - (double)xh);
    dd[i] = x;
    (void)o_unused;
}

template <int NS, class T>
void launch_adj(const AdjKernelArgs &ka, dim3 grid, hipStream_t s)
{
    if (ka.lj_cut)
        hipLaunchKernelGGL((k_adjoint_direct<NS, T, true>), grid, kBlock, 0, s, ka);
    else
        hipLaunchKernelGGL((k_adjoint_direct<NS, T, false>), grid, kBlock, 0, s, ka);
}

}  // namespace

int build_axis_tables(const GridParams &g, Workspace &ws, const float *axh[3], const float *axl[3],
                      const double *axd[3], hipStream_t s)
{
    int dims[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        float *hi = ws.get<float>(dims[a]);
        float *lo = ws.get<float>(dims[a]);
        double *dd = ws.get<double>(dims[a]);
        if (ws.status()) return ws.status();
        hipLaunchKernelGGL(k_axis_tables, (dims[a] + 255) / 256, 256, 0, s, 0.0, g.h[a], dims[a],
                           hi, lo, dd);
        RISM_HIP(hipGetLastError());
        axh[a] = hi;
        axl[a] = lo;
        axd[a] = dd;
    }
    return RISM_OK;
}

int adjoint_direct(const AdjointArgs &a, bool f64, Workspace &ws, rism_stats &st, hipStream_t s)
{
    AdjKernelArgs ka{};
    ka.atoms = a.atoms;
    ka.ns = a.sp.ns;
    ka.nx = a.g.nx;
    ka.ny = a.g.ny;
    ka.nz = a.g.nz;
    ka.m = a.g.m;
    ka.w = a.w;
    ka.w_f64 = a.w_f64;
    for (int g = 0; g < kMaxSites; ++g) ka.sq[g] = a.sp.q[g];
    ka.kc = a.kc;
    ka.lj_cut = a.lj_mode == LJ_CUT;
    // atoms per workgroup: 256; records are padded to kAtomPad only, so the
    // last workgroup's idle lanes read record 0 and store nothing.
    int64_t abl = (a.npad + kBlock - 1) / kBlock;
    int64_t want = 4096;
    int64_t nch = (want + abl - 1) / abl;
    if (nch > a.g.m) nch = a.g.m;
    if (nch < 1) nch = 1;
    ka.chunk = (a.g.m + nch - 1) / nch;
    ka.nchunks = (int)((a.g.m + ka.chunk - 1) / ka.chunk);
    ka.npad = a.npad;
    int rc = build_axis_tables(a.g, ws, ka.axh, ka.axl, ka.axd, s);
    if (rc) return rc;
    ka.part = ws.get<double>((size_t)ka.nchunks * 6 * a.npad);
    if (!ka.part) return ws.status();
    dim3 grid((unsigned)abl, (unsigned)ka.nchunks);
    const bool ev = a.opts->flags & RISM_FLAG_PHASE_EVENTS;
    {
    PhaseTimer pt(ev, RISM_PHASE_ADJOINT, s);
    switch (a.sp.ns_pad) {
    case 1: f64 ? launch_adj<1, double>(ka, grid, s) : launch_adj<1, float>(ka, grid, s); break;
    case 2: f64 ? launch_adj<2, double>(ka, grid, s) : launch_adj<2, float>(ka, grid, s); break;
    case 4: f64 ? launch_adj<4, double>(ka, grid, s) : launch_adj<4, float>(ka, grid, s); break;
    default: f64 ? launch_adj<8, double>(ka, grid, s) : launch_adj<8, float>(ka, grid, s); break;
    }
    }
    RISM_HIP(hipGetLastError());
    PhaseTimer pt2(ev, RISM_PHASE_ADJ_REDUCE, s);
    hipLaunchKernelGGL(k_adjoint_reduce, (unsigned)((a.n + kBlock - 1) / kBlock), kBlock, 0, s,
                       ka.part, ka.nchunks, a.n, a.npad, a.eps_in, a.sig_in, a.dxyz, a.dq, a.deps,
                       a.dsig);
    RISM_HIP(hipGetLastError());
    st.pairs_direct = (double)a.n * a.g.m;
    return RISM_OK;
}

}  // namespace rism
