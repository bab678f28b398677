// Reciprocal-space long-range asymptotics (Sec. 2.2, Eqs. 5 and 7, times
// k_C) with the frequency cut-off of Sec. 2.5, on the half grid of a
// real-to-complex transform of the [nz][ny][nx] grid.
//
// Everything hinges on the structure factor S(k) = sum_a Q_a exp(-i k.(R_a - o))
// at the k-points of the grid, k = 2 pi (jx/(nx hx), fy/(ny hy), fz/(nz hz)).
// It factorises per axis: exp(-i k.(R - o)) = ex[a][jx] ey[a][jy] ez[a][jz],
// so the phases are evaluated once per (atom, axis index) in FP64 and
// rounded to FP32 complex tables, and the sum over atoms is a separable
// contraction:
//   S[jz][jy][jx] = sum_a (Q_a ez[a][jz]) (ey[a][jy] ex[a][jx]).
// A workgroup owns 256 consecutive (jy, jx) entries and kAkZ consecutive jz;
// per atom a thread forms ey ex once (4 FP32 ops) and adds it, scaled by the
// kAkZ wave-uniform Q ez factors (scalar loads), into its kAkZ accumulators
// (4 ops each).  The (atom, jx) and (atom, jy) factors of a chunk of atoms
// are staged in LDS (shared by the block's rows and columns).  FP32 partial
// sums over a chunk are flushed into FP64.
// Entries beyond the cut-off are written as zero without being summed.
#include <cmath>

#include "pair.h"

namespace rism {

namespace {

constexpr int kAkThreads = 256;
constexpr int kAkZ = 8;        // jz values per workgroup

__device__ __forceinline__ int freq_of(int j, int n)
{
    return j <= (n - 1) / 2 ? j : j - n;
}

// Phase tables: for atom a, ex[a][0..nxh), ey[a][0..ny), ezq[a][0..nz) with
// ez scaled by Q_a; FP64 phase and sincos, stored as (re, im) FP32.
__global__ __launch_bounds__(kAkThreads) void k_phase_tables(const double *xyz, const double *q,
                                                             int64_t n, AkGrid g, float2 *ex,
                                                             float2 *ey, float2 *ezq)
{
    const int per = g.nxh + g.ny + g.nz;
    const int64_t tot = n * per;
    for (int64_t t = blockIdx.x * (int64_t)kAkThreads + threadIdx.x; t < tot;
         t += (int64_t)gridDim.x * kAkThreads) {
        const int64_t a = t / per;
        int j = (int)(t - a * per);
        int ax, f, nn;
        if (j < g.nxh) {
            ax = 0;
            f = j;
            nn = g.nx;
        } else if (j < g.nxh + g.ny) {
            ax = 1;
            j -= g.nxh;
            f = freq_of(j, g.ny);
            nn = g.ny;
        } else {
            ax = 2;
            j -= g.nxh + g.ny;
            f = freq_of(j, g.nz);
            nn = g.nz;
        }
        const double k = 2.0 * kPi * f / (nn * g.h[ax]);
        const double ph = k * (xyz[3 * a + ax] - g.o[ax]);
        double sn, cs;
        sincos(ph, &sn, &cs);
        if (ax == 0) {
            ex[a * g.nxh + j] = make_float2((float)cs, (float)-sn);
        } else if (ax == 1) {
            ey[a * g.ny + j] = make_float2((float)cs, (float)-sn);
        } else {
            ezq[a * g.nz + j] = make_float2((float)(q[a] * cs), (float)(-q[a] * sn));
        }
    }
}

struct Quad2 {
    float x, y;
};

// LDS stage of one chunk of atoms: the ex factors of the block's jx values
// (all of them when the row has at most kAkThreads entries, else one per
// thread) and the ey factors of its rows.
struct AkStage {
    int xs, ys;   // entries per atom
};
__host__ __device__ inline AkStage ak_stage(int nxh)
{
    AkStage st;
    st.xs = nxh <= kAkThreads ? nxh : kAkThreads;
    st.ys = (kAkThreads + nxh - 1) / nxh + 1;
    return st;
}

__global__ __launch_bounds__(kAkThreads) void k_asym_k(AkArgs a)
{
    extern __shared__ float2 stage[];
    const AkGrid &g = a.g;
    const AkStage st = ak_stage(g.nxh);
    const int chunk = a.chunk;
    float2 *sx = stage;                 // [chunk][xs]
    float2 *sy = stage + chunk * st.xs; // [chunk][ys]
    const int nxy = g.nxh * g.ny;
    const int p0 = blockIdx.x * kAkThreads;
    const int p = p0 + threadIdx.x;
    const bool valid = p < nxy;
    const int pc = valid ? p : p0;
    const int jy = pc / g.nxh, jx = pc % g.nxh;
    const int jy0 = p0 / g.nxh;
    const int rows = (min(p0 + kAkThreads, nxy) - 1) / g.nxh - jy0 + 1;
    const int xi = g.nxh <= kAkThreads ? jx : (int)threadIdx.x;   // column in sx
    const int jz0 = blockIdx.y * kAkZ;
    const double kx = 2.0 * kPi * jx / (g.nx * g.h[0]);
    const double ky = 2.0 * kPi * freq_of(jy, g.ny) / (g.ny * g.h[1]);
    auto k2_of = [&](int z) {
        const int jz = jz0 + z;
        const double kz = 2.0 * kPi * freq_of(jz < g.nz ? jz : 0, g.nz) / (g.nz * g.h[2]);
        return kx * kx + ky * ky + kz * kz;
    };
    const double k2c = as_const(a.k2cut)[0], k2h = as_const(a.k2cut)[1];
    const double k2max = k2c > k2h ? k2c : k2h;
    bool any = false;
#pragma unroll
    for (int z = 0; z < kAkZ; ++z) any |= valid && jz0 + z < g.nz && k2_of(z) <= k2max;
    double Sr[kAkZ], Si[kAkZ];
#pragma unroll
    for (int z = 0; z < kAkZ; ++z) Sr[z] = Si[z] = 0.0;
    if (__syncthreads_or(any)) {
        ConstAS<Quad2> *ezq = as_const(reinterpret_cast<const Quad2 *>(a.ezq));
        for (int64_t a0 = 0; a0 < a.n; a0 += chunk) {
            const int cnt = (int)min((int64_t)chunk, a.n - a0);
            __syncthreads();
            for (int t = threadIdx.x; t < cnt * st.xs; t += kAkThreads) {
                const int at = t / st.xs, l = t % st.xs;
                const int col = g.nxh <= kAkThreads ? l : min(p0 + l, nxy - 1) % g.nxh;
                sx[at * st.xs + l] = a.ex[(a0 + at) * g.nxh + col];
            }
            for (int t = threadIdx.x; t < cnt * rows; t += kAkThreads) {
                const int at = t / rows, r = t % rows;
                sy[at * st.ys + r] = a.ey[(a0 + at) * g.ny + jy0 + r];
            }
            __syncthreads();
            float pr[kAkZ], pi[kAkZ];
#pragma unroll
            for (int z = 0; z < kAkZ; ++z) pr[z] = pi[z] = 0.f;
            for (int at = 0; at < cnt; ++at) {
                const float2 vx = sx[at * st.xs + xi], vy = sy[at * st.ys + (jy - jy0)];
                const float tr = fmaf(vy.x, vx.x, -vy.y * vx.y);
                const float ti = fmaf(vy.x, vx.y, vy.y * vx.x);
                ConstAS<Quad2> *ez = ezq + (a0 + at) * g.nz;
#pragma unroll
                for (int z = 0; z < kAkZ; ++z) {
                    const int jz = jz0 + z < g.nz ? jz0 + z : g.nz - 1;   // in range; unused past nz
                    const float wr = ez[jz].x, wi = ez[jz].y;
                    pr[z] = fmaf(wr, tr, fmaf(-wi, ti, pr[z]));
                    pi[z] = fmaf(wr, ti, fmaf(wi, tr, pi[z]));
                }
            }
#pragma unroll
            for (int z = 0; z < kAkZ; ++z) {
                Sr[z] += (double)pr[z];
                Si[z] += (double)pi[z];
            }
        }
    }
    if (!valid) return;
    if (p == 0 && jz0 == 0) {
        // k = 0: S is the net charge; its FP32 terms would leave ~1e-7 sum |Q|
        Sr[0] = as_const(a.k2cut)[2];
        Si[0] = 0.0;
    }
    const int64_t mk = (int64_t)nxy * g.nz;
#pragma unroll
    for (int z = 0; z < kAkZ; ++z) {
        const int jz = jz0 + z;
        if (jz >= g.nz) continue;
        const int64_t e = (int64_t)jz * nxy + p;
        const double k2 = k2_of(z);
        const bool in_c = k2 > 0.0 && k2 <= k2c;
        const bool in_h = k2 <= k2h && k2 + a.kappa2 > 0.0;   // h(0) at kappa = 0 is 0, as c(0)
        const double gauss = exp(-k2 * a.eta2_4);
        const double fc = in_c ? gauss / k2 : 0.0;
        const double fh = in_h ? gauss / (k2 + a.kappa2) : 0.0;
        if (a.c)
            for (int s = 0; s < a.ns; ++s) {
                const double f = a.c_scale[s] * fc;
                store_val(a.c, a.f64, 2 * (s * mk + e), f * Sr[z]);
                store_val(a.c, a.f64, 2 * (s * mk + e) + 1, f * Si[z]);
            }
        if (a.h)
            for (int s = 0; s < a.n_ionic; ++s) {
                const double f = a.h_scale[s] * fh;
                store_val(a.h, a.f64, 2 * (s * mk + e), f * Sr[z]);
                store_val(a.h, a.f64, 2 * (s * mk + e) + 1, f * Si[z]);
            }
    }
}

}  // namespace

// Root of the Sec. 2.5 bound: pref exp(-k^2 eta^2/4) / den(k) = tol, with
// den = k^2 (c^lr) or eps (k^2 + kappa^2) (h^lr), by Newton's method on the
// logarithm, kept inside a bracket that every step shrinks.  0 when no
// positive k reaches the tolerance (then nothing is cut).
__host__ __device__ static double ak_log_bound(bool for_h, double k, double lpt, double eta,
                                               double kappa, double diel)
{
    const double den = for_h ? diel * (k * k + kappa * kappa) : k * k;
    return lpt - k * k * eta * eta / 4.0 - log(den);
}

__host__ __device__ double ak_kcut(bool for_h, double tol, double pref, double eta, double kappa,
                                   double diel)
{
    if (!(tol > 0.0) || !(pref > 0.0)) return 0.0;
    const double lpt = log(pref / tol);
    double lo = 1e-12, hi = 1.0;
    if (ak_log_bound(for_h, lo, lpt, eta, kappa, diel) <= 0.0) return 0.0;
    while (ak_log_bound(for_h, hi, lpt, eta, kappa, diel) > 0.0 && hi < 1e6) hi *= 2.0;
    double k = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double v = ak_log_bound(for_h, k, lpt, eta, kappa, diel);
        if (v > 0.0) lo = k;
        else hi = k;
        const double dv = -k * eta * eta / 2.0 - (for_h ? 2.0 * k / (k * k + kappa * kappa) : 2.0 / k);
        double kn = k - v / dv;
        if (!(kn > lo && kn < hi)) kn = 0.5 * (lo + hi);
        const bool done = fabs(kn - k) <= 1e-15 * k;
        k = kn;
        if (done) break;
    }
    return k;
}

namespace {

__global__ __launch_bounds__(kAkThreads) void k_ak_cutoffs(const double *q, int64_t n, double tol,
                                                           double pref_c, double pref_h,
                                                           double eta, double kappa, double diel,
                                                           double *k2cut)
{
    __shared__ double red[2][kAkThreads / 64];
    double s = 0.0, sq = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kAkThreads) {
        s += fabs(q[i]);
        sq += q[i];
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        sq += __shfl_xor(sq, off);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s;
        red[1][threadIdx.x >> 6] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0, tq = 0.0;
        for (int w = 0; w < kAkThreads / 64; ++w) {
            t += red[0][w];
            tq += red[1][w];
        }
        k2cut[2] = tq;   // S(0), the net charge, in FP64
        const double kc = ak_kcut(false, tol, pref_c * t, eta, kappa, diel);
        const double kh = ak_kcut(true, tol, pref_h * t, eta, kappa, diel);
        k2cut[0] = kc > 0.0 ? kc * kc : INFINITY;
        k2cut[1] = kh > 0.0 ? kh * kh : INFINITY;
    }
}

}  // namespace

int launch_ak_cutoffs(const double *q, int64_t n, double tol, double pref_c, double pref_h,
                      double eta, double kappa, double diel, double *k2cut, hipStream_t s)
{
    hipLaunchKernelGGL(k_ak_cutoffs, 1, kAkThreads, 0, s, q, n, tol, pref_c, pref_h, eta, kappa,
                       diel, k2cut);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

int launch_asym_k(const AkArgs &a, const double *xyz, const double *q, float2 *ex, float2 *ey,
                  float2 *ezq, hipStream_t s)
{
    const int64_t tot = a.n * (int64_t)(a.g.nxh + a.g.ny + a.g.nz);
    if (tot > 0) {
        const int blocks = (int)std::min<int64_t>((tot + kAkThreads - 1) / kAkThreads, 65536);
        hipLaunchKernelGGL(k_phase_tables, blocks, kAkThreads, 0, s, xyz, q, a.n, a.g, ex, ey,
                           ezq);
    }
    AkArgs b = a;
    b.ex = ex;
    b.ey = ey;
    b.ezq = ezq;
    const AkStage st = ak_stage(a.g.nxh);
    const size_t per_atom = (size_t)(st.xs + st.ys) * sizeof(float2);
    b.chunk = (int)std::max<size_t>(1, std::min<size_t>(64, (48 * 1024) / per_atom));
    const int nxy = a.g.nxh * a.g.ny;
    dim3 grid((nxy + kAkThreads - 1) / kAkThreads, (a.g.nz + kAkZ - 1) / kAkZ);
    hipLaunchKernelGGL(k_asym_k, grid, kAkThreads, b.chunk * per_atom, s, b);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

}  // namespace rism
