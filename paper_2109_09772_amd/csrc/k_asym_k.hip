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
// The contraction is a complex matrix product per jy (or per jx) and runs on
// the matrix cores (below).  Entries beyond the cut-off are written as zero;
// whole tiles beyond it are not summed.
#include <cmath>

#include "pair.h"

namespace rism {

namespace {

constexpr int kAkThreads = 256;   // phase tables and cut-offs

__device__ __forceinline__ int freq_of(int j, int n)
{
    return j <= (n - 1) / 2 ? j : j - n;
}

// Phase tables: for atom a, ex[a][0..nxh), ey[a][0..ny), ezq[a][0..nz) with
// ez scaled by Q_a; FP64 phase and sincos, stored as (re, im) FP32.  Rows
// n .. npad - 1 are padding: ex = ey = 1, ezq = 0.
__global__ __launch_bounds__(kAkThreads) void k_phase_tables(const double *xyz, const double *q,
                                                             int64_t n, int64_t npad, AkGrid g,
                                                             float2 *ex, float2 *ey, float2 *ezq)
{
    const int per = g.nxh + g.ny + g.nz;
    const int64_t tot = npad * per;
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
        double sn = 0.0, cs = 1.0, qa = 0.0;
        if (a < n) {
            const double k = 2.0 * kPi * f / (nn * g.h[ax]);
            const double ph = k * (xyz[3 * a + ax] - g.o[ax]);
            sincos(ph, &sn, &cs);
            qa = q[a];
        }
        if (ax == 0) {
            ex[a * g.nxh + j] = make_float2((float)cs, (float)-sn);
        } else if (ax == 1) {
            ey[a * g.ny + j] = make_float2((float)cs, (float)-sn);
        } else {
            ezq[a * g.nz + j] = make_float2((float)(qa * cs), (float)(-qa * sn));
        }
    }
}

// ------------------------------------------------------- matrix-core path
// For each jy the structure factor is a complex matrix product over atoms,
//   S[jz][jx] = sum_a Z[a][jz] T[a][jx],   Z = Q ez,  T = ey[a][jy] ex[a][jx],
// run on v_mfma_f32_32x32x2_f32 with K = 2 holding the real and imaginary
// parts of one atom's factors: A[i][k] = (Re, Im) Z[a][jz_i], and
//   B = (Re T, -Im T) for Re S,   B = (Im T, Re T) for Im S.
// A workgroup owns 32 MFMA columns, 4 rows (one per wave) and 32 jz (one
// 32-row tile per wave: two accumulator chains, real and imaginary).  The
// single tile keeps a wave at about 160 registers, so three waves share a
// SIMD and one wave's FP64 flushes and operand preparation run under another
// wave's matrix instructions (two tiles per wave needed 312 registers, one
// wave per SIMD, and kept the matrix pipe busy 56 % of the time).  Columns
// are 32 consecutive jx and rows are jy (YC = false: the full 32-column tiles
// of the half grid), or columns are jy and rows the jx past the last full
// tile (YC = true: the Nyquist column of an even nx, or every jx of a half
// grid narrower than 32).  The phase factors of 32 atoms at a time (the
// columns' and rows' ex / ey and the 32 jz's Q ez: 17 KB) are staged in LDS,
// double buffered: the next 32 atoms are fetched into registers while the
// matrix cores work on the current ones.  T is formed per lane.  FP32 matrix
// sums over 32 atoms are flushed into FP64 registers.
// The tables are padded to a multiple of 32 atoms with Q = 0, so no atom
// needs a test; columns and rows past the grid run on clamped indices and
// are not stored.
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMfCols = 32;    // MFMA columns per workgroup
constexpr int kMfZT = 1;       // 32-row jz tiles per wave
constexpr int kMfZ = 32 * kMfZT;   // jz per workgroup
constexpr int kMfWaves = 4;    // rows per workgroup, one per wave
constexpr int kMfFlush = 32;   // atoms per LDS stage and per FP32 matrix sum
constexpr int kMfThreads = 64 * kMfWaves;
constexpr int kMfZPer = kMfFlush * kMfZ / kMfThreads;      // staged Q ez values per thread
constexpr int kMfCPer = kMfFlush * kMfCols / kMfThreads;   // staged column factors per thread
static_assert(kMfZPer >= 1 && kMfCPer >= 1 && kMfFlush * kMfWaves <= kMfThreads, "staging");

struct MfStage {
    float2 c[kMfFlush][kMfCols];   // column factors
    float z[kMfFlush][kMfZ][2];    // Q ez
    float2 r[kMfFlush][kMfWaves];  // row factors
};

// Output of one half-grid entry from its structure factor (sr, si): the
// Eq. 5 / Eq. 7 factors, the cut-offs, and S(0) = the FP64 net charge.
__device__ void ak_store(const AkArgs &a, int jx, int jy, int jz, double sr, double si)
{
    const AkGrid &g = a.g;
    if (jx == 0 && jy == 0 && jz == 0) {
        // k = 0: S is the net charge; its FP32 terms would leave ~1e-7 sum |Q|
        sr = as_const(a.k2cut)[2];
        si = 0.0;
    }
    const double kx = 2.0 * kPi * jx / (g.nx * g.h[0]);
    const double ky = 2.0 * kPi * freq_of(jy, g.ny) / (g.ny * g.h[1]);
    const double kz = 2.0 * kPi * freq_of(jz, g.nz) / (g.nz * g.h[2]);
    const double k2 = kx * kx + ky * ky + kz * kz;
    const double k2c = as_const(a.k2cut)[0], k2h = as_const(a.k2cut)[1];
    const bool in_c = k2 > 0.0 && k2 <= k2c;
    const bool in_h = k2 <= k2h && k2 + a.kappa2 > 0.0;   // h(0) at kappa = 0 is 0
    const double gauss = exp(-k2 * a.eta2_4);
    const double fc = in_c ? gauss / k2 : 0.0;
    const double fh = in_h ? gauss / (k2 + a.kappa2) : 0.0;
    const int64_t nxy = (int64_t)g.nxh * g.ny, mk = nxy * g.nz;
    const int64_t e = (int64_t)jz * nxy + (int64_t)jy * g.nxh + jx;
    if (a.c)
        for (int s = 0; s < a.ns; ++s) {
            const double f = a.c_scale[s] * fc;
            store_val(a.c, a.f64, 2 * (s * mk + e), f * sr);
            store_val(a.c, a.f64, 2 * (s * mk + e) + 1, f * si);
        }
    if (a.h)
        for (int s = 0; s < a.n_ionic; ++s) {
            const double f = a.h_scale[s] * fh;
            store_val(a.h, a.f64, 2 * (s * mk + e), f * sr);
            store_val(a.h, a.f64, 2 * (s * mk + e) + 1, f * si);
        }
}

// A region: the jx in [x0, x0 + xw), every jy and jz; its entry idx =
// (jz ny + jy) xw + jx - x0.  With ks > 1 the atoms are split into ks
// contiguous groups of 32-atom chunks, one per workgroup layer, and each
// layer writes its FP64 partial sums to part[layer][idx][re, im]; a second
// kernel adds the layers in order.
struct AkRegion {
    int x0, xw, ks;
    int64_t count;     // entries
    double *part;      // [ks][count][2] when ks > 1
};

template <bool YC>
__global__ __launch_bounds__(kMfThreads, 2) void k_asym_k_mfma(AkArgs a, AkRegion rg)
{
    const int x0 = rg.x0;
    __shared__ MfStage st[2];
    const AkGrid &g = a.g;
    const int tid = threadIdx.x;
    const int lane = tid & 63, half = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // columns c0 + col below clim, rows r0 + wave below rlim
    const int c0 = blockIdx.x * kMfCols, clim = YC ? g.ny : g.nxh;
    const int r0 = (YC ? x0 : 0) + blockIdx.y * kMfWaves, rlim = YC ? g.nxh : g.ny;
    const float2 *ctab = YC ? a.ey : a.ex, *rtab = YC ? a.ex : a.ey;
    const int cstride = YC ? g.ny : g.nxh, rstride = YC ? g.nxh : g.ny;
    const int ci = c0 + col, ri = r0 + wave;
    const int jx = YC ? ri : ci, jy = YC ? ci : ri;
    const int zt = (g.nz + kMfZ - 1) / kMfZ;
    const int layer = blockIdx.z / zt;
    const int jz0 = (blockIdx.z % zt) * kMfZ;
    const int nch_all = (int)((a.n + kMfFlush - 1) / kMfFlush);
    const int cb = (int)((int64_t)layer * nch_all / rg.ks);
    const int ce = (int)((int64_t)(layer + 1) * nch_all / rg.ks);
    auto kx_of = [&](int x) { return 2.0 * kPi * x / (g.nx * g.h[0]); };
    auto ky_of = [&](int y) { return 2.0 * kPi * freq_of(y, g.ny) / (g.ny * g.h[1]); };
    auto kz_of = [&](int z) { return 2.0 * kPi * freq_of(z, g.nz) / (g.nz * g.h[2]); };
    const double k2c = as_const(a.k2cut)[0], k2h = as_const(a.k2cut)[1];
    const double k2max = k2c > k2h ? k2c : k2h;
    // smallest |k|^2 of the workgroup's tile: skip the sum beyond both cut-offs
    // (kx grows with jx; the first column or row holds the smallest)
    double ky2min = INFINITY, kz2min = INFINITY;
    const int ylo = YC ? c0 : r0, yn = YC ? kMfCols : kMfWaves;
    for (int y = ylo; y < ylo + yn && y < g.ny; ++y) ky2min = fmin(ky2min, ky_of(y) * ky_of(y));
    for (int z = jz0; z < jz0 + kMfZ && z < g.nz; ++z) kz2min = fmin(kz2min, kz_of(z) * kz_of(z));
    const double kx2min = kx_of(YC ? r0 : c0) * kx_of(YC ? r0 : c0);
    const bool work = ce > cb && kx2min + ky2min + kz2min <= k2max;

    // staging: thread tid carries kMfCPer column, kMfZPer Q ez and (tid < kMfFlush kMfWaves)
    // one row value per stage
    float2 rc[kMfCPer], rz[kMfZPer], rr = make_float2(0.f, 0.f);
    auto fetch = [&](int64_t a0) {
#pragma unroll
        for (int u = 0; u < kMfCPer; ++u) {
            const int e = tid + u * kMfThreads, at = e / kMfCols, c = e % kMfCols;
            rc[u] = ctab[(a0 + at) * cstride + min(c0 + c, clim - 1)];
        }
#pragma unroll
        for (int u = 0; u < kMfZPer; ++u) {
            const int e = tid + u * kMfThreads, at = e / kMfZ, z = e % kMfZ;
            rz[u] = a.ezq[(a0 + at) * g.nz + min(jz0 + z, g.nz - 1)];
        }
        if (tid < kMfFlush * kMfWaves) {
            const int at = tid / kMfWaves, w = tid % kMfWaves;
            rr = rtab[(a0 + at) * rstride + min(r0 + w, rlim - 1)];
        }
    };
    auto stash = [&](MfStage &b) {
#pragma unroll
        for (int u = 0; u < kMfCPer; ++u) {
            const int e = tid + u * kMfThreads;
            b.c[e / kMfCols][e % kMfCols] = rc[u];
        }
#pragma unroll
        for (int u = 0; u < kMfZPer; ++u) {
            const int e = tid + u * kMfThreads;
            b.z[e / kMfZ][e % kMfZ][0] = rz[u].x;
            b.z[e / kMfZ][e % kMfZ][1] = rz[u].y;
        }
        if (tid < kMfFlush * kMfWaves) b.r[tid / kMfWaves][tid % kMfWaves] = rr;
    };

    double Sr[kMfZT][16], Si[kMfZT][16];
#pragma unroll
    for (int t = 0; t < kMfZT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) Sr[t][r] = Si[t][r] = 0.0;
    if (work) {
        fetch((int64_t)cb * kMfFlush);
        stash(st[0]);
        __syncthreads();
        for (int c = cb; c < ce; ++c) {
            const MfStage &b = st[(c - cb) & 1];
            if (c + 1 < ce) fetch((int64_t)(c + 1) * kMfFlush);
            f32x16 accR[kMfZT], accI[kMfZT];
#pragma unroll
            for (int t = 0; t < kMfZT; ++t) accR[t] = accI[t] = f32x16{};
#pragma unroll 8
            for (int i = 0; i < kMfFlush; ++i) {
                const float2 X = b.c[i][col], Y = b.r[i][wave];
                const float tr = fmaf(Y.x, X.x, -Y.y * X.y);
                const float ti = fmaf(Y.x, X.y, Y.y * X.x);
                const float bre = half ? -ti : tr, bim = half ? tr : ti;
#pragma unroll
                for (int t = 0; t < kMfZT; ++t) {
                    const float z = b.z[i][32 * t + col][half];
                    accR[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(z, bre, accR[t], 0, 0, 0);
                    accI[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(z, bim, accI[t], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < kMfZT; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    Sr[t][r] += (double)accR[t][r];
                    Si[t][r] += (double)accI[t][r];
                }
            if (c + 1 < ce) stash(st[(c + 1 - cb) & 1]);
            __syncthreads();
        }
    }
    if (ri >= rlim || ci >= clim) return;
    // output: register r of this lane is row 8 (r / 4) + 4 half + r % 4 of
    // the tile, column col
#pragma unroll
    for (int t = 0; t < kMfZT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int jz = jz0 + 32 * t + 8 * (r / 4) + 4 * half + (r % 4);
            if (jz >= g.nz) continue;
            if (rg.ks == 1) {
                ak_store(a, jx, jy, jz, Sr[t][r], Si[t][r]);
            } else {
                const int64_t idx = ((int64_t)jz * g.ny + jy) * rg.xw + (jx - rg.x0);
                double *q = rg.part + 2 * (layer * rg.count + idx);
                q[0] = Sr[t][r];
                q[1] = Si[t][r];
            }
        }
}

__global__ __launch_bounds__(kAkThreads) void k_ak_reduce(AkArgs a, AkRegion rg)
{
    for (int64_t idx = blockIdx.x * (int64_t)kAkThreads + threadIdx.x; idx < rg.count;
         idx += (int64_t)gridDim.x * kAkThreads) {
        double sr = 0.0, si = 0.0;
        for (int l = 0; l < rg.ks; ++l) {
            sr += rg.part[2 * (l * rg.count + idx)];
            si += rg.part[2 * (l * rg.count + idx) + 1];
        }
        const int jx = rg.x0 + (int)(idx % rg.xw);
        const int jy = (int)((idx / rg.xw) % a.g.ny);
        const int jz = (int)(idx / ((int64_t)rg.xw * a.g.ny));
        ak_store(a, jx, jy, jz, sr, si);
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

int launch_asym_k(const AkArgs &a, const double *xyz, const double *q, Workspace &ws, bool ev,
                  hipStream_t s)
{
    // phase tables padded to a multiple of kMfFlush atoms (padding rows carry Q = 0)
    const int64_t npad = (std::max<int64_t>(a.n, 1) + kMfFlush - 1) / kMfFlush * kMfFlush;
    const int nch = (int)(npad / kMfFlush);
    float2 *ex = ws.get<float2>((size_t)npad * a.g.nxh);
    float2 *ey = ws.get<float2>((size_t)npad * a.g.ny);
    float2 *ezq = ws.get<float2>((size_t)npad * a.g.nz);
    // full 32-column jx tiles with jy rows; the remaining jx (the Nyquist
    // column of an even nx) as rows against 32-column jy tiles.  A region
    // with fewer waves than the chip holds twice over splits its atoms.
    int cus = 0, dev = 0;
    RISM_HIP(hipGetDevice(&dev));
    RISM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int nxm = a.g.nxh / kMfCols * kMfCols, xw = a.g.nxh - nxm;
    const int zt = (a.g.nz + kMfZ - 1) / kMfZ;
    dim3 grids[2];
    AkRegion rg[2];
    for (int yc = 0; yc < 2; ++yc) {
        const int w = yc ? xw : nxm;
        rg[yc] = AkRegion{yc ? nxm : 0, w, 1, (int64_t)w * a.g.ny * a.g.nz, nullptr};
        if (w == 0) continue;
        grids[yc] = yc ? dim3((a.g.ny + kMfCols - 1) / kMfCols, (w + kMfWaves - 1) / kMfWaves, zt)
                       : dim3(w / kMfCols, (a.g.ny + kMfWaves - 1) / kMfWaves, zt);
        const int64_t waves = (int64_t)grids[yc].x * grids[yc].y * grids[yc].z * kMfWaves;
        const int64_t want = (int64_t)12 * std::max(cus, 1);   // 3 waves per SIMD
        rg[yc].ks = (int)std::max<int64_t>(1, std::min<int64_t>(nch, want / waves));
        if (rg[yc].ks > 1) rg[yc].part = ws.get<double>((size_t)2 * rg[yc].ks * rg[yc].count);
        grids[yc].z *= rg[yc].ks;
    }
    if (ws.status()) return ws.status();
    {
        PhaseTimer pt(ev, RISM_PHASE_OTHER, s);
        const int64_t tot = npad * (int64_t)(a.g.nxh + a.g.ny + a.g.nz);
        const int blocks = (int)std::min<int64_t>((tot + kAkThreads - 1) / kAkThreads, 65536);
        hipLaunchKernelGGL(k_phase_tables, blocks, kAkThreads, 0, s, xyz, q, a.n, npad, a.g, ex,
                           ey, ezq);
    }
    AkArgs b = a;
    b.ex = ex;
    b.ey = ey;
    b.ezq = ezq;
    for (int yc = 0; yc < 2; ++yc) {
        if (rg[yc].xw == 0) continue;
        if (yc) {
            PhaseTimer pt(ev, RISM_PHASE_OTHER, s);
            hipLaunchKernelGGL(k_asym_k_mfma<true>, grids[yc], kMfThreads, 0, s, b, rg[yc]);
        } else {
            PhaseTimer pt(ev, RISM_PHASE_RECIP, s);
            hipLaunchKernelGGL(k_asym_k_mfma<false>, grids[yc], kMfThreads, 0, s, b, rg[yc]);
        }
        if (rg[yc].ks > 1) {
            PhaseTimer pt(ev, RISM_PHASE_OTHER, s);
            const int blocks =
                (int)std::min<int64_t>((rg[yc].count + kAkThreads - 1) / kAkThreads, 8192);
            hipLaunchKernelGGL(k_ak_reduce, blocks, kAkThreads, 0, s, b, rg[yc]);
        }
    }
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

}  // namespace rism
