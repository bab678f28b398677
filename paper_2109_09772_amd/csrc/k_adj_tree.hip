// Adjoint treecode: the transpose of the cluster-particle forward.
//
// Coulomb part.  With W(x) = k_C sum_g q_g w_g(x), the forward tree computes
// Phi(x) = sum_a Q_a G(x, a), where G is 1/|x - y_a| for an atom summed
// directly at x's level-0 block, and otherwise the interpolant (down the
// chain of target clusters) of 1/|s_k - y_a| at the proxies s_k of the
// cluster the atom was assigned to.  Its adjoint runs the same operators
// transposed:
//   1. level-1 proxy weights  What_C[k] = sum_{x in C} L_k(x) W(x)
//      (separable contraction of W over the cluster's points);
//   2. upward through the levels: What_P[m] += sum_k L^P_m(s^C_k) What_C[k];
//   3. per atom, the same walk as the forward's assignment (coarsest level
//      where r_C < theta |y - c_C|): proxies of an accepted cluster give
//        dL/dQ_a += sum_k What_k / |s_k - y_a|,
//        dL/dR_a += Q_a sum_k What_k (s_k - y_a)/|s_k - y_a|^3,
//      and a level-0 block reached without acceptance is summed directly
//      over its grid points with W(x).
// So <W, Phi_tree(Q)> = sum_a Q_a dL/dQ_a holds to rounding: the gradient is
// that of the tree's own approximation.  The assignment is piecewise
// constant in the atom positions; like the LJ cut-off, its jumps are ignored.
//
// LJ part (truncated): each atom gathers the grid points within its largest
// cut-off radius, per site masked by its own radius, as in the direct
// adjoint.
//
// Determinism: every atom is reduced by one wave in a fixed order; no
// floating-point atomics.
#include <cmath>

#include "cheb.h"
#include "cp.h"
#include "pair.h"
#include "tree.h"

namespace rism {

namespace {

constexpr int kStackPerWave = 256;

__global__ __launch_bounds__(kBlock) void k_adj_w(const void *w, int w_f64, int ns, int64_t m,
                                                  SiteParams sp, double kc, double *W, float *Wf)
{
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * kBlock) {
        double s = 0.0;
        for (int g = 0; g < ns; ++g) {
            double v = w_f64 ? static_cast<const double *>(w)[g * m + p]
                             : (double)static_cast<const float *>(w)[g * m + p];
            s += sp.q[g] * v;
        }
        W[p] = kc * s;
        Wf[p] = (float)(kc * s);
    }
}

// Level-1 proxy weights: What[k3][k2][k1] = sum_{z,y,x} Lz[z][k3] Ly[y][k2] Lx[x][k1] W[z][y][x].
__global__ __launch_bounds__(kBlock) void k_adj_up1(CpLevels L, int deg, const double *W,
                                                    double *What)
{
    extern __shared__ double sm[];
    const int n1 = deg + 1, np = n1 * n1 * n1;
    const int q = blockIdx.x;
    const int I = q % L.cx[1], J = (q / L.cx[1]) % L.cy[1], K = q / (L.cx[1] * L.cy[1]);
    const int e = 2 * L.B;
    const int i0 = I * e, j0 = J * e, k0 = K * e;
    const int ex = min(e, L.nx - i0), ey = min(e, L.ny - j0), ez = min(e, L.nz - k0);
    double *Lx = sm;                 // [e][n1]
    double *Ly = Lx + e * n1;
    double *Lz = Ly + e * n1;
    double *T1 = Lz + e * n1;        // [ez][ey][n1]
    double *T2 = T1 + e * e * n1;    // [ez][n1][n1]
    double pb[6];
    cp_proxy_box(L, 1, I, J, K, pb);
    for (int t = threadIdx.x; t < 3 * e; t += kBlock) {
        const int ax = t / e, l = t % e;
        const int ext = ax == 0 ? ex : (ax == 1 ? ey : ez);
        const int base = ax == 0 ? i0 : (ax == 1 ? j0 : k0);
        double *Lt = ax == 0 ? Lx : (ax == 1 ? Ly : Lz);
        if (l < ext)
            lagrange_to((base + l) * pick3(L.h, ax), pick3(pb, ax), pick3(pb + 3, ax), deg,
                        Lt + l * n1, 1);
        else
            for (int k = 0; k < n1; ++k) Lt[l * n1 + k] = 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ez * ey * n1; t += kBlock) {
        const int k1 = t % n1, y = (t / n1) % ey, z = t / (n1 * ey);
        const double *row = W + ((int64_t)(k0 + z) * L.ny + (j0 + y)) * L.nx + i0;
        double s = 0;
        for (int x = 0; x < ex; ++x) s += row[x] * Lx[x * n1 + k1];
        T1[(z * e + y) * n1 + k1] = s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ez * n1 * n1; t += kBlock) {
        const int k1 = t % n1, k2 = (t / n1) % n1, z = t / (n1 * n1);
        double s = 0;
        for (int y = 0; y < ey; ++y) s += T1[(z * e + y) * n1 + k1] * Ly[y * n1 + k2];
        T2[(z * n1 + k2) * n1 + k1] = s;
    }
    __syncthreads();
    const int id = cp_id(L, 1, I, J, K);
    for (int k = threadIdx.x; k < np; k += kBlock) {
        const int k12 = k % (n1 * n1), k3 = k / (n1 * n1);
        double s = 0;
        for (int z = 0; z < ez; ++z) s += T2[z * n1 * n1 + k12] * Lz[z * n1 + k3];
        What[(size_t)id * np + k] = s;
    }
}

// Parent proxy weights from the children: What_P = sum_c (Mx (x) My (x) Mz)^T What_c,
// M[k][m] = L^P_m(s^c_k), children in (z, y, x) order.
__global__ __launch_bounds__(kBlock) void k_adj_up(CpLevels L, int lvl, int deg, double *What)
{
    extern __shared__ double sm[];
    const int n1 = deg + 1, np = n1 * n1 * n1;
    double *M = sm;                  // [3][n1 (k)][n1 (m)]
    double *src = M + 3 * n1 * n1;   // [np]
    double *t1 = src + np;
    double *t2 = t1 + np;
    double *acc = t2 + np;           // [np], each entry owned by one thread
    const int q = blockIdx.x;
    const int I = q % L.cx[lvl], J = (q / L.cx[lvl]) % L.cy[lvl], K = q / (L.cx[lvl] * L.cy[lvl]);
    const int id = cp_id(L, lvl, I, J, K);
    double pbx[6];
    cp_proxy_box(L, lvl, I, J, K, pbx);
    for (int k = threadIdx.x; k < np; k += kBlock) acc[k] = 0.0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const int ci = 2 * I + cx, cj = 2 * J + cy, ck = 2 * K + cz;
                if (ci >= L.cx[lvl - 1] || cj >= L.cy[lvl - 1] || ck >= L.cz[lvl - 1]) continue;
                const int cid = cp_id(L, lvl - 1, ci, cj, ck);
                double cb[6];
                cp_proxy_box(L, lvl - 1, ci, cj, ck, cb);
                __syncthreads();
                if (threadIdx.x < 3 * n1) {
                    const int ax = threadIdx.x / n1, k = threadIdx.x % n1;
                    lagrange_to(cheb_point(pick3(cb, ax), pick3(cb + 3, ax), k, deg), pick3(pbx, ax),
                                pick3(pbx + 3, ax), deg, M + (ax * n1 + k) * n1, 1);
                }
                for (int k = threadIdx.x; k < np; k += kBlock) src[k] = What[(size_t)cid * np + k];
                __syncthreads();
                // t1[k3][k2][m1] = sum_k1 M[0][k1][m1] src[k3][k2][k1]
                for (int k = threadIdx.x; k < np; k += kBlock) {
                    const int m1 = k % n1, rest = k / n1;
                    double s = 0;
                    for (int k1 = 0; k1 < n1; ++k1) s += M[(0 * n1 + k1) * n1 + m1] * src[rest * n1 + k1];
                    t1[k] = s;
                }
                __syncthreads();
                // t2[k3][m2][m1] = sum_k2 M[1][k2][m2] t1[k3][k2][m1]
                for (int k = threadIdx.x; k < np; k += kBlock) {
                    const int m1 = k % n1, m2 = (k / n1) % n1, k3 = k / (n1 * n1);
                    double s = 0;
                    for (int k2 = 0; k2 < n1; ++k2) s += M[(1 * n1 + k2) * n1 + m2] * t1[(k3 * n1 + k2) * n1 + m1];
                    t2[k] = s;
                }
                __syncthreads();
                // What_P[m3][m2][m1] += sum_k3 M[2][k3][m3] t2[k3][m2][m1]
                for (int k = threadIdx.x; k < np; k += kBlock) {
                    const int m12 = k % (n1 * n1), m3 = k / (n1 * n1);
                    double s = acc[k];
                    for (int k3 = 0; k3 < n1; ++k3) s += M[(2 * n1 + k3) * n1 + m3] * t2[k3 * n1 * n1 + m12];
                    acc[k] = s;
                }
            }
    for (int k = threadIdx.x; k < np; k += kBlock) What[(size_t)id * np + k] = acc[k];
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

struct AdjWalkArgs {
    CpLevels L;
    const float4 *rec;     // staged FP32 records, input order
    int stride_f4;
    int64_t n;
    int deg, np;
    const double *What;
    const float *Wf;       // W on the grid (FP32)
    double *dxyz, *dq;
};

// One wave per atom: the forward's assignment walk, proxies or direct points.
__global__ __launch_bounds__(kBlock) void k_adj_walk(AdjWalkArgs a)
{
    __shared__ long long stack[kBlock / 64][kStackPerWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t atom = blockIdx.x * (int64_t)(kBlock / 64) + wave;
    if (atom >= a.n) return;   // whole wave leaves together; no block barrier below
    const CpLevels &L = a.L;
    const float4 r0 = a.rec[(size_t)atom * a.stride_f4];
    const float4 r1 = a.rec[(size_t)atom * a.stride_f4 + 1];
    const double y[3] = {(double)r0.x + r1.x, (double)r0.y + r1.y, (double)r0.z + r1.z};
    const int n1 = a.deg + 1;
    double pot = 0, fx = 0, fy = 0, fz = 0;
    long long *st = stack[wave];
    int sp = 0;
    auto enc = [](int lvl, int I, int J, int K) -> long long {
        return ((long long)lvl << 54) | ((long long)I << 36) | ((long long)J << 18) | (long long)K;
    };
    // the stack is wave-uniform: every lane writes the same value
    st[0] = enc(L.T, 0, 0, 0);
    sp = 1;
    __builtin_amdgcn_wave_barrier();
    while (sp > 0) {
        --sp;
        const long long c = st[sp];
        __builtin_amdgcn_wave_barrier();
        const int lvl = (int)(c >> 54), I = (int)((c >> 36) & 0x3ffff),
                  J = (int)((c >> 18) & 0x3ffff), K = (int)(c & 0x3ffff);
        if (lvl >= 1 && cp_mac(L, lvl, I, J, K, y)) {
            // accepted: potential and field of the cluster's proxy weights
            double pb[6], cc[3], rr;
            cp_proxy_box(L, lvl, I, J, K, pb);
            cp_centre(L, lvl, I, J, K, cc, rr);
            const float yx = (float)(y[0] - cc[0]), yy = (float)(y[1] - cc[1]), yz = (float)(y[2] - cc[2]);
            const double *Wh = a.What + (size_t)cp_id(L, lvl, I, J, K) * a.np;
            // lane l < 3 (n+1) holds Chebyshev node l % (n+1) of axis l / (n+1),
            // relative to the atom; other lanes read it by shuffle
            float node = 0.f;
            if (lane < 3 * n1) {
                const int ax = lane / n1, kk = lane % n1;
                const float yc = ax == 0 ? yx : (ax == 1 ? yy : yz);
                node = (float)(cheb_point(pb[ax], pb[3 + ax], kk, a.deg) - cc[ax]) - yc;
            }
            float p = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
            int cnt = 0;
            for (int k0 = 0; k0 < a.np; k0 += 64) {
                const int k = k0 + lane;
                const int kc = k < a.np ? k : 0;
                const int k1 = kc % n1, k2 = (kc / n1) % n1, k3 = kc / (n1 * n1);
                const float dx = __shfl(node, k1);
                const float dy = __shfl(node, n1 + k2);
                const float dz = __shfl(node, 2 * n1 + k3);
                if (k < a.np) {
                    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float ri = __builtin_amdgcn_rsqf(d2);
                    const float wr = (float)Wh[k] * ri;
                    const float wr3 = wr * ri * ri;
                    p += wr;
                    gx = fmaf(wr3, dx, gx);
                    gy = fmaf(wr3, dy, gy);
                    gz = fmaf(wr3, dz, gz);
                }
                if (++cnt == 8) {
                    pot += p; fx += gx; fy += gy; fz += gz;
                    p = gx = gy = gz = 0.f;
                    cnt = 0;
                }
            }
            pot += p; fx += gx; fy += gy; fz += gz;
        } else if (lvl >= 1) {
            for (int cz = 1; cz >= 0; --cz)
                for (int cy = 1; cy >= 0; --cy)
                    for (int cx = 1; cx >= 0; --cx) {
                        const int ci = 2 * I + cx, cj = 2 * J + cy, ck = 2 * K + cz;
                        if (ci < L.cx[lvl - 1] && cj < L.cy[lvl - 1] && ck < L.cz[lvl - 1] &&
                            sp < kStackPerWave) {
                            st[sp] = enc(lvl - 1, ci, cj, ck);
                            ++sp;
                        }
                    }
            __builtin_amdgcn_wave_barrier();
        } else {
            // level-0 block reached unassigned: direct over its grid points
            const int i0 = I * L.B, j0 = J * L.B, k0 = K * L.B;
            const int ex = min(L.B, L.nx - i0), ey = min(L.B, L.ny - j0), ez = min(L.B, L.nz - k0);
            const int npts = ex * ey * ez;
            const float yxh = r0.x, yyh = r0.y, yzh = r0.z, yxl = r1.x, yyl = r1.y, yzl = r1.z;
            float p = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
            int cnt = 0;
            for (int t = lane; t < npts; t += 64) {
                const int li = t % ex, lj = (t / ex) % ey, lk = t / (ex * ey);
                const int gi = i0 + li, gj = j0 + lj, gk = k0 + lk;
                const double xd = gi * L.h[0], yd = gj * L.h[1], zd = gk * L.h[2];
                const float xh = (float)xd, yh = (float)yd, zh = (float)zd;
                const float dx = (xh - yxh) + ((float)(xd - (double)xh) - yxl);
                const float dy = (yh - yyh) + ((float)(yd - (double)yh) - yyl);
                const float dz = (zh - yzh) + ((float)(zd - (double)zh) - yzl);
                const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float ri = d2 > 0.f ? __builtin_amdgcn_rsqf(d2) : 0.f;
                const float wr = a.Wf[((int64_t)gk * L.ny + gj) * L.nx + gi] * ri;
                const float wr3 = wr * ri * ri;
                p += wr;
                gx = fmaf(wr3, dx, gx);
                gy = fmaf(wr3, dy, gy);
                gz = fmaf(wr3, dz, gz);
                if (++cnt == 8) {
                    pot += p; fx += gx; fy += gy; fz += gz;
                    p = gx = gy = gz = 0.f;
                    cnt = 0;
                }
            }
            pot += p; fx += gx; fy += gy; fz += gz;
        }
    }
    pot = wave_sum(pot);
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    fz = wave_sum(fz);
    if (lane == 0) {
        const double q = (double)r0.w;
        if (a.dq) a.dq[atom] = pot;
        if (a.dxyz) {
            a.dxyz[3 * atom] = q * fx;
            a.dxyz[3 * atom + 1] = q * fy;
            a.dxyz[3 * atom + 2] = q * fz;
        }
    }
}

struct AdjLjArgs {
    GridParams g;
    const void *rec;
    int64_t n;
    int ns;
    const void *w;
    int w_f64;
    double rcut_max;
    const double *eps_in;
    double *dxyz, *deps, *dsig;
    int add_xyz;           // dxyz already holds the Coulomb part
};

// One wave per atom: LJ adjoint over the grid points inside the cut-off box.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_adj_lj(AdjLjArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t atom = blockIdx.x * (int64_t)(kBlock / 64) + wave;
    if (atom >= a.n) return;
    const AtomF32<NS> &rc = static_cast<const AtomF32<NS> *>(a.rec)[atom];
    const GridParams &g = a.g;
    const double y[3] = {(double)rc.xh + rc.xl, (double)rc.yh + rc.yl, (double)rc.zh + rc.zl};
    int lo[3], hi[3];
    const int dims[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        lo[k] = (int)ceil((y[k] - a.rcut_max) / g.h[k]);
        hi[k] = (int)floor((y[k] + a.rcut_max) / g.h[k]);
        lo[k] = lo[k] < 0 ? 0 : lo[k];
        hi[k] = hi[k] > dims[k] - 1 ? dims[k] - 1 : hi[k];
    }
    float sg6[NS], e24[NS], rc2[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const float A = rc.A[s], B = rc.B[s];
        sg6[s] = B > 0.f ? A / B : 0.f;
        e24[s] = A > 0.f ? 6.f * B * B / A : 0.f;
        rc2[s] = rc.rc2[s];
    }
    double gx = 0, gy = 0, gz = 0, gE[NS], gS[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) { gE[s] = 0; gS[s] = 0; }
    if (lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2]) {
        const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
        const int64_t npts = (int64_t)ex * ey * ez;
        float fx = 0, fy = 0, fz = 0, fE[NS], fS[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) { fE[s] = 0; fS[s] = 0; }
        int cnt = 0;
        for (int64_t t = lane; t < npts; t += 64) {
            const int li = (int)(t % ex), lj = (int)((t / ex) % ey), lk = (int)(t / ((int64_t)ex * ey));
            const int gi = lo[0] + li, gj = lo[1] + lj, gk = lo[2] + lk;
            const double xd = gi * g.h[0], yd = gj * g.h[1], zd = gk * g.h[2];
            const float xh = (float)xd, yh = (float)yd, zh = (float)zd;
            const float dx = (xh - rc.xh) + ((float)(xd - (double)xh) - rc.xl);
            const float dy = (yh - rc.yh) + ((float)(yd - (double)yh) - rc.yl);
            const float dz = (zh - rc.zh) + ((float)(zd - (double)zh) - rc.zl);
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const float ri = d2 > 0.f ? __builtin_amdgcn_rsqf(d2) : 0.f;
            const float r2 = ri * ri, r6 = r2 * r2 * r2;
            const int64_t p = ((int64_t)gk * g.ny + gj) * g.nx + gi;
            float Flj = 0.f;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (s >= a.ns) break;
                float ws = a.w_f64 ? (float)static_cast<const double *>(a.w)[s * g.m + p]
                                   : static_cast<const float *>(a.w)[s * g.m + p];
                ws = d2 < rc2[s] ? ws : 0.f;
                const float s6 = sg6[s] * r6;
                const float ws6 = ws * s6;
                const float v = ws6 * (s6 + s6 - 1.f);
                fS[s] += v;
                fE[s] += ws6 * (s6 - 1.f);
                Flj = fmaf(e24[s], v, Flj);
            }
            const float F = Flj * r2;
            fx = fmaf(F, dx, fx);
            fy = fmaf(F, dy, fy);
            fz = fmaf(F, dz, fz);
            if (++cnt == 8) {
                gx += fx; gy += fy; gz += fz;
                fx = fy = fz = 0.f;
#pragma unroll
                for (int s = 0; s < NS; ++s) { gE[s] += fE[s]; gS[s] += fS[s]; fE[s] = fS[s] = 0.f; }
                cnt = 0;
            }
        }
        gx += fx; gy += fy; gz += fz;
#pragma unroll
        for (int s = 0; s < NS; ++s) { gE[s] += fE[s]; gS[s] += fS[s]; }
    }
    gx = wave_sum(gx);
    gy = wave_sum(gy);
    gz = wave_sum(gz);
    double e_sum = 0, s_sum = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double E = wave_sum(gE[s]), Sg = wave_sum(gS[s]);
        const double A = (double)rc.A[s], B = (double)rc.B[s];
        const double e_ga = A > 0 ? B * B / (4.0 * A) : 0.0;
        const double sg = B > 0 ? pow(A / B, 1.0 / 6.0) : 0.0;
        e_sum += 2.0 * e_ga * E;
        s_sum += sg > 0 ? 12.0 * e_ga / sg * Sg : 0.0;
    }
    if (lane == 0) {
        if (a.dxyz) {
            if (a.add_xyz) {
                a.dxyz[3 * atom] += gx;
                a.dxyz[3 * atom + 1] += gy;
                a.dxyz[3 * atom + 2] += gz;
            } else {
                a.dxyz[3 * atom] = gx;
                a.dxyz[3 * atom + 1] = gy;
                a.dxyz[3 * atom + 2] = gz;
            }
        }
        if (a.deps) a.deps[atom] = e_sum / a.eps_in[atom];
        if (a.dsig) a.dsig[atom] = s_sum;
    }
}

}  // namespace

int adjoint_tree(const AdjointArgs &a, Workspace &ws, rism_stats &st, hipStream_t s)
{
    const bool ev = a.opts->flags & RISM_FLAG_PHASE_EVENTS;
    const int B = a.opts->batch_edge;
    const int deg = a.opts->degree;
    const int n1 = deg + 1, np = n1 * n1 * n1;
    CpLevels L;
    if (cp_levels(a.g, B, a.opts->theta, L) != RISM_OK) {
        set_error("treecode backward: grid too large for the target octree");
        return RISM_E_UNSUPPORTED;
    }
    const int ncl = L.T >= 1 ? L.off[L.T + 1] : 0;
    int dev = 0, lds_max = 0;
    RISM_HIP(hipGetDevice(&dev));
    RISM_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t shm_up1 = (3 * (size_t)(2 * B) * n1 + (size_t)(2 * B) * (2 * B) * n1 +
                            (size_t)(2 * B) * n1 * n1) * sizeof(double);
    const size_t shm_up = (3 * (size_t)n1 * n1 + 4 * (size_t)np) * sizeof(double);
    if (std::max(shm_up1, shm_up) > (size_t)lds_max) {
        set_error("treecode backward: degree / batch edge too large for the LDS of this device");
        return RISM_E_UNSUPPORTED;
    }
    double *W = ws.get<double>(a.g.m);
    float *Wf = ws.get<float>(a.g.m);
    double *What = ws.get<double>((size_t)(ncl + 1) * np);
    if (ws.status()) return ws.status();
    {
        PhaseTimer pt(ev, RISM_PHASE_UPWARD, s);
        hipLaunchKernelGGL(k_adj_w, 2048, kBlock, 0, s, a.w, a.w_f64, a.sp.ns, a.g.m, a.sp, a.kc, W, Wf);
        if (L.T >= 1) {
            hipLaunchKernelGGL(k_adj_up1, L.cx[1] * L.cy[1] * L.cz[1], kBlock, shm_up1, s, L, deg, W,
                               What);
            for (int lvl = 2; lvl <= L.T; ++lvl)
                hipLaunchKernelGGL(k_adj_up, L.cx[lvl] * L.cy[lvl] * L.cz[lvl], kBlock, shm_up, s, L,
                                   lvl, deg, What);
        }
    }
    RISM_HIP(hipGetLastError());
    const int stride_f4 = (int)(rec32_bytes_of(a.sp.ns_pad) / sizeof(float4));
    const int nblk = (int)((a.n + 3) / 4);
    {
        PhaseTimer pt(ev, RISM_PHASE_ADJOINT, s);
        if (a.dq || a.dxyz) {
            AdjWalkArgs wa{};
            wa.L = L;
            wa.rec = static_cast<const float4 *>(a.atoms);
            wa.stride_f4 = stride_f4;
            wa.n = a.n;
            wa.deg = deg;
            wa.np = np;
            wa.What = What;
            wa.Wf = Wf;
            wa.dxyz = a.dxyz;
            wa.dq = a.dq;
            hipLaunchKernelGGL(k_adj_walk, nblk, kBlock, 0, s, wa);
        }
        if (a.dxyz || a.deps || a.dsig) {
            AdjLjArgs la{};
            la.g = a.g;
            la.rec = a.atoms;
            la.n = a.n;
            la.ns = a.sp.ns;
            la.w = a.w;
            la.w_f64 = a.w_f64;
            la.rcut_max = a.rmax_lj;
            la.eps_in = a.eps_in;
            la.dxyz = a.dxyz;
            la.deps = a.deps;
            la.dsig = a.dsig;
            la.add_xyz = 1;
            switch (a.sp.ns_pad) {
            case 1: hipLaunchKernelGGL(k_adj_lj<1>, nblk, kBlock, 0, s, la); break;
            case 2: hipLaunchKernelGGL(k_adj_lj<2>, nblk, kBlock, 0, s, la); break;
            case 4: hipLaunchKernelGGL(k_adj_lj<4>, nblk, kBlock, 0, s, la); break;
            default: hipLaunchKernelGGL(k_adj_lj<8>, nblk, kBlock, 0, s, la); break;
            }
        }
    }
    RISM_HIP(hipGetLastError());
    st.n_nodes = ncl;
    return RISM_OK;
}

}  // namespace rism
