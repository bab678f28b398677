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
#include <type_traits>

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
                                                    double *What, float *Whatf)
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
        Whatf[(size_t)id * np + k] = (float)s;
    }
}

// Parent proxy weights from the children: What_P = sum_c (Mx (x) My (x) Mz)^T What_c,
// M[k][m] = L^P_m(s^c_k).  One workgroup per child writes its term; a second
// kernel adds the (up to 8) terms of each parent in the fixed (z, y, x) order.
__global__ __launch_bounds__(kBlock) void k_adj_up_child(CpLevels L, int lvl, int deg,
                                                         const double *What, double *term)
{
    extern __shared__ double sm[];
    const int n1 = deg + 1, np = n1 * n1 * n1;
    double *M = sm;                  // [3][n1 (k)][n1 (m)]
    double *src = M + 3 * n1 * n1;   // [np]
    double *t1 = src + np;
    double *t2 = t1 + np;
    const int cl = lvl - 1;
    const int q = blockIdx.x;
    const int ci = q % L.cx[cl], cj = (q / L.cx[cl]) % L.cy[cl], ck = q / (L.cx[cl] * L.cy[cl]);
    double pbx[6], cb[6];
    cp_proxy_box(L, lvl, ci >> 1, cj >> 1, ck >> 1, pbx);
    cp_proxy_box(L, cl, ci, cj, ck, cb);
    if (threadIdx.x < 3 * n1) {
        const int ax = threadIdx.x / n1, k = threadIdx.x % n1;
        lagrange_to(cheb_point(pick3(cb, ax), pick3(cb + 3, ax), k, deg), pick3(pbx, ax),
                    pick3(pbx + 3, ax), deg, M + (ax * n1 + k) * n1, 1);
    }
    const int cid = cp_id(L, cl, ci, cj, ck);
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
    // term[m3][m2][m1] = sum_k3 M[2][k3][m3] t2[k3][m2][m1]
    for (int k = threadIdx.x; k < np; k += kBlock) {
        const int m12 = k % (n1 * n1), m3 = k / (n1 * n1);
        double s = 0;
        for (int k3 = 0; k3 < n1; ++k3) s += M[(2 * n1 + k3) * n1 + m3] * t2[k3 * n1 * n1 + m12];
        term[(size_t)q * np + k] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_adj_up_sum(CpLevels L, int lvl, int np,
                                                       const double *term, double *What,
                                                       float *Whatf)
{
    const int q = blockIdx.x;
    const int I = q % L.cx[lvl], J = (q / L.cx[lvl]) % L.cy[lvl], K = q / (L.cx[lvl] * L.cy[lvl]);
    const int cl = lvl - 1;
    const int id = cp_id(L, lvl, I, J, K);
    for (int k = threadIdx.x; k < np; k += kBlock) {
        double s = 0;
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    const int ci = 2 * I + cx, cj = 2 * J + cy, ck = 2 * K + cz;
                    if (ci >= L.cx[cl] || cj >= L.cy[cl] || ck >= L.cz[cl]) continue;
                    s += term[((size_t)(ck * L.cy[cl] + cj) * L.cx[cl] + ci) * np + k];
                }
        What[(size_t)id * np + k] = s;
        Whatf[(size_t)id * np + k] = (float)s;
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ------------------------------------------------------------ atom schedule
// The per-atom kernels below read the grid data (W, w) around their atom.
// They visit the atoms in a spatial order, a counting sort by the level-0
// block that holds the atom (z-major, atoms off the grid clamped to the
// nearest block), and workgroup b takes position (b mod 8) ceil(n/8) + b/8
// of it: consecutive workgroups go to the 8 XCDs in turn, so each XCD works
// through one contiguous stretch of space and its L2 keeps serving it.  The
// order within a block comes from atomics; it only decides which workgroup
// handles an atom, and every atom's result is computed the same way by one
// workgroup, so results do not depend on it.
constexpr int kXcds = 8;

__global__ __launch_bounds__(kBlock) void k_adj_fill(int *p, int n)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_adj_cell(const float4 *rec, int stride_f4, int n,
                                                     CpLevels L, int *cell, int *count)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float4 r0 = rec[(size_t)i * stride_f4];
    const float4 r1 = rec[(size_t)i * stride_f4 + 1];
    const double y[3] = {(double)r0.x + r1.x, (double)r0.y + r1.y, (double)r0.z + r1.z};
    const int nb[3] = {L.cx[0], L.cy[0], L.cz[0]};
    int c[3];
    for (int k = 0; k < 3; ++k) {
        const double f = floor(y[k] / (L.h[k] * L.B));
        c[k] = f >= 0 ? (f <= nb[k] - 1 ? (int)f : nb[k] - 1) : 0;   // NaN -> 0
    }
    const int id = (c[2] * nb[1] + c[1]) * nb[0] + c[0];
    cell[i] = id;
    atomicAdd(&count[id], 1);
}

// In-place exclusive scan of count[0..m) by one workgroup of 1024 threads,
// each owning a contiguous run.
__global__ __launch_bounds__(1024) void k_adj_scan(int *count, int m)
{
    __shared__ int sums[1024];
    const int t = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int b = min(t * per, m), e = min(b + per, m);
    int s = 0;
    for (int i = b; i < e; ++i) s += count[i];
    sums[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? sums[t - off] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    int run = sums[t] - s;
    for (int i = b; i < e; ++i) {
        const int c = count[i];
        count[i] = run;
        run += c;
    }
}

__global__ __launch_bounds__(kBlock) void k_adj_scatter(const int *cell, int n, int *next,
                                                        int *order)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    order[atomicAdd(&next[cell[i]], 1)] = i;
}

// The atom of this workgroup, or -1 for the few padding workgroups.
__device__ __forceinline__ int64_t adj_atom(const int *order, int64_t n)
{
    const int64_t per = (n + kXcds - 1) / kXcds;
    const int64_t pos = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    return pos < n ? order[pos] : -1;
}

// Absolute Chebyshev node coordinates of every cluster's proxy box:
// nodes[id][axis][k], so the walk forms node - atom offsets with one FP64
// subtraction each.
__global__ __launch_bounds__(kBlock) void k_adj_nodes(CpLevels L, int deg, double *nodes)
{
    const int n1 = deg + 1;
    const int ncl = L.off[L.T + 1];
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < ncl * 3 * n1; t += gridDim.x * kBlock) {
        const int id = t / (3 * n1), r = t % (3 * n1), ax = r / n1, k = r % n1;
        int lvl, I, J, K;
        cp_decode(L, id, lvl, I, J, K);
        double pb[6];
        cp_proxy_box(L, lvl, I, J, K, pb);
        nodes[t] = cheb_point(pb[ax], pb[3 + ax], k, deg);
    }
}

struct AdjWalkArgs {
    CpLevels L;
    const float4 *rec;     // staged FP32 records, input order
    int stride_f4;
    int64_t n;
    int deg, np;
    const float *Whatf;    // proxy weights rounded to FP32
    const double *nodes;   // [cluster][3][n + 1] node coordinates
    const float *Wf;       // W on the grid (FP32)
    const int *order;      // spatial order of the atoms
    double *dxyz, *dq;
};

// Waves that share one atom in the adjoint kernels; their partial sums meet
// in LDS and are added in wave order, so the result does not depend on timing.
constexpr int kAdjWaves = kBlock / 64;
constexpr int kAdjMaxDegree = 16;

__device__ __forceinline__ void block_reduce_store(double (*part)[8], const double *v, int nv,
                                                   int lane, int wave)
{
    for (int i = 0; i < nv; ++i) {
        const double s = wave_sum(v[i]);
        if (lane == 0) part[wave][i] = s;
    }
}

// One workgroup per atom: every wave repeats the forward's assignment walk
// (a few hundred MAC tests) and evaluates every kAdjWaves-th of the items it
// meets, an item being an accepted cluster (its proxies) or a level-0 block
// reached unassigned (its grid points).
__global__ __launch_bounds__(kBlock) void k_adj_walk(AdjWalkArgs a)
{
    __shared__ long long stack[kAdjWaves][kStackPerWave];
    __shared__ double part[kAdjWaves][8];
    __shared__ float nodes[kAdjWaves][64];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t atom = adj_atom(a.order, a.n);
    if (atom < 0) return;   // whole workgroup, before any barrier
    const CpLevels &L = a.L;
    const float4 r0 = a.rec[(size_t)atom * a.stride_f4];
    const float4 r1 = a.rec[(size_t)atom * a.stride_f4 + 1];
    const double y[3] = {(double)r0.x + r1.x, (double)r0.y + r1.y, (double)r0.z + r1.z};
    const int n1 = a.deg + 1;
    // q / n1 for 0 <= q < n1^3 as (int)((q + 1/2) / n1) in FP32: the
    // quotient's fractional part stays >= 1/(2 n1) away from an integer
    const float rn1 = 1.f / (float)n1;
    double pot = 0, fx = 0, fy = 0, fz = 0;
    int item = 0;

    // accepted cluster: potential and field of its proxy weights at the atom
    auto far_item = [&](int cid) {
        if (item++ % kAdjWaves != wave) return;
        const float *Wh = a.Whatf + (size_t)cid * a.np;
        // nd[l], l < 3 (n+1): Chebyshev node l % (n+1) of axis l / (n+1),
        // relative to the atom, in the wave's LDS row (LDS reads, unlike
        // shuffles, let the compiler unroll the loops below)
        float *nd = nodes[wave];
        __builtin_amdgcn_wave_barrier();
        if (lane < 3 * n1) {
            const int ax = lane >= 2 * n1 ? 2 : (lane >= n1 ? 1 : 0);
            nd[lane] = (float)(a.nodes[(size_t)cid * 3 * n1 + lane] - (ax == 0 ? y[0] : ax == 1 ? y[1] : y[2]));
        }
        __builtin_amdgcn_wave_barrier();
        // Lanes take (k1, k2) pairs, each running over k3, so dx, dy and
        // their squares are formed once per pass; the weights of one k3 are
        // consecutive.  A pass of 64 pairs walks k3 in step (dz is
        // wave-uniform); a last pass of r < 64 pairs runs 64 / r values of
        // k3 side by side.  Idle lanes run on a clamped index, so the loads
        // of an unrolled stretch carry no lane mask and issue together;
        // their sums are dropped.
        const int P = n1 * n1;
        for (int pb = 0; pb < P; pb += 64) {
            const int r = min(64, P - pb);
            float p = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
            if (r == 64) {
                const int pair = pb + lane;
                const int k2 = (int)(((float)pair + 0.5f) * rn1), k1 = pair - k2 * n1;
                const float dx = nd[k1], dy = nd[n1 + k2];
                const float dxy2 = fmaf(dx, dx, dy * dy);
                const float *col = Wh + pair;
#pragma unroll 4
                for (int k3 = 0; k3 < n1; ++k3) {
                    const float dz = nd[2 * n1 + k3];
                    const float ri = __builtin_amdgcn_rsqf(fmaf(dz, dz, dxy2));
                    const float wr = col[k3 * P] * ri;
                    const float wr3 = wr * ri * ri;
                    p += wr;
                    gx = fmaf(wr3, dx, gx);
                    gy = fmaf(wr3, dy, gy);
                    gz = fmaf(wr3, dz, gz);
                }
                pot += p; fx += gx; fy += gy; fz += gz;
                continue;
            }
            const int G = 64 / r;   // k3 values per pass (uniform)
            const int g = (int)(((float)lane + 0.5f) / (float)r);
            const int pair = pb + lane - g * r;
            const bool act = g < G;
            const int pc = act ? pair : pb;
            const int k2 = (int)(((float)pc + 0.5f) * rn1), k1 = pc - k2 * n1;
            const float dx = nd[k1], dy = nd[n1 + k2];
            const float dxy2 = fmaf(dx, dx, dy * dy);
            const float *col = Wh + pc;
#pragma unroll 4
            for (int k3b = 0; k3b < n1; k3b += G) {
                const int k3 = min(k3b + g, n1 - 1);
                const bool live = act && k3b + g < n1;
                const float dz = nd[2 * n1 + k3];
                const float w = col[k3 * P];
                const float ri = live ? __builtin_amdgcn_rsqf(fmaf(dz, dz, dxy2)) : 0.f;
                const float wr = w * ri;
                const float wr3 = wr * ri * ri;
                p += wr;
                gx = fmaf(wr3, dx, gx);
                gy = fmaf(wr3, dy, gy);
                gz = fmaf(wr3, dz, gz);
            }
            pot += p; fx += gx; fy += gy; fz += gz;
        }
    };

    // level-0 block reached unassigned: direct over its grid points, offsets
    // formed in FP64 and rounded once
    auto direct_item = [&](int I, int J, int K) {
        if (item++ % kAdjWaves != wave) return;
        const int i0 = I * L.B, j0 = J * L.B, k0 = K * L.B;
        const int ex = min(L.B, L.nx - i0), ey = min(L.B, L.ny - j0), ez = min(L.B, L.nz - k0);
        const int P = ex * ey;
        if (P <= 64) {
            // lanes take (x, y) columns of the block, several z per pass
            // when the column count is below 64; unmasked loads as above
            // small quotients in FP32 as in the far items
            const int g = (int)(((float)lane + 0.5f) / (float)P), pair = lane - g * P;
            const int G = (int)((64.5f) / (float)P);
            const bool act = g < G;
            const int lj = (int)(((float)pair + 0.5f) / (float)ex), li = pair - lj * ex;
            const float dx = (float)fma((double)(i0 + li), L.h[0], -y[0]);
            const float dy = (float)fma((double)(j0 + lj), L.h[1], -y[1]);
            const float dxy2 = fmaf(dx, dx, dy * dy);
            const int64_t plane = (int64_t)L.ny * L.nx;
            const float *col = a.Wf + ((int64_t)k0 * L.ny + (j0 + lj)) * L.nx + (i0 + li);
            float p = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
            if (G == 1) {
                // 33 to 64 columns: every lane walks the block's z in step,
                // dz from a per-wave LDS row
                float *dzs = nodes[wave];
                __builtin_amdgcn_wave_barrier();
                if (lane < ez) dzs[lane] = (float)fma((double)(k0 + lane), L.h[2], -y[2]);
                __builtin_amdgcn_wave_barrier();
#pragma unroll 4
                for (int lk = 0; lk < ez; ++lk) {
                    const float dz = dzs[lk];
                    const float d2 = fmaf(dz, dz, dxy2);
                    const float w = col[lk * plane];
                    const float ri = d2 > 0.f ? __builtin_amdgcn_rsqf(d2) : 0.f;
                    const float wr = w * ri;
                    const float wr3 = wr * ri * ri;
                    p += wr;
                    gx = fmaf(wr3, dx, gx);
                    gy = fmaf(wr3, dy, gy);
                    gz = fmaf(wr3, dz, gz);
                }
                if (act) { pot += p; fx += gx; fy += gy; fz += gz; }
                return;
            }
#pragma unroll 4
            for (int lkb = 0; lkb < ez; lkb += G) {
                const int lk = min(lkb + g, ez - 1);
                const bool live = act && lkb + g < ez;
                const float dz = (float)fma((double)(k0 + lk), L.h[2], -y[2]);
                const float w = col[lk * plane];
                const float d2 = fmaf(dz, dz, dxy2);
                const float ri = live && d2 > 0.f ? __builtin_amdgcn_rsqf(d2) : 0.f;
                const float wr = w * ri;
                const float wr3 = wr * ri * ri;
                p += wr;
                gx = fmaf(wr3, dx, gx);
                gy = fmaf(wr3, dy, gy);
                gz = fmaf(wr3, dz, gz);
            }
            pot += p; fx += gx; fy += gy; fz += gz;
            return;
        }
        const int npts = P * ez;
        float p = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        int cnt = 0;
        // lane's point (li, lj, lk) of the block, stepped by 64 points
        const int s1 = 64 % ex, s2 = (64 / ex) % ey, s3 = 64 / (ex * ey);
        int li = lane % ex, lj = (lane / ex) % ey, lk = lane / (ex * ey);
        for (int t = lane; t < npts; t += 64) {
            const int gi = i0 + li, gj = j0 + lj, gk = k0 + lk;
            li += s1; lj += s2; lk += s3;
            if (li >= ex) { li -= ex; ++lj; }
            if (lj >= ey) { lj -= ey; ++lk; }
            const float dx = (float)fma((double)gi, L.h[0], -y[0]);
            const float dy = (float)fma((double)gj, L.h[1], -y[1]);
            const float dz = (float)fma((double)gk, L.h[2], -y[2]);
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
    };

    // The walk: depth first over the clusters that fail the MAC; the (up to
    // 8) children of a popped cluster are classified by lanes 0..7 at once.
    // The stack is wave-uniform: every lane writes the same value.
    long long *st = stack[wave];
    int sp = 0;
    auto enc = [](int lvl, int I, int J, int K) -> long long {
        return ((long long)lvl << 54) | ((long long)I << 36) | ((long long)J << 18) | (long long)K;
    };
    if (L.T == 0)
        direct_item(0, 0, 0);
    else if (cp_mac(L, L.T, 0, 0, 0, y))
        far_item(cp_id(L, L.T, 0, 0, 0));
    else
        st[sp++] = enc(L.T, 0, 0, 0);
    __builtin_amdgcn_wave_barrier();
    while (sp > 0) {
        --sp;
        // every lane holds the same entry: make it scalar, so the walk's
        // indices, CpLevels lookups and counters stay in SGPRs
        const long long cv = st[sp];
        const long long c =
            ((long long)__builtin_amdgcn_readfirstlane((int)(cv >> 32)) << 32) |
            (unsigned)__builtin_amdgcn_readfirstlane((int)cv);
        __builtin_amdgcn_wave_barrier();
        const int lvl = (int)(c >> 54), I = (int)((c >> 36) & 0x3ffff),
                  J = (int)((c >> 18) & 0x3ffff), K = (int)(c & 0x3ffff);
        const int cl = lvl - 1;
        // the children's level extents and first id, read once as scalars
        const int ncx = __builtin_amdgcn_readfirstlane(L.cx[cl]);
        const int ncy = __builtin_amdgcn_readfirstlane(L.cy[cl]);
        const int ncz = __builtin_amdgcn_readfirstlane(L.cz[cl]);
        const int off = __builtin_amdgcn_readfirstlane(cl >= 1 ? L.off[cl] : 0);
        bool valid = false, acc = false;
        if (lane < 8) {
            const int ci = 2 * I + (lane & 1), cj = 2 * J + ((lane >> 1) & 1), ck = 2 * K + (lane >> 2);
            valid = ci < ncx && cj < ncy && ck < ncz;
            acc = valid && cl >= 1 && cp_mac(L, cl, ci, cj, ck, y);
        }
        const unsigned long long vm = __ballot(valid), am = __ballot(acc);
        for (int ch = 7; ch >= 0; --ch) {
            if (!((vm >> ch) & 1)) continue;
            const int ci = 2 * I + (ch & 1), cj = 2 * J + ((ch >> 1) & 1), ck = 2 * K + (ch >> 2);
            if (cl == 0)
                direct_item(ci, cj, ck);
            else if ((am >> ch) & 1)
                far_item(off + (ck * ncy + cj) * ncx + ci);
            else if (sp < kStackPerWave)
                st[sp++] = enc(cl, ci, cj, ck);
        }
        __builtin_amdgcn_wave_barrier();
    }
    const double v[4] = {pot, fx, fy, fz};
    block_reduce_store(part, v, 4, lane, wave);
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[4] = {0, 0, 0, 0};
        for (int w = 0; w < kAdjWaves; ++w)
            for (int i = 0; i < 4; ++i) s[i] += part[w][i];
        const double q = (double)r0.w;
        if (a.dq) a.dq[atom] = s[0];
        if (a.dxyz) {
            a.dxyz[3 * atom] = q * s[1];
            a.dxyz[3 * atom + 1] = q * s[2];
            a.dxyz[3 * atom + 2] = q * s[3];
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
    int off_cap;           // LDS entries reserved for the x offsets
    const int *order;      // spatial order of the atoms
    const double *eps_in;
    double *dxyz, *deps, *dsig;
    int add_xyz;           // dxyz already holds the Coulomb part
};

// Fourth word of a raw (stride 0) buffer resource on gfx9-family GPUs.
constexpr int kBufferWord3 = 0x00020000;

// Grid points of one axis within r of the coordinate y (ih = 1 / spacing):
// the closed index range [lo, hi], empty when lo > hi.  Products by 1/h may
// misplace a point lying exactly at distance r; callers widen r so that such
// points lie beyond every cut-off.
__device__ __forceinline__ void axis_range(double y, double r, double ih, int n, int &lo, int &hi)
{
    lo = max((int)ceil((y - r) * ih), 0);
    hi = min((int)floor((y + r) * ih), n - 1);
}

// One workgroup per atom: the LJ adjoint over the grid points within the
// atom's largest cut-off radius, per site masked by its own radius (UNI: one
// radius for all pairs, a single test).  Wave w takes the z planes w,
// w + kAdjWaves, ... of the cut-off box; in each plane it visits the square
// bounding the sphere's section (2/3 of the box's points), 64 points per
// step over a uniform step count: lanes past the end run on a clamped point
// with a zero kernel, so no load carries a lane mask.  Point offsets come
// from per-axis tables of FP64 differences rounded once to FP32.  Padded
// sites (A = B = 0) read the last real site's plane and add zero.
template <int NS, bool W64, bool UNI>
__global__ __launch_bounds__(kBlock) void k_adj_lj(AdjLjArgs a)
{
    extern __shared__ float offs[];    // [off_cap] x offsets, then y offsets
    __shared__ double part[kAdjWaves][8];
    __shared__ double part2[kAdjWaves][2 * NS];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t atom = adj_atom(a.order, a.n);
    if (atom < 0) return;   // whole workgroup, before any barrier
    const AtomF32<NS> &rc = static_cast<const AtomF32<NS> *>(a.rec)[atom];
    const GridParams &g = a.g;
    const double y[3] = {(double)rc.xh + rc.xl, (double)rc.yh + rc.yl, (double)rc.zh + rc.zl};
    // the sphere is widened by 1e-6 of its radius, far more than FP32
    // rounding of a distance, so that the per-site FP32 masks decide at the edge
    const double R = a.rcut_max * (1.0 + 1e-6);
    const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
    int lo[3], hi[3];
    axis_range(y[0], R, ih[0], g.nx, lo[0], hi[0]);
    axis_range(y[1], R, ih[1], g.ny, lo[1], hi[1]);
    axis_range(y[2], R, ih[2], g.nz, lo[2], hi[2]);
    float *ox = offs, *oy = offs + a.off_cap;
    for (int t = threadIdx.x; t <= hi[0] - lo[0]; t += kBlock)
        ox[t] = (float)fma((double)(lo[0] + t), g.h[0], -y[0]);
    for (int t = threadIdx.x; t <= hi[1] - lo[1]; t += kBlock)
        oy[t] = (float)fma((double)(lo[1] + t), g.h[1], -y[1]);
    __syncthreads();
    float sg6[NS], e24[NS], rc2[NS];
    const void *wp[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const float A = rc.A[s], B = rc.B[s];
        sg6[s] = B > 0.f ? A / B : 0.f;
        e24[s] = A > 0.f ? 6.f * B * B / A : 0.f;
        rc2[s] = rc.rc2[s];
        const int64_t off = (int64_t)min(s, a.ns - 1) * g.m;
        wp[s] = W64 ? (const void *)(static_cast<const double *>(a.w) + off)
                    : (const void *)(static_cast<const float *>(a.w) + off);
    }
    double gx = 0, gy = 0, gz = 0, gE[NS], gS[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) { gE[s] = 0; gS[s] = 0; }
    for (int gk = lo[2] + wave; gk <= hi[2]; gk += kAdjWaves) {
        const double dzd = fma((double)gk, g.h[2], -y[2]);
        const double r2p = R * R - dzd * dzd;
        if (r2p < 0) continue;
        const double half = sqrt(r2p);
        int ilo, ihi, jlo, jhi;
        axis_range(y[0], half, ih[0], g.nx, ilo, ihi);
        axis_range(y[1], half, ih[1], g.ny, jlo, jhi);
        ilo = max(ilo, lo[0]); ihi = min(ihi, hi[0]);
        jlo = max(jlo, lo[1]); jhi = min(jhi, hi[1]);
        if (ilo > ihi || jlo > jhi) continue;
        const int ex = ihi - ilo + 1, ey = jhi - jlo + 1, npl = ex * ey;
        const float dz = (float)dzd;
        const float dz2 = dz * dz;
        // per-site buffer resource (SGPRs) based at the rectangle's first
        // point, covering the rest of the site's grid up to 2 GiB; points
        // add a 32-bit byte offset, and a load past the range returns 0
        const int64_t rect = ((int64_t)gk * g.ny + jlo) * g.nx + ilo;
        constexpr int esz = W64 ? 8 : 4;
        const int32_t nbytes = (int32_t)min((g.m - rect) * esz, (int64_t)0x7fffffff);
        __amdgpu_buffer_rsrc_t rb[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s)
            rb[s] = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<char *>(static_cast<const char *>(wp[s])) + rect * esz, 0, nbytes,
                kBufferWord3);
        const float *oxp = ox + (ilo - lo[0]), *oyp = oy + (jlo - lo[1]);
        // lane's (li, lj) in the plane's rectangle, stepped by 64 points
        // (quotients in FP32: (q + 1/2) / ex stays 1/(2 ex) off an integer)
        const float rex = 1.f / (float)ex;
        int lj = (int)(((float)lane + 0.5f) * rex), li = lane - lj * ex;
        const int qs = (int)(64.5f * rex), rs = 64 - qs * ex;
        const int nit = (npl + 63) >> 6;
        float fx = 0, fy = 0, fz = 0, fE[NS], fS[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) { fE[s] = 0; fS[s] = 0; }
        int cnt = 0;
#pragma unroll 2
        for (int it = 0; it < nit; ++it) {
            const bool valid = lane + (it << 6) < npl;
            const int ljc = min(lj, ey - 1);
            const float dx = oxp[li], dy = oyp[ljc];
            const int p = (ljc * g.nx + li) * esz;
            li += rs;
            lj += qs;
            if (li >= ex) { li -= ex; ++lj; }
            float wv[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (W64) {
                    const auto b = __builtin_amdgcn_raw_buffer_load_b64(rb[s], p, 0, 0);
                    wv[s] = (float)__builtin_bit_cast(double, b);
                } else {
                    wv[s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb[s], p, 0, 0));
                }
            }
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz2));
            const bool ok = valid && d2 > 0.f && (!UNI || d2 < rc2[0]);
            const float r2 = ok ? __builtin_amdgcn_rcpf(d2) : 0.f;
            const float r6 = r2 * r2 * r2;
            float Flj = 0.f;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float ws = UNI || d2 < rc2[s] ? wv[s] : 0.f;
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
    const double v[3] = {gx, gy, gz};
    block_reduce_store(part, v, 3, lane, wave);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double E = wave_sum(gE[s]), Sg = wave_sum(gS[s]);
        if (lane == 0) { part2[wave][2 * s] = E; part2[wave][2 * s + 1] = Sg; }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double sx = 0, sy = 0, sz = 0, e_sum = 0, s_sum = 0;
    for (int w = 0; w < kAdjWaves; ++w) { sx += part[w][0]; sy += part[w][1]; sz += part[w][2]; }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        double E = 0, Sg = 0;
        for (int w = 0; w < kAdjWaves; ++w) { E += part2[w][2 * s]; Sg += part2[w][2 * s + 1]; }
        const double A = (double)rc.A[s], B = (double)rc.B[s];
        const double e_ga = A > 0 ? B * B / (4.0 * A) : 0.0;
        const double sg = B > 0 ? pow(A / B, 1.0 / 6.0) : 0.0;
        e_sum += 2.0 * e_ga * E;
        s_sum += sg > 0 ? 12.0 * e_ga / sg * Sg : 0.0;
    }
    if (a.dxyz) {
        if (a.add_xyz) {
            a.dxyz[3 * atom] += sx;
            a.dxyz[3 * atom + 1] += sy;
            a.dxyz[3 * atom + 2] += sz;
        } else {
            a.dxyz[3 * atom] = sx;
            a.dxyz[3 * atom + 1] = sy;
            a.dxyz[3 * atom + 2] = sz;
        }
    }
    if (a.deps) a.deps[atom] = e_sum / a.eps_in[atom];
    if (a.dsig) a.dsig[atom] = s_sum;
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
    const size_t shm_up = (3 * (size_t)n1 * n1 + 3 * (size_t)np) * sizeof(double);
    if (std::max(shm_up1, shm_up) > (size_t)lds_max) {
        set_error("treecode backward: degree / batch edge too large for the LDS of this device");
        return RISM_E_UNSUPPORTED;
    }
    double *W = ws.get<double>(a.g.m);
    float *Wf = ws.get<float>(a.g.m);
    double *What = ws.get<double>((size_t)(ncl + 1) * np);
    float *Whatf = ws.get<float>((size_t)(ncl + 1) * np);
    double *nodes = ws.get<double>((size_t)(ncl + 1) * 3 * n1);
    // per-child terms of the upward pass, sized for the level-1 clusters
    double *term = L.T >= 2 ? ws.get<double>((size_t)L.cx[1] * L.cy[1] * L.cz[1] * np) : nullptr;
    if (ws.status()) return ws.status();
    {
        PhaseTimer pt(ev, RISM_PHASE_UPWARD, s);
        hipLaunchKernelGGL(k_adj_w, 2048, kBlock, 0, s, a.w, a.w_f64, a.sp.ns, a.g.m, a.sp, a.kc, W, Wf);
        if (L.T >= 1) {
            hipLaunchKernelGGL(k_adj_nodes, std::min((ncl * 3 * n1 + kBlock - 1) / kBlock, 1024),
                               kBlock, 0, s, L, deg, nodes);
            hipLaunchKernelGGL(k_adj_up1, L.cx[1] * L.cy[1] * L.cz[1], kBlock, shm_up1, s, L, deg, W,
                               What, Whatf);
            for (int lvl = 2; lvl <= L.T; ++lvl) {
                hipLaunchKernelGGL(k_adj_up_child, L.cx[lvl - 1] * L.cy[lvl - 1] * L.cz[lvl - 1],
                                   kBlock, shm_up, s, L, lvl, deg, What, term);
                hipLaunchKernelGGL(k_adj_up_sum, L.cx[lvl] * L.cy[lvl] * L.cz[lvl], kBlock, 0, s, L,
                                   lvl, np, term, What, Whatf);
            }
        }
    }
    RISM_HIP(hipGetLastError());
    const int stride_f4 = (int)(rec32_bytes_of(a.sp.ns_pad) / sizeof(float4));
    if (a.n == 0) return RISM_OK;
    if (deg > kAdjMaxDegree) {
        set_error("treecode backward: degree above 16");
        return RISM_E_UNSUPPORTED;
    }
    // LJ gather: per-axis offset tables in LDS, sized for the widest cut-off box
    auto axis_cap = [&](double h, int n) {
        return (int)std::min<double>(n, std::floor(2.0 * a.rmax_lj * (1.0 + 1e-6) / h) + 2.0);
    };
    const int off_cap = axis_cap(a.g.h[0], a.g.nx), off_cap_y = axis_cap(a.g.h[1], a.g.ny);
    const size_t shm_lj = (size_t)(off_cap + off_cap_y) * sizeof(float);
    if ((int64_t)a.g.nx * a.g.ny >= (int64_t(1) << 28)) {
        set_error("treecode backward: grid planes above 2^28 points");
        return RISM_E_UNSUPPORTED;
    }
    if ((a.dxyz || a.deps || a.dsig) && shm_lj + 4096 > (size_t)lds_max) {
        set_error("treecode backward: LJ cut-off box too wide for the LDS of this device");
        return RISM_E_UNSUPPORTED;
    }
    if (a.n > INT32_MAX / 2) {
        set_error("treecode backward: too many atoms");
        return RISM_E_UNSUPPORTED;
    }
    const int n = (int)a.n;
    const int ncell = L.cx[0] * L.cy[0] * L.cz[0];
    int *cell = ws.get<int>(n);
    int *next = ws.get<int>(ncell);
    int *order = ws.get<int>(n);
    if (ws.status()) return ws.status();
    {
        PhaseTimer pt(ev, RISM_PHASE_TREE_BUILD, s);   // atom schedule
        const int nb = (n + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_adj_fill, std::min((ncell + kBlock - 1) / kBlock, 1024), kBlock, 0, s,
                           next, ncell);
        hipLaunchKernelGGL(k_adj_cell, nb, kBlock, 0, s, static_cast<const float4 *>(a.atoms),
                           stride_f4, n, L, cell, next);
        hipLaunchKernelGGL(k_adj_scan, 1, 1024, 0, s, next, ncell);
        hipLaunchKernelGGL(k_adj_scatter, nb, kBlock, 0, s, cell, n, next, order);
    }
    const int nblk = (int)(((int64_t)n + kXcds - 1) / kXcds * kXcds);
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
            wa.Whatf = Whatf;
            wa.Wf = Wf;
            wa.order = order;
            wa.nodes = nodes;
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
            la.off_cap = off_cap;
            la.order = order;
            la.eps_in = a.eps_in;
            la.dxyz = a.dxyz;
            la.deps = a.deps;
            la.dsig = a.dsig;
            la.add_xyz = 1;
            const bool uni = a.opts->lj_tol <= 0 && a.opts->lj_cutoff > 0;
            auto launch = [&](auto ns_c) {
                constexpr int NS = decltype(ns_c)::value;
                auto go = [&](auto kern) { hipLaunchKernelGGL(kern, nblk, kBlock, shm_lj, s, la); };
                if (a.w_f64)
                    uni ? go(k_adj_lj<NS, true, true>) : go(k_adj_lj<NS, true, false>);
                else
                    uni ? go(k_adj_lj<NS, false, true>) : go(k_adj_lj<NS, false, false>);
            };
            switch (a.sp.ns_pad) {
            case 1: launch(std::integral_constant<int, 1>{}); break;
            case 2: launch(std::integral_constant<int, 2>{}); break;
            case 4: launch(std::integral_constant<int, 4>{}); break;
            default: launch(std::integral_constant<int, 8>{}); break;
            }
        }
    }
    RISM_HIP(hipGetLastError());
    st.n_nodes = ncl;
    return RISM_OK;
}

}  // namespace rism
