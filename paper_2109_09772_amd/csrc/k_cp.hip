// Cluster-particle treecode: the orientation of the paper (Sec. 2.3), where
// the tree is built on the grid targets, written with barycentric Chebyshev
// interpolation on the target clusters instead of Taylor expansions.
//
// Target tree: the implicit octree of the grid.  Level 0 are blocks of B^3
// points (leaves); a level-l cluster is a block of (B 2^l)^3 points, clipped to
// the grid; the top level T is a single cluster covering the grid.
//
// For an atom y and the chain of clusters C_T ... C_1 that contain a target
// leaf, the atom is assigned to the coarsest level l at which it is well
// separated, r_{C_l} < theta |y - c_{C_l}| (the paper's MAC r/R < theta), and
// to the leaf's direct sum if it is well separated at no level >= 1
// (Eq. 10).  Clusters at level >= 1 hold (n+1)^3 proxy values: the far field
// of their assigned atoms evaluated at the Chebyshev points of the cluster
// box.  The proxies are pushed down level by level (each child's proxy
// values += the parent's interpolant evaluated at the child's proxy points),
// and finally interpolated to the grid points of every leaf.  Level 0 sums
// its assigned atoms directly, since a B^3 leaf has fewer points than proxies.
//
// Far field: 1/d (Coulomb, c^lr) and e^{-kappa d}/d (h^lr), FP32 pair
// arithmetic, FP64 accumulation per proxy and in the interpolation passes.
// Short range (LJ within its cut-off, smeared-kernel corrections within R_s)
// is evaluated per leaf for every atom within reach, whatever level the atom
// was assigned to.
#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>

#include "cheb.h"
#include "cp.h"
#include "pair.h"
#include "tree.h"

namespace rism {

namespace {


// ----------------------------------------------------------------- scans

// Exclusive scans in place of up to four arrays of n entries each (one
// launch per step for all of them): tile sums, a scan of the tile sums per
// array (its total to *total[k]), then each tile scanned from LDS with its
// offset added.  Tiles are 2048 entries, 8 per thread.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

struct ScanBatch {
    uint32_t *a[5];
    uint32_t *total[5];
    int n[5], na;
    // optional capacity check: a total above cap[k] (or a set *overflow)
    // sets *bad, which starts at 0
    uint32_t cap[5];
    int *bad;
    const int *overflow;
};

// The capacity check of array k's total.
__device__ __forceinline__ void scan_check(const ScanBatch &b, int k, uint32_t tot)
{
    if (!b.bad) return;
    if (tot > b.cap[k] || (k == 0 && *b.overflow)) atomicOr(b.bad, 1);
}

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(ScanBatch b, uint32_t *bsum,
                                                            int ntiles)
{
    __shared__ uint32_t red[kScanThreads / 64];
    const uint32_t *a = b.a[blockIdx.y];
    const int base = blockIdx.x * kScanTile;
    uint32_t v = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const int i = base + k * kScanThreads + threadIdx.x;
        if (i < b.n[blockIdx.y]) v += a[i];
    }
    v = block_sum_u32(v, red);
    if (threadIdx.x == 0) bsum[blockIdx.y * ntiles + blockIdx.x] = v;
}

__global__ __launch_bounds__(1024) void k_scan_sums(ScanBatch b, uint32_t *bsum, int ntiles)
{
    __shared__ uint32_t sc[1024];
    uint32_t *bs = bsum + blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < ntiles; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < ntiles ? bs[i] : 0u;
        sc[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t u = threadIdx.x >= off ? sc[threadIdx.x - off] : 0u;
            __syncthreads();
            sc[threadIdx.x] += u;
            __syncthreads();
        }
        if (i < ntiles) bs[i] = carry + sc[threadIdx.x] - v;
        carry += sc[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *b.total[blockIdx.x] = carry;
        scan_check(b, blockIdx.x, carry);
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(ScanBatch b, const uint32_t *bsum,
                                                            int ntiles)
{
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t tsum[kScanThreads];
    uint32_t *a = b.a[blockIdx.y];
    const int n = b.n[blockIdx.y];
    const int base = blockIdx.x * kScanTile;
    for (int k = 0; k < kScanPer; ++k) {
        const int j = k * kScanThreads + threadIdx.x;
        tile[j] = base + j < n ? a[base + j] : 0u;
    }
    __syncthreads();
    uint32_t loc[kScanPer], run = 0;
    for (int k = 0; k < kScanPer; ++k) {
        loc[k] = run;
        run += tile[threadIdx.x * kScanPer + k];
    }
    tsum[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t u = threadIdx.x >= off ? tsum[threadIdx.x - off] : 0u;
        __syncthreads();
        tsum[threadIdx.x] += u;
        __syncthreads();
    }
    const uint32_t off0 = bsum[blockIdx.y * ntiles + blockIdx.x] + tsum[threadIdx.x] - run;
    for (int k = 0; k < kScanPer; ++k) tile[threadIdx.x * kScanPer + k] = off0 + loc[k];
    __syncthreads();
    for (int k = 0; k < kScanPer; ++k) {
        const int j = k * kScanThreads + threadIdx.x;
        if (base + j < n) a[base + j] = tile[j];
    }
}

// The whole scan of one array per workgroup (arrays of up to kScanOneMax
// entries): kScanOnePer consecutive entries per thread, a workgroup scan of
// the thread sums, the total to *total[k].
constexpr int kScanOneThreads = 1024;
constexpr int kScanOnePer = 16;
constexpr int kScanOneMax = kScanOneThreads * kScanOnePer;

__global__ __launch_bounds__(kScanOneThreads) void k_scan_one(ScanBatch b)
{
    __shared__ uint32_t wsum[kScanOneThreads / 64];
    uint32_t *a = b.a[blockIdx.x];
    const int n = b.n[blockIdx.x];
    const int per = (n + kScanOneThreads - 1) / kScanOneThreads;
    const int i0 = threadIdx.x * per;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t v[kScanOnePer], run = 0;
#pragma unroll
    for (int k = 0; k < kScanOnePer; ++k) {
        const int i = i0 + k;
        v[k] = k < per && i < n ? a[i] : 0u;
        run += v[k];
    }
    uint32_t x = run;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int w = 0; w < kScanOneThreads / 64; ++w) {
        const uint32_t t = wsum[w];
        base += w < wave ? t : 0u;
        tot += t;
    }
    uint32_t o = base + x - run;
#pragma unroll
    for (int k = 0; k < kScanOnePer; ++k) {
        const int i = i0 + k;
        if (k < per && i < n) a[i] = o;
        o += v[k];
    }
    if (threadIdx.x == 0) {
        *b.total[blockIdx.x] = tot;
        scan_check(b, blockIdx.x, tot);
    }
}

static int scan_batch(const ScanBatch &b, Workspace &ws, hipStream_t s)
{
    if (b.na <= 0) return RISM_OK;
    int nmax = 0;
    for (int k = 0; k < b.na; ++k) nmax = std::max(nmax, b.n[k]);
    if (nmax <= 0) return RISM_OK;
    if (nmax <= kScanOneMax) {
        hipLaunchKernelGGL(k_scan_one, b.na, kScanOneThreads, 0, s, b);
        RISM_HIP(hipGetLastError());
        return RISM_OK;
    }
    const int ntiles = (nmax + kScanTile - 1) / kScanTile;
    uint32_t *bsum = ws.get<uint32_t>((size_t)ntiles * b.na);
    if (!bsum) return ws.status();
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles, b.na), kScanThreads, 0, s, b, bsum, ntiles);
    hipLaunchKernelGGL(k_scan_sums, b.na, 1024, 0, s, b, bsum, ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles, b.na), kScanThreads, 0, s, b, bsum, ntiles);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

// ----------------------------------------------------------------- queries

// Candidate source leaves of every target query.
//  mode 0 (clusters, levels 1..T): leaves reaching the ball around the
//         parent P beyond which every atom is well separated from P
//         (cp_sep_radius), or every leaf for the top cluster;
//  mode 1 (level-0 blocks): leaves reaching the ball of the level-1 ancestor
//         or the short range of the block.
// ----------------------------------------------------------------- tables

// One-axis tables of the target octree, formed once per call (they depend on
// the grid, the batch edge and the degree only): the interpolation matrix
// M[k][m] of every downward step, for each level lvl = 1..T-1, axis and
// cluster index along that axis, and the level-1 basis at every grid
// coordinate of each axis (rounded up to whole level-0 blocks).  One row of
// n + 1 values per thread; the same arithmetic as forming them in place.
struct CpTabArgs {
    CpLevels L;
    int degree, taylor;
    int mrow0[kCpMaxLev + 1][3];   // first M row of (lvl, axis)
    int nrow_m;                    // M rows in all
    int lrow0[3], nrow_l;          // first level-1 basis row of each axis; rows in all
    double *M, *Lg;
    // optional: the input check's flag words of err_n staging workgroups
    // (three each), reduced into err_dst[0] (non-finite input) and err_dst[1]
    // (tolerance), gathered with the lists' counts for one read-back
    const int *err_src;
    int err_n;
    uint32_t *err_dst;
};

// Threads of the neighbour-query workgroups (one wave), which also form the
// tables: the workgroups after the queries, one row per thread.
constexpr int kQueryThreads = 64;
inline int cp_table_blocks(const CpTabArgs &t)
{
    return (t.nrow_m + t.nrow_l + kQueryThreads - 1) / kQueryThreads;
}

inline void cp_tab_layout(const CpLevels &L, int n1, CpTabArgs &t)
{
    int r = 0;
    for (int lvl = 1; lvl < L.T; ++lvl)
        for (int ax = 0; ax < 3; ++ax) {
            t.mrow0[lvl][ax] = r;
            r += (ax == 0 ? L.cx[lvl] : (ax == 1 ? L.cy[lvl] : L.cz[lvl])) * n1;
        }
    t.nrow_m = r;
    r = 0;
    for (int ax = 0; ax < 3; ++ax) {
        t.lrow0[ax] = r;
        r += (ax == 0 ? L.cx[0] : (ax == 1 ? L.cy[0] : L.cz[0])) * L.B;
    }
    t.nrow_l = r;
}

// Row r of the tables; cosk holds cos(k pi / n), k = 0..n.
__device__ __forceinline__ void cp_table_row(const CpTabArgs &a, int r, const double *cosk)
{
    const CpLevels &L = a.L;
    const int n1 = a.degree + 1;
    if (r < a.nrow_m) {
        int lvl = 1, ax = 0;
        for (int l = 1; l < L.T; ++l)
            for (int x = 0; x < 3; ++x)
                if (r >= a.mrow0[l][x]) {
                    lvl = l;
                    ax = x;
                }
        const int rel = r - a.mrow0[lvl][ax], I = rel / n1, k = rel % n1;
        double *row = a.M + (size_t)r * n1;
        if (a.taylor) {
            // C(m, k) delta^(m - k), delta = child centre - parent centre
            const double dl = cp_centre_axis(L, lvl, ax, I) - cp_centre_axis(L, lvl + 1, ax, I >> 1);
            for (int m = 0; m < k; ++m) row[m] = 0.0;
            double c = 1.0;
            for (int m = k; m < n1; ++m) {
                row[m] = c;
                c = c * dl * (double)(m + 1) / (double)(m + 1 - k);
            }
        } else {
            double clo, chi, plo, phi;
            cp_proxy_axis(L, lvl, ax, I, clo, chi);
            cp_proxy_axis(L, lvl + 1, ax, I >> 1, plo, phi);
            lagrange_to_cos(clo + (chi - clo) * 0.5 * (1.0 + cosk[k]), plo, phi, a.degree, cosk,
                            row, 1);
        }
    } else if (r < a.nrow_m + a.nrow_l) {
        const int rl = r - a.nrow_m;
        const int ax = rl >= a.lrow0[2] ? 2 : (rl >= a.lrow0[1] ? 1 : 0);
        const int i = rl - a.lrow0[ax];   // grid coordinate along ax
        const int I1 = (i / L.B) >> 1;     // level-1 cluster along ax
        const double x = i * (ax == 0 ? L.h[0] : (ax == 1 ? L.h[1] : L.h[2]));
        double *row = a.Lg + (size_t)rl * n1;
        if (a.taylor) {   // (x - c)^k about the level-1 centre
            const double dx = x - cp_centre_axis(L, 1, ax, I1);
            double pw = 1.0;
            for (int k = 0; k < n1; ++k, pw *= dx) row[k] = pw;
        } else {          // L_k(x) of the level-1 proxy points
            double lo, hi;
            cp_proxy_axis(L, 1, ax, I1, lo, hi);
            lagrange_to_cos(x, lo, hi, a.degree, cosk, row, 1);
        }
    }
}

// Candidate atoms of a family that its fill workgroup assigns (eight rounds
// of 512); above kAssignExtraMinAtoms atoms the rest go, in chunks of as
// many, to the workgroups of a second launch (k_cp_assign_extra), so that a
// family whose candidates are most of the atoms does not hold up the pass.
// Below it the groups' classification spans the fill launch about as long
// as the largest family, and the second launch would only add its own time
// (at 14,000 atoms the lists took 0.233 ms with it, 0.214 without).
constexpr int kAssignChunk = 4096;
constexpr int64_t kAssignExtraMinAtoms = 32768;

struct CpQueryArgs {
    CpLevels L;
    int mode, nq;
    double rshort;
    const int *begin, *end, *child0, *nchild;
    const double *box;
    const int *n_nodes;
    uint32_t *cnt, *acnt;           // count pass (nq + 1 entries each; acnt optional)
    uint32_t *ecnt;                 // count pass, optional (nq + 1): chunks of
                                    // kAssignChunk candidate atoms after the first
    const uint32_t *off;            // fill pass
    int *list;
    const int *bad;                 // fill pass: lists sized too small, write nothing
    int *overflow;
    int fill;
    int stack_w;   // LDS stack entries (cp_query_stack)
};

// Per-wave DFS stack of the neighbour queries (LDS, one wave per
// workgroup).  A step pops up to 64 nodes from the top and pushes at most 8
// children each; below the newest layer the stack keeps at most one partial
// layer of at most 7 x 64 nodes per tree depth, so a tree of depth D =
// kMortonBits needs at most 448 (D - 1) + 512 = 4544 slots.  Each node is
// also pushed at most once per query (it has one parent), so the tree's node
// capacity bounds the stack as well: the launch sizes the LDS stack to the
// smaller bound, which lets more queries share a CU.
constexpr int kQStackW = 4608;
// Trees of at most this many nodes are scanned flat instead of descended.
constexpr int kQFlatNodes = 256;
static_assert(kQStackW >= 448 * (kMortonBits - 1) + 512, "query stack bound");
inline int cp_query_stack(int cap_nodes) { return cap_nodes < kQStackW ? cap_nodes : kQStackW; }

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

// Families of target clusters (siblings share one query and one pass over
// their candidates): family f < nfam - 1 is the children of the f-th cluster
// at levels 2..T (its parent, at level lp); the last family is the top
// cluster alone (lp = T + 1).
__device__ __forceinline__ void cp_family(const CpLevels &L, int f, int nfam, int &lp, int &I,
                                          int &J, int &K)
{
    if (f == nfam - 1) {
        lp = L.T + 1;
        I = J = K = 0;
    } else {
        cp_decode(L, L.off[2] + f, lp, I, J, K);
    }
}

// One wave per query.  Small trees are scanned flat, node by node; larger
// ones descended: the DFS pops up to 64 nodes at a time (one per lane),
// appends the hit leaves in lane order and pushes the children of the other
// hits.  Either way the candidate order is deterministic.
__device__ __forceinline__ void cp_query(const CpQueryArgs &a, int q, int *stk)
{
    const int lane = threadIdx.x;
    if (a.fill && *a.bad) return;
    if (!a.fill && q == 0 && threadIdx.x == 0) {
        a.cnt[a.nq] = 0;
        if (a.acnt) a.acnt[a.nq] = 0;
        if (a.ecnt) a.ecnt[a.nq] = 0;
    }
    if (q >= a.nq) return;   // the whole wave leaves together
    const CpLevels &L = a.L;
    bool all = false, has_ball = false, has_box = false;
    double bc[3] = {0, 0, 0}, br2 = 0, blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
    if (a.mode == 0) {
        // a family of target clusters: the leaves near their parent
        int lp, I, J, K;
        cp_family(L, q, a.nq, lp, I, J, K);
        if (lp > L.T) {
            all = true;
        } else {
            double r;
            cp_centre(L, lp, I, J, K, bc, r);
            const double rb = cp_sep_radius(L, r);
            br2 = rb * rb;
            has_ball = true;
        }
    } else if (L.T == 0) {
        all = true;   // one level-0 block
    } else {
        // the level-0 blocks of level-1 cluster q: atoms not well separated
        // from it, and atoms within the short range of its box
        const int I = q % L.cx[1], J = (q / L.cx[1]) % L.cy[1], K = q / (L.cx[1] * L.cy[1]);
        double r;
        cp_centre(L, 1, I, J, K, bc, r);
        const double rb = cp_sep_radius(L, r);
        br2 = rb * rb;
        has_ball = true;
        if (a.rshort > 0) {
            cp_box(L, 1, I, J, K, blo, bhi);
            has_box = true;
        }
    }
    const double rs2 = a.rshort * a.rshort;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t o = a.fill ? a.off[q] : 0u;
    uint32_t n = 0, nat = 0;   // wave-uniform running counts of leaves and atoms
    // appends this lane's leaf (lf) of sz atoms in lane order
    auto append = [&](bool lf, int node, int sz) {
        const uint64_t m = __ballot(lf);
        if (!lf) sz = 0;
        const int incl = wave_incl_scan(sz, lane);
        if (lf && a.fill) a.list[o + n + (uint32_t)__popcll(m & lt)] = node;
        n += (uint32_t)__popcll(m);
        nat += (uint32_t)__shfl(incl, 63);
    };
    const int nn = *a.n_nodes;
    if (nn <= kQFlatNodes) {
        // small trees: every node tested directly, in node order, with all
        // loads issued up front (a leaf that meets the query has every
        // ancestor meeting it as well, so this is the set the descent finds)
        constexpr int NCH = kQFlatNodes / 64;
        double nb[NCH][6];
        int nch[NCH], sz[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int node = c * 64 + lane;
            nch[c] = -1;
            sz[c] = 0;
            if (node < nn) {
                nch[c] = a.nchild[node];
                sz[c] = a.end[node] - a.begin[node];
                if (!all)
                    for (int k = 0; k < 6; ++k) nb[c][k] = a.box[6 * node + k];
            }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (c * 64 >= nn) break;   // wave-uniform
            bool lf = nch[c] == 0;
            if (lf && !all) {
                bool hit = has_ball && gap2_point_box(bc, nb[c]) < br2;
                if (!hit && has_box) hit = gap2_box_box(blo, bhi, nb[c]) < rs2;
                lf = hit;
            }
            append(lf, c * 64 + lane, sz[c]);
        }
    } else if (all) {
        // every leaf, in node order
        for (int i0 = 0; i0 < nn; i0 += 64) {
            const int node = i0 + lane;
            const bool lf = node < nn && a.nchild[node] == 0;
            append(lf, node, lf ? a.end[node] - a.begin[node] : 0);
        }
    } else {
        int *st = stk;
        st[0] = 0;   // every lane writes the same value
        int sp = 1;
        while (sp > 0) {
            const int take = sp < 64 ? sp : 64;
            const int base = sp - take;
            const int node = lane < take ? st[base + lane] : -1;
            sp = base;
            bool hit = false;
            if (node >= 0) {
                const double *nb = a.box + 6 * node;
                if (has_ball) hit = gap2_point_box(bc, nb) < br2;
                if (!hit && has_box) hit = gap2_box_box(blo, bhi, nb) < rs2;
            }
            const int nch = node >= 0 ? a.nchild[node] : 0;
            const bool lf = hit && nch == 0;
            append(lf, node, lf ? a.end[node] - a.begin[node] : 0);
            const int nc = (hit && nch > 0) ? nch : 0;
            const int incl = wave_incl_scan(nc, lane);
            const int total = __shfl(incl, 63);
            if (sp + total > a.stack_w) {
                if (lane == 0) *a.overflow = 1;
                break;
            }
            const int c0 = nc > 0 ? a.child0[node] : 0;
            for (int k = 0; k < nc; ++k) st[sp + incl - nc + k] = c0 + k;
            sp += total;
        }
    }
    if (!a.fill && lane == 0) {
        a.cnt[q] = n;
        if (a.acnt) a.acnt[q] = nat;
        if (a.ecnt) a.ecnt[q] = nat > (uint32_t)kAssignChunk ? (nat - 1) / kAssignChunk : 0u;
    }
}

// Both query sets in one launch: workgroups [0, a.nq) take a's queries,
// the next b.nq b's (b.nq may be 0), and any further ones form the per-call
// tables (cp_table_row, one row per thread).
__global__ __launch_bounds__(kQueryThreads) void k_cp_query(CpQueryArgs a, CpQueryArgs b,
                                                            CpTabArgs t)
{
    extern __shared__ int stk[];   // [a.stack_w]
    const int q = blockIdx.x;
    if (q < a.nq) {
        cp_query(a, q, stk);
    } else if (q < a.nq + b.nq) {
        cp_query(b, q - a.nq, stk);
    } else {
        __shared__ double cosk[kMaxDeg + 1];   // cos(k pi / n), shared by the rows
        const int n1 = t.degree + 1;
        if ((int)threadIdx.x < n1) cosk[threadIdx.x] = cos(kPi * threadIdx.x / t.degree);
        __syncthreads();
        const int r = (q - a.nq - b.nq) * kQueryThreads + (int)threadIdx.x;
        if (r < t.nrow_m + t.nrow_l) cp_table_row(t, r, cosk);
        if (t.err_src && q == a.nq + b.nq) {   // the first table workgroup (one wave)
            int f0 = 0, f1 = 0;
            for (int i = threadIdx.x; i < t.err_n; i += kQueryThreads) {
                f0 |= t.err_src[3 * i];
                f1 |= t.err_src[3 * i + 1];
            }
            const bool b0 = __ballot(f0 != 0) != 0, b1 = __ballot(f1 != 0) != 0;
            if (threadIdx.x == 0) {
                t.err_dst[0] = b0 ? 1u : 0u;
                t.err_dst[1] = b1 ? 1u : 0u;
            }
        }
    }
}

// Level-0 blocks are classified in groups: the (up to eight) blocks of one
// level-1 cluster (the one block when the tree has no level 1).  The blocks
// of a group share every ancestor, so an atom assigned to no level >= 1 is
// direct for all of them: one direct list per group.  An atom assigned to
// some level is short-range for each block of the group within whose short
// range it lies: one short list per block.
__host__ __device__ inline int cp_groups(const CpLevels &L)
{
    return L.T >= 1 ? L.cx[1] * L.cy[1] * L.cz[1] : 1;
}

// Group of level-0 block (I, J, K) and its place (0..7) in the group.
__device__ __forceinline__ int cp_group_of(const CpLevels &L, int I, int J, int K, int &child)
{
    child = (I & 1) | ((J & 1) << 1) | ((K & 1) << 2);
    return L.T >= 1 ? ((K >> 1) * L.cy[1] + (J >> 1)) * L.cx[1] + (I >> 1) : 0;
}

// Classification of every candidate atom of a group, once: direct, short-range
// for some of its blocks, or skipped.  One workgroup per group, its candidate
// atoms dealt 256 at a time to the threads in candidate order; every list
// keeps that order.  The direct list of group g starts at aoff[g], the short
// list of its block c at 8 aoff[g] + c (aoff[g + 1] - aoff[g]): each has room
// for all of the group's candidate atoms.
struct CpClassArgs {
    CpLevels L;
    int nq;                    // groups
    double rshort;
    const uint32_t *cand_off;  // candidate leaves of each group (prefix)
    const int *cand;
    const int *begin, *end;
    const float4 *rec;
    int stride_f4;
    const uint32_t *aoff;      // candidate atoms of each group (prefix)
    int *dlist, *slist;
    uint32_t *nd;              // direct atoms per group
    uint32_t *on_grid;         // per group: 1 if a direct atom sits on a grid point
    uint32_t *ns;              // short-range atoms per level-0 block
    uint32_t *cost;            // per level-0 block: its direct and short-range atoms
};

// Threads of the classification, and candidate leaves per LDS window (one
// per thread).
constexpr int kClsThreads = 512;
constexpr int kClsWin = kClsThreads;
constexpr int kClsLists = 9;   // the direct list and eight short lists

// Exclusive scan of v over the workgroup of NT threads, in thread order, and
// the total.  `ws` holds NT / 64 ints; the call contains two barriers.
template <int NT>
__device__ __forceinline__ int group_excl_scan(int v, int *ws, int &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int incl = wave_incl_scan(v, lane);
    if (lane == 63) ws[wave] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int x = ws[w];
        base += w < wave ? x : 0;
        tot += x;
    }
    __syncthreads();   // ws is rewritten by the next scan
    total = tot;
    return base + incl - v;
}

// Offsets of NL ordered compactions over the NW waves of a workgroup, from
// the per-wave counts cnt[l][w] in LDS: lane l < NL of every wave gets list
// l's count in the waves before its own (o) and over all waves (tot), so that
// each wave forms the sums once, in parallel over the lists, and reads them
// back per list with lane_word.
template <int NL, int NW>
__device__ __forceinline__ void list_offsets(const uint32_t *cnt, int lane, int wave, uint32_t &o,
                                             uint32_t &tot)
{
    o = tot = 0;
    if (lane < NL) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t c = cnt[lane * NW + w];
            o += w < wave ? c : 0u;
            tot += c;
        }
    }
}

// Lane l's value of v (wave-uniform result).
__device__ __forceinline__ uint32_t lane_word(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// Set bits of the wave mask m below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One workgroup of kClsThreads threads classifies group g.
__device__ __forceinline__ void cp_classify_group(const CpClassArgs &a, int g)
{
    constexpr int NW = kClsThreads / 64;
    __shared__ int beg[kClsWin];
    __shared__ int pre[kClsWin + 1];
    __shared__ int ws[NW];
    __shared__ uint32_t cnt[2][kClsLists][NW];
    __shared__ CpMac mac[kCpMaxLev + 1];   // the group's ancestors, levels 1..T
    __shared__ double cbox[8][6];          // its blocks' boxes (empty if absent)
    __shared__ int cleaf[8];               // their ids (-1 if absent)
    __shared__ int on_any;                 // a direct atom sits on a grid point
    const CpLevels &L = a.L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int I1 = 0, J1 = 0, K1 = 0;
    if (L.T >= 1) {
        I1 = g % L.cx[1];
        J1 = (g / L.cx[1]) % L.cy[1];
        K1 = g / (L.cx[1] * L.cy[1]);
    }
    if (tid >= 1 && tid <= L.T) {
        const int sh = tid - 1;
        cp_mac_terms(L, tid, I1 >> sh, J1 >> sh, K1 >> sh, mac[tid]);
    }
    if (tid < 8) {
        const int I = 2 * I1 + (tid & 1), J = 2 * J1 + ((tid >> 1) & 1), K = 2 * K1 + (tid >> 2);
        const bool in = (L.T >= 1 || tid == 0) && I < L.cx[0] && J < L.cy[0] && K < L.cz[0];
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        if (in) cp_box(L, 0, I, J, K, lo, hi);
        for (int k = 0; k < 3; ++k) {
            cbox[tid][k] = lo[k];
            cbox[tid][3 + k] = hi[k];
        }
        cleaf[tid] = in ? (K * L.cy[0] + J) * L.cx[0] + I : -1;
    }
    if (tid == 0) on_any = 0;
    __syncthreads();
    const double rs2 = a.rshort * a.rshort;
    const uint32_t base = a.aoff[g], na = a.aoff[g + 1] - base;
    uint32_t nl[kClsLists];   // workgroup-uniform list lengths
#pragma unroll
    for (int l = 0; l < kClsLists; ++l) nl[l] = 0;
    const int c0 = (int)a.cand_off[g], c1 = (int)a.cand_off[g + 1];
    for (int cw = c0; cw < c1; cw += kClsWin) {
        // window of candidate leaves: first atom and atom prefix, in list order
        const int nw = min(kClsWin, c1 - cw);
        int sz = 0;
        if (tid < nw) {
            const int leaf = a.cand[cw + tid];
            beg[tid] = a.begin[leaf];
            sz = a.end[leaf] - a.begin[leaf];
        }
        int run;
        const int ex = group_excl_scan<kClsThreads>(sz, ws, run);
        if (tid < nw) pre[tid] = ex;
        if (tid == 0) pre[nw] = run;
        __syncthreads();
        // the window's atoms, one per thread per round
        for (int t0 = 0, par = 0; t0 < run; t0 += kClsThreads, par ^= 1) {
            const int t = t0 + tid;
            uint32_t cls = 0;   // bit 0: direct; bit 1 + c: short-range for block c
            int i = 0;
            if (t < run) {
                int lo = 0, hi = nw - 1;   // last k with pre[k] <= t
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                i = beg[lo] + (t - pre[lo]);
                double y[3];
                atom_pos(a.rec, a.stride_f4, i, y);
                int lvl = 0;   // coarsest ancestor at which y is well separated
                for (int l = L.T; l >= 1; --l)
                    if (cp_mac_at(L, mac[l], y)) {
                        lvl = l;
                        break;
                    }
                if (lvl == 0) {
                    cls = 1u;
                    if (a.rec[(size_t)i * a.stride_f4 + 1].w != 0.f) on_any = 1;   // on_grid
                } else {
                    // the blocks' boxes share their extents along each axis
                    // (block c takes the lower or upper one by bit k of c), so
                    // the gaps are formed once per axis and extent; a block
                    // beyond the grid has an empty box and an infinite gap
                    double gg[3][2];
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int c = h << k;
                            gg[k][h] = fmax(0.0, fmax(cbox[c][k] - y[k], y[k] - cbox[c][3 + k]));
                        }
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const double gx = gg[0][c & 1], gy = gg[1][(c >> 1) & 1], gz = gg[2][c >> 2];
                        const double g2 = fma(gz, gz, fma(gy, gy, gx * gx));
                        if (g2 < rs2) cls |= 2u << c;
                    }
                }
            }
            // ordered compaction of every list over the workgroup: wave counts
            // through LDS (two count buffers alternate, so one barrier per
            // round suffices)
            uint64_t m[kClsLists];
#pragma unroll
            for (int l = 0; l < kClsLists; ++l) {
                m[l] = __ballot((cls >> l) & 1u);
                if (lane == 0) cnt[par][l][wave] = (uint32_t)__popcll(m[l]);
            }
            __syncthreads();
            uint32_t ol, tl;
            list_offsets<kClsLists, NW>(&cnt[par][0][0], lane, wave, ol, tl);
#pragma unroll
            for (int l = 0; l < kClsLists; ++l) {
                if ((cls >> l) & 1u) {
                    const uint32_t at = nl[l] + lane_word(ol, l) + lanes_below(m[l]);
                    if (l == 0) a.dlist[base + at] = i;
                    else a.slist[8 * (size_t)base + (size_t)(l - 1) * na + at] = i;
                }
                nl[l] += lane_word(tl, l);
            }
        }
        __syncthreads();   // the window is read before the next one is written
    }
    if (tid == 0) {
        a.nd[g] = nl[0];
        a.on_grid[g] = on_any;   // set before the last barrier of the window loop
    }
    if (tid < 8 && cleaf[tid] >= 0) {
        uint32_t nsc = 0;
#pragma unroll
        for (int l = 1; l < kClsLists; ++l) nsc = l - 1 == tid ? nl[l] : nsc;
        a.ns[cleaf[tid]] = nsc;
        a.cost[cleaf[tid]] = nl[0] + nsc;
    }
}

// Launch orders: work items sorted by decreasing cost (c1 + c2, in
// power-of-two classes), so that the heaviest items start first and the light
// ones fill the end of the launch.  Results do not depend on the order.  One
// workgroup per order.
constexpr int kCostClasses = 33;
constexpr int kPlanThreads = 1024;
// Atoms per far work item at most: a cluster's assigned atoms are swept in
// runs of this many, one workgroup each (kSweepGroups ranges of kBlock).
constexpr int kItemAtoms = 1024;
// The Taylor sweep takes one atom per wave at a time (four waves), through
// recurrences of dependent steps: runs of 64 atoms give it more workgroups.
constexpr int kTaylorItemAtoms = 64;
__device__ __forceinline__ int cost_class(uint32_t c)
{
    return c == 0 ? 0 : 32 - __clz(c);
}
struct OrderJob {
    int n;                         // items (an upper bound if n_dev is set)
    const uint32_t *n_dev;         // optional: item count on the device
    const uint32_t *c1, *c2;       // costs (c2 optional)
    int *order;
};
__device__ __forceinline__ void order_by_cost(const OrderJob &j)
{
    __shared__ unsigned int cnt[kCostClasses];
    const uint32_t *c1 = j.c1, *c2 = j.c2;
    int *order = j.order;
    int n = j.n;
    if (j.n_dev) n = min(n, (int)*j.n_dev);
    __syncthreads();   // a previous order of this workgroup is done with cnt
    if (threadIdx.x < kCostClasses) cnt[threadIdx.x] = 0u;
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += blockDim.x)
        atomicAdd(&cnt[cost_class(c1[q] + (c2 ? c2[q] : 0u))], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int run = 0;
        for (int c = kCostClasses - 1; c >= 0; --c) {
            const unsigned int k = cnt[c];
            cnt[c] = run;
            run += k;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += blockDim.x)
        order[atomicAdd(&cnt[cost_class(c1[q] + (c2 ? c2[q] : 0u))], 1u)] = q;
}

// Far work items: each cluster's assigned atoms in runs of at most amax (at
// least one item per cluster, so that every cluster's far field is formed),
// numbered cluster by cluster; item_off[cl] is the first item of cluster cl.
// A cluster's atoms come in pieces, one per assignment chunk of its family
// (chunk c from position c kAssignChunk of the cluster's region on).
struct CpItemArgs {
    CpLevels L;
    int ncl, nfam;
    const uint32_t *n;     // assigned atoms per cluster (chunk 0)
    const uint32_t *eoff;  // extra chunks before each family (prefix), or null
    const uint32_t *pc;    // atoms of each extra chunk per child (CpAssignArgs::pc)
    uint32_t amax;         // atoms per item at most
    uint32_t *item_off;    // [ncl + 1]
    int *it_cl;            // cluster of each item
    uint32_t *it_a0;       // first atom of the item within its cluster's region
    uint32_t *it_na;       // atoms of the item
    uint32_t *n_items;     // items in all
};

// Cluster cl's family and its place (child) in it.
__device__ __forceinline__ void cp_family_of(const CpLevels &L, int nfam, int cl, int &f, int &j)
{
    int lvl, I, J, K;
    cp_decode(L, cl, lvl, I, J, K);
    if (lvl >= L.T) {
        f = nfam - 1;
        j = 0;
    } else {
        f = cp_id(L, lvl + 1, I >> 1, J >> 1, K >> 1) - L.off[2];
        j = (I & 1) | ((J & 1) << 1) | ((K & 1) << 2);
    }
}

// The items of a piece of count atoms from position first: runs of at most
// amax atoms, each passed to emit(a0, na); returns their number.
template <class F>
__device__ __forceinline__ uint32_t piece_items(uint32_t first, uint32_t count, uint32_t amax,
                                                F emit)
{
    uint32_t k = 0;
    for (uint32_t u = 0; u * amax < count; ++u, ++k) emit(first + u * amax, min(amax, count - u * amax));
    return k;
}

__device__ __forceinline__ void cp_make_items(const CpItemArgs &a)
{
    __shared__ uint32_t wsum[kPlanThreads / 64];
    __shared__ uint32_t carry;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < a.ncl; c0 += kPlanThreads) {
        const int cl = c0 + tid;
        const uint32_t na = cl < a.ncl ? a.n[cl] : 0u;
        int f = 0, jc = 0;
        uint32_t e0 = 0, e1 = 0;   // the family's extra chunks
        if (cl < a.ncl && a.eoff) {
            cp_family_of(a.L, a.nfam, cl, f, jc);
            e0 = a.eoff[f];
            e1 = a.eoff[f + 1];
        }
        uint32_t k = 0;
        if (cl < a.ncl) {
            k = (na + a.amax - 1) / a.amax;
            for (uint32_t e = e0; e < e1; ++e) k += (a.pc[8 * (size_t)e + jc] + a.amax - 1) / a.amax;
            k = max(1u, k);
        }
        uint32_t x = k;   // inclusive scan over the workgroup
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t base = carry, tot = 0;
        for (int w = 0; w < kPlanThreads / 64; ++w) {
            base += w < wave ? wsum[w] : 0u;
            tot += wsum[w];
        }
        const uint32_t first = base + x - k;
        if (cl < a.ncl) {
            a.item_off[cl] = first;
            uint32_t w = first;
            auto emit = [&](uint32_t a0, uint32_t n_at) {
                a.it_cl[w] = cl;
                a.it_a0[w] = a0;
                a.it_na[w] = n_at;
                ++w;
            };
            piece_items(0u, na, a.amax, emit);
            for (uint32_t e = e0; e < e1; ++e)
                piece_items((e - e0 + 1) * (uint32_t)kAssignChunk, a.pc[8 * (size_t)e + jc], a.amax,
                            emit);
            if (w == first) emit(0u, 0u);   // an empty cluster still has its item
        }
        __syncthreads();   // every thread has read carry and wsum
        if (tid == 0) carry += tot;
        __syncthreads();
    }
    if (tid == 0) {
        a.item_off[a.ncl] = carry;
        *a.n_items = carry;
    }
}

// The launch plan after the lists: workgroup 0 orders the level-0 blocks;
// workgroup 1 (with clusters) forms the far work items and orders them.
// Workgroup 0 first copies the call's nflags flag words to host_flags
// (mapped pinned host memory), which the host reads after the call's last
// kernel, without a copy of its own.
__global__ __launch_bounds__(kPlanThreads) void k_cp_plan(OrderJob leaves, CpItemArgs items,
                                                         OrderJob item_order, const int *bad,
                                                         const uint32_t *flags,
                                                         uint32_t *host_flags, int nflags)
{
    if (blockIdx.x == 0 && host_flags && (int)threadIdx.x < nflags) {
        // system-scope stores into coherent host memory, complete before the
        // wave ends: the event the host waits on needs no cache write-back
        __hip_atomic_store(&host_flags[threadIdx.x], flags[threadIdx.x], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
        __builtin_amdgcn_s_waitcnt(0);
    }
    if (*bad) return;
    if (blockIdx.x == 0) {
        order_by_cost(leaves);
    } else {
        cp_make_items(items);
        __syncthreads();   // the items are written before they are ordered
        order_by_cost(item_order);
    }
}

// Far-field assignment by families: the children of one parent cluster share
// their candidates (the leaves near the parent), so each candidate atom is
// read and tested once for all of them; the top cluster forms a family of its
// own, every leaf a candidate.  An atom belongs to a child when the child
// satisfies the MAC and the parent and its ancestors do not (the coarsest
// cluster on the atom's chain that satisfies it).  Child j's assigned atoms
// are written, in candidate order, as (position relative to the child's
// centre, charge) from 8 aoff[f] + j (aoff[f + 1] - aoff[f]) on, where aoff
// is the prefix of the families' candidate atoms; the counts go to n[cl], the
// first positions to slot[cl].
struct CpAssignArgs {
    CpLevels L;
    int nfam;                  // families: parents at levels 2..T, then the top cluster
    const uint32_t *cand_off;  // candidate leaves of each family (prefix)
    const int *cand;
    const int *begin, *end;
    const float4 *rec;
    int stride_f4;
    const uint32_t *aoff;      // candidate atoms of each family (prefix)
    float4 *abuf;              // assigned atoms
    uint32_t *n;               // assigned atoms per cluster
    uint32_t *slot;            // first position of each cluster's atoms in abuf
    unsigned long long *work;  // optional: (atom, proxy) pairs
    int np;
    double psc;                // scale of the assigned atoms' positions and charges
                               // (CpSweepArgs::psc)
    // families of more than kAssignChunk candidate atoms: chunk c >= 1 (atoms
    // [c, c + 1) kAssignChunk in candidate order) is extra chunk
    // eoff[f] + c - 1, assigned by k_cp_assign_extra
    const uint32_t *eoff;      // [nfam + 1] extra chunks before each family (prefix)
    uint32_t *apre;            // per candidate leaf (as cand): atoms before it in its
                               // family's order, written by chunk 0 when there are extra
                               // chunks; or null
    uint32_t *pc;              // [8 per extra chunk]: its atoms assigned to each child
    const int *bad;
};

// One workgroup of NT threads assigns chunk c of family f's candidate atoms
// (atoms [c, c + 1) kAssignChunk in candidate order; chunk 0 is the fill
// workgroup's, extra chunk e = eoff[f] + c - 1 a workgroup of the extra
// launch), windows of NT candidate leaves at a time, their atoms dealt NT at a
// time to the threads.  Child j's atoms of the chunk go to its part of the
// family's region from position c kAssignChunk on, in candidate order.
template <int NT>
__device__ __forceinline__ void cp_assign_family(const CpAssignArgs &a, int f, int c, int e)
{
    constexpr int NW = NT / 64;
    __shared__ int beg[NT];
    __shared__ int pre[NT + 1];
    __shared__ int ws[NW];
    __shared__ uint32_t wcnt[2][8][NW];
    __shared__ CpMac mac[kCpMaxLev + 1];   // the parent and its ancestors, levels lp..T
    __shared__ CpMac cmac[8];              // the children
    __shared__ double ccen64[8][3];        // their centres
    __shared__ int cid[8];                 // their cluster ids (-1: beyond the grid)
    const CpLevels &L = a.L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int lp, Ip, Jp, Kp;
    cp_family(L, f, a.nfam, lp, Ip, Jp, Kp);
    const int lc = lp - 1;   // the children's level
    if (tid >= lp && tid <= L.T) {
        const int sh = tid - lp;
        cp_mac_terms(L, tid, Ip >> sh, Jp >> sh, Kp >> sh, mac[tid]);
    }
    if (tid >= 64 && tid < 72) {
        const int j = tid - 64;
        const int I = lp > L.T ? 0 : 2 * Ip + (j & 1), J = lp > L.T ? 0 : 2 * Jp + ((j >> 1) & 1);
        const int K = lp > L.T ? 0 : 2 * Kp + (j >> 2);
        const bool in = (lp <= L.T || j == 0) && I < L.cx[lc] && J < L.cy[lc] && K < L.cz[lc];
        cid[j] = in ? cp_id(L, lc, I, J, K) : -1;
        if (in) {
            cp_mac_terms(L, lc, I, J, K, cmac[j]);
            double cc[3], rr;
            cp_centre(L, lc, I, J, K, cc, rr);
            for (int k = 0; k < 3; ++k) ccen64[j][k] = cc[k];
        }
    }
    __syncthreads();
    const uint32_t base0 = a.aoff[f], naf = a.aoff[f + 1] - base0;
    const uint32_t alo = (uint32_t)c * kAssignChunk;
    // (without extra chunks, chunk 0 is every candidate)
    const uint32_t ahi = a.eoff ? min(naf, alo + (uint32_t)kAssignChunk) : naf;
    const bool write_pre = c == 0 && a.apre && naf > (uint32_t)kAssignChunk;
    float4 *out = a.abuf + 8 * (size_t)base0 + alo;
    uint32_t filled[8];   // workgroup-uniform
#pragma unroll
    for (int j = 0; j < 8; ++j) filled[j] = 0;
    const int c0 = (int)a.cand_off[f], c1 = (int)a.cand_off[f + 1];
    int cstart = c0;
    uint32_t wbase = 0;   // the family's atoms before the window (workgroup-uniform)
    if (c > 0) {
        // the chunk's first candidate leaf: the last with apre <= alo
        __shared__ int kstart;
        if (tid == 0) {
            int lo = c0, hi = c1 - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.apre[mid] <= alo) lo = mid;
                else hi = mid - 1;
            }
            kstart = lo;
        }
        __syncthreads();
        cstart = kstart;
        wbase = a.apre[cstart];
    }
    // (chunk 0 of a family with extra chunks runs through every window, for
    // the prefixes; the others stop after their chunk's last atom)
    for (int cw = cstart; cw < c1 && (write_pre || wbase < ahi); cw += NT) {
        // window of candidate leaves: first atom and atom prefix, in list order
        const int nw = min(NT, c1 - cw);
        int sz = 0;
        if (tid < nw) {
            const int leaf = a.cand[cw + tid];
            const int b = a.begin[leaf];
            beg[tid] = b;
            sz = a.end[leaf] - b;
        }
        int run;
        const int ex = group_excl_scan<NT>(sz, ws, run);
        if (tid < nw) pre[tid] = ex;
        if (tid == 0) pre[nw] = run;
        if (write_pre && tid < nw) a.apre[cw + tid] = wbase + (uint32_t)ex;
        __syncthreads();
        // the window's atoms within the chunk: [tlo, thi) of its run
        const uint32_t wend = wbase + (uint32_t)run;
        const uint32_t glo = max(wbase, alo), ghi = min(wend, ahi);
        const int tlo = (int)(glo - wbase), thi = ghi > glo ? (int)(ghi - wbase) : tlo;
        wbase = wend;
        for (int t0 = tlo, par = 0; t0 < thi; t0 += NT, par ^= 1) {
            const int t = t0 + tid;
            uint32_t acc = 0;   // bit j: assigned to child j
            double y[3] = {0.0, 0.0, 0.0};
            float q = 0.f;
            if (t < thi) {
                int lo = 0, hi = nw - 1;   // last k with pre[k] <= t
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                const int i = beg[lo] + (t - pre[lo]);
                atom_pos(a.rec, a.stride_f4, i, y);
                q = a.rec[(size_t)i * a.stride_f4].w;
                // well separated from none of the parent's chain ...
                bool up = true;
                for (int l = lp; up && l <= L.T; ++l) up = !cp_mac_at(L, mac[l], y);
                // ... and from the child
                if (up)
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (cid[j] >= 0 && cp_mac_at(L, cmac[j], y)) acc |= 1u << j;
            }
            // ordered compaction of every child's list (two count buffers
            // alternate: one barrier a round)
            uint64_t m[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                m[j] = __ballot((acc >> j) & 1u);
                if (lane == 0) wcnt[par][j][wave] = (uint32_t)__popcll(m[j]);
            }
            __syncthreads();
            uint32_t oj, tj;
            list_offsets<8, NW>(&wcnt[par][0][0], lane, wave, oj, tj);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if ((acc >> j) & 1u) {
                    const float4 v = make_float4((float)((y[0] - ccen64[j][0]) * a.psc),
                                                 (float)((y[1] - ccen64[j][1]) * a.psc),
                                                 (float)((y[2] - ccen64[j][2]) * a.psc),
                                                 (float)((double)q * a.psc));
                    out[(size_t)j * naf + filled[j] + lane_word(oj, j) + lanes_below(m[j])] = v;
                }
                filled[j] += lane_word(tj, j);   // workgroup-uniform
            }
        }
        __syncthreads();   // the window is read before the next one is written
    }
    if (tid < 8) {
        uint32_t fj = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) fj = j == tid ? filled[j] : fj;
        if (c > 0) {
            a.pc[8 * (size_t)e + tid] = fj;
        } else if (cid[tid] >= 0) {
            a.n[cid[tid]] = fj;
            a.slot[cid[tid]] = 8 * base0 + (uint32_t)tid * naf;
        }
    }
    if (tid == 0 && a.work) {
        unsigned long long tot = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) tot += filled[j];
        atomicAdd(a.work, tot * (unsigned long long)a.np);
    }
}

// Fill pass of the neighbour queries with the work that reads their lists:
// workgroups [0, qc.nq) query a family of target clusters and assign their
// far-field atoms, the rest query a group of level-0 blocks and classify its
// near field.  The query runs on the first wave; the whole workgroup then reads
// the list it wrote.
constexpr int kFillThreads = kClsThreads;

__global__ __launch_bounds__(kFillThreads, 4) void k_cp_fill(CpQueryArgs qc, CpQueryArgs ql,
                                                         CpAssignArgs aa, CpClassArgs ca)
{
    extern __shared__ int stk[];   // [qc.stack_w]
    if (*qc.bad) return;           // whole workgroup: lists sized too small
    const int q = blockIdx.x;
    if (q < qc.nq) {
        if (threadIdx.x < 64) cp_query(qc, q, stk);
        __syncthreads();
        cp_assign_family<kFillThreads>(aa, q, 0, 0);
    } else {
        if (threadIdx.x < 64) cp_query(ql, q - qc.nq, stk);
        __syncthreads();
        cp_classify_group(ca, q - qc.nq);
    }
}

// Extra chunks of the families with more than kAssignChunk candidate atoms
// (after k_cp_fill, which wrote their candidate lists and prefixes): one
// workgroup per chunk, grid from an upper bound (the workgroups past the
// device's count leave at once).  Workgroup e takes the family f with
// eoff[f] <= e < eoff[f + 1], found in two rounds of loads.
__global__ __launch_bounds__(kFillThreads, 4) void k_cp_assign_extra(CpAssignArgs aa)
{
    if (*aa.bad) return;   // whole workgroup: lists sized too small
    const uint32_t e = blockIdx.x;
    if (e >= aa.eoff[aa.nfam]) return;
    const int n = aa.nfam + 1;
    const int stride = (n + kFillThreads - 1) / kFillThreads;
    const int t = threadIdx.x;
    const int k1 = __syncthreads_count(t * stride < n && aa.eoff[t * stride] <= e) - 1;
    const int base = k1 * stride;
    const int f = base - 1 + __syncthreads_count(t < stride && base + t < n && aa.eoff[base + t] <= e);
    cp_assign_family<kFillThreads>(aa, f, (int)(e - aa.eoff[f]) + 1, (int)e);
}

// Far field of one work item into its cluster's proxies: every thread owns NR
// proxies per pass (NR = ceil(np / 256) up to 4, so that no lane sweeps an
// empty slot for the common degrees) and sweeps the item's assigned atoms.
// The atoms pass through LDS in chunks of one per thread, double-buffered:
// the vector load of the next chunk is in flight while the current one is
// swept, and each atom reaches the lanes as one broadcast LDS read.  Items
// are launched heaviest first.
struct CpSweepArgs {
    CpLevels L;
    const int *order;              // items, heaviest first (one workgroup each)
    const int *it_cl;              // item -> cluster
    const uint32_t *it_a0, *it_na; // item's first atom in its cluster's run, atoms
    const uint32_t *slot;          // each cluster's first assigned atom in abuf
    const float4 *abuf;
    int degree, np;
    float yk;
    double kappa;   // Taylor moments of the screened kernel
    double eta;     // Taylor moments of the erf kernel (paper far field)
    int nc;         // components per item and cluster: 2, or 3 with the erf kernel
    double *part;   // [items][nc][np]: each item's part of its cluster's far field
    const uint32_t *n_items;   // items on the device (the launch may have more)
    const int *bad;
    // scale s of the assigned atoms' positions (relative to their cluster's
    // centre) and charges, and of the proxies' positions: with s = -yk =
    // kappa log2(e), the scaled distance d' = s d gives exp(-kappa d) =
    // exp2(-d') and q'/d' = q/d, which saves the product by yk per pair; 1
    // where unused
    double psc;
};

// Workgroup's item: its cluster, atom count and first atom.
struct SweepItem {
    int item, cl, n;
    const float4 *at;
};
__device__ __forceinline__ SweepItem sweep_item(const CpSweepArgs &a)
{
    SweepItem r;
    r.item = as_const(a.order)[blockIdx.x];
    r.cl = as_const(a.it_cl)[r.item];
    r.n = (int)as_const(a.it_na)[r.item];
    r.at = a.abuf + as_const(a.slot)[r.cl] + as_const(a.it_a0)[r.item];
    return r;
}

struct Quad {
    float x, y, z, w;
};

template <bool ASYM, int NR>
__global__ __launch_bounds__(kBlock) void k_cp_sweep(CpSweepArgs a)
{
    __shared__ float node[3][kMaxDeg + 1];
    __shared__ float4 stage[2][kBlock];
    if (*a.bad || (int)blockIdx.x >= (int)*a.n_items) return;   // whole workgroup
    const SweepItem w = sweep_item(a);
    const int cl = w.cl, item = w.item, n = w.n;
    const float4 *at = w.at;
    const int n1 = a.degree + 1;
    if (threadIdx.x < 3 * n1) {
        int lvl, I, J, K;
        cp_decode(a.L, cl, lvl, I, J, K);
        double pb[6], cc[3], rr;
        cp_proxy_box(a.L, lvl, I, J, K, pb);
        cp_centre(a.L, lvl, I, J, K, cc, rr);
        const int ax = threadIdx.x / n1, k = threadIdx.x % n1;
        node[ax][k] = (float)(cheb_point(pick3(pb, ax), pick3(pb + 3, ax), k, a.degree) -
                              pick3(cc, ax));
    }
    __syncthreads();
    for (int k0 = 0; k0 < a.np; k0 += NR * kBlock) {
        float px[NR], py[NR], pz[NR];
        double aC[NR], aY[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int k = k0 + r * kBlock + threadIdx.x;
            const int kk = k < a.np ? k : 0;
            const int k1 = kk % n1, k2 = (kk / n1) % n1, k3 = kk / (n1 * n1);
            px[r] = node[0][k1];
            py[r] = node[1][k2];
            pz[r] = node[2][k3];
            aC[r] = aY[r] = 0.0;
        }
        float4 nxt = threadIdx.x < n ? at[threadIdx.x] : float4{0.f, 0.f, 0.f, 0.f};
        for (int c0 = 0, buf = 0; c0 < n; c0 += kBlock, buf ^= 1) {
            // buffer buf was last read two chunks ago, before the barrier
            // that every thread passed after it
            stage[buf][threadIdx.x] = nxt;
            __syncthreads();
            if (c0 + kBlock + (int)threadIdx.x < n) nxt = at[c0 + kBlock + threadIdx.x];
            const float4 *st = stage[buf];
            const int m = min(kBlock, n - c0);
            for (int s0 = 0; s0 < m; s0 += 16) {
                float pC[NR], pY[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r) pC[r] = pY[r] = 0.f;
                const int s1 = min(s0 + 16, m);
#pragma unroll 4
                for (int s = s0; s < s1; ++s) {
                    const float4 v = st[s];
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const float dx = px[r] - v.x, dy = py[r] - v.y, dz = pz[r] - v.z;
                        const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        const float ri = __builtin_amdgcn_rsqf(d2);
                        const float qr = v.w * ri;
                        pC[r] += qr;
                        if (ASYM)
                            pY[r] = fmaf(qr, __builtin_amdgcn_exp2f(a.yk * (d2 * ri)), pY[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    aC[r] += (double)pC[r];
                    aY[r] += (double)pY[r];
                }
            }
        }
        __syncthreads();   // the stage is rewritten by the next pass
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int k = k0 + r * kBlock + threadIdx.x;
            if (k < a.np) {
                a.part[((size_t)item * a.nc + 0) * a.np + k] = aC[r];
                a.part[((size_t)item * a.nc + 1) * a.np + k] = aY[r];
            }
        }
    }
}

// k_cp_sweep with the proxies taken along x-lines: every thread owns NI
// proxies of one line (fixed y and z nodes), so dy^2 + dz^2 is formed once
// per atom and shared by the NI proxies, and a pair costs a subtraction and
// an FMA for its distance instead of three subtractions, a product and two
// FMAs.  d2 = fma(dx, dx, fma(dy, dy, dz dz)) is the same expression in the
// same order as in k_cp_sweep.  G = ceil(n1 / NI) threads share a line;
// threads beyond the n1^2 lines and slots beyond n1 on a line compute on
// node 0 and store nothing.
//
// Work items differ in size by up to two orders of magnitude, and all of
// them are resident at once, so the heaviest one sets the launch's length:
// kSweepGroups groups of kBlock threads split an item's atoms into as many
// contiguous ranges, each group sweeping its range over all proxies, and
// their sums are added in group order at the end (the result does not
// depend on the schedule).
constexpr int kSweepGroups = 4;
constexpr int kSweepThreads = kSweepGroups * kBlock;
// Launches of more items than this many per CU take the atom loop unrolled
// twice instead of four times: fewer registers (60 against 83), so two
// workgroups share a CU, which pays once there are enough items to fill
// them; with fewer items the deeper unrolling is faster.
constexpr int kSweepItemsPerCuUnroll2 = 16;

template <bool ASYM, int NI, int UNROLL, bool SC>
__global__ __launch_bounds__(kSweepThreads) void k_cp_sweep_lines(CpSweepArgs a)
{
    __shared__ float node[3][kMaxDeg + 1];
    __shared__ float4 stage[kSweepGroups][2][kBlock];
    __shared__ double red[kSweepGroups - 1][2 * NI][kBlock];
    if (*a.bad || (int)blockIdx.x >= (int)*a.n_items) return;   // whole workgroup
    const SweepItem w = sweep_item(a);
    const int cl = w.cl, item = w.item, n = w.n;
    const int n1 = a.degree + 1;
    if (threadIdx.x < 3 * n1) {
        int lvl, I, J, K;
        cp_decode(a.L, cl, lvl, I, J, K);
        double pb[6], cc[3], rr;
        cp_proxy_box(a.L, lvl, I, J, K, pb);
        cp_centre(a.L, lvl, I, J, K, cc, rr);
        const int ax = threadIdx.x / n1, k = threadIdx.x % n1;
        node[ax][k] = (float)((cheb_point(pick3(pb, ax), pick3(pb + 3, ax), k, a.degree) -
                               pick3(cc, ax)) * a.psc);
    }
    __syncthreads();
    // this thread's group, its atom range, and its place in the group
    const int grp = (int)threadIdx.x / kBlock, tl = (int)threadIdx.x % kBlock;
    const int b0 = (int)((long long)n * grp / kSweepGroups);
    const int na = (int)((long long)n * (grp + 1) / kSweepGroups) - b0;
    const float4 *at = w.at + b0;
    // chunks per group: the same count in every group (barriers inside)
    const int nchunk = ((n + kSweepGroups - 1) / kSweepGroups + kBlock - 1) / kBlock;
    const int G = (n1 + NI - 1) / NI;
    const int line = tl / G, i0 = (tl % G) * NI;
    const bool live = line < n1 * n1;
    const float py = node[1][live ? line % n1 : 0], pz = node[2][live ? line / n1 : 0];
    float px[NI];
    double aC[NI], aY[NI];
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        px[r] = node[0][i0 + r < n1 ? i0 + r : 0];
        aC[r] = aY[r] = 0.0;
    }
    float4 nxt = tl < na ? at[tl] : float4{0.f, 0.f, 0.f, 0.f};
    for (int ch = 0, buf = 0; ch < nchunk; ++ch, buf ^= 1) {
        const int c0 = ch * kBlock;
        // buffer buf was last read two chunks ago, before the barrier that
        // every thread passed after it
        stage[grp][buf][tl] = nxt;
        __syncthreads();
        if (c0 + kBlock + tl < na) nxt = at[c0 + kBlock + tl];
        const float4 *st = stage[grp][buf];
        const int m = max(0, min(kBlock, na - c0));
        for (int s0 = 0; s0 < m; s0 += 16) {
            float pC[NI], pY[NI];
#pragma unroll
            for (int r = 0; r < NI; ++r) pC[r] = pY[r] = 0.f;
            const int s1 = min(s0 + 16, m);
#pragma unroll UNROLL
            for (int s = s0; s < s1; ++s) {
                const float4 v = st[s];
                const float dy = py - v.y, dz = pz - v.z;
                const float e = fmaf(dy, dy, dz * dz);
#pragma unroll
                for (int r = 0; r < NI; ++r) {
                    const float dx = px[r] - v.x;
                    const float d2 = fmaf(dx, dx, e);
                    const float ri = __builtin_amdgcn_rsqf(d2);
                    const float qr = v.w * ri;
                    pC[r] += qr;
                    if (ASYM)
                        pY[r] = fmaf(qr, __builtin_amdgcn_exp2f(SC ? -(d2 * ri) : a.yk * (d2 * ri)),
                                     pY[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < NI; ++r) {
                aC[r] += (double)pC[r];
                aY[r] += (double)pY[r];
            }
        }
    }
    // the groups' sums, added in group order by group 0 (all of a thread's
    // sums through LDS at once: one barrier)
    if (grp > 0) {
#pragma unroll
        for (int r = 0; r < NI; ++r) {
            red[grp - 1][r][tl] = aC[r];
            red[grp - 1][NI + r][tl] = aY[r];
        }
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
        for (int r = 0; r < NI; ++r)
            for (int g = 0; g < kSweepGroups - 1; ++g) {
                aC[r] += red[g][r][tl];
                aY[r] += red[g][NI + r][tl];
            }
    }
    if (grp == 0 && live) {
#pragma unroll
        for (int r = 0; r < NI; ++r) {
            if (i0 + r < n1) {
                const int k = i0 + r + n1 * line;
                a.part[((size_t)item * a.nc + 0) * a.np + k] = aC[r];
                a.part[((size_t)item * a.nc + 1) * a.np + k] = aY[r];
            }
        }
    }
}

// Proxies per thread of k_cp_sweep_lines for n1 nodes per axis: the fewest
// that fit the n1^2 lines into one group of kBlock threads, if the lines then keep at
// least 90 % of its threads busy and that count is instantiated (n1 = 8, 9
// and 11); otherwise 0 (k_cp_sweep).
inline int sweep_line_ni(int n1)
{
    for (int ni = 1; ni <= n1; ++ni) {
        const int busy = n1 * n1 * ((n1 + ni - 1) / ni);
        if (busy <= kBlock)
            return 10 * busy >= 9 * kBlock && (ni == 2 || ni == 3 || ni == 6) ? ni : 0;
    }
    return 0;
}

template <bool ASYM>
void launch_sweep(int nitems, int np, int degree, int n_cu, const CpSweepArgs &sa,
                  hipStream_t s)
{
    const bool many = nitems > kSweepItemsPerCuUnroll2 * n_cu;
    // (the scaled variant exists for the screened kernel only)
    const bool sc = ASYM && sa.psc != 1.0;
    switch (sweep_line_ni(degree + 1)) {
    case 2:
        if (sc) hipLaunchKernelGGL((k_cp_sweep_lines<ASYM, 2, 4, ASYM>), nitems, kSweepThreads, 0, s, sa);
        else hipLaunchKernelGGL((k_cp_sweep_lines<ASYM, 2, 4, false>), nitems, kSweepThreads, 0, s, sa);
        return;
    case 3:
        if (many && sc)
            hipLaunchKernelGGL((k_cp_sweep_lines<ASYM, 3, 2, ASYM>), nitems, kSweepThreads, 0, s, sa);
        else if (many)
            hipLaunchKernelGGL((k_cp_sweep_lines<ASYM, 3, 2, false>), nitems, kSweepThreads, 0, s, sa);
        else if (sc)
            hipLaunchKernelGGL((k_cp_sweep_lines<ASYM, 3, 4, ASYM>), nitems, kSweepThreads, 0, s, sa);
        else
            hipLaunchKernelGGL((k_cp_sweep_lines<ASYM, 3, 4, false>), nitems, kSweepThreads, 0, s, sa);
        return;
    case 6:
        if (sc) hipLaunchKernelGGL((k_cp_sweep_lines<ASYM, 6, 4, ASYM>), nitems, kSweepThreads, 0, s, sa);
        else hipLaunchKernelGGL((k_cp_sweep_lines<ASYM, 6, 4, false>), nitems, kSweepThreads, 0, s, sa);
        return;
    default: break;
    }
    const int nr = np <= 3 * kBlock ? (np + kBlock - 1) / kBlock : 4;
    switch (nr) {
    case 1: hipLaunchKernelGGL((k_cp_sweep<ASYM, 1>), nitems, kBlock, 0, s, sa); break;
    case 2: hipLaunchKernelGGL((k_cp_sweep<ASYM, 2>), nitems, kBlock, 0, s, sa); break;
    case 3: hipLaunchKernelGGL((k_cp_sweep<ASYM, 3>), nitems, kBlock, 0, s, sa); break;
    default: hipLaunchKernelGGL((k_cp_sweep<ASYM, 4>), nitems, kBlock, 0, s, sa); break;
    }
}

// ----------------------------------------------------- Taylor far field
// The paper's own far field (Secs. 2.3.1, 2.3.2, 2.4.1, 2.4.2), as the method
// RISM_TREECODE_TAYLOR: per target cluster the moments
//   m_k = sum_atoms Q t_k(y - c),   |k| <= p,
// of the order-p Taylor polynomials about the cluster centre c of 1/d (u),
// exp(-kappa d)/d (h^lr; the factor 2 of the TCF's far-field form is applied
// with h's other terms) and, in the paper's form, erf(d/eta)/d (c^lr), by the
// recurrences in terms of v = y - c:
//   t_k = [(2 - 1/|k|) sum_i v_i t_{k-e_i} - (1 - 1/|k|) sum_i t_{k-2e_i}
//          + X_k] / R^2,
//   screened:  X_k = (kappa/|k|)(sum_i v_i b_{k-e_i} - sum_i b_{k-2e_i}),
//              b_k = (kappa/|k|)(sum_i v_i t_{k-e_i} - sum_i t_{k-2e_i}),
//              t_0 = exp(-kappa R)/R, b_0 = exp(-kappa R);
//   erf:       X_k = g_k = (2/(eta^2 |k|))(sum_i v_i g_{k-e_i} - sum_i g_{k-2e_i}),
//              t_0 = erf(R/eta)/R, g_0 = -(eta/sqrt(pi)) exp(-R^2/eta^2);
//   1/R:       X_k = 0, t_0 = 1/R.
// The moments take the place of the proxy values: the downward pass shifts
// them to the children's centres and the leaves evaluate the polynomials at
// their points.
//
// One workgroup per work item; its atoms are dealt to the four waves.  A
// wave runs one atom's recurrences degree by degree, a lane per coefficient
// of the degree, with the coefficients in LDS in FP64 (tetrahedral layout:
// degree d starts at d(d+1)(d+2)/6; within it, k = (k1, k2, k3) sits at
// (d-k1)(d-k1+1)/2 + k3).  The wave's moments are in LDS too, each entry
// owned by one lane; the four waves' moments are added in wave order into
// the item's partial, in the cube layout [(p+1)^3] of the proxy values
// (zero above order p): component 0 the 1/d moments, 1 the screened ones,
// 2 the erf ones.
constexpr int kMaxTaylor = 12;

__host__ __device__ inline int tet_off(int d) { return d * (d + 1) * (d + 2) / 6; }

// Coefficient arrays per wave: tC, mC [, tS, bS, mS [, tE, gE, mE]].
__host__ __device__ inline int cp_taylor_arrays(bool asym, bool paper)
{
    return asym ? (paper ? 8 : 5) : 2;
}

inline size_t cp_taylor_lds(int p, bool asym, bool paper)
{
    return (size_t)(kBlock / 64) * cp_taylor_arrays(asym, paper) * tet_off(p + 1) *
           sizeof(double);
}

template <bool ASYM, bool PAPER>
__global__ __launch_bounds__(kBlock) void k_cp_taylor(CpSweepArgs a)
{
    extern __shared__ double sm[];
    if (*a.bad || (int)blockIdx.x >= (int)*a.n_items) return;   // whole workgroup
    const SweepItem w = sweep_item(a);
    const int cl = w.cl, item = w.item, n = w.n;
    ConstAS<Quad> *at = as_const(reinterpret_cast<const Quad *>(w.at));
    const int p = a.degree, n1 = p + 1, nt = tet_off(p + 1);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int NA = ASYM ? (PAPER ? 8 : 5) : 2;
    double *tC = sm + (size_t)wave * NA * nt, *mC = tC + nt;
    double *tS = tC + 2 * nt, *bS = tC + 3 * nt, *mS = tC + 4 * nt;
    double *tE = tC + 5 * nt, *gE = tC + 6 * nt, *mE = tC + 7 * nt;
    for (int i = lane; i < nt; i += 64) {
        mC[i] = 0.0;
        if (ASYM) mS[i] = 0.0;
        if (ASYM && PAPER) mE[i] = 0.0;
    }
    const double kap = a.kappa, eta = a.eta;
    const double ge = PAPER ? 2.0 / (eta * eta) : 0.0;
    for (int s = wave; s < n; s += kBlock / 64) {
        ConstAS<Quad> &av = at[s];
        const double v[3] = {av.x, av.y, av.z}, q = av.w;
        const double R2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double R = sqrt(R2), iR2 = 1.0 / R2;
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            tC[0] = 1.0 / R;
            mC[0] += q * tC[0];
            if (ASYM) {
                const double e = exp(-kap * R);
                tS[0] = e / R;
                bS[0] = e;
                mS[0] += q * tS[0];
            }
            if (ASYM && PAPER) {
                tE[0] = erf(R / eta) / R;
                gE[0] = -(eta / sqrt(kPi)) * exp(-R2 / (eta * eta));
                mE[0] += q * tE[0];
            }
        }
        for (int d = 1; d <= p; ++d) {
            __builtin_amdgcn_wave_barrier();   // degree d - 1 written by every lane
            const int Ld = (d + 1) * (d + 2) / 2;
            const int o0 = tet_off(d), o1 = tet_off(d - 1), o2 = d >= 2 ? tet_off(d - 2) : 0;
            const double c1 = 2.0 - 1.0 / d, c2 = 1.0 - 1.0 / d, kd = kap / d, gd = ge / d;
            for (int pos = lane; pos < Ld; pos += 64) {
                // pos = m(m+1)/2 + k3 with m = d - k1
                int m = (int)((sqrtf(8.f * pos + 1.f) - 1.f) * 0.5f);
                m -= m * (m + 1) / 2 > pos;
                m += (m + 1) * (m + 2) / 2 <= pos;
                const int k3 = pos - m * (m + 1) / 2, k1 = d - m, k2 = m - k3;
                const int T1 = m >= 1 ? (m - 1) * m / 2 : 0, T2 = m >= 2 ? (m - 2) * (m - 1) / 2 : 0;
                // sum_i v_i f_{k-e_i} and sum_i f_{k-2e_i} over one coefficient array
                auto sums = [&](const double *f, double &s2) {
                    double s1 = 0.0;
                    s2 = 0.0;
                    if (k1 >= 1) s1 += v[0] * f[o1 + pos];
                    if (k2 >= 1) s1 += v[1] * f[o1 + T1 + k3];
                    if (k3 >= 1) s1 += v[2] * f[o1 + T1 + k3 - 1];
                    if (k1 >= 2) s2 += f[o2 + pos];
                    if (k2 >= 2) s2 += f[o2 + T2 + k3];
                    if (k3 >= 2) s2 += f[o2 + T2 + k3 - 2];
                    return s1;
                };
                double s2;
                const double s1 = sums(tC, s2);
                const double tc = (c1 * s1 - c2 * s2) * iR2;
                tC[o0 + pos] = tc;
                mC[o0 + pos] += q * tc;
                if (ASYM) {
                    double a2, b2;
                    const double a1 = sums(tS, a2), b1 = sums(bS, b2);
                    const double ts = (c1 * a1 - c2 * a2 + kd * (b1 - b2)) * iR2;
                    tS[o0 + pos] = ts;
                    bS[o0 + pos] = kd * (a1 - a2);
                    mS[o0 + pos] += q * ts;
                }
                if (ASYM && PAPER) {
                    double e2, g2;
                    const double e1 = sums(tE, e2), g1 = sums(gE, g2);
                    const double gk = gd * (g1 - g2);
                    const double te = (c1 * e1 - c2 * e2 + gk) * iR2;
                    gE[o0 + pos] = gk;
                    tE[o0 + pos] = te;
                    mE[o0 + pos] += q * te;
                }
            }
        }
    }
    __syncthreads();
    double *out = a.part + (size_t)item * a.nc * a.np;
    for (int k = threadIdx.x; k < a.np; k += kBlock) {
        const int k1 = k % n1, k2 = (k / n1) % n1, k3 = k / (n1 * n1), d = k1 + k2 + k3;
        double sc = 0.0, ss = 0.0, se = 0.0;
        if (d <= p) {
            const int idx = tet_off(d) + (d - k1) * (d - k1 + 1) / 2 + k3;
            for (int w = 0; w < kBlock / 64; ++w) {
                sc += sm[(size_t)w * NA * nt + nt + idx];
                if (ASYM) ss += sm[(size_t)w * NA * nt + 4 * nt + idx];
                if (ASYM && PAPER) se += sm[(size_t)w * NA * nt + 7 * nt + idx];
            }
        }
        out[k] = sc;
        out[a.np + k] = ss;
        if (a.nc > 2) out[2 * a.np + k] = se;
    }
}

// ----------------------------------------------------------------- downward

// The far field of every level-1 cluster in one launch.  With P_l cluster
// l's own far field (the sum of its items' parts, in item order), the
// downward pass is V_T = P_T and V_l = P_l + (Mx (x) My (x) Mz)_l V_{l+1}
// for l = T-1 .. 1: the parent's far field carried onto the child's proxies.
// M[k][m] = L^P_m(s^C_k), the parent's interpolant evaluated at the child's
// proxy points, separably, in FP64; Taylor moments (taylor != 0) take
// M[k][m] = C(m, k) delta^(m - k) for m >= k, delta = child centre - parent
// centre: the parent's polynomial re-expanded about the child's centre, again
// separably.  The rows come from the per-call tables (cp_table_row).
//
// One workgroup per cluster of level lo walks its chain of ancestors from
// level hi down in LDS and writes V_lo only.  Two launches: the level-2
// clusters from the top (each ancestor's V formed by every one of its
// level-2 descendants: a few redundant contractions in place of one
// dependent launch per level), then the level-1 clusters from the level-2
// V (the leaves read nothing else).  nc of the ncomp components per pass, as
// the LDS allows.
constexpr int kDownThreads = 512;
static_assert(3 * (kMaxDeg + 1) * (kMaxDeg + 1) <= 2 * kDownThreads, "two matrix entries per thread");

inline size_t cp_down_lds(int degree, int nc)
{
    const size_t n1 = degree + 1, np = n1 * n1 * n1;
    return (3 * n1 * n1 + 3 * (size_t)nc * np) * sizeof(double);
}

// s = sum_m row[m] src[m stride], m < n1, unrolled to the largest degree so
// that the LDS reads of a sum are issued together.
__device__ __forceinline__ double dot_lds(const double *row, const double *src, int stride,
                                          int n1)
{
    double s = 0;
#pragma unroll
    for (int m = 0; m <= kMaxDeg; ++m)
        if (m < n1) s += row[m] * src[m * stride];
    return s;
}

struct CpDownArgs {
    CpLevels L;
    int degree;
    int ncomp;                     // components per cluster in part and V
    int nc;                        // components per pass
    const double *M;               // rows of the per-call tables
    int mrow0[kCpMaxLev + 1][3];   // first row of (lvl, axis)
    const uint32_t *item_off;      // first work item of each cluster (clusters + 1)
    const int *bad;                // buffers sized too small: do nothing
    const double *part;            // [item][ncomp][np]
    double *V;                     // [cluster][ncomp][np]; level-lo entries written
    int lo, hi;                    // one workgroup per level-lo cluster, from level hi down
    int top_v;                     // level hi's V is final in V (else its items' sum)
};

// Parts of one cluster's first few items at this thread's S entries, loaded
// ahead of the contractions that precede their sum (fewer items for more
// entries, within the registers of two workgroups per CU).
template <int S>
struct DownPartials {
    static constexpr int PF = S <= 2 ? 6 : (S == 4 ? 4 : (S == 8 ? 2 : 1));
    double v[S][PF];
    int i0, ni;   // the cluster's first item and item count (workgroup-uniform)
};

template <int S>
__device__ __forceinline__ void down_fetch(const CpDownArgs &a, int cl, int e0, int ne, int stride,
                                           DownPartials<S> &p)
{
    p.i0 = (int)a.item_off[cl];
    p.ni = (int)a.item_off[cl + 1] - p.i0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int e = threadIdx.x + j * kDownThreads;
#pragma unroll
        for (int k = 0; k < DownPartials<S>::PF; ++k)
            p.v[j][k] = e < ne && k < p.ni ? a.part[(size_t)(p.i0 + k) * stride + e0 + e] : 0.0;
    }
}

// Sum of the cluster's parts at entry e (slot j), in item order.
template <int S>
__device__ __forceinline__ double down_sum(const CpDownArgs &a, const DownPartials<S> &p, int j,
                                           int e0, int e, int stride)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DownPartials<S>::PF; ++k)
        if (k < p.ni) s += p.v[j][k];
    for (int it = DownPartials<S>::PF; it < p.ni; ++it)
        s += a.part[(size_t)(p.i0 + it) * stride + e0 + e];
    return s;
}

// Matrix entry t of the step to level lvl for the level-lo cluster (I0, J0,
// K0): row of its level-lvl ancestor along axis t / n1^2 (per-call tables).
__device__ __forceinline__ double down_mrow(const CpDownArgs &a, int lvl, int t, int I0, int J0,
                                            int K0, int n1)
{
    if (lvl < a.lo || t >= 3 * n1 * n1) return 0.0;
    const int sh = lvl - a.lo, ax = t / (n1 * n1), km = t % (n1 * n1);
    const int ix = ax == 0 ? I0 >> sh : (ax == 1 ? J0 >> sh : K0 >> sh);
    return a.M[(size_t)(a.mrow0[lvl][ax] + ix * n1) * n1 + km];
}

// dot_lds with the number of terms fixed at compile time (N1 > 0) or not.
template <int N1>
__device__ __forceinline__ double dot_n(const double *row, const double *src, int stride, int n1)
{
    if (N1 == 0) return dot_lds(row, src, stride, n1);
    double s = 0;
#pragma unroll
    for (int m = 0; m < N1; ++m) s += row[m] * src[m * stride];
    return s;
}

// S: entry slots per thread, nc np <= S kDownThreads; N1: degree + 1 when
// fixed at compile time, else 0.  The parts of each level are fetched
// before the two contractions that precede their sum, and each step's
// matrix rows one step ahead.
template <int S, int N1>
__global__ __launch_bounds__(kDownThreads) void k_cp_down_chain(CpDownArgs a)
{
    extern __shared__ double sm[];
    const CpLevels &L = a.L;
    const int n1 = N1 > 0 ? N1 : a.degree + 1;
    const int np = n1 * n1 * n1, stride = a.ncomp * np, nm = 3 * n1 * n1;
    double *M = sm;                   // [3][n1][n1]
    double *src = M + nm;             // [nc][np]: V of the current level
    double *t1 = src + a.nc * np;     // [nc][np]
    double *t2 = t1 + a.nc * np;      // [nc][np]
    if (*a.bad) return;   // whole workgroup
    const int lo = a.lo, hi = a.hi;
    const int q = blockIdx.x;   // level-lo cluster
    const int I0 = q % L.cx[lo], J0 = (q / L.cx[lo]) % L.cy[lo], K0 = q / (L.cx[lo] * L.cy[lo]);
    const int tid = threadIdx.x;
    for (int comp0 = 0; comp0 < a.ncomp; comp0 += a.nc) {
        const int ne = min(a.nc, a.ncomp - comp0) * np, e0 = comp0 * np;
        DownPartials<S> p;
        const int sh_top = hi - lo;
        const int top = cp_id(L, hi, I0 >> sh_top, J0 >> sh_top, K0 >> sh_top);
        if (!a.top_v) down_fetch<S>(a, top, e0, ne, stride, p);
        double mr0 = down_mrow(a, hi - 1, tid, I0, J0, K0, n1);
        double mr1 = down_mrow(a, hi - 1, tid + kDownThreads, I0, J0, K0, n1);
        __syncthreads();   // the previous pass is done with src
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int e = tid + j * kDownThreads;
            if (e < ne)
                src[e] = a.top_v ? a.V[(size_t)top * stride + e0 + e]
                                 : down_sum<S>(a, p, j, e0, e, stride);
        }
        for (int lvl = hi - 1; lvl >= lo; --lvl) {
            const int sh = lvl - lo;
            down_fetch<S>(a, cp_id(L, lvl, I0 >> sh, J0 >> sh, K0 >> sh), e0, ne, stride, p);
            __syncthreads();   // src written; the previous step's z pass is done with M
            if (tid < nm) M[tid] = mr0;
            if (tid + kDownThreads < nm) M[tid + kDownThreads] = mr1;
            mr0 = down_mrow(a, lvl - 1, tid, I0, J0, K0, n1);
            mr1 = down_mrow(a, lvl - 1, tid + kDownThreads, I0, J0, K0, n1);
            __syncthreads();
            // entry e = c np + k, k = (z, y, x) with x fastest; contract x,
            // then y, then z
            for (int e = tid; e < ne; e += kDownThreads) {
                const int c = e / np, k = e - c * np;
                const int k1 = k % n1, rest = k / n1;
                t1[e] = dot_n<N1>(M + (0 * n1 + k1) * n1, src + c * np + rest * n1, 1, n1);
            }
            __syncthreads();
            for (int e = tid; e < ne; e += kDownThreads) {
                const int c = e / np, k = e - c * np;
                const int k1 = k % n1, k2 = (k / n1) % n1, m3 = k / (n1 * n1);
                t2[e] = dot_n<N1>(M + (1 * n1 + k2) * n1, t1 + c * np + m3 * n1 * n1 + k1, n1, n1);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const int e = tid + j * kDownThreads;
                if (e < ne) {
                    const int c = e / np, k = e - c * np;
                    const int k12 = k % (n1 * n1), k3 = k / (n1 * n1);
                    src[e] = down_sum<S>(a, p, j, e0, e, stride) +
                             dot_n<N1>(M + (2 * n1 + k3) * n1, t2 + c * np + k12, n1 * n1, n1);
                }
            }
        }
        __syncthreads();
        const int id = cp_id(L, lo, I0, J0, K0);
        for (int e = tid; e < ne; e += kDownThreads) a.V[(size_t)id * stride + e0 + e] = src[e];
    }
}

// Above this many atoms the downward pass takes one launch per level: each
// workgroup of a chain sums the items of every ancestor again, and a large
// solute gives the top clusters up to n / kItemAtoms items each.
constexpr int64_t kChainMaxAtoms = 32768;

// Entry slots per thread of the downward kernel for nc components of degree
// `degree`: 1, 2, 4, 8 or 16 (enough for every degree the LDS admits).
inline int cp_down_slots(int degree, int nc)
{
    const int n1 = degree + 1, ne = nc * n1 * n1 * n1;
    int sl = 1;
    while (sl < 16 && sl * kDownThreads < ne) sl *= 2;
    return sl;
}

// ----------------------------------------------------------------- leaves

struct CpLeafArgs {
    CpLevels L;
    GridParams g;
    OutParams out;
    AsymParams asym;
    const void *rec;
    const uint32_t *aoff;      // candidate atoms of each group (prefix; cp_classify_group)
    const int *dlist, *slist;  // direct atoms per group / short-range atoms per block
    const uint32_t *nd, *ns;   // their counts
    const uint32_t *on_grid;   // per group: a direct atom sits on a grid point
    const int *order;          // block -> level-0 block, heaviest first
    const int *bad;            // lists sized too small: do nothing
    const double *V;           // proxy values (Taylor: moments) of level-1 clusters
    const double *Lg;          // level-1 basis rows per grid coordinate (per-call tables)
    int lrow0[3];              // first row of each axis in Lg
    int degree, np;
    int taylor;                // basis: Lagrange (0) or monomials about the centre (1)
    int ncomp;                 // components per cluster in V (2, or 3 with the erf kernel)
    int paper;                 // Taylor far fields of the paper: u from the 1/d
                               // moments, c^lr from the erf moments (component 2),
                               // short-range atoms contribute LJ only
    unsigned long long *work;  // optional: [0] direct pairs, [1] short-range pairs
};

// Far-field components the leaf interpolates: 1/d [, exp(-kappa d)/d [, erf]].
__host__ __device__ inline int cp_leaf_ncomp(bool asym, bool paper)
{
    return asym ? (paper ? 3 : 2) : 1;
}

// One grid point per thread, up to 512 threads per block.
template <int B>
struct LeafShape {
    static constexpr int threads = B * B * B < 512 ? B * B * B : 512;
    static constexpr int passes = (B * B * B) / threads;
};

// Atoms per LDS chunk of the leaf kernel (a multiple of kAtomPad, so the
// flushes fall where they would without chunks).
constexpr int kLeafStage = 256;
static_assert(kLeafStage % kAtomPad == 0, "leaf chunks must keep the flush points");

// Doubles of the leaf kernel's LDS before the atom chunk, rounded up to an
// even count so that the 16-byte records start aligned.
__host__ __device__ inline size_t cp_leaf_head(int B, int degree, bool asym, bool paper)
{
    const size_t n1 = degree + 1, np = n1 * n1 * n1;
    const size_t ncomp = cp_leaf_ncomp(asym, paper);
    const size_t d = (asym ? 4 * (size_t)kSmearIntervals : 0) + ncomp * n1 * B * B +
                     3 * (size_t)B * n1 + np + n1 * n1 * B;
    return (d + 1) & ~(size_t)1;
}

// Dynamic LDS of the leaf kernel, in bytes (layout in k_cp_leaf), for atom
// records of rec_bytes.
inline size_t cp_leaf_lds(int B, int degree, bool asym, bool paper, size_t rec_bytes)
{
    return cp_leaf_head(B, degree, asym, paper) * sizeof(double) + kLeafStage * rec_bytes;
}

// Staged atoms [s0, s1) against this thread's point, into fresh partial sums.
template <int NS, int LJM, bool ASYM, bool EXACT, bool FULL, bool GUARD>
__device__ __forceinline__ PairAcc<NS> leaf_group(const AtomF32<NS> *stg, int s0, int s1,
                                                  const GridPt &gp, const PairConst &kc,
                                                  const float4 *tab, bool &hit)
{
    PairAcc<NS> p;
    p.zero();
#pragma unroll 1
    for (int s = s0; s < s1; ++s)
        pair_eval<NS, LJM, ASYM, EXACT, FULL, GUARD>(stg[s], gp, kc, tab, p, hit);
    return p;
}

// The staged atoms [0, m) against this thread's point, flushed every
// 2 kAtomPad atoms.  guard (full pairs): some staged atom sits on a grid
// point.  The choice is made per group of atoms, so that the running sums
// stay outside the two versions of the loop.
template <int NS, int LJM, bool ASYM, bool EXACT, bool FULL>
__device__ __forceinline__ void leaf_chunk(const AtomF32<NS> *stg, int m, bool guard,
                                           const GridPt &gp, const PairConst &kc,
                                           const float4 *tab, PointAcc<NS> &acc)
{
    for (int s0 = 0; s0 < m; s0 += 2 * kAtomPad) {
        const int s1 = min(s0 + 2 * kAtomPad, m);
        const PairAcc<NS> p =
            !FULL || guard
                ? leaf_group<NS, LJM, ASYM, EXACT, FULL, true>(stg, s0, s1, gp, kc, tab, acc.hit)
                : leaf_group<NS, LJM, ASYM, EXACT, FULL, false>(stg, s0, s1, gp, kc, tab,
                                                                acc.hit);
        acc.template flush<LJM != LJ_NONE, ASYM>(p);
    }
}

// The atoms of one index list against this thread's point.  The workgroup
// copies the records to LDS kLeafStage at a time (one per thread), and every
// pair reads its atom's fields from there into vector registers: a vector
// instruction takes one scalar operand at most, so with the fields in scalar
// registers each site's fma(A, r^-6, -B) would need a move of B first.
// guard: the list holds an atom that sits on a grid point (full pairs only;
// without one the pair loop leaves out the coincidence handling).  Every
// thread of the workgroup calls this with the same list (barriers inside).
template <int NS, int LJM, bool ASYM, bool EXACT, bool FULL, int NT>
__device__ __forceinline__ void leaf_atoms(const AtomF32<NS> *rec, ConstAS<int> *il, int cnt,
                                           bool guard, AtomF32<NS> *stg, const GridPt &gp,
                                           const PairConst &kc, const float4 *tab,
                                           PointAcc<NS> &acc)
{
    for (int c0 = 0; c0 < cnt; c0 += kLeafStage) {
        const int m = min(kLeafStage, cnt - c0);
        __syncthreads();   // every wave is done with the previous chunk
        for (int t = threadIdx.x; t < m; t += NT) stg[t] = rec[il[c0 + t]];
        __syncthreads();
        leaf_chunk<NS, LJM, ASYM, EXACT, FULL>(stg, m, guard, gp, kc, tab, acc);
    }
}

// One workgroup per level-0 block, blocks launched heaviest first.  Far
// field: the level-1 ancestor's proxy values interpolated onto the block by
// three one-axis contractions (the first two once per block, into LDS; the
// last per point).  Near field: the block's direct atoms (full pair) and
// short-range atoms (LJ and the smeared kernels less their far-field forms)
// from the block's index lists.
//
// LDS: [smeared table (ASYM)] [T2 per component: n1 x B x B] [Lb: 3 x B x n1]
//      [Vs (np)] [T1 (n1 x n1 x B)] [atom chunk: kLeafStage records]
// N1: degree + 1 when fixed at compile time (the contractions unrolled), else 0.
template <int NS, int LJM, bool ASYM, int B, int N1>
__global__ __launch_bounds__(LeafShape<B>::threads) void k_cp_leaf(CpLeafArgs a)
{
    using S = LeafShape<B>;
    constexpr int NT = S::threads;
    const bool paper = ASYM && a.paper;
    const int NCOMP = cp_leaf_ncomp(ASYM, paper);
    extern __shared__ double sm[];
    const int n1 = N1 > 0 ? N1 : a.degree + 1, np = N1 > 0 ? N1 * N1 * N1 : a.np;
    float4 *tab = reinterpret_cast<float4 *>(sm);
    double *T2 = sm + (ASYM ? 4 * kSmearIntervals : 0);   // [NCOMP][n1][B][B]
    double *Lb = T2 + NCOMP * n1 * B * B;                  // [3][B][n1]
    double *Vs = Lb + 3 * B * n1;                          // [np]
    double *T1 = Vs + np;                                  // [n1][n1][B]
    AtomF32<NS> *stg =
        reinterpret_cast<AtomF32<NS> *>(sm + cp_leaf_head(B, a.degree, ASYM, paper));
    if (*a.bad) return;   // whole workgroup
    const CpLevels &L = a.L;
    const GridParams &g = a.g;
    const int q = as_const(a.order)[blockIdx.x];
    const int I = q % L.cx[0], J = (q / L.cx[0]) % L.cy[0], K = q / (L.cx[0] * L.cy[0]);
    const int i0 = I * B, j0 = J * B, k0 = K * B;
    const PairConst kc = make_pair_const(a.asym);
    const AtomF32<NS> *grec = static_cast<const AtomF32<NS> *>(a.rec);
    int child;
    const int grp = cp_group_of(L, I, J, K, child);
    const uint32_t base = as_const(a.aoff)[grp], na = as_const(a.aoff)[grp + 1] - base;
    ConstAS<int> *dl = as_const(a.dlist + base);
    ConstAS<int> *sl = as_const(a.slist + 8 * (size_t)base + (size_t)child * na);
    const int ndir = (int)as_const(a.nd)[grp], nsh = (int)as_const(a.ns)[q];
    const bool dguard = as_const(a.on_grid)[grp] != 0;
    if (ASYM)
        for (int i = threadIdx.x; i < 2 * kSmearIntervals; i += NT) tab[i] = a.asym.tab[i];

    // ------------------------------- far: first two contractions, per block
    if (L.T >= 1) {
        // level-1 ancestor basis at the block's point coordinates, L_k(x) or
        // (x - c)^k for Taylor moments, copied from the per-call table
        for (int t = threadIdx.x; t < 3 * B * n1; t += NT) {
            const int ax = t / (B * n1), lk = t % (B * n1);
            const int b0 = ax == 0 ? i0 : (ax == 1 ? j0 : k0);
            Lb[t] = a.Lg[(size_t)(a.lrow0[ax] + b0) * n1 + lk];
        }
        const int a1 = cp_id(L, 1, I >> 1, J >> 1, K >> 1);
        for (int comp = 0; comp < NCOMP; ++comp) {
            __syncthreads();
            for (int k = threadIdx.x; k < np; k += NT)
                Vs[k] = a.V[((size_t)a1 * a.ncomp + comp) * np + k];
            __syncthreads();
            // T1[k1][k2][z] = sum_k3 V[k3][k2][k1] Lz[z][k3]
            for (int t = threadIdx.x; t < n1 * n1 * B; t += NT) {
                const int z = t % B, k12 = t / B;
                double s = 0;
                for (int k3 = 0; k3 < n1; ++k3) s += Vs[k3 * n1 * n1 + k12] * Lb[(2 * B + z) * n1 + k3];
                T1[t] = s;
            }
            __syncthreads();
            // T2[k1][y][z] = sum_k2 T1[k1][k2][z] Ly[y][k2]     (k12 = k2 n1 + k1)
            double *T2c = T2 + comp * n1 * B * B;
            for (int t = threadIdx.x; t < n1 * B * B; t += NT) {
                const int z = t % B, y = (t / B) % B, k1 = t / (B * B);
                double s = 0;
                for (int k2 = 0; k2 < n1; ++k2)
                    s += T1[(k2 * n1 + k1) * B + z] * Lb[(1 * B + y) * n1 + k2];
                T2c[t] = s;
            }
        }
    }
    __syncthreads();

    if (a.work && threadIdx.x == 0) {
        const unsigned long long np_blk =
            (unsigned long long)(min(B, g.nx - i0) * min(B, g.ny - j0) * min(B, g.nz - k0));
        atomicAdd(&a.work[0], (unsigned long long)ndir * np_blk);
        atomicAdd(&a.work[1], (unsigned long long)nsh * np_blk);
    }

    for (int pass = 0; pass < S::passes; ++pass) {
        const int l = pass * NT + threadIdx.x;
        const int li = l % B, lj = (l / B) % B, lk = l / (B * B);
        const bool valid = i0 + li < g.nx && j0 + lj < g.ny && k0 + lk < g.nz;
        const GridPt gp = grid_pt(g, valid ? i0 + li : i0, valid ? j0 + lj : j0,
                                  valid ? k0 + lk : k0);
        PointAcc<NS> acc;
        acc.zero();
        // paper's Taylor far fields: u and c^lr take the 1/d and erf(d/eta)/d
        // expansions, so both stay out of acc.C
        double far_u = 0.0, far_c = 0.0;

        // ---------------------------------------------- far: last contraction
        if (L.T >= 1) {
            for (int comp = 0; comp < NCOMP; ++comp) {
                const double *T2c = T2 + comp * n1 * B * B;
                double s = 0;
                for (int k1 = 0; k1 < n1; ++k1)
                    s += T2c[(k1 * B + lj) * B + lk] * Lb[(0 * B + li) * n1 + k1];
                if (comp == 1) acc.Y = s;
                else if (comp == 2) far_c = s;
                else if (paper) far_u = s;
                else acc.C = s;
            }
        }

        // ---------------------------------------------- direct and short
        // short-range atoms (far field from the clusters): LJ, and for the
        // exact-split far fields the smeared kernels' remainders
        if (g.exact) {
            leaf_atoms<NS, LJM, ASYM, true, true, NT>(grec, dl, ndir, dguard,
                                                      stg, gp, kc, tab, acc);
            if (ASYM && !paper)
                leaf_atoms<NS, LJM, ASYM, true, false, NT>(grec, sl, nsh, true,
                                                           stg, gp, kc, tab, acc);
            else if (LJM != LJ_NONE)
                leaf_atoms<NS, LJM, false, true, false, NT>(grec, sl, nsh, true,
                                                            stg, gp, kc, tab, acc);
        } else {
            leaf_atoms<NS, LJM, ASYM, false, true, NT>(grec, dl, ndir, dguard,
                                                       stg, gp, kc, tab, acc);
            if (ASYM && !paper)
                leaf_atoms<NS, LJM, ASYM, false, false, NT>(grec, sl, nsh, true,
                                                            stg, gp, kc, tab, acc);
            else if (LJM != LJ_NONE)
                leaf_atoms<NS, LJM, false, false, false, NT>(grec, sl, nsh, true,
                                                             stg, gp, kc, tab, acc);
        }

        if (valid) {
            const int64_t p = ((int64_t)(k0 + lk) * g.ny + (j0 + lj)) * g.nx + (i0 + li);
            store_point<NS, LJM, ASYM>(a.out, g, p, acc, far_u, far_c);
        }
    }
}

template <int NS, int LJM, bool ASYM>
void launch_leaf_b(int B, int nleaf, size_t shm, const CpLeafArgs &a, hipStream_t s)
{
    if (B == 4)
        hipLaunchKernelGGL((k_cp_leaf<NS, LJM, ASYM, 4, 0>), nleaf, LeafShape<4>::threads, shm, s,
                           a);
    else if (B == 8 && a.degree == 8)   // the usual batch edge and degree
        hipLaunchKernelGGL((k_cp_leaf<NS, LJM, ASYM, 8, 9>), nleaf, LeafShape<8>::threads, shm, s,
                           a);
    else if (B == 8)
        hipLaunchKernelGGL((k_cp_leaf<NS, LJM, ASYM, 8, 0>), nleaf, LeafShape<8>::threads, shm, s,
                           a);
    else
        hipLaunchKernelGGL((k_cp_leaf<NS, LJM, ASYM, 16, 0>), nleaf, LeafShape<16>::threads, shm,
                           s, a);
}

template <int NS>
void launch_leaf_ns(int lj_mode, bool asym, int B, int nleaf, size_t shm, const CpLeafArgs &a,
                    hipStream_t s)
{
    if (lj_mode == LJ_CUT1) {
        if (asym) launch_leaf_b<NS, LJ_CUT1, true>(B, nleaf, shm, a, s);
        else launch_leaf_b<NS, LJ_CUT1, false>(B, nleaf, shm, a, s);
    } else if (lj_mode == LJ_CUT) {
        if (asym) launch_leaf_b<NS, LJ_CUT, true>(B, nleaf, shm, a, s);
        else launch_leaf_b<NS, LJ_CUT, false>(B, nleaf, shm, a, s);
    } else {
        if (asym) launch_leaf_b<NS, LJ_NONE, true>(B, nleaf, shm, a, s);
        else launch_leaf_b<NS, LJ_NONE, false>(B, nleaf, shm, a, s);
    }
}

__global__ void k_fill_int(int *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Pinned, coherent host memory for the flag words read at the end of a pass.
uint32_t *pinned_u32(int n)
{
    static thread_local uint32_t *p = nullptr;
    if (!p && hipHostMalloc((void **)&p, 64 * sizeof(uint32_t), hipHostMallocCoherent) != hipSuccess)
        p = nullptr;
    return n <= 64 ? p : nullptr;
}

// Flag words of a cluster-particle call (layout at their allocation).
constexpr int kFlagWords = 10;

// Event recorded after the plan kernel, which copies the flag words to host
// memory: the host waits for it, and the far sweep, the downward pass and the
// leaves keep running after the call returns.  One per device and host thread.
// Without the system-scope fence: the flags reach host memory through the
// plan kernel's own system-scope stores.
constexpr int kMaxEventDevices = 64;
hipEvent_t flags_event(int dev)
{
    static thread_local hipEvent_t ev[kMaxEventDevices] = {};
    if (dev < 0 || dev >= kMaxEventDevices) return nullptr;
    if (!ev[dev] && hipEventCreateWithFlags(&ev[dev], hipEventDisableTiming |
                                                          hipEventDisableSystemFence) != hipSuccess)
        ev[dev] = nullptr;
    return ev[dev];
}

// Sizes of the list buffers: [0] cluster candidates, [1] unused (0), [2]
// group candidates, [3] group candidate atoms, [4] cluster candidate atoms.
struct CpCaps {
    uint32_t c[5];
};


// Capacities seen for a problem shape (device, atoms, blocks, clusters,
// degree, theta, leaf size, short range): a later call of the same shape sizes
// its buffers from them and enqueues all its kernels without waiting for the
// counts; the kernels do nothing when the device-side check fails, and the
// call then runs again with the counts it read back.
struct CpShape {
    int dev, leaf, deg;
    int64_t n;
    int nleaf, ncl;
    double theta, rshort, guard;
    bool operator<(const CpShape &o) const
    {
        if (dev != o.dev) return dev < o.dev;
        if (n != o.n) return n < o.n;
        if (nleaf != o.nleaf) return nleaf < o.nleaf;
        if (ncl != o.ncl) return ncl < o.ncl;
        if (deg != o.deg) return deg < o.deg;
        if (leaf != o.leaf) return leaf < o.leaf;
        if (theta != o.theta) return theta < o.theta;
        if (rshort != o.rshort) return rshort < o.rshort;
        return guard < o.guard;
    }
};
std::mutex g_cp_caps_mu;
std::map<CpShape, CpCaps> g_cp_caps;

}  // namespace

int tree_forward_cp(const TreeCallArgs &a, Workspace &ws, rism_stats &st, hipStream_t s)
{
    const bool ev = a.opts->flags & RISM_FLAG_PHASE_EVENTS;
    const int B = a.opts->batch_edge;
    const int deg = a.opts->degree;
    const int n1 = deg + 1, np = n1 * n1 * n1;
    // implicit target octree
    CpLevels L;
    if (cp_levels(a.g, B, a.opts->theta, L) != RISM_OK) {
        set_error("treecode_cp: grid too large for the target octree");
        return RISM_E_UNSUPPORTED;
    }
    const int ncl = L.T >= 1 ? L.off[L.T + 1] : 0;
    const int nleaf = L.cx[0] * L.cy[0] * L.cz[0];
    const int ngrp = cp_groups(L);   // groups of level-0 blocks (cp_classify_group)
    const bool taylor = a.opts->method == RISM_TREECODE_TAYLOR;
    // the paper's Taylor far fields (expansions of 1/d, erf(d/eta)/d and
    // 2 exp(-kappa d)/d), unless the exact-split variant is asked for
    const bool paper = taylor && !(a.opts->flags & RISM_FLAG_TAYLOR_SPLIT);
    const int item_atoms = taylor ? kTaylorItemAtoms : kItemAtoms;
    // with h^lr expanded as 2 exp(-kappa d)/d (the erfc -> 2/0 step), no
    // target of an accepting cluster may come within eta (6 + kappa eta/2)
    // of the atom, where that step is off by more than erfc(6) ~ 2e-17
    if (paper && a.out.want_h)
        L.guard = a.asym.eta * (6.0 + 0.5 * a.asym.kappa * a.asym.eta);
    // components per cluster in the proxy / moment arrays
    const int nc = paper && a.asym_on ? 3 : 2;

    // [0..4] totals as in CpCaps, [5] query stack overflow, [6] capacity
    // check failed, [8..9] the input check's flags: one block, read back with
    // one copy; the tree build clears [0..6]
    uint32_t *flags = ws.get<uint32_t>(kFlagWords);
    if (ws.status()) return ws.status();
    uint32_t *tot = flags;
    int *overflow = reinterpret_cast<int *>(flags + 5);
    int *bad = reinterpret_cast<int *>(flags + 6);

    // source tree on the atoms (Morton sort, boxes) for the neighbour queries
    TreeDev t{};
    t.clear = reinterpret_cast<int *>(flags);
    t.n_clear = 7;
    int rc;
    {
        PhaseTimer pt(ev, RISM_PHASE_TREE_BUILD, s);
        rc = build_source_tree(a, ws, t, st, s);
    }
    if (rc) return rc;
    const int stride_f4 = (int)(rec32_bytes_of(a.sp.ns_pad) / sizeof(float4));
    // short range of the leaves: LJ within its cut-off and, unless the far
    // fields are the paper's own expansions of the smeared kernels, their
    // remainders within R_s
    double rshort = a.asym_on && !paper ? std::sqrt(a.asym.rs2) : 0.0;
    if (a.lj_mode == LJ_CUT) rshort = std::max(rshort, a.rmax_short);

    // queries: clusters (mode 0) and groups of leaves (mode 1), count pass
    // families of target clusters: the children of each cluster at levels
    // 2..T, and the top cluster alone
    const int nfam = ncl > 0 ? ncl - L.off[2] + 1 : 0;
    uint32_t *ccnt = ws.get<uint32_t>(nfam + 1), *cacnt = ws.get<uint32_t>(nfam + 1);
    // extra assignment chunks per family (prefix after the scan)
    const bool extra_chunks = ncl > 0 && a.solute->n > kAssignExtraMinAtoms;
    uint32_t *ecnt = extra_chunks ? ws.get<uint32_t>(nfam + 1) : nullptr;
    uint32_t *lcnt = ws.get<uint32_t>(ngrp + 1), *lacnt = ws.get<uint32_t>(ngrp + 1);
    if (ws.status()) return ws.status();
    int dev = 0;
    RISM_HIP(hipGetDevice(&dev));
    int n_cu = 0;
    RISM_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    CpQueryArgs qa{};
    qa.L = L;
    qa.rshort = rshort;
    qa.begin = t.begin;
    qa.end = t.end;
    qa.child0 = t.child0;
    qa.nchild = t.nchild;
    qa.box = t.box;
    qa.n_nodes = t.n_nodes;
    qa.overflow = overflow;
    qa.stack_w = cp_query_stack(t.cap_nodes);
    const size_t qshm = (size_t)qa.stack_w * sizeof(int);
    // the per-call tables, formed by the count pass's launch
    CpTabArgs ta{};
    ta.L = L;
    ta.degree = deg;
    ta.taylor = taylor;
    cp_tab_layout(L, n1, ta);
    ta.err_src = a.stage_err;
    ta.err_n = a.n_stage_err;
    ta.err_dst = flags + 8;
    ta.M = ws.get<double>((size_t)(ta.nrow_m + 1) * n1);
    ta.Lg = ws.get<double>((size_t)ta.nrow_l * n1);
    if (ws.status()) return ws.status();
    // list capacities of an earlier call of the same shape: the scans check
    // the counts against them, and the lists are filled speculatively
    const CpShape shape{dev,   a.opts->leaf_size, deg,    a.solute->n, nleaf,
                        ncl,   a.opts->theta,     rshort, L.guard};
    CpCaps cached{};
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_cp_caps_mu);
        auto it = g_cp_caps.find(shape);
        if (it != g_cp_caps.end()) {
            cached = it->second;
            have = true;
        }
    }
    {
        // count pass of both query sets (and the tables) in one launch, then
        // the four scans
        PhaseTimer pt(ev, RISM_PHASE_LISTS, s);
        CpQueryArgs qc = qa;   // families of clusters (none when ncl = 0)
        qc.mode = 0;
        qc.nq = nfam;
        qc.cnt = ccnt;
        qc.acnt = cacnt;
        qc.ecnt = ecnt;
        qc.fill = 0;
        CpQueryArgs ql = qa;   // groups of level-0 blocks
        ql.mode = 1;
        ql.nq = ngrp;
        ql.cnt = lcnt;
        ql.acnt = lacnt;
        ql.fill = 0;
        hipLaunchKernelGGL(k_cp_query, nfam + ngrp + cp_table_blocks(ta), kQueryThreads, qshm, s,
                           qc, ql, ta);
        ScanBatch sb{};
        int na = 0;
        auto add = [&](uint32_t *arr, int k, int n) {
            sb.a[na] = arr;
            sb.total[na] = tot + k;
            sb.n[na] = n;
            sb.cap[na] = cached.c[k];
            ++na;
        };
        if (ncl > 0) {   // (otherwise their totals stay 0)
            add(ccnt, 0, nfam + 1);
            add(cacnt, 4, nfam + 1);
        }
        if (ecnt) {   // total into flags[7], no capacity of its own
            sb.a[na] = ecnt;
            sb.total[na] = tot + 7;
            sb.n[na] = nfam + 1;
            sb.cap[na] = 0xffffffffu;
            ++na;
        }
        add(lcnt, 2, ngrp + 1);
        add(lacnt, 3, ngrp + 1);
        sb.na = na;
        if (have) {
            sb.bad = bad;
            sb.overflow = overflow;
        }
        if ((rc = scan_batch(sb, ws, s))) return rc;
    }
    RISM_HIP(hipGetLastError());

    int lds_max = 0;
    RISM_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t leaf_shm = cp_leaf_lds(B, deg, a.asym_on, paper, rec32_bytes_of(a.sp.ns_pad));
    if (taylor && (deg > kMaxTaylor || cp_taylor_lds(deg, a.asym_on, paper) > (size_t)lds_max)) {
        set_error("Taylor treecode: order above 12 or its LDS beyond this device");
        return RISM_E_UNSUPPORTED;
    }
    if (leaf_shm + 2048 > (size_t)lds_max || cp_down_lds(deg, 1) > (size_t)lds_max) {
        set_error("treecode_cp: degree / batch edge too large for the LDS of this device");
        return RISM_E_UNSUPPORTED;
    }
    // components per pass of the downward kernel: all of them if the LDS allows
    int down_nc = nc;
    while (down_nc > 1 && cp_down_lds(deg, down_nc) > (size_t)lds_max) --down_nc;
    const bool want_stats = a.opts->flags & RISM_FLAG_STATS;
    unsigned long long *work = want_stats ? ws.get<unsigned long long>(4) : nullptr;
    uint32_t *nd = ws.get<uint32_t>(ngrp), *nsh = ws.get<uint32_t>(nleaf);
    uint32_t *dguard = ws.get<uint32_t>(ngrp);
    uint32_t *cost = ws.get<uint32_t>(nleaf);
    int *order = ws.get<int>(nleaf);
    double *V = ws.get<double>((size_t)(ncl + 1) * nc * np);
    if (ws.status()) return ws.status();

    // totals and flags read back at the end of a pass: [0..4] counts as in
    // CpCaps, [5] query stack overflow, [6] capacity check failed, [8..9] the
    // input check's flags (when deferred to here)
    uint32_t *hres = pinned_u32(kFlagWords);
    const hipEvent_t fev = flags_event(dev);
    if (!fev) {
        set_error("treecode_cp: event creation failed");
        return RISM_E_HIP;
    }
    if (!hres) {
        set_error("treecode_cp: pinned host buffer allocation failed");
        return RISM_E_HIP;
    }
    // scale of the far-field sweep's atom and proxy positions (CpSweepArgs::psc):
    // the line kernels with the screened kernel, kappa > 0
    const double psc = !taylor && a.asym_on && a.asym.kappa > 0.0 && sweep_line_ni(deg + 1) != 0
                           ? -a.asym.yk
                           : 1.0;
    // Everything after the counts, with buffers of the given capacities.
    auto second_half = [&](const CpCaps &cap) -> int {
        int *ccand = ws.get<int>(cap.c[0] + 1), *lcand = ws.get<int>(cap.c[2] + 1);
        uint32_t *cl_n = ws.get<uint32_t>(ncl + 1), *item_off = ws.get<uint32_t>(ncl + 1);
        uint32_t *cslot = ws.get<uint32_t>(ncl + 1);
        // far work items: runs of at most item_atoms of a cluster's atoms (a
        // family's children have room for all of its candidate atoms each)
        const size_t max_assigned = 8 * (size_t)cap.c[4];
        // extra assignment chunks (at most one per kAssignChunk candidate
        // atoms), each adding up to eight partial items
        const int n_extra = ecnt ? (int)(cap.c[4] / kAssignChunk) : 0;
        const int max_items = ncl + (int)((max_assigned + item_atoms - 1) / item_atoms) + 8 * n_extra;
        uint32_t *apre = n_extra > 0 ? ws.get<uint32_t>(cap.c[0] + 1) : nullptr;
        uint32_t *pc = n_extra > 0 ? ws.get<uint32_t>(8 * (size_t)n_extra) : nullptr;
        int *it_cl = ws.get<int>(max_items + 1), *it_order = ws.get<int>(max_items + 1);
        uint32_t *it_a0 = ws.get<uint32_t>(max_items + 1), *it_na = ws.get<uint32_t>(max_items + 1);
        uint32_t *n_items = ws.get<uint32_t>(1);
        double *part = ws.get<double>((size_t)(max_items + 1) * nc * np);
        float4 *abuf = ws.get<float4>(max_assigned + 1);
        int *dlist = ws.get<int>(cap.c[3] + 1), *slist = ws.get<int>(8 * (size_t)cap.c[3] + 1);
        if (ws.status()) return ws.status();
        if (work) hipLaunchKernelGGL(k_fill_u64, 1, 64, 0, s, work, 4);
        qa.bad = bad;
        // fill pass of both query sets in one launch, with the far-field
        // assignment of every cluster and the near-field classification of
        // every group; then the launch orders
        {
            PhaseTimer pt(ev, RISM_PHASE_LISTS, s);
            CpQueryArgs qc = qa;
            qc.mode = 0;
            qc.nq = nfam;
            qc.off = ccnt;
            qc.list = ccand;
            qc.fill = 1;
            qc.acnt = nullptr;
            CpQueryArgs ql = qa;
            ql.mode = 1;
            ql.nq = ngrp;
            ql.off = lcnt;
            ql.list = lcand;
            ql.fill = 1;
            ql.acnt = nullptr;
            CpAssignArgs aa{};
            aa.L = L;
            aa.nfam = nfam;
            aa.cand_off = ccnt;
            aa.cand = ccand;
            aa.begin = t.begin;
            aa.end = t.end;
            aa.rec = static_cast<const float4 *>(t.sorted_rec);
            aa.stride_f4 = stride_f4;
            aa.aoff = cacnt;
            aa.abuf = abuf;
            aa.n = cl_n;
            aa.slot = cslot;
            aa.work = work ? work + 2 : nullptr;
            aa.np = np;
            aa.psc = psc;
            aa.eoff = n_extra > 0 ? ecnt : nullptr;
            aa.apre = apre;
            aa.pc = pc;
            aa.bad = bad;
            CpClassArgs ca{};
            ca.L = L;
            ca.nq = ngrp;
            ca.rshort = rshort;
            ca.cand_off = lcnt;
            ca.cand = lcand;
            ca.begin = t.begin;
            ca.end = t.end;
            ca.rec = static_cast<const float4 *>(t.sorted_rec);
            ca.stride_f4 = stride_f4;
            ca.aoff = lacnt;
            ca.dlist = dlist;
            ca.slist = slist;
            ca.nd = nd;
            ca.on_grid = dguard;
            ca.ns = nsh;
            ca.cost = cost;
            hipLaunchKernelGGL(k_cp_fill, nfam + ngrp, kFillThreads, qshm, s, qc, ql, aa, ca);
            if (n_extra > 0)
                hipLaunchKernelGGL(k_cp_assign_extra, n_extra, kFillThreads, 0, s, aa);
            const OrderJob leaf_order{nleaf, nullptr, cost, nullptr, order};
            CpItemArgs ia{};
            ia.L = L;
            ia.ncl = ncl;
            ia.nfam = nfam;
            ia.n = cl_n;
            ia.eoff = n_extra > 0 ? ecnt : nullptr;
            ia.pc = pc;
            ia.amax = item_atoms;
            ia.item_off = item_off;
            ia.it_cl = it_cl;
            ia.it_a0 = it_a0;
            ia.it_na = it_na;
            ia.n_items = n_items;
            const OrderJob item_order{max_items, n_items, it_na, nullptr, it_order};
            hipLaunchKernelGGL(k_cp_plan, ncl > 0 ? 2 : 1, kPlanThreads, 0, s, leaf_order, ia,
                               item_order, (const int *)bad, (const uint32_t *)flags, hres,
                               kFlagWords);
            RISM_HIP(hipEventRecord(fev, s));
        }
        RISM_HIP(hipGetLastError());

        // far field of every item into its part of its cluster's proxies
        // (heaviest first), then the downward pass
        if (ncl > 0) {
            PhaseTimer pu(ev, RISM_PHASE_UPWARD, s);
            CpSweepArgs sa{};
            sa.L = L;
            sa.order = it_order;
            sa.it_cl = it_cl;
            sa.it_a0 = it_a0;
            sa.it_na = it_na;
            sa.slot = cslot;
            sa.abuf = abuf;
            sa.degree = deg;
            sa.np = np;
            sa.yk = (float)a.asym.yk;
            sa.kappa = a.asym.kappa;
            sa.eta = a.asym.eta;
            sa.nc = nc;
            sa.part = part;
            sa.n_items = n_items;
            sa.bad = bad;
            sa.psc = psc;
            if (taylor) {
                const size_t tshm = cp_taylor_lds(deg, a.asym_on, paper);
                if (a.asym_on && paper)
                    hipLaunchKernelGGL((k_cp_taylor<true, true>), max_items, kBlock, tshm, s, sa);
                else if (a.asym_on)
                    hipLaunchKernelGGL((k_cp_taylor<true, false>), max_items, kBlock, tshm, s, sa);
                else
                    hipLaunchKernelGGL((k_cp_taylor<false, false>), max_items, kBlock, tshm, s,
                                       sa);
            } else if (a.asym_on) {
                launch_sweep<true>(max_items, np, deg, n_cu, sa, s);
            } else {
                launch_sweep<false>(max_items, np, deg, n_cu, sa, s);
            }
        }
        if (ncl > 0) {
            PhaseTimer pt(ev, RISM_PHASE_DOWNWARD, s);
            CpDownArgs da{};
            da.L = L;
            da.degree = deg;
            da.ncomp = nc;
            da.nc = down_nc;
            da.M = ta.M;
            for (int l = 0; l <= kCpMaxLev; ++l)
                for (int ax = 0; ax < 3; ++ax) da.mrow0[l][ax] = ta.mrow0[l][ax];
            da.item_off = item_off;
            da.bad = bad;
            da.part = part;
            da.V = V;
            const size_t dshm = cp_down_lds(deg, down_nc);
            const int slots = cp_down_slots(deg, down_nc);
            auto chain = [&](int lo, int hi, int top_v) {
                da.lo = lo;
                da.hi = hi;
                da.top_v = top_v;
                const int ng = L.cx[lo] * L.cy[lo] * L.cz[lo];
                if (deg == 8 && slots == 4)   // the usual degree, two components
                    hipLaunchKernelGGL((k_cp_down_chain<4, 9>), ng, kDownThreads, dshm, s, da);
                else
                    switch (slots) {
                    case 1: hipLaunchKernelGGL((k_cp_down_chain<1, 0>), ng, kDownThreads, dshm, s, da); break;
                    case 2: hipLaunchKernelGGL((k_cp_down_chain<2, 0>), ng, kDownThreads, dshm, s, da); break;
                    case 4: hipLaunchKernelGGL((k_cp_down_chain<4, 0>), ng, kDownThreads, dshm, s, da); break;
                    case 8: hipLaunchKernelGGL((k_cp_down_chain<8, 0>), ng, kDownThreads, dshm, s, da); break;
                    default: hipLaunchKernelGGL((k_cp_down_chain<16, 0>), ng, kDownThreads, dshm, s, da); break;
                    }
            };
            if (a.solute->n > kChainMaxAtoms) {
                // one launch per level: every cluster's items are summed once
                chain(L.T, L.T, 0);
                for (int l = L.T - 1; l >= 1; --l) chain(l, l + 1, 1);
            } else if (L.T >= 3) {
                chain(2, L.T, 0);   // V_2 from the top
                chain(1, 2, 1);     // V_1 from V_2
            } else {
                chain(1, L.T, 0);
            }
        }
        RISM_HIP(hipGetLastError());

        // leaves
        CpLeafArgs la{};
        la.L = L;
        la.g = a.g;
        la.out = a.out;
        la.asym = a.asym;
        la.rec = t.sorted_rec;
        la.aoff = lacnt;
        la.dlist = dlist;
        la.slist = slist;
        la.nd = nd;
        la.on_grid = dguard;
        la.ns = nsh;
        la.order = order;
        la.bad = bad;
        la.V = V;
        la.Lg = ta.Lg;
        for (int ax = 0; ax < 3; ++ax) la.lrow0[ax] = ta.lrow0[ax];
        la.degree = deg;
        la.np = np;
        la.taylor = taylor;
        la.ncomp = nc;
        la.paper = paper;
        la.work = work;
        {
            PhaseTimer pt(ev, RISM_PHASE_EVAL, s);
            const int ljm = a.lj_mode == LJ_CUT && a.lj_uniform ? LJ_CUT1 : a.lj_mode;
            switch (a.sp.ns_pad) {
            case 1: launch_leaf_ns<1>(ljm, a.asym_on, B, nleaf, leaf_shm, la, s); break;
            case 2: launch_leaf_ns<2>(ljm, a.asym_on, B, nleaf, leaf_shm, la, s); break;
            case 4: launch_leaf_ns<4>(ljm, a.asym_on, B, nleaf, leaf_shm, la, s); break;
            default: launch_leaf_ns<8>(ljm, a.asym_on, B, nleaf, leaf_shm, la, s); break;
            }
        }
        RISM_HIP(hipGetLastError());
        return RISM_OK;
    };

    // copied: the flags reached hres through k_cp_plan (a full pass); only
    // that kernel is waited for
    auto read_back = [&](bool copied) -> int {
        if (copied) {
            RISM_HIP(hipEventSynchronize(fev));
        } else {
            RISM_HIP(hipMemcpyAsync(hres, flags, kFlagWords * sizeof(uint32_t),
                                    hipMemcpyDeviceToHost, s));
            RISM_HIP(hipStreamSynchronize(s));
        }
        if (a.stage_err && (hres[8] || hres[9])) {
            set_error(hres[8] ? "non-finite atom input or negative sigma/eps"
                              : "lj_tol must be below eps_ga of every pair");
            return RISM_E_INVALID;
        }
        if (hres[5]) {
            set_error("treecode_cp: neighbour query stack overflow");
            return RISM_E_UNSUPPORTED;
        }
        if (ncl == 0) hres[0] = hres[1] = hres[4] = 0;
        return RISM_OK;
    };
    bool done = false;
    if (have) {
        // speculative pass with the cached capacities (checked by the scans)
        if ((rc = second_half(cached))) return rc;
        if ((rc = read_back(true))) return rc;
        done = hres[6] == 0;
    } else {
        if ((rc = read_back(false))) return rc;
    }
    if (!done) {
        // exact capacities from the counts just read
        CpCaps exact{};
        for (int k = 0; k < 5; ++k) exact.c[k] = hres[k];
        hipLaunchKernelGGL(k_fill_int, 1, 64, 0, s, bad, 1, 0);
        if ((rc = second_half(exact))) return rc;
        std::lock_guard<std::mutex> lk(g_cp_caps_mu);
        if (g_cp_caps.size() > 64) g_cp_caps.clear();
        CpCaps &c = g_cp_caps[shape];
        for (int k = 0; k < 5; ++k) c.c[k] = std::max(c.c[k], exact.c[k]);
    }
    RISM_HIP(hipGetLastError());
    st.n_batches = nleaf;
    st.n_nodes = ncl;
    if (work) {
        unsigned long long hw[4];
        RISM_HIP(hipMemcpyAsync(hw, work, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        RISM_HIP(hipStreamSynchronize(s));
        st.pairs_direct = (double)hw[0];
        st.pairs_short = (double)hw[1];
        st.pairs_far = (double)hw[2];
    }
    return RISM_OK;
}

}  // namespace rism
