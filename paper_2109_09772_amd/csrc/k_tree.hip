// Particle-cluster treecode on the GPU: source octree on the atoms (Morton
// keys, LSD radix sort, level-by-level split), node boxes, barycentric
// Chebyshev proxy charges (upward pass), and the per-batch interaction lists
// that drive the evaluation kernel (k_tree_eval.hip).
//
// Reading of the paper (Sec. 2.3): the paper builds its tree on the grid
// targets and expands each source atom about target clusters (cluster-
// particle, Taylor).  This file is the particle-cluster orientation with
// interpolation proxies: the far field of a source cluster C seen from a
// batch B of grid points is sum_k qhat_k phi(x, s_k) over the (n+1)^3
// Chebyshev points s_k of C's box, with qhat_k = sum_{j in C} L_k(y_j) q_j.
// It is accepted when (r_B + r_C) < theta |c_B - c_C| and C holds more
// atoms than proxies; otherwise C is opened, and leaves are summed directly.
#include <algorithm>
#include <cmath>
#include <utility>

#include "cheb.h"
#include "pair.h"
#include "tree.h"

namespace rism {

namespace {

constexpr int kRsItems = 8;
constexpr int kRsTile = kBlock * kRsItems;   // keys per radix-sort workgroup

// ------------------------------------------------------------ bounding box

__global__ __launch_bounds__(kBlock) void k_bbox_partial(const float4 *rec, int stride_f4, int n,
                                                         double *part)
{
    __shared__ double red[6][kBlock];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        float4 a = rec[(size_t)i * stride_f4];       // xh, yh, zh, q
        float4 b = rec[(size_t)i * stride_f4 + 1];   // xl, yl, zl, pad
        double v[3] = {(double)a.x + b.x, (double)a.y + b.y, (double)a.z + b.z};
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], v[k]);
            hi[k] = fmax(hi[k], v[k]);
        }
    }
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = lo[k];
        red[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 3; ++k) {
                red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
                red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Key cube of the atoms: lower corner and edge (the largest extent, padded).
__device__ __forceinline__ void bbox_cube(const double lo[3], const double hi[3], double *bbox)
{
    double ext = fmax(fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    ext = fmax(ext, 1e-3) * (1.0 + 1e-9);
    for (int k = 0; k < 3; ++k) {
        bbox[k] = lo[k];
        bbox[3 + k] = ext;   // cube edge
    }
}

// The key cube from per-workgroup boxes: one workgroup of kBlock threads.
__global__ __launch_bounds__(kBlock) void k_bbox_final(const double *part, int nparts,
                                                       double *bbox)
{
    __shared__ double red[6][kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int p = threadIdx.x; p < nparts; p += kBlock)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], part[6 * p + k]);
            hi[k] = fmax(hi[k], part[6 * p + 3 + k]);
        }
    for (int off = 32; off > 0; off >>= 1)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmax(hi[k], __shfl_xor(hi[k], off));
        }
    if (lane == 0)
        for (int k = 0; k < 3; ++k) {
            red[k][wave] = lo[k];
            red[3 + k][wave] = hi[k];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w)
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], red[k][w]);
                hi[k] = fmax(hi[k], red[3 + k][w]);
            }
        bbox_cube(lo, hi, bbox);
    }
}

// ------------------------------------------------------------ Morton keys

__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

// 30-bit Morton key of atom i in the key cube.
__device__ __forceinline__ uint32_t atom_key(const float4 *rec, int stride_f4, int i,
                                             const double *bbox)
{
    float4 a = rec[(size_t)i * stride_f4];
    float4 b = rec[(size_t)i * stride_f4 + 1];
    double v[3] = {(double)a.x + b.x, (double)a.y + b.y, (double)a.z + b.z};
    uint32_t c[3];
    for (int k = 0; k < 3; ++k) {
        double t = (v[k] - bbox[k]) / bbox[3 + k] * (double)(1 << kMortonBits);
        int ci = (int)floor(t);
        ci = ci < 0 ? 0 : (ci > (1 << kMortonBits) - 1 ? (1 << kMortonBits) - 1 : ci);
        c[k] = (uint32_t)ci;
    }
    return spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
}

__global__ __launch_bounds__(kBlock) void k_morton(const float4 *rec, int stride_f4, int n,
                                                   const double *bbox, uint32_t *keys, int *idx)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    keys[i] = atom_key(rec, stride_f4, i, bbox);
    idx[i] = i;
}

// ------------------------------------------------------------ radix sort

__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t *keys, int n, int shift,
                                                    int nblocks, uint32_t *hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        int i = base + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of a[0..n) in place by one 1024-thread workgroup; n is read
// from n_dev if given.  If total_out is given it receives the sum.
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t *a, int n_host, const int *n_dev,
                                                    uint32_t *total_out)
{
    __shared__ uint32_t s[1024];
    const int n = n_dev ? *n_dev : n_host;
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int lo = t * per < n ? t * per : n;
    const int hi = lo + per < n ? lo + per : n;
    // each thread's segment in runs of kScanRun loads issued together
    constexpr int kScanRun = 16;
    uint32_t sum = 0;
    for (int i0 = lo; i0 < hi; i0 += kScanRun) {
        uint32_t v[kScanRun];
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) v[u] = i0 + u < hi ? a[i0 + u] : 0u;
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) sum += v[u];
    }
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    uint32_t run = s[t] - sum;
    for (int i0 = lo; i0 < hi; i0 += kScanRun) {
        uint32_t v[kScanRun];
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) v[u] = i0 + u < hi ? a[i0 + u] : 0u;
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) {
            if (i0 + u < hi) a[i0 + u] = run;
            run += v[u];
        }
    }
    if (total_out && t == 1023) *total_out = s[1023];
}

__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t *kin, const int *vin,
                                                       uint32_t *kout, int *vout, int n, int shift,
                                                       int nblocks, const uint32_t *offs)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kBlock / 64][256];
    __shared__ uint32_t wbase[kBlock / 64][256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    run[t] = offs[(size_t)t * nblocks + blockIdx.x];
    for (int w = 0; w < kBlock / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int base = blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        const int i = base + r * kBlock + t;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t dig = (key >> shift) & 255u;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const int rank = __popcll(m & lt);
        if (valid && rank == 0) wcnt[wave][dig] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t acc = run[t];
        for (int w = 0; w < kBlock / 64; ++w) {
            wbase[w][t] = acc;
            acc += wcnt[w][t];
        }
        run[t] = acc;
        __syncthreads();
        if (valid) {
            const uint32_t dst = wbase[wave][dig] + (uint32_t)rank;
            kout[dst] = key;
            vout[dst] = vin[i];
        }
        __syncthreads();
        for (int w = 0; w < kBlock / 64; ++w) wcnt[w][t] = 0;
        __syncthreads();
    }
}

// ------------------------------------------------------------ octree

__global__ void k_tree_root(int n, int *begin, int *end, int *level, int *level_start, int *n_nodes,
                            int *flags, int *clear, int n_clear)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int k = 0; k < n_clear; ++k) clear[k] = 0;
    begin[0] = 0;
    end[0] = n;
    level[0] = 0;
    level_start[0] = 0;
    level_start[1] = 1;
    for (int l = 2; l < kMortonBits + 2; ++l) level_start[l] = 1;
    *n_nodes = 1;
    flags[0] = 0;
}

__global__ void k_level_count(const int *level_start, int lvl, int *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = level_start[lvl + 1] - level_start[lvl];
}

__device__ __forceinline__ int lower_digit(const uint32_t *keys, int lo, int hi, int shift, int d)
{
    // first index in [lo, hi) whose 3-bit digit at `shift` is >= d (digits are
    // non-decreasing inside a node's range)
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((int)((keys[mid] >> shift) & 7u) < d) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_split_count(const uint32_t *keys, const int *begin,
                                                        const int *end, const int *level_start,
                                                        int lvl, int leaf, uint32_t *cnt)
{
    const int s0 = level_start[lvl], s1 = level_start[lvl + 1];
    const int shift = 3 * (kMortonBits - 1 - lvl);
    for (int i = s0 + blockIdx.x * kBlock + threadIdx.x; i < s1; i += gridDim.x * kBlock) {
        const int b = begin[i], e = end[i];
        uint32_t c = 0;
        if (e - b > leaf && lvl < kMortonBits) {
            int prev = b;
            for (int d = 1; d <= 8; ++d) {
                int nx = d == 8 ? e : lower_digit(keys, prev, e, shift, d);
                if (nx > prev) ++c;
                prev = nx;
            }
        }
        cnt[i - s0] = c;
    }
}

__global__ __launch_bounds__(kBlock) void k_split_write(const uint32_t *keys, int *begin, int *end,
                                                        int *level, int *child0, int *nchild,
                                                        int *level_start, int lvl, int leaf,
                                                        const uint32_t *off, const uint32_t *total,
                                                        int cap, int *n_nodes, int *flags)
{
    const int s0 = level_start[lvl], s1 = level_start[lvl + 1];
    const int shift = 3 * (kMortonBits - 1 - lvl);
    const int first_child = s1;   // children of this level start right after it
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int tot = s1 + (int)*total;
        if (tot > cap) {
            flags[0] = 1;
            tot = cap;   // never let a later level index past the node arrays
        }
        level_start[lvl + 2] = tot;
        *n_nodes = tot;
    }
    for (int i = s0 + blockIdx.x * kBlock + threadIdx.x; i < s1; i += gridDim.x * kBlock) {
        const int b = begin[i], e = end[i];
        int c = 0;
        if (e - b > leaf && lvl < kMortonBits) {
            const int base = first_child + (int)off[i - s0];
            child0[i] = base;
            int prev = b;
            for (int d = 1; d <= 8; ++d) {
                int nx = d == 8 ? e : lower_digit(keys, prev, e, shift, d);
                if (nx > prev) {
                    int j = base + c;
                    if (j < cap) {
                        begin[j] = prev;
                        end[j] = nx;
                        level[j] = lvl + 1;
                        child0[j] = -1;
                        nchild[j] = 0;
                    }
                    ++c;
                }
                prev = nx;
            }
        } else {
            child0[i] = -1;
        }
        nchild[i] = c;
    }
}

// ------------------------------------------------- one-workgroup builder

// Small trees: keys formed and ranked by many workgroups (each forms every
// key, since it counts over all of them), which also place the atom records
// in key order; then one workgroup builds the octree level by level with
// block-wide scans.
// Produces the same permutation and nodes as the multi-kernel build.
constexpr int kSmallThreads = 1024;
constexpr int kRankTargets = 64;   // atoms ranked per workgroup
// Largest tree built this way: the ranking costs n^2 / 64 comparisons per
// lane, about 20 us at 16K atoms, still below the multi-kernel radix sort and
// level-by-level split (about 0.3 ms at 14,000 atoms).
constexpr int kSmallTreeMax = 16384;
static_assert(kSmallTreeMax <= (1 << 14), "k_tree_rank packs the atom index into 14 bits");

// Stores node's box and its centre and radius (half-diagonal) from the
// box's corners.
__device__ __forceinline__ void store_node_box(int node, const double lo[3], const double hi[3],
                                               double *box, double *centre)
{
    double r2 = 0;
    for (int k = 0; k < 3; ++k) {
        box[6 * node + k] = lo[k];
        box[6 * node + 3 + k] = hi[k];
        centre[4 * node + k] = 0.5 * (lo[k] + hi[k]);
        r2 += 0.25 * (hi[k] - lo[k]) * (hi[k] - lo[k]);
    }
    centre[4 * node + 3] = sqrt(r2);
}

// Key cube of a small tree's atoms by one workgroup of kSmallThreads: a
// block-wide reduction of the positions.  bb: 6 doubles in LDS.
__device__ __forceinline__ void small_key_cube(const float4 *rec, int stride_f4, int n,
                                               const double *bpart, int nbpart, double *bb,
                                               double *tight)
{
    __shared__ double red[6][kSmallThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    if (bpart) {   // the staging's per-workgroup boxes of the same positions
        for (int i = tid; i < nbpart; i += kSmallThreads)
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], bpart[6 * i + k]);
                hi[k] = fmax(hi[k], bpart[6 * i + 3 + k]);
            }
    } else {
        for (int i = tid; i < n; i += kSmallThreads) {
            float4 a = rec[(size_t)i * stride_f4];
            float4 b = rec[(size_t)i * stride_f4 + 1];
            double v[3] = {(double)a.x + b.x, (double)a.y + b.y, (double)a.z + b.z};
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], v[k]);
                hi[k] = fmax(hi[k], v[k]);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmax(hi[k], __shfl_xor(hi[k], off));
        }
    if (lane == 0)
        for (int k = 0; k < 3; ++k) {
            red[k][wave] = lo[k];
            red[3 + k][wave] = hi[k];
        }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kSmallThreads / 64; ++w)
            for (int k = 0; k < 3; ++k) {
                red[k][0] = fmin(red[k][0], red[k][w]);
                red[3 + k][0] = fmax(red[3 + k][0], red[3 + k][w]);
            }
        const double l3[3] = {red[0][0], red[1][0], red[2][0]};
        const double h3[3] = {red[3][0], red[4][0], red[5][0]};
        for (int k = 0; k < 3; ++k) {
            tight[k] = l3[k];
            tight[3 + k] = h3[k];
        }
        bbox_cube(l3, h3, bb);
    }
    __syncthreads();
}

// Sorted position of every atom by (key, index), i.e. the position a stable
// sort by key gives: each workgroup forms all keys in LDS (workgroup 0 also
// stores them) and ranks 64 atoms, each of its sixteen waves counting over a
// sixteenth of the keys (four keys per broadcast read).  The ranked atoms'
// records are then placed at their sorted positions (the padding records,
// n <= i < npad, stay last).  Workgroup 0 also stores the box of the root
// node (all n atoms, node 0) from the same reduction, so that the node-box
// pass can leave out its longest node.
constexpr int kRankThreads = kSmallThreads;
constexpr int kRankWaves = kRankThreads / 64;

__global__ __launch_bounds__(kRankThreads) void k_tree_rank(const float4 *rec, int stride_f4,
                                                            int n, int npad,
                                                            const double *bpart, int nbpart,
                                                            int *rank, uint32_t *keys, int *perm,
                                                            float4 *sorted, double *root_box,
                                                            double *root_centre)
{
    // every atom's (key, index) as one 64-bit word, key << 14 | index (the
    // index is below kSmallTreeMax = 2^14): the words are distinct, so one
    // unsigned comparison orders them as the stable sort does
    extern __shared__ uint4 k4[];   // [round_up(n, 4 kRankWaves) / 2]
    __shared__ int part[kRankWaves][kRankTargets];
    __shared__ double bb[6], tb[6];
    unsigned long long *kk = reinterpret_cast<unsigned long long *>(k4);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    small_key_cube(rec, stride_f4, n, bpart, nbpart, bb, tb);
    if (blockIdx.x == 0 && tid == 0) store_node_box(0, tb, tb + 3, root_box, root_centre);
    const int np = (n + 4 * kRankWaves - 1) / (4 * kRankWaves) * (4 * kRankWaves);
    for (int i = tid; i < np; i += kRankThreads) {
        const uint32_t key = i < n ? atom_key(rec, stride_f4, i, bb) : 0u;
        kk[i] = i < n ? ((unsigned long long)key << 14) | (unsigned)i : ~0ull;
        if (blockIdx.x == 0 && i < n) keys[i] = key;
    }
    __syncthreads();
    const int t = blockIdx.x * kRankTargets + lane;
    const int q = np / 2 / kRankWaves;   // units of two words per wave
    int c = 0;
    if (t < n) {
        const unsigned long long w = kk[t];
#pragma unroll 4
        for (int j = wave * q; j < (wave + 1) * q; ++j) {
            const uint4 v = k4[j];   // the same j on every lane: one broadcast read
            c += (((unsigned long long)v.y << 32) | v.x) < w ? 1 : 0;
            c += (((unsigned long long)v.w << 32) | v.z) < w ? 1 : 0;
        }
    }
    part[wave][lane] = c;
    __syncthreads();
    __shared__ int rk[kRankTargets];
    if (wave == 0 && t < n) {
        int r = 0;
        for (int w = 0; w < kRankWaves; ++w) r += part[w][lane];
        rank[t] = r;
        perm[r] = t;
        rk[lane] = r;
    }
    __syncthreads();
    // the ranked atoms' records, one float4 per thread
    for (int u = tid; u < kRankTargets * stride_f4; u += kRankThreads) {
        const int j = u / stride_f4, k = u - j * stride_f4, tj = blockIdx.x * kRankTargets + j;
        if (tj < n) sorted[(size_t)rk[j] * stride_f4 + k] = rec[(size_t)tj * stride_f4 + k];
    }
    if (blockIdx.x == 0)
        for (int u = tid; u < (npad - n) * stride_f4; u += kRankThreads)
            sorted[(size_t)n * stride_f4 + u] = rec[(size_t)n * stride_f4 + u];
}

__device__ __forceinline__ int block_excl_scan(int v, int *wsum, int &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < kSmallThreads / 64; ++w) {
        if (w < wave) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();   // wsum is reused by the next scan
    total = tot;
    return base + x - v;
}

__device__ __forceinline__ int lower_digit_lds(const unsigned long long *sk, int lo, int hi,
                                               int shift, int d)
{
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((int)((sk[mid] >> (32 + shift)) & 7u) < d) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct SmallTreeArgs {
    const uint32_t *keys;
    const int *rank;
    int n, leaf, cap;
    int *begin, *end, *level, *child0, *nchild, *level_start, *n_nodes, *flags;
    int *clear, n_clear;   // words set to 0 (TreeDev::clear)
};

// Dynamic LDS of k_tree_small: the sorted keys.
inline size_t small_tree_lds(int n)
{
    return (size_t)n * sizeof(unsigned long long);
}

__global__ __launch_bounds__(kSmallThreads) void k_tree_small(SmallTreeArgs a)
{
    extern __shared__ unsigned long long sk[];   // [n] (key << 32) | index, sorted
    __shared__ int wsum[kSmallThreads / 64];
    __shared__ int ls[kMortonBits + 2];
    const int tid = threadIdx.x, lane = tid & 63;
    const int n = a.n, leaf = a.leaf, cap = a.cap;
    int *begin = a.begin, *end = a.end, *level = a.level, *child0 = a.child0,
        *nchild = a.nchild, *flags = a.flags;

    if (tid < a.n_clear) a.clear[tid] = 0;
    for (int i = tid; i < n; i += kSmallThreads)
        sk[a.rank[i]] = ((unsigned long long)a.keys[i] << 32) | (unsigned)i;
    __syncthreads();
    // octree, level by level
    if (tid == 0) {
        begin[0] = 0;
        end[0] = n;
        level[0] = 0;
        ls[0] = 0;
        for (int l = 1; l < kMortonBits + 2; ++l) ls[l] = 1;
        flags[0] = 0;
    }
    __syncthreads();
    for (int lvl = 0; lvl < kMortonBits; ++lvl) {
        const int s0 = ls[lvl], s1 = ls[lvl + 1];
        const int shift = 3 * (kMortonBits - 1 - lvl);
        int running = 0;
        // eight threads per node: thread d finds the first atom of the node
        // whose digit is >= d (the node's atoms are sorted, so the children
        // are the runs between these boundaries)
        for (int c0 = s0; c0 < s1; c0 += kSmallThreads / 8) {
            const int i = c0 + (tid >> 3), d = tid & 7;
            int b = 0, e = 0;
            const bool split = i < s1 && (e = end[i]) - (b = begin[i]) > leaf;
            const int lo = split ? (d == 0 ? b : lower_digit_lds(sk, b, e, shift, d)) : 0;
            int hi = __shfl_down(lo, 1);
            if (d == 7) hi = e;
            const bool ne = split && hi > lo;   // child of digit d is not empty
            const unsigned long long m = __ballot(ne);
            const int g0 = lane & ~7;
            const unsigned gm = (unsigned)((m >> g0) & 0xffull);
            const int c = __popc(gm);
            int tot;
            const int off = block_excl_scan(d == 0 ? c : 0, wsum, tot);
            const int base = s1 + running + __shfl(off, g0);
            if (i < s1) {
                if (ne) {
                    const int j = base + __popc(gm & ((1u << d) - 1u));
                    if (j < cap) {
                        begin[j] = lo;
                        end[j] = hi;
                        level[j] = lvl + 1;
                        child0[j] = -1;
                        nchild[j] = 0;
                    }
                }
                if (d == 0) {
                    child0[i] = split ? base : -1;
                    nchild[i] = c;
                }
            }
            running += tot;
        }
        __syncthreads();   // children written before the next level reads them
        if (tid == 0) {
            int t = s1 + running;
            if (t > cap) {
                flags[0] = 1;
                t = cap;
            }
            ls[lvl + 2] = t;
        }
        __syncthreads();
        if (ls[lvl + 2] == s1) {
            // no node at the next level, so none at any later one
            if (tid > lvl + 2 && tid < kMortonBits + 2) ls[tid] = s1;
            __syncthreads();
            break;
        }
    }
    if (tid < kMortonBits + 2) a.level_start[tid] = ls[tid];
    if (tid == 0) *a.n_nodes = ls[kMortonBits + 1];
}

template <int NS>
__global__ __launch_bounds__(kBlock) void k_permute(const AtomF32<NS> *in, const int *perm, int n,
                                                    int npad, AtomF32<NS> *out)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = in[perm[i]];
    else if (i < npad) out[i] = in[i];   // padding records stay last
}

// Atoms per chunk of the chunk boxes: a node of more than 2 kBoxChunk atoms
// takes the boxes of the whole chunks it covers and reads only the atoms of
// its two partial chunks.
constexpr int kBoxChunk = 2048;

// Box of the sorted atoms [b, e) of this wave, accumulated into lo / hi
// (lane-partial; four atoms per lane per step, their loads issued together).
__device__ __forceinline__ void atoms_box(const float4 *rec, int stride_f4, int b, int e,
                                          int lane, double lo[3], double hi[3])
{
    for (int i0 = b + lane; i0 < e; i0 += 4 * 64) {
        float4 a[4], c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + 64 * u;
            if (i < e) {
                a[u] = rec[(size_t)i * stride_f4];
                c[u] = rec[(size_t)i * stride_f4 + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i0 + 64 * u >= e) break;
            const double v[3] = {(double)a[u].x + c[u].x, (double)a[u].y + c[u].y,
                                 (double)a[u].z + c[u].z};
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], v[k]);
                hi[k] = fmax(hi[k], v[k]);
            }
        }
    }
}

__device__ __forceinline__ void wave_box(double lo[3], double hi[3])
{
    for (int off = 32; off > 0; off >>= 1)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmax(hi[k], __shfl_xor(hi[k], off));
        }
}

// Box of every chunk of kBoxChunk sorted atoms: one wave per chunk.
__global__ __launch_bounds__(kBlock) void k_chunk_box(const float4 *rec, int stride_f4, int n,
                                                      double *cbox)
{
    const int lane = threadIdx.x & 63;
    const int c = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int b = c * kBoxChunk;
    if (b >= n) return;   // whole wave
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    atoms_box(rec, stride_f4, b, min(b + kBoxChunk, n), lane, lo, hi);
    wave_box(lo, hi);
    if (lane == 0)
        for (int k = 0; k < 3; ++k) {
            cbox[6 * c + k] = lo[k];
            cbox[6 * c + 3 + k] = hi[k];
        }
}

// Tight box, centre and radius of every node from `first` on (the nodes
// before it are done): one wave per node.  With cbox (the chunk boxes), a
// node of more than 2 kBoxChunk atoms reads the boxes of its whole chunks
// instead of their atoms.
__global__ __launch_bounds__(kBlock) void k_node_box(const float4 *rec, int stride_f4,
                                                     const int *begin, const int *end,
                                                     const int *n_nodes, const double *cbox,
                                                     double *box, double *centre, int first)
{
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int nw = gridDim.x * (kBlock / 64);
    const int nn = *n_nodes;
    for (int node = first + wave; node < nn; node += nw) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        const int b = begin[node], e = end[node];
        if (cbox && e - b > 2 * kBoxChunk) {
            const int c0 = (b + kBoxChunk - 1) / kBoxChunk, c1 = e / kBoxChunk;
            atoms_box(rec, stride_f4, b, c0 * kBoxChunk, lane, lo, hi);
            atoms_box(rec, stride_f4, c1 * kBoxChunk, e, lane, lo, hi);
            for (int c = c0 + lane; c < c1; c += 64)
                for (int k = 0; k < 3; ++k) {
                    lo[k] = fmin(lo[k], cbox[6 * c + k]);
                    hi[k] = fmax(hi[k], cbox[6 * c + 3 + k]);
                }
        } else {
            atoms_box(rec, stride_f4, b, e, lane, lo, hi);
        }
        wave_box(lo, hi);
        if (lane == 0) store_node_box(node, lo, hi, box, centre);
    }
}

// ------------------------------------------------------------ upward pass

constexpr int kTile = 64;

// Leaves: qhat_k = sum_j q_j Lx_k1(x_j) Ly_k2(y_j) Lz_k3(z_j) from the atoms.
// Internal nodes: qhat_P = sum_children (Mx (x) My (x) Mz) qhat_c, with
// M[k][m] = L^P_k(s^c_m): exact, since each L^P_k is a polynomial of degree n
// that the child's degree-n interpolation reproduces.
__global__ __launch_bounds__(kBlock) void k_upward_level(const float4 *rec, int stride_f4,
                                                         const int *begin, const int *end,
                                                         const int *child0, const int *nchild,
                                                         const double *box, const int *level_start,
                                                         int lvl, int deg, double *pq, double *pbox)
{
    extern __shared__ double sm[];
    const int n1 = deg + 1, np = n1 * n1 * n1;
    const int s0 = level_start[lvl], s1 = level_start[lvl + 1];
    double *Lx = sm;                        // [kTile][n1] (leaf) / [n1][n1] (internal)
    double *Ly = Lx + kTile * n1;
    double *Lz = Ly + kTile * n1;
    double *qa = Lz + kTile * n1;           // [kTile]
    double *qc = qa + kTile;                // [np] child proxies
    double *t1 = qc + np;                   // [np]
    double *t2 = t1 + np;                   // [np]
    double *acc = t2 + np;                  // [np], each entry owned by one thread
    for (int node = s0 + blockIdx.x; node < s1; node += gridDim.x) {
        double pb[6];
        proxy_box(box + 6 * node, pb);
        if (threadIdx.x < 6) pbox[6 * node + threadIdx.x] = pick3(threadIdx.x < 3 ? pb : pb + 3, threadIdx.x % 3);
        for (int k = threadIdx.x; k < np; k += kBlock) acc[k] = 0.0;
        if (nchild[node] == 0) {
            for (int t0 = begin[node]; t0 < end[node]; t0 += kTile) {
                const int cnt = min(kTile, end[node] - t0);
                __syncthreads();
                if (threadIdx.x < cnt) {
                    const int i = t0 + threadIdx.x;
                    float4 a = rec[(size_t)i * stride_f4];
                    float4 b = rec[(size_t)i * stride_f4 + 1];
                    lagrange_to((double)a.x + b.x, pb[0], pb[3], deg, Lx + threadIdx.x * n1, 1);
                    lagrange_to((double)a.y + b.y, pb[1], pb[4], deg, Ly + threadIdx.x * n1, 1);
                    lagrange_to((double)a.z + b.z, pb[2], pb[5], deg, Lz + threadIdx.x * n1, 1);
                    qa[threadIdx.x] = (double)a.w;
                }
                __syncthreads();
                for (int k = threadIdx.x; k < np; k += kBlock) {
                    const int k1 = k % n1, k2 = (k / n1) % n1, k3 = k / (n1 * n1);
                    double s = acc[k];
                    for (int j = 0; j < cnt; ++j)
                        s += qa[j] * Lx[j * n1 + k1] * Ly[j * n1 + k2] * Lz[j * n1 + k3];
                    acc[k] = s;
                }
            }
        } else {
            for (int c = child0[node]; c < child0[node] + nchild[node]; ++c) {
                __syncthreads();
                double cb[6];
                proxy_box(box + 6 * c, cb);
                // interpolation matrices M[k][m] = L^P_k(s^c_m), per axis
                if (threadIdx.x < 3 * n1) {
                    const int ax = threadIdx.x / n1, m = threadIdx.x % n1;
                    double *M = ax == 0 ? Lx : (ax == 1 ? Ly : Lz);
                    lagrange_to(cheb_point(pick3(cb, ax), pick3(cb + 3, ax), m, deg), pick3(pb, ax),
                                pick3(pb + 3, ax), deg, M + m, n1);
                }
                for (int k = threadIdx.x; k < np; k += kBlock) qc[k] = pq[(size_t)c * np + k];
                __syncthreads();
                // t1[k1][m2][m3] = sum_m1 Mx[k1][m1] qc[m1][m2][m3]   (x fastest)
                for (int k = threadIdx.x; k < np; k += kBlock) {
                    const int k1 = k % n1, rest = k / n1;
                    double s = 0;
                    for (int m1 = 0; m1 < n1; ++m1) s += Lx[k1 * n1 + m1] * qc[rest * n1 + m1];
                    t1[k] = s;
                }
                __syncthreads();
                for (int k = threadIdx.x; k < np; k += kBlock) {
                    const int k1 = k % n1, k2 = (k / n1) % n1, m3 = k / (n1 * n1);
                    double s = 0;
                    for (int m2 = 0; m2 < n1; ++m2) s += Ly[k2 * n1 + m2] * t1[(m3 * n1 + m2) * n1 + k1];
                    t2[k] = s;
                }
                __syncthreads();
                for (int k = threadIdx.x; k < np; k += kBlock) {
                    const int k12 = k % (n1 * n1), k3 = k / (n1 * n1);
                    double s = acc[k];
                    for (int m3 = 0; m3 < n1; ++m3) s += Lz[k3 * n1 + m3] * t2[m3 * n1 * n1 + k12];
                    acc[k] = s;
                }
            }
        }
        for (int k = threadIdx.x; k < np; k += kBlock) pq[(size_t)node * np + k] = acc[k];
        __syncthreads();
    }
}

// ------------------------------------------------------------ lists

struct ListArgs {
    int nx, ny, nz, B, bx, by, bz, nb;
    double h[3];
    double theta, rshort;
    int np;
    const int *begin, *end, *child0, *nchild;
    const double *box, *centre;
    const int *n_nodes;
    // count pass
    uint32_t *cnt_far, *cnt_near, *cnt_short;
    // fill pass
    const uint32_t *off_far, *off_near, *off_short;
    int *far, *near_l, *shrt;
    unsigned long long *work;   // [3]: far pairs, near pairs, short pairs (point x source)
    int fill;
};

__device__ __forceinline__ double box_gap2(const double *bl, const double *bh, const double *box)
{
    double s = 0;
    for (int k = 0; k < 3; ++k) {
        double g = fmax(0.0, fmax(box[k] - bh[k], bl[k] - box[3 + k]));
        s += g * g;
    }
    return s;
}

constexpr int kStack = 128;

__global__ __launch_bounds__(kBlock) void k_lists(ListArgs a)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (!a.fill && b == 0) {
        // sentinel slot: the exclusive scan over nb + 1 entries then leaves
        // the total in slot nb
        a.cnt_far[a.nb] = 0;
        a.cnt_near[a.nb] = 0;
        a.cnt_short[a.nb] = 0;
    }
    if (b >= a.nb) return;
    const int bi = b % a.bx, bj = (b / a.bx) % a.by, bk = b / (a.bx * a.by);
    const int i0 = bi * a.B, j0 = bj * a.B, k0 = bk * a.B;
    const int i1 = min(i0 + a.B, a.nx), j1 = min(j0 + a.B, a.ny), k1 = min(k0 + a.B, a.nz);
    const double bl[3] = {i0 * a.h[0], j0 * a.h[1], k0 * a.h[2]};
    const double bh[3] = {(i1 - 1) * a.h[0], (j1 - 1) * a.h[1], (k1 - 1) * a.h[2]};
    double cb[3], rb2 = 0;
    for (int k = 0; k < 3; ++k) {
        cb[k] = 0.5 * (bl[k] + bh[k]);
        rb2 += 0.25 * (bh[k] - bl[k]) * (bh[k] - bl[k]);
    }
    const double rb = sqrt(rb2);
    const double npts = (double)(i1 - i0) * (j1 - j0) * (k1 - k0);
    const double rs2 = a.rshort * a.rshort;
    uint32_t nf = 0, nn = 0, ns = 0;
    uint32_t of = 0, on = 0, os = 0;
    if (a.fill) {
        of = a.off_far[b];
        on = a.off_near[b];
        os = a.off_short[b];
    }
    unsigned long long wf = 0, wn = 0, ws = 0;
    int stack[kStack];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const int node = stack[--sp];
        const double *c = a.centre + 4 * node;
        const double dx = c[0] - cb[0], dy = c[1] - cb[1], dz = c[2] - cb[2];
        const double R = sqrt(dx * dx + dy * dy + dz * dz);
        const int cnt = a.end[node] - a.begin[node];
        if (cnt > a.np && rb + c[3] < a.theta * R) {
            if (a.fill) a.far[of + nf] = node;
            ++nf;
            wf += (unsigned long long)a.np;
            // leaves of this cluster that reach the batch's short range
            if (a.rshort > 0 && box_gap2(bl, bh, a.box + 6 * node) < rs2) {
                int st2[kStack];
                int sp2 = 0;
                st2[sp2++] = node;
                while (sp2 > 0) {
                    const int m = st2[--sp2];
                    if (box_gap2(bl, bh, a.box + 6 * m) >= rs2) continue;
                    if (a.nchild[m] == 0) {
                        if (a.fill) a.shrt[os + ns] = m;
                        ++ns;
                        ws += (unsigned long long)(a.end[m] - a.begin[m]);
                    } else {
                        for (int ch = a.child0[m] + a.nchild[m] - 1; ch >= a.child0[m]; --ch)
                            if (sp2 < kStack) st2[sp2++] = ch;
                    }
                }
            }
        } else if (a.nchild[node] == 0) {
            if (a.fill) a.near_l[on + nn] = node;
            ++nn;
            wn += (unsigned long long)cnt;
        } else {
            for (int ch = a.child0[node] + a.nchild[node] - 1; ch >= a.child0[node]; --ch)
                if (sp < kStack) stack[sp++] = ch;
        }
    }
    if (!a.fill) {
        a.cnt_far[b] = nf;
        a.cnt_near[b] = nn;
        a.cnt_short[b] = ns;
        atomicAdd(&a.work[0], (unsigned long long)(wf * npts));
        atomicAdd(&a.work[1], (unsigned long long)(wn * npts));
        atomicAdd(&a.work[2], (unsigned long long)(ws * npts));
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}


}  // namespace

// ------------------------------------------------------------ drivers

int build_source_tree(const TreeCallArgs &a, Workspace &ws, TreeDev &t, rism_stats &st,
                      hipStream_t s)
{
    const int n = (int)a.solute->n;
    const int leaf = a.opts->leaf_size;
    const int stride_f4 = (int)(rec32_bytes_of(a.sp.ns_pad) / sizeof(float4));
    const float4 *rec = static_cast<const float4 *>(a.rec32);
    t.n_atoms = n;
    // node capacity: at most 8 * floor(n / (leaf + 1)) nodes per level below
    // the root (parents are disjoint and hold more than `leaf` atoms)
    long cap = 1;
    long split_max = (long)n / (leaf + 1);
    for (int l = 1; l <= kMortonBits; ++l) {
        long p8 = 1;
        for (int k = 0; k < l && p8 < (1L << 40); ++k) p8 *= 8;
        cap += std::min(p8, 8 * split_max);
    }
    t.cap_nodes = (int)std::min<long>(cap, 1L << 30);
    const int nparts = 64;
    double *part = ws.get<double>(6 * nparts);
    double *bbox = ws.get<double>(6);
    uint32_t *k0 = ws.get<uint32_t>(n), *k1 = ws.get<uint32_t>(n);
    int *v0 = ws.get<int>(n), *v1 = ws.get<int>(n);
    const int nrs = (n + kRsTile - 1) / kRsTile;
    uint32_t *hist = ws.get<uint32_t>((size_t)256 * nrs);
    t.n_nodes = ws.get<int>(1);
    t.level_start = ws.get<int>(kMortonBits + 2);
    int *flags = ws.get<int>(2);
    t.begin = ws.get<int>(t.cap_nodes);
    t.end = ws.get<int>(t.cap_nodes);
    t.child0 = ws.get<int>(t.cap_nodes);
    t.nchild = ws.get<int>(t.cap_nodes);
    t.level = ws.get<int>(t.cap_nodes);
    t.box = ws.get<double>((size_t)6 * t.cap_nodes);
    t.centre = ws.get<double>((size_t)4 * t.cap_nodes);
    uint32_t *cnt = ws.get<uint32_t>(t.cap_nodes);
    uint32_t *total = ws.get<uint32_t>(1);
    t.sorted_rec = ws.alloc(rec32_bytes_of(a.sp.ns_pad) * a.npad);
    if (ws.status()) return ws.status();

    // small trees: keys formed and ranked (and the records placed) by many
    // workgroups, the octree built by one
    int dev = 0, lds_max = 0;
    RISM_HIP(hipGetDevice(&dev));
    RISM_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // (up to kSmallTreeMax atoms, and keys that fit the LDS of one workgroup)
    const bool small = n <= kSmallTreeMax && small_tree_lds(n) + 4096 <= (size_t)lds_max;
    if (small) {
        {
            // (one workgroup at least: it also places the padding records)
            const int npad = (n + 4 * kRankWaves - 1) / (4 * kRankWaves) * (4 * kRankWaves);
            hipLaunchKernelGGL(k_tree_rank, std::max(1, (n + kRankTargets - 1) / kRankTargets),
                               kRankThreads, (size_t)npad * sizeof(unsigned long long), s, rec, stride_f4,
                               n, (int)a.npad, a.bbox_part, a.n_bbox_part, v1, k0, v0,
                               static_cast<float4 *>(t.sorted_rec), t.box, t.centre);
        }
        SmallTreeArgs sa{};
        sa.keys = k0;
        sa.rank = v1;
        sa.n = n;
        sa.leaf = leaf;
        sa.cap = t.cap_nodes;
        sa.begin = t.begin;
        sa.end = t.end;
        sa.level = t.level;
        sa.child0 = t.child0;
        sa.nchild = t.nchild;
        sa.level_start = t.level_start;
        sa.n_nodes = t.n_nodes;
        sa.flags = flags;
        sa.clear = t.clear;
        sa.n_clear = t.n_clear;
        hipLaunchKernelGGL(k_tree_small, 1, kSmallThreads, small_tree_lds(n), s, sa);
        t.perm = v0;
    } else {
    const int nb = (n + kBlock - 1) / kBlock;
    if (a.bbox_part) {
        hipLaunchKernelGGL(k_bbox_final, 1, kBlock, 0, s, a.bbox_part, a.n_bbox_part, bbox);
    } else {
        hipLaunchKernelGGL(k_bbox_partial, nparts, kBlock, 0, s, rec, stride_f4, n, part);
        hipLaunchKernelGGL(k_bbox_final, 1, kBlock, 0, s, part, nparts, bbox);
    }
    hipLaunchKernelGGL(k_morton, nb, kBlock, 0, s, rec, stride_f4, n, bbox, k0, v0);
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_rs_hist, nrs, kBlock, 0, s, k0, n, shift, nrs, hist);
        hipLaunchKernelGGL(k_scan_excl, 1, 1024, 0, s, hist, 256 * nrs, (const int *)nullptr,
                           (uint32_t *)nullptr);
        hipLaunchKernelGGL(k_rs_scatter, nrs, kBlock, 0, s, k0, v0, k1, v1, n, shift, nrs, hist);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    t.perm = v0;
    hipLaunchKernelGGL(k_tree_root, 1, 1, 0, s, n, t.begin, t.end, t.level, t.level_start,
                       t.n_nodes, flags, t.clear, t.n_clear);
    const int gb = 256;
    for (int lvl = 0; lvl < kMortonBits; ++lvl) {
        hipLaunchKernelGGL(k_split_count, gb, kBlock, 0, s, k0, t.begin, t.end, t.level_start, lvl,
                           leaf, cnt);
        // scan the split counts of this level's nodes (count read on device)
        hipLaunchKernelGGL(k_level_count, 1, 1, 0, s, t.level_start, lvl, flags + 1);
        hipLaunchKernelGGL(k_scan_excl, 1, 1024, 0, s, cnt, 0, (const int *)(flags + 1), total);
        hipLaunchKernelGGL(k_split_write, gb, kBlock, 0, s, k0, t.begin, t.end, t.level, t.child0,
                           t.nchild, t.level_start, lvl, leaf, cnt, total, t.cap_nodes, t.n_nodes,
                           flags);
    }
    }
    RISM_HIP(hipGetLastError());
    if (!small) {
    switch (a.sp.ns_pad) {
    case 1: hipLaunchKernelGGL(k_permute<1>, (int)((a.npad + kBlock - 1) / kBlock), kBlock, 0, s, (const AtomF32<1> *)a.rec32, t.perm, n, (int)a.npad, (AtomF32<1> *)t.sorted_rec); break;
    case 2: hipLaunchKernelGGL(k_permute<2>, (int)((a.npad + kBlock - 1) / kBlock), kBlock, 0, s, (const AtomF32<2> *)a.rec32, t.perm, n, (int)a.npad, (AtomF32<2> *)t.sorted_rec); break;
    case 4: hipLaunchKernelGGL(k_permute<4>, (int)((a.npad + kBlock - 1) / kBlock), kBlock, 0, s, (const AtomF32<4> *)a.rec32, t.perm, n, (int)a.npad, (AtomF32<4> *)t.sorted_rec); break;
    default: hipLaunchKernelGGL(k_permute<8>, (int)((a.npad + kBlock - 1) / kBlock), kBlock, 0, s, (const AtomF32<8> *)a.rec32, t.perm, n, (int)a.npad, (AtomF32<8> *)t.sorted_rec); break;
    }
    }
    double *cbox = nullptr;
    if (n > 2 * kBoxChunk) {
        const int nch = (n + kBoxChunk - 1) / kBoxChunk;
        cbox = ws.get<double>(6 * (size_t)nch);
        if (ws.status()) return ws.status();
        hipLaunchKernelGGL(k_chunk_box, (nch + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, s,
                           (const float4 *)t.sorted_rec, stride_f4, n, cbox);
    }
    hipLaunchKernelGGL(k_node_box, 1024, kBlock, 0, s, (const float4 *)t.sorted_rec, stride_f4,
                       t.begin, t.end, t.n_nodes, cbox, t.box, t.centre, small ? 1 : 0);
    RISM_HIP(hipGetLastError());
    (void)st;
    return RISM_OK;
}

int build_proxies(const TreeDev &t, int degree, Workspace &ws, ProxyDev &p, int n_nodes,
                  hipStream_t s, int stride_f4, int max_level)
{
    p.degree = degree;
    const int n1 = degree + 1;
    p.np = n1 * n1 * n1;
    p.q = ws.get<double>((size_t)n_nodes * p.np);
    p.pbox = ws.get<double>((size_t)n_nodes * 6);
    if (ws.status()) return ws.status();
    const size_t shm = (3 * (size_t)kTile * n1 + kTile + 4 * (size_t)p.np) * sizeof(double);
    int dev = 0, lds_max = 0;
    RISM_HIP(hipGetDevice(&dev));
    RISM_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (shm > (size_t)lds_max) {
        set_error("treecode: degree too high for the LDS of this device");
        return RISM_E_UNSUPPORTED;
    }
    for (int lvl = max_level; lvl >= 0; --lvl)
        hipLaunchKernelGGL(k_upward_level, 1024, kBlock, shm, s, (const float4 *)t.sorted_rec,
                           stride_f4, t.begin, t.end, t.child0, t.nchild, t.box, t.level_start,
                           lvl, degree, p.q, p.pbox);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

int build_lists(const TreeCallArgs &a, const TreeDev &t, int n_nodes, double r_short,
                Workspace &ws, ListsDev &l, rism_stats &st, hipStream_t s)
{
    const int B = a.opts->batch_edge;
    const int n1 = a.opts->degree + 1;
    ListArgs la{};
    la.nx = a.g.nx;
    la.ny = a.g.ny;
    la.nz = a.g.nz;
    la.B = B;
    la.bx = (a.g.nx + B - 1) / B;
    la.by = (a.g.ny + B - 1) / B;
    la.bz = (a.g.nz + B - 1) / B;
    la.nb = la.bx * la.by * la.bz;
    for (int k = 0; k < 3; ++k) la.h[k] = a.g.h[k];
    la.theta = a.opts->theta;
    la.rshort = r_short;
    la.np = n1 * n1 * n1;
    la.begin = t.begin;
    la.end = t.end;
    la.child0 = t.child0;
    la.nchild = t.nchild;
    la.box = t.box;
    la.centre = t.centre;
    la.n_nodes = t.n_nodes;
    l.nb = la.nb;
    l.bx = la.bx;
    l.by = la.by;
    l.bz = la.bz;
    uint32_t *cf = ws.get<uint32_t>(la.nb + 1), *cn = ws.get<uint32_t>(la.nb + 1),
             *cs = ws.get<uint32_t>(la.nb + 1);
    uint32_t *tot = ws.get<uint32_t>(4);
    la.work = ws.get<unsigned long long>(4);
    if (ws.status()) return ws.status();
    la.cnt_far = cf;
    la.cnt_near = cn;
    la.cnt_short = cs;
    const int grid = (la.nb + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_zero_u64, 1, 64, 0, s, la.work, 4);
    la.fill = 0;
    {
        PhaseTimer pt(a.opts->flags & RISM_FLAG_PHASE_EVENTS, RISM_PHASE_LISTS, s);
        hipLaunchKernelGGL(k_lists, grid, kBlock, 0, s, la);
        hipLaunchKernelGGL(k_scan_excl, 1, 1024, 0, s, cf, la.nb + 1, (const int *)nullptr, tot + 0);
        hipLaunchKernelGGL(k_scan_excl, 1, 1024, 0, s, cn, la.nb + 1, (const int *)nullptr, tot + 1);
        hipLaunchKernelGGL(k_scan_excl, 1, 1024, 0, s, cs, la.nb + 1, (const int *)nullptr, tot + 2);
    }
    RISM_HIP(hipGetLastError());
    uint32_t htot[4];
    unsigned long long hwork[4];
    RISM_HIP(hipMemcpyAsync(htot, tot, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RISM_HIP(hipMemcpyAsync(hwork, la.work, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    RISM_HIP(hipStreamSynchronize(s));
    l.far_off = (int *)cf;
    l.near_off = (int *)cn;
    l.short_off = (int *)cs;
    l.far = ws.get<int>(htot[0] + 1);
    l.near = ws.get<int>(htot[1] + 1);
    l.shrt = ws.get<int>(htot[2] + 1);
    if (ws.status()) return ws.status();
    la.off_far = cf;
    la.off_near = cn;
    la.off_short = cs;
    la.far = l.far;
    la.near_l = l.near;
    la.shrt = l.shrt;
    la.fill = 1;
    {
        PhaseTimer pt(a.opts->flags & RISM_FLAG_PHASE_EVENTS, RISM_PHASE_LISTS, s);
        hipLaunchKernelGGL(k_lists, grid, kBlock, 0, s, la);
    }
    RISM_HIP(hipGetLastError());
    st.pairs_far = (double)hwork[0];
    st.pairs_direct = (double)hwork[1];
    st.pairs_short = (double)hwork[2];
    st.n_batches = la.nb;
    (void)n_nodes;
    return RISM_OK;
}

int tree_forward(const TreeCallArgs &a, Workspace &ws, rism_stats &st, hipStream_t s)
{
    const bool ev = a.opts->flags & RISM_FLAG_PHASE_EVENTS;
    TreeDev t{};
    int rc;
    {
        PhaseTimer pt(ev, RISM_PHASE_TREE_BUILD, s);
        rc = build_source_tree(a, ws, t, st, s);
    }
    if (rc) return rc;
    int hn[2 + kMortonBits + 2];
    RISM_HIP(hipMemcpyAsync(hn, t.n_nodes, sizeof(int), hipMemcpyDeviceToHost, s));
    RISM_HIP(hipMemcpyAsync(hn + 2, t.level_start, (kMortonBits + 2) * sizeof(int),
                            hipMemcpyDeviceToHost, s));
    RISM_HIP(hipStreamSynchronize(s));
    const int n_nodes = hn[0];
    int hflag = 0;
    (void)hflag;
    int max_level = 0;
    for (int l = 0; l <= kMortonBits; ++l)
        if (hn[2 + l + 1] > hn[2 + l]) max_level = l;
    st.n_nodes = n_nodes;
    if (n_nodes > t.cap_nodes) {
        set_error("treecode: node capacity exceeded");
        return RISM_E_NOMEM;
    }
    const int stride_f4 = (int)(rec32_bytes_of(a.sp.ns_pad) / sizeof(float4));
    ProxyDev p{};
    {
        PhaseTimer pt(ev, RISM_PHASE_UPWARD, s);
        rc = build_proxies(t, a.opts->degree, ws, p, n_nodes, s, stride_f4, max_level);
    }
    if (rc) return rc;
    // short-range radius: the LJ cut-off (largest per-pair radius) and R_s
    double rshort = a.asym_on ? std::sqrt(a.asym.rs2) : 0.0;
    if (a.lj_mode == LJ_CUT) rshort = std::max(rshort, a.rmax_short);
    ListsDev l{};
    rc = build_lists(a, t, n_nodes, rshort, ws, l, st, s);
    if (rc) return rc;
    TreeEvalArgs ea{};
    ea.g = a.g;
    ea.out = a.out;
    ea.asym = a.asym;
    ea.rec = t.sorted_rec;
    ea.begin = t.begin;
    ea.end = t.end;
    ea.pq = p.q;
    ea.pbox = p.pbox;
    ea.degree = p.degree;
    ea.np = p.np;
    ea.l = l;
    ea.rshort2 = (float)(rshort * rshort);
    {
        PhaseTimer pt(ev, RISM_PHASE_EVAL, s);
        rc = launch_tree_eval(a.sp, a.lj_mode, a.asym_on, a.opts->batch_edge, ea, s);
    }
    return rc;
}

}  // namespace rism
