// Device data of the particle-cluster treecode (source octree on the atoms).
#pragma once

#include "rism_internal.h"

namespace rism {

constexpr int kMortonBits = 10;   // per axis: 30-bit keys, 10 tree levels below the root

// Octree over Morton-sorted atoms.  Nodes are stored level by level; node i
// owns the sorted atoms [begin[i], end[i]).
struct TreeDev {
    int n_atoms;
    int cap_nodes;
    int *n_nodes;          // device: total nodes
    int *level_start;      // device: [kMortonBits + 2]
    int *begin, *end;      // [cap]
    int *child0, *nchild;  // first child (children are contiguous), count (0: leaf)
    int *level;            // [cap]
    double *box;           // [cap][6]: tight lo[3], hi[3] (relative to the grid origin)
    double *centre;        // [cap][4]: centre x, y, z, radius (half-diagonal)
    int *perm;             // sorted position -> input index
    void *sorted_rec;      // AtomF32<ns_pad> in sorted order
    // in: n_clear words the build sets to 0 (flags of the caller's later
    // kernels), or none
    int *clear;
    int n_clear;
};

// Proxy charges of the barycentric Chebyshev interpolation (upward pass).
struct ProxyDev {
    int degree;            // n: (n+1)^3 proxies per node
    int np;                // (n+1)^3
    double *q;             // [n_nodes][np] FP64 proxy charges
    double *pbox;          // [n_nodes][6] box on which the proxies sit (lo, hi)
};

// Per-batch interaction lists (CSR).
struct ListsDev {
    int nb;                // batches
    int bx, by, bz;        // batches per axis
    int *far_off, *far;    // proxy interactions: node ids
    int *near_off, *near;  // leaves: full near-field evaluation
    int *short_off, *shrt; // leaves: short-range terms only (Coulomb from proxies)
};

int build_source_tree(const TreeCallArgs &a, Workspace &ws, TreeDev &t, rism_stats &st,
                      hipStream_t s);
int build_proxies(const TreeDev &t, int degree, Workspace &ws, ProxyDev &p, int n_nodes,
                  hipStream_t s, int stride_f4, int max_level);
int build_lists(const TreeCallArgs &a, const TreeDev &t, int n_nodes, double r_short,
                Workspace &ws, ListsDev &l, rism_stats &st, hipStream_t s);

struct TreeEvalArgs {
    GridParams g;
    OutParams out;
    AsymParams asym;
    const void *rec;       // sorted AtomF32 records
    const int *begin, *end;
    const double *pq;      // proxy charges
    const double *pbox;
    int degree, np;
    ListsDev l;
    float rshort2;         // squared short-range radius (LJ cut-off / R_s)
};
int launch_tree_eval(const SiteParams &sp, int lj_mode, bool asym, int batch_edge,
                     const TreeEvalArgs &a, hipStream_t s);

}  // namespace rism
