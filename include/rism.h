/*
 * rism.h -- C ABI of librism.so: the 3D-RISM initialisation hot path on
 * AMD Instinct MI355X (gfx950).
 *
 * Paper: Wilson, Krasny & Luchko, "Accelerating the 3D-RISM theory of
 * molecular solvation with treecode summation and cut-offs".
 *
 * Units: lengths in angstrom, charges in e, energies in kcal/mol.
 * Grid: point (i, j, k) sits at origin + (i*spacing[0], j*spacing[1],
 * k*spacing[2]); every grid buffer is C-contiguous [site][nz][ny][nx]
 * (x fastest), of the element type named by rism_opts.out_dtype.
 *
 * Memory: pointers marked [device] must point to device memory of the
 * current HIP device; [host] pointers to host memory.  The caller owns all
 * buffers.  Outputs are overwritten, never accumulated into.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Work is
 * enqueued on it; outputs are valid once the stream has been synchronised.
 * A call may synchronise the stream internally (tree sizes, device-side
 * input checks, host outputs such as lj_tail); RISM_TREECODE_CP returns only
 * after its work has completed (it reads back list sizes at the end and, if
 * buffers sized from an earlier call of the same problem shape were too
 * small, runs its second half again).  Calls that use the same
 * device and stream from several host threads must be serialised by the
 * caller; scratch memory is kept per (device, stream) and reused.
 *
 * Errors: every entry point returns RISM_OK (0) or a negative code and
 * never throws; rism_last_error() gives the message of the calling thread's
 * last failure.  On failure outputs are unspecified.
 */
#ifndef RISM_H
#define RISM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RISM_OK 0
#define RISM_E_INVALID (-1)      /* bad argument (null, out of range, non-finite) */
#define RISM_E_NOMEM (-2)        /* scratch would exceed max_workspace_bytes, or allocation failed */
#define RISM_E_HIP (-3)          /* a HIP runtime call failed */
#define RISM_E_UNSUPPORTED (-4)  /* valid but not implemented combination */

#define RISM_MAX_SITES 8

/* Summation methods.
 * RISM_DIRECT_F64   plain FP64 direct sum of every (atom, point) pair, the
 *                   definitions term by term (GPU reference).
 * RISM_DIRECT_F32C  FP32 pair arithmetic over every pair (hi/lo
 *                   coordinates), blocked partial sums flushed into FP64
 *                   (electrostatics) or compensated FP32 (LJ) accumulators;
 *                   the smeared kernels are 1/d and
 *                   2 exp(-kappa d)/d beyond R_s (to < 1e-12) and come from a
 *                   cubic table (FP64-fitted) within R_s.
 * RISM_TREECODE     as DIRECT_F32C, but the far parts 1/d and exp(-kappa d)/d
 *                   come from a particle-cluster treecode: Morton-sorted
 *                   octree on the atoms, barycentric Chebyshev proxy charges,
 *                   batches of grid points as targets; LJ needs a cut-off.
 * RISM_TREECODE_CP  as RISM_TREECODE with the cluster-particle orientation of
 *                   the paper (Sec. 2.3): the tree is built on the grid
 *                   targets and atoms are interpolated into target clusters.
 * RISM_TREECODE_TAYLOR  as RISM_TREECODE_CP with the paper's own far fields:
 *                   order-p Taylor polynomials about the target clusters'
 *                   centres of 1/d (u), erf(d/eta)/d (c^lr) and
 *                   2 exp(-kappa d)/d (h^lr: the TCF kernel's large-distance
 *                   form), coefficients from the recurrences of Secs. 2.3.2,
 *                   2.4.1 and 2.4.2 (p = degree, 1..12); atoms not accepted
 *                   take the exact kernels.  When h^lr is requested the MAC
 *                   also requires |y - c| - r >= eta (6 + kappa eta / 2), so
 *                   that the erfc -> 2/0 step is exact to ~1e-17 at every
 *                   target.  RISM_FLAG_TAYLOR_SPLIT selects the exact-split
 *                   variant.  No adjoint (rism_potential_backward:
 *                   RISM_E_UNSUPPORTED). */
#define RISM_DIRECT_F64 0
#define RISM_DIRECT_F32C 1
#define RISM_TREECODE 2
#define RISM_TREECODE_CP 3
#define RISM_TREECODE_TAYLOR 4

#define RISM_F32 0
#define RISM_F64 1

/* rism_opts.flags */
#define RISM_FLAG_NO_DEVICE_CHECK 1u  /* skip the device-side finiteness check
                                          of atom inputs (saves one stream sync) */
#define RISM_FLAG_PHASE_EVENTS 2u     /* record HIP events around every kernel
                                          phase (read with rism_phase_times) */
#define RISM_FLAG_STATS 4u            /* count evaluated interactions of the
                                          treecodes exactly (one extra sync) */
#define RISM_FLAG_TAYLOR_SPLIT 8u     /* RISM_TREECODE_TAYLOR: the exact-split
                                          variant (far fields 1/d and
                                          exp(-kappa d)/d only, the smeared
                                          kernels' remainders added exactly
                                          within R_s) instead of the paper's
                                          expansions of the smeared kernels */

/* Kernel phases reported by rism_phase_times. */
#define RISM_PHASE_STAGE 0        /* mixing, cut-offs, FP32/FP64 atom records */
#define RISM_PHASE_DIRECT_F64 1   /* FP64 direct sum */
#define RISM_PHASE_DIRECT_F32 2   /* FP32 compensated direct sum */
#define RISM_PHASE_TREE_BUILD 3   /* Morton keys, sort, octree, boxes */
#define RISM_PHASE_UPWARD 4       /* proxy charges / proxy potentials */
#define RISM_PHASE_LISTS 5        /* interaction lists */
#define RISM_PHASE_EVAL 6         /* far + near evaluation on grid batches */
#define RISM_PHASE_DOWNWARD 7     /* target-side interpolation to grid points */
#define RISM_PHASE_ADJOINT 8      /* adjoint pair kernels */
#define RISM_PHASE_ADJ_REDUCE 9   /* adjoint partial-sum reduction */
#define RISM_PHASE_OTHER 10
#define RISM_PHASE_RECIP 11       /* reciprocal-space structure factor on the matrix cores */
#define RISM_NUM_PHASES 12

/* Regular grid (Sec. 2.1: u, c and h live on one 3-D grid). */
typedef struct rism_grid {
    double origin[3];
    double spacing[3];   /* > 0 */
    int32_t dims[3];     /* nx, ny, nz > 0 */
} rism_grid;

/* Solute atoms (the sources R_a, Q_a of Sec. 2.2 and the LJ parameters of
 * Sec. 2.6).  All arrays [device], FP64, length n; xyz is [n][3]. */
typedef struct rism_solute {
    int64_t n;            /* >= 0; n == 0 gives zero grids */
    const double *xyz;
    const double *q;
    const double *sigma;  /* LJ sigma_a >= 0 */
    const double *eps;    /* LJ epsilon_a >= 0 */
} rism_solute;

/* Solvent sites gamma.  All arrays [host], length n (1..RISM_MAX_SITES).
 * LJ pair parameters use Lorentz-Berthelot mixing:
 * sigma_ga = (sigma_g + sigma_a)/2, eps_ga = sqrt(eps_g eps_a),
 * A = 4 eps_ga sigma_ga^12, B = 4 eps_ga sigma_ga^6.
 * ionic[g] != 0 marks the ionic species that get h^lr (Sec. 2.2). */
typedef struct rism_sites {
    int32_t n;
    const double *q;
    const double *sigma;
    const double *eps;
    const int32_t *ionic;   /* may be NULL: no ionic sites */
} rism_sites;

typedef struct rism_opts {
    int32_t method;        /* RISM_DIRECT_F64 / _F32C / RISM_TREECODE / _CP / _TAYLOR */
    int32_t out_dtype;     /* RISM_F32 or RISM_F64 for every grid buffer */
    double coulomb_k;      /* k_C in kcal*A/(mol*e^2); default 332.0522173 */
    double lj_cutoff;      /* A; > 0: LJ pairs with d >= lj_cutoff are dropped
                              (Sec. 2.6, Eq. 28); <= 0: no cut-off */
    double lj_tol;         /* > 0: per-pair cut-off r_cut with |u_LJ(r_cut)| =
                              lj_tol beyond the minimum (Sec. 2.6); overrides
                              lj_cutoff; must be < eps_ga for every pair */
    double theta;          /* treecode MAC parameter, in (0, 1) */
    int32_t degree;        /* interpolation degree n, (n+1)^3 proxies, 1..16 */
    int32_t leaf_size;     /* treecode leaf size N0 (atoms, or grid points per
                              leaf edge^3 for _CP), >= 1 */
    int32_t batch_edge;    /* target batch edge in grid points: 4, 8 or 16 */
    uint32_t flags;        /* RISM_FLAG_* */
    uint64_t max_workspace_bytes;  /* 0 = unlimited */
} rism_opts;

/* Counters of the last successful call on this thread. */
typedef struct rism_stats {
    double pairs_direct;     /* (point, atom) pairs evaluated directly */
    double pairs_far;        /* (point, proxy) or (atom, proxy) pairs */
    double pairs_short;      /* short-range (LJ / smeared correction) pairs tested */
    double upward_flops;     /* proxy construction / interpolation work */
    int64_t n_nodes;         /* tree nodes */
    int64_t n_batches;       /* target batches */
    int64_t workspace_bytes; /* scratch in use */
} rism_stats;

/* Fills *opts with defaults: RISM_TREECODE_CP, RISM_F32, k_C 332.0522173,
 * lj_cutoff 9, lj_tol 0, theta 0.6, degree 8, leaf 64, batch 8, flags 0
 * (theta 0.6 with degree 8 keeps the cluster-particle treecode within 1e-6
 * rel-L2 of the direct sums on the 2,500- and 14,000-atom workloads). */
void rism_default_opts(rism_opts *opts);

/*
 * u_gamma(r) for every site on the grid (Sec. 2.1; LJ truncation Sec. 2.6,
 * Eq. 28):
 *   u_g(r) = sum_a [ k_C Q_a q_g / d + [d < r_cut,ga] (A_ga/d^12 - B_ga/d^6) ]
 * with d = |r - R_a|.  A point that coincides with an atom gets +inf.
 * u:       [device] [S][nz][ny][nx], out_dtype.
 * lj_tail: [host] [S] or NULL; if given, receives
 *   T_g = 4 pi sum_a int_{r_cut}^inf u_LJ,ga(r) r^2 dr
 *       = (4 pi/3) sum_a (A_ga/(3 r_c^9) - B_ga/r_c^3)
 * (Sec. 2.6, the analytic correction; the correction to the excess chemical
 * potential of a truncated calculation is + sum_g rho_g T_g).  Zero without
 * a cut-off.  Requesting it synchronises the stream.
 */
int rism_potential(const rism_solute *solute, const rism_sites *sites,
                   const rism_grid *grid, const rism_opts *opts,
                   void *u, double *lj_tail, void *stream);

/*
 * Real-space long-range asymptotics (Sec. 2.2, Eqs. 4 and 6, with k_C):
 *   c_g(r) = -beta k_C q_g sum_a Q_a erf(d/eta)/d                for all sites
 *   h_j(r) = -(beta k_C q_j/(2 eps)) exp(kappa^2 eta^2/4)
 *            sum_a Q_a [e^{-kappa d} erfc(kappa eta/2 - d/eta)
 *                      - e^{kappa d} erfc(kappa eta/2 + d/eta)]/d  for ionic j
 * (d -> 0 limits at coincident points).  kappa is the total inverse Debye
 * length; eps the solvent dielectric constant.
 * c_lr: [device] [S][..] or NULL;  h_lr: [device] [n_ionic][..] (ionic sites
 * in site order) or NULL.  eta > 0, kappa >= 0, beta > 0, dielectric > 0.
 */
int rism_asymptotics(const rism_solute *solute, const rism_sites *sites,
                     const rism_grid *grid, const rism_opts *opts,
                     double eta, double kappa, double beta, double dielectric,
                     void *c_lr, void *h_lr, void *stream);

/*
 * Reciprocal-space long-range asymptotics (Sec. 2.2, Eqs. 5 and 7, times
 * coulomb_k) on the half grid of a real-to-complex transform of the grid:
 *   c_k [device] [S][nz][ny][nx/2+1][2]       (re, im), of out_dtype;
 *   h_k [device] [n_ionic][nz][ny][nx/2+1][2] (ionic sites only).
 * Entry (jz, jy, jx) is k = 2 pi (jx/(nx hx), fy/(ny hy), fz/(nz hz)) with
 * fy = jy for jy <= (ny-1)/2, else jy - ny (likewise fz): the order of a
 * forward discrete transform.  The structure factor is
 *   S(k) = sum_a Q_a exp(-i k.(R_a - origin)),
 * i.e. the transform of a grid anchored at `origin` with the exp(-i k.r)
 * sign (the paper's exp(+i k.R) is the same quantity under the opposite
 * sign convention).  c_k at k = 0 is 0, and so is h_k at k = 0 when kappa = 0.
 * tol > 0 applies the frequency cut-off of Sec. 2.5: entries with |k| above
 * the root of the error bound (Eq. 26 for c, its analogue for h; the bound
 * uses sum_a |Q_a| and the largest |q| of the sites concerned) are 0 and not
 * summed; tol <= 0 sums every entry.  Either output may be NULL (h_k is
 * ignored without ionic sites).  opts->method is not used.
 */
int rism_asymptotics_k(const rism_solute *solute, const rism_sites *sites,
                       const rism_grid *grid, const rism_opts *opts,
                       double eta, double kappa, double beta, double dielectric, double tol,
                       void *c_k, void *h_k, void *stream);

/*
 * Fused initialisation: rism_potential and rism_asymptotics in one pass
 * over the atoms (they share the Coulomb sum).  Any of u, c_lr, h_lr may be
 * NULL; arguments as in the two calls above.
 */
int rism_initialize(const rism_solute *solute, const rism_sites *sites,
                    const rism_grid *grid, const rism_opts *opts,
                    double eta, double kappa, double beta, double dielectric,
                    void *u, double *lj_tail, void *c_lr, void *h_lr, void *stream);

/*
 * rism_initialize without any allocation, for callers that cannot allocate
 * device or host memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): arguments and results as rism_initialize,
 * for methods RISM_DIRECT_F64 and RISM_DIRECT_F32C (others:
 * RISM_E_UNSUPPORTED).  Scratch (atom records, cut-off radii, the smeared-
 * kernel table, flags) comes from a fixed 32 MiB device array that the
 * library holds per GPU until the process ends; a call needing more
 * (beyond about 116,000 atoms with 8 sites or 209,000 with 4 on the FP64
 * path with lj_tail, 299,000 with 4 on the FP32 path) fails with
 * RISM_E_INVALID before any work is enqueued.  Calls on one GPU
 * share that array: calls that overlap on one GPU (several host threads or
 * streams) race and must be serialised by the caller.  Phase events and
 * statistics counters are not recorded.  The device-side input check and a
 * requested lj_tail still synchronise the stream, through copies into
 * caller or stack memory.
 */
int rism_initialize_noalloc(const rism_solute *solute, const rism_sites *sites,
                            const rism_grid *grid, const rism_opts *opts,
                            double eta, double kappa, double beta, double dielectric,
                            void *u, double *lj_tail, void *c_lr, void *h_lr, void *stream);

/*
 * Adjoint of rism_potential.  Given dL_du = dL/du_g(r) ([device],
 * [S][nz][ny][nx], out_dtype), returns ([device], FP64, each may be NULL)
 *   dL_dxyz[n][3], dL_dq[n], dL_deps[n], dL_dsigma[n]
 * of L = sum_g sum_r dL_du_g(r) u_g(r), differentiating the definition
 * above term by term (the jump of a truncated LJ term at r_cut is ignored).
 * Points that coincide with an atom are skipped.  dL_deps requires
 * eps_a > 0 for every atom (RISM_E_INVALID otherwise, checked on device).
 * Methods: DIRECT_F64, DIRECT_F32C, TREECODE and TREECODE_CP (both: the
 * grid-source treecode, the transpose of the cluster-particle forward, for
 * the Coulomb part, and a per-atom gather for the truncated LJ part);
 * TREECODE_TAYLOR returns RISM_E_UNSUPPORTED.
 */
int rism_potential_backward(const rism_solute *solute, const rism_sites *sites,
                            const rism_grid *grid, const rism_opts *opts,
                            const void *dL_du, double *dL_dxyz, double *dL_dq,
                            double *dL_deps, double *dL_dsigma, void *stream);

/*
 * Error report of a computed grid against a reference (FP64) grid, both
 * [device] with n elements.  x has element type x_dtype.  mask: [device]
 * n bytes or NULL; points whose byte is 0 are left out of every count (for
 * instance rism_near_mask's points near atoms).  Reduces, in FP64 and in a
 * fixed order, over the points the mask keeps:
 *   out[0] = sum (x - ref)^2 over points where both are finite and
 *            |x|, |ref| <= ref_cap (ref_cap <= 0: no cap)
 *   out[1] = sum ref^2 over the same points
 *   out[2] = max |x - ref| over the same points
 *   out[3] = number of points excluded (non-finite on either side or over
 *            the cap)
 *   out[4] = number of excluded points where x and ref disagree in kind:
 *            one finite and within the cap, the other not
 *   out[5] = number of points compared (those of out[0])
 * rel-L2 = sqrt(out[0] / out[1]).  out: [host] double[6].  Synchronises the
 * stream.
 */
int rism_compare(const void *x, int32_t x_dtype, const double *ref, int64_t n,
                 double ref_cap, const uint8_t *mask, double *out, void *stream);

/*
 * Mask of the grid points away from the solute, for the error report:
 * mask[p] = 1 when every atom is at least `radius` from grid point p
 * (distances in FP64 from the absolute coordinates), else 0.  mask: [device]
 * [nz][ny][nx] bytes, overwritten.  radius 1 A gives the report's
 * {min_a d >= 1 A} region, which leaves out the LJ cores that dominate u's
 * norm.  solute->q, sigma and eps are not read.
 */
int rism_near_mask(const rism_solute *solute, const rism_grid *grid, double radius,
                   uint8_t *mask, void *stream);

/* Counters of the calling thread's last successful call. */
int rism_last_stats(rism_stats *stats);

/*
 * Elapsed GPU time per phase (ms, summed) and number of timed launches per
 * phase, over every call made by this thread with RISM_FLAG_PHASE_EVENTS
 * since the previous rism_phase_times call.  ms and count are [host] arrays
 * of RISM_NUM_PHASES.  Waits for the recorded events, then clears the log.
 */
int rism_phase_times(double *ms, int64_t *count);

/* Message of the calling thread's last failure ("" if none). */
const char *rism_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RISM_H */
