// Internal declarations shared by the HIP translation units of librism.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "rism.h"

namespace rism {

constexpr int kMaxSites = RISM_MAX_SITES;
constexpr int kBlock = 256;           // threads per workgroup (4 wave64)
constexpr int kAtomPad = 8;           // atom arrays are padded to a multiple of this
constexpr double kPi = 3.14159265358979323846;
constexpr double kFarAway = 1.0e5;    // padding atoms sit this far from the grid (A)

// ---------------------------------------------------------------- staged data
// Atom records are read wave-uniformly by every grid-point thread, so the
// compiler serves them through the scalar data cache (read-only loads) and
// the VALU takes their fields as SGPR operands: no LDS staging needed.
//
// FP32 record: coordinates relative to the grid origin split into hi + lo
// FP32 words (x = xh + xl to ~48 bits), so that FP32 differences d = g - x are
// accurate to a few ulp of d itself even 100+ A from the origin.
template <int NS>
struct alignas(16) AtomF32 {
    float xh, yh, zh, q;
    float xl, yl, zl;
    float on_grid;   // 1 when the atom sits on a grid point (d2 == 0 in the
                     // FP32 pair arithmetic for that point), else 0
    float A[NS];     // 4 eps_ga sigma_ga^12
    float B[NS];     // 4 eps_ga sigma_ga^6
    float rc2[NS];   // squared LJ cut-off radius (inf: no cut-off)
};

template <int NS>
struct alignas(16) AtomF64 {
    double x, y, z, q;
    double A[NS];
    double B[NS];
    double rc2[NS];
};

struct SiteParams {
    int ns;          // real sites
    int ns_pad;      // template width (1, 2, 4 or 8)
    double q[kMaxSites], sig[kMaxSites], eps[kMaxSites];
    int ionic[kMaxSites];
};

// LJ_CUT1 is a kernel template value only: LJ_CUT where every site of an atom
// has the same cut-off radius (a fixed lj_cutoff), so one test serves all sites.
enum LjMode { LJ_NONE = 0, LJ_ALL = 1, LJ_CUT = 2, LJ_CUT1 = 3 };

struct GridParams {
    double o[3];
    double h[3];
    int nx, ny, nz;
    int64_t m;       // nx*ny*nz
    int exact;       // i*h is exact in FP32 for every index on every axis
};

// Output scaling of the three electrostatic sums and the LJ sums.
struct OutParams {
    void *u, *c, *h;
    int f64;                    // element type of u, c, h
    int want_u, want_c, want_h;
    int ns, n_ionic;
    double u_coul[kMaxSites];   // k_C q_g
    double c_scale[kMaxSites];  // -beta k_C q_g
    double h_scale[kMaxSites];  // per ionic slot: -(beta k_C q_j/(2 eps)) e^{kappa^2 eta^2/4}
};

// Cubic table of the smeared kernels on [0, R_s] (FP32 coefficients in the
// local variable t in [0, 1) of each interval): tab[2 i] for erf(d/eta)/d and
// tab[2 i + 1] for the Eq. 6 bracket over d, each as (c0, c1, c2, c3).
constexpr int kSmearIntervals = 256;
// workgroups of kBlock threads that form the table (four threads per interval)
constexpr int kSmearBlocks = (4 * kSmearIntervals + kBlock - 1) / kBlock;

struct AsymParams {
    const float4 *tab;  // device table, 2 * kSmearIntervals entries (FP32 paths)
    double tab_inv_h;   // intervals per angstrom: kSmearIntervals / R_s
    double eta, kappa;
    double inv_eta;     // 1/eta
    double a;           // kappa eta / 2
    double rs2;         // squared radius of the short-range correction
    double dcf0;        // lim_{d->0} erf(d/eta)/d = 2/(eta sqrt(pi))
    double tcf0;        // lim_{d->0} of the Eq. 6 bracket over d
    double yk;          // -kappa * log2(e): exp(-kappa d) = exp2(yk d)
};

// ---------------------------------------------------------------- workspace
// Grow-only scratch kept per (device, stream).  Chunks never move, so pointers
// carved earlier in a call stay valid when a later request adds a chunk.
class Workspace {
public:
    struct Arena;
    Workspace(int device, void *stream, uint64_t cap_bytes);
    // Fixed mode: carves every request from [base, base + bytes) and never
    // allocates; a request beyond it fails with RISM_E_NOMEM.
    Workspace(void *base, size_t bytes);
    ~Workspace();
    bool fixed() const { return fixed_ != nullptr; }
    // Returns nullptr (and sets the error) on failure.
    void *alloc(size_t bytes);
    template <class T> T *get(size_t count) { return static_cast<T *>(alloc(count * sizeof(T))); }
    uint64_t in_use() const { return used_total_; }
    int status() const { return status_; }
private:
    Arena *arena_ = nullptr;
    char *fixed_ = nullptr;
    size_t fixed_size_ = 0;
    uint64_t cap_ = 0;
    uint64_t used_total_ = 0;
    size_t chunk_ = 0, off_ = 0;
    int status_ = RISM_OK;
};

// ---------------------------------------------------------------- phase events
// RAII recorder: with RISM_FLAG_PHASE_EVENTS set, records a start event on
// construction and a stop event on destruction, on the call's stream.
class PhaseTimer {
public:
    PhaseTimer(bool on, int phase, hipStream_t s);
    ~PhaseTimer();
private:
    int slot_ = -1;
    hipStream_t s_;
};

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define RISM_HIP(call)                                            \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::rism::hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return RISM_OK or an error code.

struct StageArgs {
    const double *xyz, *q, *sig, *eps;
    int64_t n, npad;
    double origin[3];
    double lj_cutoff;   // > 0 global radius
    double lj_tol;      // > 0 per-pair radius from tolerance (overrides)
    int lj_mode;        // LjMode
    int check_eps;      // flag eps_a <= 0 as an error (backward dL/deps)
    int *err_part;      // device int[3] per staging workgroup (the first npad / kBlock), all
                        // written: [0] non-finite input, [1] tol >= eps_ga / eps <= 0,
                        // [2] bits of the largest squared cut-off radius (float)
    void *rec32;        // AtomF32<ns_pad>[npad] or null
    void *rec64;        // AtomF64<ns_pad>[npad] or null
    double *rcut;       // [ns][n] FP64 cut-off radii or null
    float4 *smear_tab;  // or null: the smeared-kernel table of `smear` (cubic
    AsymParams smear;   // pieces per interval), formed by the same launch
    GridParams grid;    // for AtomF32::on_grid
    double *bbox_part;  // or null: per staging workgroup (the first npad / kBlock),
                        // the box of its atoms' FP32 record positions: lo[3], hi[3]
};
int launch_stage(const SiteParams &sp, const StageArgs &a, hipStream_t s);
// Reduces the staging workgroups' words (err_part of nparts workgroups) into
// flags[0..2]: OR, OR, max.
int launch_stage_flags(const int *part, int nparts, int *flags, hipStream_t s);
int launch_lj_tail(const SiteParams &sp, const double *rcut, const double *sig, const double *eps,
                   int64_t n, double *tail_dev, hipStream_t s);

struct DirectArgs {
    const void *atoms;  // AtomF32 or AtomF64 records
    int64_t n;          // real atoms
    int64_t npad;
    GridParams g;
    OutParams out;
    AsymParams asym;
    int lj_mode;
    int lj_uniform;     // LJ_CUT with one radius for all sites (fixed lj_cutoff)
    int asym_on;        // compute the smeared sums (c and/or h)
};
int launch_direct_f64(const SiteParams &sp, const DirectArgs &a, hipStream_t s);
// Fills the 2 * kSmearIntervals cubic pieces of erf(d/eta)/d and of the Eq. 6
// bracket over d on [0, R_s] (FP64 evaluation, FP32 coefficients).
int launch_direct_f32(const SiteParams &sp, const DirectArgs &a, hipStream_t s);

int launch_compare(const void *x, int f64, const double *ref, const uint8_t *mask, int64_t n,
                   double cap, double *partials, int nblocks, hipStream_t s);
// mask[p] = 1 where every atom is at least `radius` from grid point p, else 0.
int launch_near_mask(const double *xyz, int64_t n, const GridParams &g, double radius,
                     uint8_t *mask, hipStream_t s);

// Tree forward (particle-cluster); defined in k_tree.hip.
struct TreeCallArgs {
    const rism_solute *solute;
    SiteParams sp;
    GridParams g;
    OutParams out;
    AsymParams asym;
    const rism_opts *opts;
    int lj_mode;
    int lj_uniform;         // LJ_CUT with one radius for all sites
    int asym_on;
    const void *rec32;      // staged FP32 atom records (input order)
    int64_t npad;
    double rmax_short;      // short-range radius: max(LJ cut-off, R_s)
    const int *stage_err;   // device flag words of the input check still to read
                            // (StageArgs::err_part), or null
    int n_stage_err;        // staging workgroups in stage_err
    const double *bbox_part;  // per-workgroup boxes of the staged atoms, or null
    int n_bbox_part;
};
int tree_forward(const TreeCallArgs &a, Workspace &ws, rism_stats &st, hipStream_t s);
int tree_forward_cp(const TreeCallArgs &a, Workspace &ws, rism_stats &st, hipStream_t s);

// Reciprocal-space asymptotics; defined in k_asym_k.hip.
struct AkGrid {
    int nx, ny, nz, nxh;   // nxh = nx / 2 + 1 entries along the halved axis
    double o[3], h[3];
};
struct AkArgs {
    AkGrid g;
    int64_t n;
    const float2 *ex, *ey, *ezq;   // phase tables (set by launch_asym_k)
    const double *k2cut;           // device [3]: squared cut-offs of c and h, net charge
    double eta2_4, kappa2;
    void *c, *h;                   // [S][nz][ny][nxh][2], [n_ionic][...][2]
    int f64, ns, n_ionic;
    double c_scale[kMaxSites];     // -4 pi beta k_C q_g
    double h_scale[kMaxSites];     // -4 pi beta k_C q_j / eps
};
// Frequency cut-off of Sec. 2.5 (Newton's method, bracketed); 0 = none.
__host__ __device__ double ak_kcut(bool for_h, double tol, double pref, double eta, double kappa,
                                   double diel);
// Phase tables, matrix-core contraction and outputs; scratch from ws.
// ev: record the phase events (RISM_PHASE_RECIP for the main matrix-core
// kernel, RISM_PHASE_OTHER for the rest).
int launch_asym_k(const AkArgs &a, const double *xyz, const double *q, Workspace &ws, bool ev,
                  hipStream_t s);
// Squared cut-offs into k2cut[0..1] (INFINITY where tol <= 0 or nothing is
// cut) and the net charge into k2cut[2]; pref_c / pref_h are the bounds'
// prefactors without sum |Q_a|.
int launch_ak_cutoffs(const double *q, int64_t n, double tol, double pref_c, double pref_h,
                      double eta, double kappa, double diel, double *k2cut, hipStream_t s);

// Adjoint; defined in k_adjoint.hip.
struct AdjointArgs {
    const void *atoms;      // AtomF32 / AtomF64 records (input order)
    int64_t n, npad;
    SiteParams sp;
    GridParams g;
    const void *w;          // dL/du [S][M]
    int w_f64;
    double kc;
    int lj_mode;
    const double *eps_in;   // device FP64 eps_a (for dL/deps)
    const double *sig_in;
    double *dxyz, *dq, *deps, *dsig;
    const rism_opts *opts;
    double rmax_lj;         // largest LJ cut-off radius (LJ_CUT)
};
int adjoint_direct(const AdjointArgs &a, bool f64, Workspace &ws, rism_stats &st, hipStream_t s);
int adjoint_tree(const AdjointArgs &a, Workspace &ws, rism_stats &st, hipStream_t s);

// Template-width helper: the kernels are instantiated for 1, 2, 4, 8 sites.
inline int pad_sites(int ns) { return ns <= 1 ? 1 : ns <= 2 ? 2 : ns <= 4 ? 4 : 8; }

}  // namespace rism
