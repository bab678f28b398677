// C-ABI entry points of librism.so: argument validation, constant
// preparation (Lorentz-Berthelot mixing, cut-offs, output scale factors),
// scratch management and dispatch to the HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "pair.h"

namespace rism {

// ------------------------------------------------------------------ errors

static thread_local std::string g_error;
static thread_local rism_stats g_stats;

void set_error(const std::string &msg) { g_error = msg; }

int hip_fail(hipError_t e, const char *what)
{
    g_error = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? RISM_E_NOMEM : RISM_E_HIP;
}

static int fail(int code, const std::string &msg)
{
    g_error = msg;
    return code;
}

// ------------------------------------------------------------ phase events

struct PhaseRec {
    int phase;
    hipEvent_t start, stop;
};
static thread_local std::vector<PhaseRec> g_phase_log;
static thread_local std::vector<hipEvent_t> g_event_pool;

static hipEvent_t take_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

PhaseTimer::PhaseTimer(bool on, int phase, hipStream_t s) : s_(s)
{
    if (!on) return;
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) return;
    if (hipEventRecord(a, s) != hipSuccess) return;
    g_phase_log.push_back({phase, a, b});
    slot_ = (int)g_phase_log.size() - 1;
}

PhaseTimer::~PhaseTimer()
{
    if (slot_ >= 0) (void)hipEventRecord(g_phase_log[slot_].stop, s_);
}

// --------------------------------------------------------------- workspace

struct Workspace::Arena {
    std::vector<std::pair<void *, size_t>> chunks;
    uint64_t total = 0;
};

static std::mutex g_arena_mu;
static std::map<std::pair<int, void *>, Workspace::Arena *> *g_arenas;

Workspace::Workspace(int device, void *stream, uint64_t cap_bytes) : cap_(cap_bytes)
{
    std::lock_guard<std::mutex> lk(g_arena_mu);
    if (!g_arenas) g_arenas = new std::map<std::pair<int, void *>, Arena *>();
    auto key = std::make_pair(device, stream);
    auto it = g_arenas->find(key);
    if (it == g_arenas->end()) it = g_arenas->emplace(key, new Arena()).first;
    arena_ = it->second;
}

Workspace::Workspace(void *base, size_t bytes)
    : fixed_(static_cast<char *>(base)), fixed_size_(bytes)
{
}

Workspace::~Workspace() {}

void *Workspace::alloc(size_t bytes)
{
    if (status_ != RISM_OK) return nullptr;
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (fixed_) {
        if (off_ + bytes > fixed_size_) {
            status_ = fail(RISM_E_NOMEM, "fixed scratch exhausted");
            return nullptr;
        }
        void *p = fixed_ + off_;
        off_ += bytes;
        used_total_ = off_;
        return p;
    }
    used_total_ += bytes;
    if (cap_ && used_total_ > cap_) {
        status_ = fail(RISM_E_NOMEM, "workspace request exceeds max_workspace_bytes");
        return nullptr;
    }
    while (chunk_ < arena_->chunks.size()) {
        auto &c = arena_->chunks[chunk_];
        if (off_ + bytes <= c.second) {
            void *p = static_cast<char *>(c.first) + off_;
            off_ += bytes;
            return p;
        }
        ++chunk_;
        off_ = 0;
    }
    size_t sz = bytes < (size_t(64) << 20) ? (size_t(64) << 20) : bytes;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
        status_ = hip_fail(e, "hipMalloc(workspace)");
        return nullptr;
    }
    arena_->chunks.emplace_back(p, sz);
    arena_->total += sz;
    chunk_ = arena_->chunks.size() - 1;
    off_ = bytes;
    return p;
}

// ----------------------------------------------------------- small kernels

// Zeroes n 32-bit words (a kernel rather than hipMemsetAsync, so that the
// call stays a plain kernel launch inside captured graphs).
__global__ void k_zero_words(uint32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Pinned host staging for small device->host reads.
static int *pinned_flags()
{
    static thread_local int *p = nullptr;
    if (!p) {
        if (hipHostMalloc((void **)&p, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess)
            p = nullptr;
    }
    return p;
}

// ------------------------------------------------------------- validation

static bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

static int check_common(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                        const rism_opts *op)
{
    if (!so || !si || !gr || !op) return fail(RISM_E_INVALID, "null solute/sites/grid/opts");
    if (so->n < 0) return fail(RISM_E_INVALID, "solute n < 0");
    if (so->n > 0 && (!so->xyz || !so->q || !so->sigma || !so->eps))
        return fail(RISM_E_INVALID, "null solute array");
    if (so->n > (int64_t(1) << 31) - 64) return fail(RISM_E_INVALID, "too many atoms");
    if (si->n < 1 || si->n > kMaxSites) return fail(RISM_E_INVALID, "sites n must be in 1..8");
    if (!si->q || !si->sigma || !si->eps) return fail(RISM_E_INVALID, "null site array");
    for (int g = 0; g < si->n; ++g) {
        if (!std::isfinite(si->q[g]) || !std::isfinite(si->sigma[g]) || !std::isfinite(si->eps[g]) ||
            si->sigma[g] < 0 || si->eps[g] < 0)
            return fail(RISM_E_INVALID, "site parameters must be finite, sigma/eps >= 0");
    }
    for (int a = 0; a < 3; ++a) {
        if (gr->dims[a] <= 0) return fail(RISM_E_INVALID, "grid dims must be > 0");
        if (!(gr->spacing[a] > 0) || !std::isfinite(gr->spacing[a]))
            return fail(RISM_E_INVALID, "grid spacing must be finite and > 0");
    }
    if (!finite3(gr->origin)) return fail(RISM_E_INVALID, "grid origin must be finite");
    if ((double)gr->dims[0] * gr->dims[1] * gr->dims[2] > 4.0e9)
        return fail(RISM_E_INVALID, "grid too large (> 4e9 points)");
    if (op->method < RISM_DIRECT_F64 || op->method > RISM_TREECODE_TAYLOR)
        return fail(RISM_E_INVALID, "unknown method");
    if (op->out_dtype != RISM_F32 && op->out_dtype != RISM_F64)
        return fail(RISM_E_INVALID, "out_dtype must be RISM_F32 or RISM_F64");
    if (!std::isfinite(op->coulomb_k)) return fail(RISM_E_INVALID, "coulomb_k must be finite");
    if (!std::isfinite(op->lj_cutoff) || !std::isfinite(op->lj_tol) || op->lj_tol < 0)
        return fail(RISM_E_INVALID, "lj_cutoff / lj_tol must be finite, lj_tol >= 0");
    if (op->method >= RISM_TREECODE) {
        if (!(op->theta > 0 && op->theta < 1)) return fail(RISM_E_INVALID, "theta must be in (0,1)");
        if (op->degree < 1 || op->degree > 16) return fail(RISM_E_INVALID, "degree must be in 1..16");
        if (op->method == RISM_TREECODE_TAYLOR && op->degree > 12)
            return fail(RISM_E_INVALID, "Taylor order (degree) must be in 1..12");
        if (op->leaf_size < 1) return fail(RISM_E_INVALID, "leaf_size must be >= 1");
        if (op->batch_edge != 4 && op->batch_edge != 8 && op->batch_edge != 16)
            return fail(RISM_E_INVALID, "batch_edge must be 4, 8 or 16");
    }
    return RISM_OK;
}

static bool grid_exact_f32(const rism_grid *gr)
{
    for (int a = 0; a < 3; ++a) {
        double h = gr->spacing[a];
        if ((double)(float)h != h) return false;
        // h = m * 2^e with m an odd integer of b bits; i*h exact iff bits(i*m) <= 24
        int e;
        double fr = std::frexp(h, &e);  // h = fr * 2^e, fr in [0.5, 1)
        double m = fr;
        int bits = 0;
        while (m != std::floor(m) && bits < 64) { m *= 2; ++bits; }
        int mbits = 0;
        for (double t = m; t >= 1.0; t /= 2) ++mbits;
        int ibits = 0;
        for (int64_t t = gr->dims[a] - 1; t > 0; t >>= 1) ++ibits;
        if (mbits + ibits > 24) return false;
    }
    return true;
}

// --------------------------------------------------------------- prep

struct Prep {
    SiteParams sp{};
    GridParams g{};
    OutParams out{};
    AsymParams asym{};
    int lj_mode = LJ_NONE;
    int64_t npad = 0;
    int n_ionic = 0;
};

static void prep_common(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                        const rism_opts *op, Prep &p)
{
    p.sp.ns = si->n;
    p.sp.ns_pad = pad_sites(si->n);
    for (int g = 0; g < kMaxSites; ++g) {
        bool r = g < si->n;
        p.sp.q[g] = r ? si->q[g] : 0.0;
        p.sp.sig[g] = r ? si->sigma[g] : 0.0;
        p.sp.eps[g] = r ? si->eps[g] : 0.0;
        p.sp.ionic[g] = r && si->ionic ? (si->ionic[g] != 0) : 0;
        if (p.sp.ionic[g]) ++p.n_ionic;
    }
    for (int a = 0; a < 3; ++a) {
        p.g.o[a] = gr->origin[a];
        p.g.h[a] = gr->spacing[a];
    }
    p.g.nx = gr->dims[0];
    p.g.ny = gr->dims[1];
    p.g.nz = gr->dims[2];
    p.g.m = (int64_t)gr->dims[0] * gr->dims[1] * gr->dims[2];
    p.g.exact = grid_exact_f32(gr) ? 1 : 0;
    p.lj_mode = (op->lj_tol > 0 || op->lj_cutoff > 0) ? LJ_CUT : LJ_ALL;
    p.npad = ((so->n + kAtomPad - 1) / kAtomPad) * kAtomPad;
    if (p.npad == 0) p.npad = kAtomPad;
    p.out.f64 = op->out_dtype == RISM_F64;
    p.out.ns = si->n;
    p.out.n_ionic = p.n_ionic;
}

static void prep_asym(double eta, double kappa, double beta, double diel, double kc, Prep &p)
{
    AsymParams &A = p.asym;
    A.eta = eta;
    A.kappa = kappa;
    A.inv_eta = 1.0 / eta;
    A.a = 0.5 * kappa * eta;
    double rs = eta * (5.0 + A.a);
    A.rs2 = rs * rs;
    A.dcf0 = 2.0 / (eta * std::sqrt(kPi));
    A.tcf0 = 4.0 * std::exp(-A.a * A.a) / (eta * std::sqrt(kPi)) - 2.0 * kappa * std::erfc(A.a);
    A.yk = -kappa / std::log(2.0);
    A.tab = nullptr;
    A.tab_inv_h = kSmearIntervals / rs;
    int j = 0;
    for (int g = 0; g < p.sp.ns; ++g) {
        p.out.c_scale[g] = -beta * kc * p.sp.q[g];
        if (p.sp.ionic[g])
            p.out.h_scale[j++] = -beta * kc * p.sp.q[g] / (2.0 * diel) *
                                 std::exp(kappa * kappa * eta * eta / 4.0);
    }
}

static size_t rec_bytes(int ns_pad, bool f64)
{
    return f64 ? rec64_bytes_of(ns_pad) : rec32_bytes_of(ns_pad);
}

// Stages the atoms into FP32 and/or FP64 records, optionally the cut-off
// table, and checks the device-side error flags (one stream sync) unless the
// caller opted out.
// defer_err: when the checks need nothing back before later kernels run (no
// per-pair cut-off radius from a tolerance, no eps check), skip the stream
// sync here and hand the staging workgroups' flag words (StageArgs::err_part,
// *defer_n workgroups) to the caller, which reads them with its own
// end-of-call read-back (the kernels in between clamp every index they
// derive from atom data).
// smear_tab: also form the smeared-kernel table of p.asym there (same launch).
static int stage_atoms(const rism_solute *so, const Prep &p, const rism_opts *op, bool want32,
                       bool want64, bool check_eps, Workspace &ws, void **rec32, void **rec64,
                       double **rcut, hipStream_t s, double *max_rcut = nullptr,
                       const int **defer_err = nullptr, int *defer_n = nullptr,
                       float4 *smear_tab = nullptr, const double **bbox_part = nullptr)
{
    StageArgs a{};
    a.smear_tab = smear_tab;
    a.smear = p.asym;
    a.xyz = so->xyz;
    a.q = so->q;
    a.sig = so->sigma;
    a.eps = so->eps;
    a.n = so->n;
    a.npad = p.npad;
    for (int k = 0; k < 3; ++k) a.origin[k] = p.g.o[k];
    a.grid = p.g;
    a.lj_cutoff = op->lj_cutoff;
    a.lj_tol = op->lj_tol;
    a.lj_mode = p.lj_mode;
    a.check_eps = check_eps;
    const int nstage = (int)((p.npad + kBlock - 1) / kBlock);
    a.err_part = ws.get<int>(3 * (size_t)nstage);
    int *err_flags = ws.get<int>(4);
    a.rec32 = want32 ? ws.alloc(rec_bytes(p.sp.ns_pad, false) * p.npad) : nullptr;
    a.rec64 = want64 ? ws.alloc(rec_bytes(p.sp.ns_pad, true) * p.npad) : nullptr;
    a.rcut = rcut ? ws.get<double>((size_t)p.sp.ns * (so->n > 0 ? so->n : 1)) : nullptr;
    a.bbox_part = bbox_part ? ws.get<double>(6 * (size_t)((p.npad + kBlock - 1) / kBlock))
                            : nullptr;
    if (bbox_part) *bbox_part = a.bbox_part;
    if (ws.status() != RISM_OK) return ws.status();
    int rc;
    {
        PhaseTimer pt(op->flags & RISM_FLAG_PHASE_EVENTS, RISM_PHASE_STAGE, s);
        rc = launch_stage(p.sp, a, s);
    }
    if (rc) return rc;
    bool need_check = !(op->flags & RISM_FLAG_NO_DEVICE_CHECK) || op->lj_tol > 0 || check_eps;
    if (defer_err) *defer_err = nullptr;
    if (need_check && defer_err && !(op->lj_tol > 0) && !check_eps && so->n > 0) {
        *defer_err = a.err_part;
        if (defer_n) *defer_n = nstage;
        need_check = false;
    }
    if (need_check && so->n > 0) {
        // pinned staging (allocated once per thread), or the stack when the
        // call may not allocate (a pageable copy, synchronous anyway here)
        int local[4] = {0, 0, 0, 0};
        int *h = ws.fixed() ? local : pinned_flags();
        if (!h) return fail(RISM_E_HIP, "pinned host buffer allocation failed");
        if ((rc = launch_stage_flags(a.err_part, nstage, err_flags, s))) return rc;
        RISM_HIP(hipMemcpyAsync(h, err_flags, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
        RISM_HIP(hipStreamSynchronize(s));
        if (h[0]) return fail(RISM_E_INVALID, "non-finite atom input or negative sigma/eps");
        if (h[1])
            return fail(RISM_E_INVALID, check_eps ? "dL/deps needs eps_a > 0 for every atom"
                                                  : "lj_tol must be below eps_ga of every pair");
        if (max_rcut) {
            float r2;
            std::memcpy(&r2, &h[2], sizeof(float));
            *max_rcut = std::sqrt((double)r2);
        }
    }
    if (rec32) *rec32 = a.rec32;
    if (rec64) *rec64 = a.rec64;
    if (rcut) *rcut = a.rcut;
    return RISM_OK;
}

// ------------------------------------------------------------ forward core

static int zero_grid(void *buf, int f64, int64_t count, hipStream_t s)
{
    if (!buf || count == 0) return RISM_OK;
    const int64_t words = count * (f64 ? 2 : 1);
    const int64_t blocks = std::min<int64_t>((words + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(k_zero_words, (int)blocks, kBlock, 0, s, static_cast<uint32_t *>(buf),
                       words);
    RISM_HIP(hipGetLastError());
    return RISM_OK;
}

static int forward(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                   const rism_opts *op, bool asym_call, double eta, double kappa, double beta,
                   double diel, void *u, double *lj_tail, void *c, void *h, void *stream,
                   void *fixed_scratch = nullptr, size_t fixed_bytes = 0)
{
    rism_stats st{};
    int rc = check_common(so, si, gr, op);
    if (rc) return rc;
    if (asym_call) {
        if (!(eta > 0) || !std::isfinite(eta)) return fail(RISM_E_INVALID, "eta must be > 0");
        if (!(kappa >= 0) || !std::isfinite(kappa)) return fail(RISM_E_INVALID, "kappa must be >= 0");
        if (!(beta > 0) || !std::isfinite(beta)) return fail(RISM_E_INVALID, "beta must be > 0");
        if (!(diel > 0) || !std::isfinite(diel)) return fail(RISM_E_INVALID, "dielectric must be > 0");
    }
    Prep p;
    prep_common(so, si, gr, op, p);
    if (!asym_call) { c = nullptr; h = nullptr; }
    if (p.n_ionic == 0) h = nullptr;
    if (!u && !c && !h && !lj_tail) {
        g_stats = st;
        return RISM_OK;
    }
    p.out.u = u;
    p.out.c = c;
    p.out.h = h;
    p.out.want_u = u != nullptr;
    p.out.want_c = c != nullptr;
    p.out.want_h = h != nullptr;
    for (int g = 0; g < p.sp.ns; ++g) p.out.u_coul[g] = op->coulomb_k * p.sp.q[g];
    if (asym_call) prep_asym(eta, kappa, beta, diel, op->coulomb_k, p);
    else prep_asym(1.0, 0.0, 1.0, 1.0, op->coulomb_k, p);
    const bool asym_on = c || h;
    if (op->method >= RISM_TREECODE && u && p.lj_mode != LJ_CUT)
        return fail(RISM_E_UNSUPPORTED, "treecode methods need an LJ cut-off (lj_cutoff or lj_tol)");

    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    RISM_HIP(hipGetDevice(&dev));
    Workspace ws = fixed_scratch ? Workspace(fixed_scratch, fixed_bytes)
                                 : Workspace(dev, stream, op->max_workspace_bytes);

    if (so->n == 0) {
        if ((rc = zero_grid(u, p.out.f64, p.sp.ns * p.g.m, s))) return rc;
        if ((rc = zero_grid(c, p.out.f64, p.sp.ns * p.g.m, s))) return rc;
        if ((rc = zero_grid(h, p.out.f64, p.n_ionic * p.g.m, s))) return rc;
        if (lj_tail)
            for (int g = 0; g < p.sp.ns; ++g) lj_tail[g] = 0.0;
        g_stats = st;
        return RISM_OK;
    }

    const bool f64path = op->method == RISM_DIRECT_F64;
    void *rec32 = nullptr, *rec64 = nullptr;
    double *rcut = nullptr;
    bool want_rcut = lj_tail && p.lj_mode == LJ_CUT;
    double max_rcut = op->lj_cutoff;
    // the cluster-particle treecodes end with a read-back of their own: the
    // input check joins it instead of synchronising here
    const bool cp_method = (op->method == RISM_TREECODE_CP || op->method == RISM_TREECODE_TAYLOR) &&
                           (u || c || h);
    const int *stage_err = nullptr;
    int n_stage_err = 0;
    const double *bbox_part = nullptr;   // per-workgroup atom boxes, for the trees
    const bool tree_method = op->method == RISM_TREECODE || cp_method;
    // the FP32 paths' smeared-kernel table, formed by the staging launch
    float4 *tab = nullptr;
    if (asym_on && !f64path) {
        tab = ws.get<float4>(2 * kSmearIntervals);
        if (!tab) return ws.status();
    }
    rc = stage_atoms(so, p, op, !f64path, f64path, false, ws, &rec32, &rec64,
                     want_rcut ? &rcut : nullptr, s, &max_rcut, cp_method ? &stage_err : nullptr,
                     &n_stage_err, tab, tree_method ? &bbox_part : nullptr);
    if (rc) return rc;
    if (tab) p.asym.tab = tab;

    if (u || c || h) {
        DirectArgs da{};
        da.n = so->n;
        da.npad = p.npad;
        da.g = p.g;
        da.out = p.out;
        da.asym = p.asym;
        da.lj_mode = u ? p.lj_mode : LJ_NONE;
        da.lj_uniform = op->lj_tol <= 0 && op->lj_cutoff > 0;
        da.asym_on = asym_on;
        const bool ev = op->flags & RISM_FLAG_PHASE_EVENTS;
        if (f64path) {
            da.atoms = rec64;
            PhaseTimer pt(ev, RISM_PHASE_DIRECT_F64, s);
            rc = launch_direct_f64(p.sp, da, s);
            st.pairs_direct = (double)so->n * p.g.m;
        } else if (op->method == RISM_DIRECT_F32C) {
            da.atoms = rec32;
            PhaseTimer pt(ev, RISM_PHASE_DIRECT_F32, s);
            rc = launch_direct_f32(p.sp, da, s);
            st.pairs_direct = (double)so->n * p.g.m;
        } else {
            TreeCallArgs ta{};
            ta.solute = so;
            ta.sp = p.sp;
            ta.g = p.g;
            ta.out = p.out;
            ta.asym = p.asym;
            ta.opts = op;
            ta.lj_mode = da.lj_mode;
            ta.lj_uniform = da.lj_uniform;
            ta.asym_on = asym_on;
            ta.rec32 = rec32;
            ta.npad = p.npad;
            // largest LJ cut-off radius (read back with the device checks,
            // which lj_tol > 0 always runs)
            ta.rmax_short = op->lj_tol > 0 ? max_rcut : op->lj_cutoff;
            ta.stage_err = stage_err;
            ta.n_stage_err = n_stage_err;
            ta.bbox_part = bbox_part;
            ta.n_bbox_part = (int)((p.npad + kBlock - 1) / kBlock);
            rc = op->method == RISM_TREECODE ? tree_forward(ta, ws, st, s)
                                             : tree_forward_cp(ta, ws, st, s);
        }
        if (rc) return rc;
    }
    if (lj_tail) {
        if (p.lj_mode != LJ_CUT) {
            for (int g = 0; g < p.sp.ns; ++g) lj_tail[g] = 0.0;
        } else {
            double *td = ws.get<double>(kMaxSites);
            if (!td) return ws.status();
            rc = launch_lj_tail(p.sp, rcut, so->sigma, so->eps, so->n, td, s);
            if (rc) return rc;
            RISM_HIP(hipMemcpyAsync(lj_tail, td, p.sp.ns * sizeof(double), hipMemcpyDeviceToHost, s));
            RISM_HIP(hipStreamSynchronize(s));
        }
    }
    st.workspace_bytes = (int64_t)ws.in_use();
    g_stats = st;
    return RISM_OK;
}

// ------------------------------------------------------- no-alloc scratch
// Device scratch of rism_initialize_noalloc: a file-scope array that every
// GPU the library runs on holds until the process ends.  In host code its
// name is not a device address; the address is taken once per device with
// hipGetSymbolAddress and only that address reaches kernels and copies.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void *> *g_scratch_ptr;

// Address of this device's scratch array (the device must be current).
static int noalloc_scratch(int dev, void **ptr)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr) g_scratch_ptr = new std::map<int, void *>();
    auto it = g_scratch_ptr->find(dev);
    if (it != g_scratch_ptr->end()) {
        *ptr = it->second;
        return RISM_OK;
    }
    void *p = nullptr;
    RISM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(RISM_E_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    (*g_scratch_ptr)[dev] = p;
    *ptr = p;
    return RISM_OK;
}

// Scratch bytes forward() carves for a direct-sum call (the fixed-mode
// workspace rounds every request up to 256 bytes).
static size_t noalloc_need(const Prep &p, int64_t n, bool f64path, bool want_rcut, bool asym)
{
    auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t need = r(4 * sizeof(int));                                 // stage error flags
    need += r(rec_bytes(p.sp.ns_pad, f64path) * (size_t)p.npad);      // atom records
    if (want_rcut) need += r(sizeof(double) * p.sp.ns * (size_t)(n > 0 ? n : 1));
    if (asym && !f64path) need += r(sizeof(float4) * 2 * kSmearIntervals);   // table
    if (want_rcut) need += r(sizeof(double) * kMaxSites);             // tail constants
    return need;
}

}  // namespace rism

using namespace rism;

extern "C" {

int rism_initialize_noalloc(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                            const rism_opts *op, double eta, double kappa, double beta,
                            double diel, void *u, double *lj_tail, void *c, void *h,
                            void *stream)
{
    int rc = check_common(so, si, gr, op);
    if (rc) return rc;
    if (op->method != RISM_DIRECT_F64 && op->method != RISM_DIRECT_F32C)
        return fail(RISM_E_UNSUPPORTED,
                    "rism_initialize_noalloc: only RISM_DIRECT_F64 and RISM_DIRECT_F32C");
    Prep p;
    prep_common(so, si, gr, op, p);
    const bool f64path = op->method == RISM_DIRECT_F64;
    const bool asym = c || (h && p.n_ionic > 0);
    const bool want_rcut = lj_tail && p.lj_mode == LJ_CUT;
    const size_t need = noalloc_need(p, so->n, f64path, want_rcut, asym);
    if (need > kNoAllocScratchBytes) {
        char msg[256];
        std::snprintf(msg, sizeof msg,
                      "rism_initialize_noalloc: %lld atoms with %d sites need %zu bytes of "
                      "scratch, above its fixed %zu bytes",
                      (long long)so->n, (int)si->n, need, kNoAllocScratchBytes);
        return fail(RISM_E_INVALID, msg);
    }
    int dev = 0;
    RISM_HIP(hipGetDevice(&dev));
    void *base = nullptr;
    if ((rc = noalloc_scratch(dev, &base))) return rc;
    // phase events and the statistics counters would create events or
    // buffers: not recorded by this entry point
    rism_opts o = *op;
    o.flags &= ~(RISM_FLAG_PHASE_EVENTS | RISM_FLAG_STATS);
    return forward(so, si, gr, &o, true, eta, kappa, beta, diel, u, lj_tail, c, h, stream, base,
                   kNoAllocScratchBytes);
}

void rism_default_opts(rism_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->method = RISM_TREECODE_CP;
    o->out_dtype = RISM_F32;
    o->coulomb_k = 332.0522173;
    o->lj_cutoff = 9.0;
    o->lj_tol = 0.0;
    o->theta = 0.6;
    o->degree = 8;
    o->leaf_size = 64;
    o->batch_edge = 8;
    o->flags = 0;
    o->max_workspace_bytes = 0;
}

int rism_potential(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                   const rism_opts *op, void *u, double *lj_tail, void *stream)
{
    if (!u && !lj_tail) return fail(RISM_E_INVALID, "no output requested (u and lj_tail are NULL)");
    return forward(so, si, gr, op, false, 1, 0, 1, 1, u, lj_tail, nullptr, nullptr, stream);
}

int rism_asymptotics(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                     const rism_opts *op, double eta, double kappa, double beta, double diel,
                     void *c, void *h, void *stream)
{
    if (!c && !h) return fail(RISM_E_INVALID, "no output requested (c_lr and h_lr are NULL)");
    return forward(so, si, gr, op, true, eta, kappa, beta, diel, nullptr, nullptr, c, h, stream);
}

int rism_asymptotics_k(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                       const rism_opts *op, double eta, double kappa, double beta, double diel,
                       double tol, void *c, void *h, void *stream)
{
    int rc = check_common(so, si, gr, op);
    if (rc) return rc;
    if (!(eta > 0) || !std::isfinite(eta)) return fail(RISM_E_INVALID, "eta must be > 0");
    if (!(kappa >= 0) || !std::isfinite(kappa)) return fail(RISM_E_INVALID, "kappa must be >= 0");
    if (!(beta > 0) || !std::isfinite(beta)) return fail(RISM_E_INVALID, "beta must be > 0");
    if (!(diel > 0) || !std::isfinite(diel)) return fail(RISM_E_INVALID, "dielectric must be > 0");
    if (!std::isfinite(tol)) return fail(RISM_E_INVALID, "tol must be finite");
    Prep p;
    prep_common(so, si, gr, op, p);
    if (p.n_ionic == 0) h = nullptr;
    if (!c && !h) return fail(RISM_E_INVALID, "no output requested (c and h are NULL)");
    AkArgs ak{};
    ak.g.nx = gr->dims[0];
    ak.g.ny = gr->dims[1];
    ak.g.nz = gr->dims[2];
    ak.g.nxh = gr->dims[0] / 2 + 1;
    for (int a = 0; a < 3; ++a) {
        ak.g.o[a] = gr->origin[a];
        ak.g.h[a] = gr->spacing[a];
    }
    ak.n = so->n;
    ak.eta2_4 = eta * eta / 4.0;
    ak.kappa2 = kappa * kappa;
    ak.c = c;
    ak.h = h;
    ak.f64 = op->out_dtype == RISM_F64;
    ak.ns = si->n;
    ak.n_ionic = p.n_ionic;
    double qc = 0.0, qh = 0.0;
    for (int g = 0, j = 0; g < si->n; ++g) {
        ak.c_scale[g] = -4.0 * kPi * beta * op->coulomb_k * si->q[g];
        qc = std::max(qc, std::fabs(si->q[g]));
        if (p.sp.ionic[g]) {
            ak.h_scale[j++] = -4.0 * kPi * beta * op->coulomb_k * si->q[g] / diel;
            qh = std::max(qh, std::fabs(si->q[g]));
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    RISM_HIP(hipGetDevice(&dev));
    Workspace ws(dev, stream, op->max_workspace_bytes);
    double *k2cut = ws.get<double>(3);
    if (ws.status()) return ws.status();
    // the bound of Sec. 2.5 per unit sum |Q_a| (summed on the device)
    const double pre = 4.0 * std::sqrt(2.0) * kPi * beta * std::fabs(op->coulomb_k);
    if ((rc = launch_ak_cutoffs(so->q, so->n, tol, pre * qc, pre * qh, eta, kappa, diel, k2cut, s)))
        return rc;
    ak.k2cut = k2cut;
    rc = launch_asym_k(ak, so->xyz, so->q, ws, op->flags & RISM_FLAG_PHASE_EVENTS, s);
    if (rc) return rc;
    rism_stats st{};
    st.pairs_direct = (double)so->n * ak.g.nxh * ak.g.ny * ak.g.nz;
    st.workspace_bytes = (int64_t)ws.in_use();
    g_stats = st;
    return RISM_OK;
}

int rism_initialize(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                    const rism_opts *op, double eta, double kappa, double beta, double diel,
                    void *u, double *lj_tail, void *c, void *h, void *stream)
{
    return forward(so, si, gr, op, true, eta, kappa, beta, diel, u, lj_tail, c, h, stream);
}

int rism_potential_backward(const rism_solute *so, const rism_sites *si, const rism_grid *gr,
                            const rism_opts *op, const void *w, double *dxyz, double *dq,
                            double *deps, double *dsig, void *stream)
{
    int rc = check_common(so, si, gr, op);
    if (rc) return rc;
    if (!w) return fail(RISM_E_INVALID, "dL_du is NULL");
    Prep p;
    prep_common(so, si, gr, op, p);
    if (op->method == RISM_TREECODE_TAYLOR)
        return fail(RISM_E_UNSUPPORTED, "the Taylor treecode has no adjoint; use RISM_TREECODE_CP");
    if (op->method >= RISM_TREECODE && p.lj_mode != LJ_CUT)
        return fail(RISM_E_UNSUPPORTED, "treecode backward needs an LJ cut-off");
    rism_stats st{};
    if (so->n == 0 || (!dxyz && !dq && !deps && !dsig)) {
        g_stats = st;
        return RISM_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    RISM_HIP(hipGetDevice(&dev));
    Workspace ws(dev, stream, op->max_workspace_bytes);
    const bool f64path = op->method == RISM_DIRECT_F64;
    void *rec32 = nullptr, *rec64 = nullptr;
    double max_rcut = op->lj_cutoff;
    rc = stage_atoms(so, p, op, !f64path, f64path, deps != nullptr, ws, &rec32, &rec64, nullptr, s,
                     &max_rcut);
    if (rc) return rc;
    AdjointArgs a{};
    a.atoms = f64path ? rec64 : rec32;
    a.n = so->n;
    a.npad = p.npad;
    a.sp = p.sp;
    a.g = p.g;
    a.w = w;
    a.w_f64 = op->out_dtype == RISM_F64;
    a.kc = op->coulomb_k;
    a.lj_mode = p.lj_mode;
    a.eps_in = so->eps;
    a.sig_in = so->sigma;
    a.dxyz = dxyz;
    a.dq = dq;
    a.deps = deps;
    a.dsig = dsig;
    a.opts = op;
    a.rmax_lj = op->lj_tol > 0 ? max_rcut : op->lj_cutoff;
    rc = op->method >= RISM_TREECODE ? adjoint_tree(a, ws, st, s)
                                     : adjoint_direct(a, f64path, ws, st, s);
    if (rc) return rc;
    st.workspace_bytes = (int64_t)ws.in_use();
    g_stats = st;
    return RISM_OK;
}

int rism_compare(const void *x, int32_t x_dtype, const double *ref, int64_t n, double ref_cap,
                 const uint8_t *mask, double *out, void *stream)
{
    if (!x || !ref || !out || n < 0) return fail(RISM_E_INVALID, "null argument or n < 0");
    if (x_dtype != RISM_F32 && x_dtype != RISM_F64) return fail(RISM_E_INVALID, "bad x_dtype");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    RISM_HIP(hipGetDevice(&dev));
    Workspace ws(dev, stream, 0);
    const int nb = 1024;
    double *part = ws.get<double>(6 * nb);
    if (!part) return ws.status();
    int rc = launch_compare(x, x_dtype == RISM_F64, ref, mask, n, ref_cap, part, nb, s);
    if (rc) return rc;
    std::vector<double> hpart(6 * nb);
    RISM_HIP(hipMemcpyAsync(hpart.data(), part, hpart.size() * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    RISM_HIP(hipStreamSynchronize(s));
    double r[6] = {0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nb; ++b) {
        r[0] += hpart[6 * b];
        r[1] += hpart[6 * b + 1];
        r[2] = std::max(r[2], hpart[6 * b + 2]);
        r[3] += hpart[6 * b + 3];
        r[4] += hpart[6 * b + 4];
        r[5] += hpart[6 * b + 5];
    }
    for (int k = 0; k < 6; ++k) out[k] = r[k];
    return RISM_OK;
}

int rism_near_mask(const rism_solute *so, const rism_grid *gr, double radius, uint8_t *mask,
                   void *stream)
{
    if (!so || !gr || !mask) return fail(RISM_E_INVALID, "null solute, grid or mask");
    if (so->n < 0 || (so->n > 0 && !so->xyz)) return fail(RISM_E_INVALID, "bad solute");
    if (so->n > (int64_t(1) << 31) - 64) return fail(RISM_E_INVALID, "too many atoms");
    if (!std::isfinite(radius) || radius < 0) return fail(RISM_E_INVALID, "radius must be >= 0");
    for (int a = 0; a < 3; ++a) {
        if (gr->dims[a] <= 0) return fail(RISM_E_INVALID, "grid dims must be > 0");
        if (!(gr->spacing[a] > 0) || !std::isfinite(gr->spacing[a]))
            return fail(RISM_E_INVALID, "grid spacing must be finite and > 0");
    }
    if (!finite3(gr->origin)) return fail(RISM_E_INVALID, "grid origin must be finite");
    GridParams g{};
    for (int a = 0; a < 3; ++a) {
        g.o[a] = gr->origin[a];
        g.h[a] = gr->spacing[a];
    }
    g.nx = gr->dims[0];
    g.ny = gr->dims[1];
    g.nz = gr->dims[2];
    g.m = (int64_t)g.nx * g.ny * g.nz;
    return launch_near_mask(so->xyz, so->n, g, radius, mask, static_cast<hipStream_t>(stream));
}

int rism_phase_times(double *ms, int64_t *count)
{
    if (!ms || !count) return fail(RISM_E_INVALID, "null output");
    for (int p = 0; p < RISM_NUM_PHASES; ++p) { ms[p] = 0; count[p] = 0; }
    int rc = RISM_OK;
    for (auto &r : g_phase_log) {
        float t = 0.f;
        if (rc == RISM_OK) {
            hipError_t e = hipEventSynchronize(r.stop);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime");
        }
        if (r.phase >= 0 && r.phase < RISM_NUM_PHASES) {
            ms[r.phase] += t;
            count[r.phase] += 1;
        }
        g_event_pool.push_back(r.start);
        g_event_pool.push_back(r.stop);
    }
    g_phase_log.clear();
    return rc;
}

int rism_last_stats(rism_stats *stats)
{
    if (!stats) return fail(RISM_E_INVALID, "null stats");
    *stats = g_stats;
    return RISM_OK;
}

const char *rism_last_error(void) { return g_error.c_str(); }

}  // extern "C"
