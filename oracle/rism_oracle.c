/*
 * FP64 CPU oracle for the 3D-RISM initialisation quantities.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP
 * path.
 *
 * Everything here is a plain direct sum over all (atom, point) pairs in
 * double precision, atoms in input order, using libm erf/erfc/exp/sqrt.
 * No tree, no splitting, no blocking.
 *
 * Paper: Wilson, Krasny & Luchko, "Accelerating the 3D-RISM theory of
 * molecular solvation with treecode summation and cut-offs".
 *
 * Definitions followed (with the readings adopted where the paper is silent):
 *  - u_gamma(r): Sec. 2.1 (potential = Coulomb + Lennard-Jones between the
 *    solvent site and every solute atom) and Sec. 2.6 (LJ A/r^12 - B/r^6,
 *    truncated form Eq. 28).  Reading: Coulomb carries the constant k_C
 *    (units A, e, kcal/mol); A = 4 eps sigma^12, B = 4 eps sigma^6 with
 *    Lorentz-Berthelot mixing sigma_ga = (sigma_g + sigma_a)/2,
 *    eps_ga = sqrt(eps_g eps_a).  Cut-off: the pair is kept iff d < r_cut.
 *    A grid point that coincides with an atom (d == 0) gets u = +inf.
 *  - c^lr_gamma(r): Sec. 2.2, Eq. 4, times k_C; d == 0 takes the limit
 *    erf(d/eta)/d -> 2/(eta sqrt(pi)).
 *  - h^lr_j(r): Sec. 2.2, Eq. 6, times k_C, for ionic sites only; d == 0
 *    takes the limit of the bracket / d:
 *      4 exp(-kappa^2 eta^2/4)/(eta sqrt(pi)) - 2 kappa erfc(kappa eta/2).
 *  - LJ cut-off from a tolerance: Sec. 2.6 (|u_LJ(r_cut)| = tol, beyond the
 *    minimum), solved here by plain bisection.
 *  - Tail constant: Sec. 2.6 (final result for the chemical-potential
 *    correction): T_gamma = 4 pi sum_a int_{r_cut}^inf u_LJ(r) r^2 dr
 *                        = (4 pi / 3) sum_a (A/(3 r_c^9) - B/r_c^3).
 *  - c^lr_gamma(k), h^lr_j(k): Sec. 2.2, Eqs. 5 and 7, times k_C, on the half
 *    grid of a real-to-complex transform of the [nz][ny][nx] grid (entries
 *    [mz][my][mx], mx = 0..nx/2; my, mz in transform order 0, 1, ..., then
 *    the negative frequencies), k = 2 pi (mx/(nx hx), my/(ny hy), mz/(nz hz)).
 *    Reading: the structure factor is S(k) = sum_a Q_a exp(-i k.(R_a - o)),
 *    o the grid origin, i.e. the sign and anchor of a forward discrete
 *    transform of the grid (the paper writes exp(+i k.R): the same quantity
 *    under the opposite sign convention).  c^lr(k = 0) is set to 0 (1/k^2
 *    with S(0) = 0 for a neutral solute), and so is h^lr(k = 0) when
 *    kappa = 0 (the same singularity).  Entries beyond the frequency
 *    cut-off are 0.
 *  - Frequency cut-off: Sec. 2.5, Eq. 26 and the h^lr bound after it.
 *    Reading: the bound uses sum_a |Q_a| (the signed sum vanishes for a
 *    neutral solute) and the largest |q| of the sites concerned; the root
 *    k_cut of bound(k) = tol is found here by plain bisection.
 *  - Backward: gradient of L = sum_gamma sum_r w_gamma(r) u_gamma(r) with
 *    respect to atom positions, charges, eps_a and sigma_a, differentiating
 *    the definition of u above term by term (the jump at r_cut is ignored).
 *
 * One part is not a direct sum: the Taylor-recurrence treecode at the end
 * of the file (Secs. 2.3 and 2.4), an approximation whose steps are taken
 * here in the paper's order, pair by pair, with no moments, shifts or
 * blocking.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846

/* ---------------------------------------------------------------- mixing */

static void lb_mix(double sig_g, double eps_g, double sig_a, double eps_a,
                   double *sig_ga, double *eps_ga)
{
    *sig_ga = 0.5 * (sig_g + sig_a);
    *eps_ga = sqrt(eps_g * eps_a);
}

static double lj_pair(double sig, double eps, double d)
{
    double s = sig / d;
    double s6 = s * s * s * s * s * s;
    return 4.0 * eps * (s6 * s6 - s6);
}

/* ---------------------------------------------------------------- points */

static void point_of(const double origin[3], const double spacing[3],
                     const int32_t dims[3], int64_t idx, double p[3])
{
    int64_t nx = dims[0], ny = dims[1];
    int64_t i = idx % nx, j = (idx / nx) % ny, k = idx / (nx * ny);
    p[0] = origin[0] + (double)i * spacing[0];
    p[1] = origin[1] + (double)j * spacing[1];
    p[2] = origin[2] + (double)k * spacing[2];
}

/*
 * u at one point for every site.  terms: bit 0 Coulomb, bit 1 LJ.
 * rcut: [ns][n] per-pair cut-off radii, or NULL for no cut-off.
 */
static void potential_at(int64_t n, const double *xyz, const double *q,
                         const double *sig, const double *eps,
                         int32_t ns, const double *sq, const double *ssig,
                         const double *seps, double kc, const double *rcut,
                         int terms, const double p[3], double *out, int64_t stride)
{
    for (int32_t g = 0; g < ns; ++g) {
        double coul = 0.0, lj = 0.0;
        int hit = 0;
        for (int64_t a = 0; a < n; ++a) {
            double dx = p[0] - xyz[3 * a + 0];
            double dy = p[1] - xyz[3 * a + 1];
            double dz = p[2] - xyz[3 * a + 2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (d == 0.0) { hit = 1; continue; }
            if (terms & 1) coul += kc * q[a] * sq[g] / d;
            if (terms & 2) {
                double s_ga, e_ga;
                lb_mix(ssig[g], seps[g], sig[a], eps[a], &s_ga, &e_ga);
                if (rcut == NULL || d < rcut[(int64_t)g * n + a])
                    lj += lj_pair(s_ga, e_ga, d);
            }
        }
        out[(int64_t)g * stride] = hit ? INFINITY : coul + lj;
    }
}

int oracle_potential_points(int64_t n, const double *xyz, const double *q,
                            const double *sig, const double *eps, int32_t ns,
                            const double *sq, const double *ssig, const double *seps,
                            double kc, const double *rcut, int terms,
                            int64_t npts, const double *pts, double *u)
{
    if (n < 0 || ns <= 0 || npts < 0) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < npts; ++i)
        potential_at(n, xyz, q, sig, eps, ns, sq, ssig, seps, kc, rcut, terms,
                     pts + 3 * i, u + i, npts);
    return 0;
}

int oracle_potential_grid(int64_t n, const double *xyz, const double *q,
                          const double *sig, const double *eps, int32_t ns,
                          const double *sq, const double *ssig, const double *seps,
                          double kc, const double *rcut, int terms,
                          const double *origin, const double *spacing,
                          const int32_t *dims, double *u)
{
    if (n < 0 || ns <= 0 || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return -1;
    int64_t m = (int64_t)dims[0] * dims[1] * dims[2];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        double p[3];
        point_of(origin, spacing, dims, i, p);
        potential_at(n, xyz, q, sig, eps, ns, sq, ssig, seps, kc, rcut, terms,
                     p, u + i, m);
    }
    return 0;
}

/* ----------------------------------------------------------- asymptotics */

/* erf(d/eta)/d, with its d -> 0 limit. */
static double dcf_kernel(double d, double eta)
{
    if (d == 0.0) return 2.0 / (eta * sqrt(ORACLE_PI));
    return erf(d / eta) / d;
}

/* The bracket of Eq. 6 divided by d, with its d -> 0 limit. */
static double tcf_kernel(double d, double eta, double kappa)
{
    double a = 0.5 * kappa * eta;
    if (d == 0.0)
        return 4.0 * exp(-a * a) / (eta * sqrt(ORACLE_PI)) - 2.0 * kappa * erfc(a);
    double x = d / eta;
    return (exp(-kappa * d) * erfc(a - x) - exp(kappa * d) * erfc(a + x)) / d;
}

static void asymptotics_at(int64_t n, const double *xyz, const double *q,
                           int32_t ns, const double *sq, const int32_t *ionic,
                           double kc, double eta, double kappa, double beta,
                           double diel, const double p[3],
                           double *c, double *h, int64_t stride)
{
    double sum_c = 0.0, sum_h = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        double dx = p[0] - xyz[3 * a + 0];
        double dy = p[1] - xyz[3 * a + 1];
        double dz = p[2] - xyz[3 * a + 2];
        double d = sqrt(dx * dx + dy * dy + dz * dz);
        if (c) sum_c += q[a] * dcf_kernel(d, eta);
        if (h) sum_h += q[a] * tcf_kernel(d, eta, kappa);
    }
    int32_t j = 0;
    for (int32_t g = 0; g < ns; ++g) {
        if (c) c[(int64_t)g * stride] = -beta * kc * sq[g] * sum_c;
        if (ionic[g]) {
            if (h)
                h[(int64_t)j * stride] = -beta * kc * sq[g] / (2.0 * diel)
                                         * exp(kappa * kappa * eta * eta / 4.0) * sum_h;
            ++j;
        }
    }
}

int oracle_asymptotics_points(int64_t n, const double *xyz, const double *q,
                              int32_t ns, const double *sq, const int32_t *ionic,
                              double kc, double eta, double kappa, double beta,
                              double diel, int64_t npts, const double *pts,
                              double *c, double *h)
{
    if (n < 0 || ns <= 0 || npts < 0 || !(eta > 0.0) || kappa < 0.0 || !(diel > 0.0))
        return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < npts; ++i)
        asymptotics_at(n, xyz, q, ns, sq, ionic, kc, eta, kappa, beta, diel,
                       pts + 3 * i, c ? c + i : NULL, h ? h + i : NULL, npts);
    return 0;
}

int oracle_asymptotics_grid(int64_t n, const double *xyz, const double *q,
                            int32_t ns, const double *sq, const int32_t *ionic,
                            double kc, double eta, double kappa, double beta,
                            double diel, const double *origin, const double *spacing,
                            const int32_t *dims, double *c, double *h)
{
    if (n < 0 || ns <= 0 || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0 ||
        !(eta > 0.0) || kappa < 0.0 || !(diel > 0.0))
        return -1;
    int64_t m = (int64_t)dims[0] * dims[1] * dims[2];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        double p[3];
        point_of(origin, spacing, dims, i, p);
        asymptotics_at(n, xyz, q, ns, sq, ionic, kc, eta, kappa, beta, diel,
                       p, c ? c + i : NULL, h ? h + i : NULL, m);
    }
    return 0;
}

/* --------------------------------------------- reciprocal-space asymptotics */

/* Frequency index of transform position j on an axis of n points. */
static int freq_index(int j, int n)
{
    return j <= (n - 1) / 2 ? j : j - n;
}

/* Entries e of the half grid (all of them when entries is NULL, else the
 * n_entries listed flat indices); outputs [site][entry][re, im]. */
int oracle_asymptotics_k_entries(int64_t n, const double *xyz, const double *q,
                                 int32_t ns, const double *sq, const int32_t *ionic,
                                 double kc, double eta, double kappa, double beta,
                                 double diel, const double *origin, const double *spacing,
                                 const int32_t *dims, double kcut_c, double kcut_h,
                                 int64_t n_entries, const int64_t *entries,
                                 double *c, double *h)
{
    if (n < 0 || ns <= 0 || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0 ||
        !(eta > 0.0) || kappa < 0.0 || !(diel > 0.0))
        return -1;
    const int nxh = dims[0] / 2 + 1;
    const int64_t mk = entries ? n_entries : (int64_t)nxh * dims[1] * dims[2];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ie = 0; ie < mk; ++ie) {
        const int64_t e = entries ? entries[ie] : ie;
        const int jx = (int)(e % nxh);
        const int jy = (int)((e / nxh) % dims[1]);
        const int jz = (int)(e / ((int64_t)nxh * dims[1]));
        double k[3];
        k[0] = 2.0 * ORACLE_PI * jx / (dims[0] * spacing[0]);
        k[1] = 2.0 * ORACLE_PI * freq_index(jy, dims[1]) / (dims[1] * spacing[1]);
        k[2] = 2.0 * ORACLE_PI * freq_index(jz, dims[2]) / (dims[2] * spacing[2]);
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double kk = sqrt(k2);
        double sre = 0.0, sim = 0.0;
        for (int64_t a = 0; a < n; ++a) {
            double ph = 0.0;
            for (int d = 0; d < 3; ++d) ph += k[d] * (xyz[3 * a + d] - origin[d]);
            sre += q[a] * cos(ph);
            sim -= q[a] * sin(ph);
        }
        const double gauss = exp(-k2 * eta * eta / 4.0);
        int32_t j = 0;
        for (int32_t g = 0; g < ns; ++g) {
            if (c) {
                double f = 0.0;
                if (k2 > 0.0 && !(kcut_c > 0.0 && kk > kcut_c))
                    f = -4.0 * ORACLE_PI * beta * kc * sq[g] * gauss / k2;
                c[2 * ((int64_t)g * mk + ie)] = f * sre;
                c[2 * ((int64_t)g * mk + ie) + 1] = f * sim;
            }
            if (ionic[g]) {
                if (h) {
                    double f = 0.0;
                    if (!(kcut_h > 0.0 && kk > kcut_h) && k2 + kappa * kappa > 0.0)
                        f = -4.0 * ORACLE_PI * beta * kc * sq[g] * gauss / (diel * (k2 + kappa * kappa));
                    h[2 * ((int64_t)j * mk + ie)] = f * sre;
                    h[2 * ((int64_t)j * mk + ie) + 1] = f * sim;
                }
                ++j;
            }
        }
    }
    return 0;
}

int oracle_asymptotics_k(int64_t n, const double *xyz, const double *q,
                         int32_t ns, const double *sq, const int32_t *ionic,
                         double kc, double eta, double kappa, double beta,
                         double diel, const double *origin, const double *spacing,
                         const int32_t *dims, double kcut_c, double kcut_h,
                         double *c, double *h)
{
    return oracle_asymptotics_k_entries(n, xyz, q, ns, sq, ionic, kc, eta, kappa, beta, diel,
                                        origin, spacing, dims, kcut_c, kcut_h, 0, NULL, c, h);
}

/* Cut-off wave number of the c^lr (which = 0) or h^lr (which = 1) bound of
 * Sec. 2.5: the k > 0 where bound(k) = tol, bound(k) =
 * 4 sqrt(2) pi beta k_C qmax sum|Q| exp(-k^2 eta^2/4) / (k^2 [+ kappa^2] [eps]).
 * The bound decreases in k, so the root is bracketed and bisected.  Returns
 * 0 if tol <= 0 or the bound never exceeds tol (no cut-off needed at k > 0
 * would be 0 too: every k is below tol). */
double oracle_kcut(int which, double tol, double qmax, double qabs_sum, double kc,
                   double eta, double kappa, double beta, double diel)
{
    if (!(tol > 0.0)) return 0.0;
    const double pref = 4.0 * sqrt(2.0) * ORACLE_PI * beta * kc * fabs(qmax) * qabs_sum;
    double lo = 1e-12, hi = 1.0;
#define BOUND(k) (which == 0 ? pref * exp(-(k) * (k) * eta * eta / 4.0) / ((k) * (k)) \
                             : pref * exp(-(k) * (k) * eta * eta / 4.0) / (diel * ((k) * (k) + kappa * kappa)))
    if (BOUND(lo) <= tol) return 0.0;
    while (BOUND(hi) > tol) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (BOUND(mid) > tol) lo = mid;
        else hi = mid;
    }
#undef BOUND
    return 0.5 * (lo + hi);
}

/* -------------------------------------------------------- LJ cut-off, tail */

/* Outermost r > r_min with |u_LJ(r)| = tol, by bisection (Sec. 2.6).
 * Returns -1 if tol >= eps (no root beyond the minimum). */
double oracle_lj_rcut_from_tol(double sig, double eps, double tol)
{
    if (!(tol > 0.0) || !(eps > 0.0) || !(sig > 0.0) || tol >= eps) return -1.0;
    double lo = pow(2.0, 1.0 / 6.0) * sig;  /* minimum, |u| = eps > tol */
    double hi = lo;
    while (fabs(lj_pair(sig, eps, hi)) > tol) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (fabs(lj_pair(sig, eps, mid)) > tol) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Per-pair cut-off table [ns][n]: global radius if tol <= 0, else from tol. */
int oracle_lj_rcut_table(int64_t n, const double *sig, const double *eps,
                         int32_t ns, const double *ssig, const double *seps,
                         double rcut, double tol, double *out)
{
    for (int32_t g = 0; g < ns; ++g)
        for (int64_t a = 0; a < n; ++a) {
            double s_ga, e_ga;
            lb_mix(ssig[g], seps[g], sig[a], eps[a], &s_ga, &e_ga);
            /* a pair with eps_ga = 0 has no LJ term: |u_LJ| = 0 <= tol at
             * every distance, so under a tolerance its radius is 0 (dropped) */
            double r = tol > 0.0 ? (e_ga == 0.0 ? 0.0 : oracle_lj_rcut_from_tol(s_ga, e_ga, tol))
                                 : rcut;
            if (!(r > 0.0) && !(tol > 0.0 && e_ga == 0.0)) return -1;
            out[(int64_t)g * n + a] = r;
        }
    return 0;
}

/* T_gamma = (4 pi / 3) sum_a (A/(3 r_c^9) - B/r_c^3)  (Sec. 2.6). */
int oracle_lj_tail(int64_t n, const double *sig, const double *eps, int32_t ns,
                   const double *ssig, const double *seps, const double *rcut,
                   double *tail)
{
    for (int32_t g = 0; g < ns; ++g) {
        double t = 0.0;
        for (int64_t a = 0; a < n; ++a) {
            double s_ga, e_ga;
            lb_mix(ssig[g], seps[g], sig[a], eps[a], &s_ga, &e_ga);
            double s3 = s_ga * s_ga * s_ga;
            double A = 4.0 * e_ga * s3 * s3 * s3 * s3;
            double B = 4.0 * e_ga * s3 * s3;
            double rc = rcut[(int64_t)g * n + a];
            double rc3 = rc * rc * rc;
            if (rc > 0.0) t += A / (3.0 * rc3 * rc3 * rc3) - B / rc3;
        }
        tail[g] = 4.0 * ORACLE_PI / 3.0 * t;
    }
    return 0;
}

/* -------------------------------------------------------------- backward */

/*
 * L = sum_g sum_r w[g][r] u_g(r).  For atom a (d = |r - R_a|, s = sigma_ga/d):
 *   dL/dQ_a     = k_C sum_g q_g sum_r w / d
 *   dL/dR_a     = sum_g sum_r w [k_C Q_a q_g (r - R_a)/d^3
 *                               + [d<rc] (4 eps_ga/d^2)(12 s^12 - 6 s^6)(r - R_a)]
 *   dL/deps_a   = sum_g sum_r w [d<rc] u_LJ,ga / (2 eps_a)
 *   dL/dsigma_a = sum_g sum_r w [d<rc] (2 eps_ga/sigma_ga)(12 s^12 - 6 s^6)
 * Points with d == 0 are skipped.  Any output pointer may be NULL.
 */
int oracle_backward_points(int64_t n, const double *xyz, const double *q,
                           const double *sig, const double *eps, int32_t ns,
                           const double *sq, const double *ssig, const double *seps,
                           double kc, const double *rcut, int64_t npts,
                           const double *pts, const double *w,
                           double *dxyz, double *dq, double *deps, double *dsig)
{
    if (n < 0 || ns <= 0 || npts < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < n; ++a) {
        double gx = 0, gy = 0, gz = 0, gq = 0, ge = 0, gs = 0;
        for (int32_t g = 0; g < ns; ++g) {
            double s_ga, e_ga;
            lb_mix(ssig[g], seps[g], sig[a], eps[a], &s_ga, &e_ga);
            double rc = rcut ? rcut[(int64_t)g * n + a] : INFINITY;
            for (int64_t i = 0; i < npts; ++i) {
                double wv = w[(int64_t)g * npts + i];
                double rx = pts[3 * i + 0] - xyz[3 * a + 0];
                double ry = pts[3 * i + 1] - xyz[3 * a + 1];
                double rz = pts[3 * i + 2] - xyz[3 * a + 2];
                double d2 = rx * rx + ry * ry + rz * rz;
                if (d2 == 0.0) continue;
                double d = sqrt(d2);
                double f = kc * q[a] * sq[g] / (d2 * d);
                gq += wv * kc * sq[g] / d;
                if (d < rc) {
                    double s = s_ga / d;
                    double s6 = s * s * s * s * s * s;
                    double s12 = s6 * s6;
                    f += 4.0 * e_ga / d2 * (12.0 * s12 - 6.0 * s6);
                    if (eps[a] > 0.0) ge += wv * 4.0 * e_ga * (s12 - s6) / (2.0 * eps[a]);
                    gs += wv * (2.0 * e_ga / s_ga) * (12.0 * s12 - 6.0 * s6);
                }
                gx += wv * f * rx;
                gy += wv * f * ry;
                gz += wv * f * rz;
            }
        }
        if (dxyz) { dxyz[3 * a] = gx; dxyz[3 * a + 1] = gy; dxyz[3 * a + 2] = gz; }
        if (dq) dq[a] = gq;
        if (deps) deps[a] = ge;
        if (dsig) dsig[a] = gs;
    }
    return 0;
}

int oracle_grid_points(const double *origin, const double *spacing,
                       const int32_t *dims, double *pts)
{
    int64_t m = (int64_t)dims[0] * dims[1] * dims[2];
    for (int64_t i = 0; i < m; ++i) point_of(origin, spacing, dims, i, pts + 3 * i);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later parallel sums (n <= 0: every processor). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

/* ------------------------------------------------ Taylor-recurrence treecode */

/*
 * Taylor coefficients of a radial kernel phi(|x - y|) about a target centre
 * x (Sec. 2.3.1, Eq. taylor_coefficients), times (-1)^|k|:
 *   t_k = ((-1)^|k| / k!) d^k phi/dy^k = (1/k!) d^k phi/dx^k,
 * so that phi(x', y) ~ sum_{|k| <= p} t_k (x' - x)^k.  In terms of v = y - x
 * the paper's recurrences keep their printed form (odd orders flip sign
 * together with x - y):
 *  kind 0, 1/R (Sec. 2.3.2): for |k| >= 1
 *    t_k = [(2 - 1/|k|) sum_i v_i t_{k-e_i} - (1 - 1/|k|) sum_i t_{k-2e_i}] / R^2;
 *  kind 1, erf(R/eta)/R (Sec. 2.4.1): the same plus g_k / R^2, g the
 *    coefficients of the auxiliary Gaussian, g_k = 2/(eta^2 |k|) [sum_i v_i
 *    g_{k-e_i} - sum_i g_{k-2e_i}].  Reading: g_0 = -(eta/sqrt(pi))
 *    exp(-R^2/eta^2); with the printed exp(-R^2/eta^2) alone the recurrence
 *    does not reproduce the kernel's derivatives;
 *  kind 2, 2 exp(-kappa R)/R (Sec. 2.4.2, the far-field form of the TCF
 *    kernel): the 1/R form plus (kappa/|k|) [sum_i v_i b_{k-e_i} - sum_i
 *    b_{k-2e_i}] / R^2, b the coefficients of 2 exp(-kappa R),
 *    b_k = (kappa/|k|) [sum_i v_i t_{k-e_i} - sum_i t_{k-2e_i}].  Reading:
 *    the printed factor kappa lacks the 1/|k| that the derivatives require.
 * Components with a negative index are zero.  out: cube [(p+1)^3] with
 * k = (k3 (p+1) + k2)(p+1) + k1, zero where |k| > p.
 */
static double tc_get(const double *t, int p, int k1, int k2, int k3)
{
    if (k1 < 0 || k2 < 0 || k3 < 0) return 0.0;
    return t[((int64_t)k3 * (p + 1) + k2) * (p + 1) + k1];
}

static double tc_rec(const double *t, int p, int k1, int k2, int k3, const double v[3],
                     double *second)
{
    /* sum_i v_i t_{k-e_i}, and sum_i t_{k-2e_i} into *second */
    *second = tc_get(t, p, k1 - 2, k2, k3) + tc_get(t, p, k1, k2 - 2, k3) +
              tc_get(t, p, k1, k2, k3 - 2);
    return v[0] * tc_get(t, p, k1 - 1, k2, k3) + v[1] * tc_get(t, p, k1, k2 - 1, k3) +
           v[2] * tc_get(t, p, k1, k2, k3 - 1);
}

int oracle_taylor_coeffs(int kind, const double v[3], int p, double eta, double kappa,
                         double *out)
{
    if (p < 0 || p > 40 || kind < 0 || kind > 2) return -1;
    const int n1 = p + 1;
    const int64_t m = (int64_t)n1 * n1 * n1;
    double *aux = calloc((size_t)m, sizeof(double));
    if (!aux) return -1;
    for (int64_t i = 0; i < m; ++i) out[i] = 0.0;
    const double R2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double R = sqrt(R2);
    if (kind == 0) {
        out[0] = 1.0 / R;
    } else if (kind == 1) {
        out[0] = erf(R / eta) / R;
        aux[0] = -(eta / sqrt(ORACLE_PI)) * exp(-R2 / (eta * eta));
    } else {
        out[0] = 2.0 * exp(-kappa * R) / R;
        aux[0] = 2.0 * exp(-kappa * R);
    }
    for (int d = 1; d <= p; ++d)
        for (int k3 = 0; k3 <= d; ++k3)
            for (int k2 = 0; k2 <= d - k3; ++k2) {
                const int k1 = d - k3 - k2;
                const int64_t idx = ((int64_t)k3 * n1 + k2) * n1 + k1;
                double s2;
                const double s1 = tc_rec(out, p, k1, k2, k3, v, &s2);
                double t = (2.0 - 1.0 / d) * s1 - (1.0 - 1.0 / d) * s2;
                if (kind == 1) {
                    double g2;
                    const double g1 = tc_rec(aux, p, k1, k2, k3, v, &g2);
                    aux[idx] = 2.0 / (eta * eta * d) * (g1 - g2);
                    t += aux[idx];
                } else if (kind == 2) {
                    double b2;
                    const double b1 = tc_rec(aux, p, k1, k2, k3, v, &b2);
                    t += kappa / d * (b1 - b2);
                    /* b_k from the t of lower orders (already final) */
                    aux[idx] = kappa / d * (s1 - s2);
                }
                out[idx] = t / R2;
            }
    free(aux);
    return 0;
}

/* Order-p Taylor polynomial of kernel `kind` about centre c, for the atom at
 * y, evaluated at x. */
static double taylor_eval(int kind, const double c[3], const double y[3], const double x[3],
                          int p, double eta, double kappa, double *coef)
{
    const double v[3] = {y[0] - c[0], y[1] - c[1], y[2] - c[2]};
    oracle_taylor_coeffs(kind, v, p, eta, kappa, coef);
    const int n1 = p + 1;
    double s = 0.0;
    for (int k3 = 0; k3 <= p; ++k3)
        for (int k2 = 0; k2 <= p - k3; ++k2)
            for (int k1 = 0; k1 <= p - k3 - k2; ++k1)
                s += coef[((int64_t)k3 * n1 + k2) * n1 + k1] * pow(x[0] - c[0], k1) *
                     pow(x[1] - c[1], k2) * pow(x[2] - c[2], k3);
    return s;
}

/*
 * The cluster-particle treecode of Sec. 2.3.1 with Taylor far fields, at
 * listed grid points (ijk [npts][3] grid indices), pair by pair.  Target
 * tree: cubes of B^3 grid points (level 0) merged 2 x 2 x 2 per level up to
 * the level T whose single cluster covers the grid (a cubic octree; reading
 * of the paper's splitting rule).  For a point x in level-0 block (I, J, K)
 * and an atom y, the atom belongs to the far field (a set I_l of Eq. 10) of
 * the coarsest ancestor cluster C (level >= 1) it is well separated from,
 * r_C < theta |y - c_C|, r_C the half-diagonal of C's box of grid points and
 * c_C its centre (reading of the garbled MAC); otherwise to the direct set D.
 * LJ is exact within each pair's cut-off either way.
 *
 * mode 0, the paper's far fields (oracle_taylor_cp_points):
 *   u:    order-p Taylor polynomial of 1/d about c_C (Sec. 2.3.2);
 *   c^lr: order-p Taylor polynomial of erf(d/eta)/d about c_C, coefficients
 *         from the erf recurrence with its Gaussian auxiliary (Sec. 2.4.1);
 *   h^lr: order-p Taylor polynomial of 2 exp(-kappa d)/d about c_C, the
 *         large-distance form of the TCF kernel (Sec. 2.4.2, Eq. tcfexp),
 *         with no correction for the erfc -> 2 and erfc -> 0 step.
 *   Direct set: the exact kernels 1/d, erf(d/eta)/d and the Eq. 6 bracket
 *   over d (d -> 0 limits at a coincident point).
 *   guard > 0 adds a distance condition to the MAC: |y - c_C| - r_C >= guard,
 *   so that no target of C lies closer to the atom than `guard`.  The
 *   erfc -> 2/0 replacement is off by about erfc(d/eta - kappa eta/2) at
 *   distance d; the paper relies on the MAC alone to make d large, which at
 *   large theta it does not (reading: guard = eta (6 + kappa eta/2) bounds
 *   that error by erfc(6) ~ 2e-17 at every target).  guard <= 0: MAC only.
 *
 * mode 1, the exact-split variant (oracle_taylor_split_cp_points): the far
 * fields are the Taylor polynomials of 1/d (u, and c^lr's long-range part)
 * and of 2 exp(-kappa d)/d (h^lr) only; for accepted atoms the remainders
 * erf(d/eta)/d - 1/d and the Eq. 6 bracket / d - 2 exp(-kappa d)/d are added
 * exactly where d < Rs = eta (5 + kappa eta/2), beyond which they are below
 * 1e-12 relative.  No guard.
 *
 * Outputs as oracle_potential_points and oracle_asymptotics_points:
 * u [S][npts], c [S][npts], h [n_ionic][npts]; any may be NULL.
 */
static int taylor_cp_points(int mode, int64_t n, const double *xyz, const double *q,
                            const double *sig, const double *eps, int32_t ns,
                            const double *sq, const double *ssig, const double *seps,
                            const int32_t *ionic, double kc, const double *rcut,
                            double eta, double kappa, double beta, double diel,
                            const double *origin, const double *spacing,
                            const int32_t *dims, int32_t B, double theta, int32_t p,
                            double guard, int64_t npts, const int32_t *ijk,
                            double *u, double *c, double *h)
{
    if (n < 0 || ns <= 0 || npts < 0 || B <= 0 || p < 0 || p > 40 || !(theta > 0.0))
        return -1;
    int32_t maxdim = dims[0];
    if (dims[1] > maxdim) maxdim = dims[1];
    if (dims[2] > maxdim) maxdim = dims[2];
    int T = 0;
    while (((int64_t)B << T) < maxdim) ++T;
    const double rs = eta * (5.0 + 0.5 * kappa * eta);
    const int64_t ncoef = (int64_t)(p + 1) * (p + 1) * (p + 1);
    int failed = 0;
#pragma omp parallel
    {
        double *coef = malloc((size_t)ncoef * sizeof(double));
        double *uacc = malloc((size_t)ns * sizeof(double));
        if (!coef || !uacc) failed = 1;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < npts; ++i) {
            if (!coef || !uacc) continue;
            const int32_t *g = ijk + 3 * i;
            const double x[3] = {origin[0] + g[0] * spacing[0], origin[1] + g[1] * spacing[1],
                                 origin[2] + g[2] * spacing[2]};
            /* coul: 1/d sum (u); sc, sh: the c^lr and h^lr kernel sums (mode
             * 0), or c^lr's remainders beside coul and h^lr's sum (mode 1) */
            double coul = 0.0, sc = 0.0, sh = 0.0;
            int hit = 0;
            for (int32_t s = 0; s < ns; ++s) uacc[s] = 0.0;
            for (int64_t a = 0; a < n; ++a) {
                const double *y = xyz + 3 * a;
                const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
                const double d = sqrt(dx * dx + dy * dy + dz * dz);
                /* coarsest ancestor cluster satisfying the MAC */
                int acc = 0;
                double cc[3] = {0, 0, 0};
                for (int lvl = T; lvl >= 1 && !acc; --lvl) {
                    const int64_t e = (int64_t)B << lvl;
                    double r2 = 0.0, R2 = 0.0, ctr[3];
                    for (int ax = 0; ax < 3; ++ax) {
                        const int64_t lo = (g[ax] / e) * e;
                        int64_t hi = lo + e - 1;
                        if (hi > dims[ax] - 1) hi = dims[ax] - 1;
                        const double xl = origin[ax] + lo * spacing[ax];
                        const double xh = origin[ax] + hi * spacing[ax];
                        ctr[ax] = 0.5 * (xl + xh);
                        r2 += 0.25 * (xh - xl) * (xh - xl);
                        R2 += (y[ax] - ctr[ax]) * (y[ax] - ctr[ax]);
                    }
                    if (r2 < theta * theta * R2 &&
                        (mode != 0 || guard <= 0.0 || sqrt(R2) - sqrt(r2) >= guard)) {
                        acc = 1;
                        for (int ax = 0; ax < 3; ++ax) cc[ax] = ctr[ax];
                    }
                }
                if (acc && mode == 0) {
                    coul += q[a] * taylor_eval(0, cc, y, x, p, eta, kappa, coef);
                    sc += q[a] * taylor_eval(1, cc, y, x, p, eta, kappa, coef);
                    sh += q[a] * taylor_eval(2, cc, y, x, p, eta, kappa, coef);
                } else if (acc) {
                    coul += q[a] * taylor_eval(0, cc, y, x, p, eta, kappa, coef);
                    sh += q[a] * taylor_eval(2, cc, y, x, p, eta, kappa, coef);
                    if (d < rs) {
                        sc += q[a] * (dcf_kernel(d, eta) - 1.0 / d);
                        sh += q[a] * (tcf_kernel(d, eta, kappa) - 2.0 * exp(-kappa * d) / d);
                    }
                } else if (d == 0.0) {
                    hit = 1;
                    sc += q[a] * dcf_kernel(d, eta);
                    sh += q[a] * tcf_kernel(d, eta, kappa);
                } else {
                    coul += q[a] / d;
                    sc += q[a] * (mode == 0 ? dcf_kernel(d, eta) : dcf_kernel(d, eta) - 1.0 / d);
                    sh += q[a] * tcf_kernel(d, eta, kappa);
                }
                if (d > 0.0)
                    for (int32_t s = 0; s < ns; ++s) {
                        double s_ga, e_ga;
                        lb_mix(ssig[s], seps[s], sig[a], eps[a], &s_ga, &e_ga);
                        if (rcut == NULL || d < rcut[(int64_t)s * n + a])
                            uacc[s] += lj_pair(s_ga, e_ga, d);
                    }
            }
            const double csum = mode == 0 ? sc : coul + sc;
            int32_t j = 0;
            for (int32_t s = 0; s < ns; ++s) {
                if (u) u[(int64_t)s * npts + i] = hit ? INFINITY : kc * sq[s] * coul + uacc[s];
                if (c) c[(int64_t)s * npts + i] = -beta * kc * sq[s] * csum;
                if (ionic[s]) {
                    if (h)
                        h[(int64_t)j * npts + i] = -beta * kc * sq[s] / (2.0 * diel) *
                                                   exp(kappa * kappa * eta * eta / 4.0) * sh;
                    ++j;
                }
            }
        }
        free(coef);
        free(uacc);
    }
    return failed ? -1 : 0;
}

int oracle_taylor_cp_points(int64_t n, const double *xyz, const double *q,
                            const double *sig, const double *eps, int32_t ns,
                            const double *sq, const double *ssig, const double *seps,
                            const int32_t *ionic, double kc, const double *rcut,
                            double eta, double kappa, double beta, double diel,
                            const double *origin, const double *spacing,
                            const int32_t *dims, int32_t B, double theta, int32_t p,
                            double guard, int64_t npts, const int32_t *ijk,
                            double *u, double *c, double *h)
{
    return taylor_cp_points(0, n, xyz, q, sig, eps, ns, sq, ssig, seps, ionic, kc, rcut, eta,
                            kappa, beta, diel, origin, spacing, dims, B, theta, p, guard, npts,
                            ijk, u, c, h);
}

int oracle_taylor_split_cp_points(int64_t n, const double *xyz, const double *q,
                                  const double *sig, const double *eps, int32_t ns,
                                  const double *sq, const double *ssig, const double *seps,
                                  const int32_t *ionic, double kc, const double *rcut,
                                  double eta, double kappa, double beta, double diel,
                                  const double *origin, const double *spacing,
                                  const int32_t *dims, int32_t B, double theta, int32_t p,
                                  int64_t npts, const int32_t *ijk,
                                  double *u, double *c, double *h)
{
    return taylor_cp_points(1, n, xyz, q, sig, eps, ns, sq, ssig, seps, ionic, kc, rcut, eta,
                            kappa, beta, diel, origin, spacing, dims, B, theta, p, 0.0, npts,
                            ijk, u, c, h);
}
