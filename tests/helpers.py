"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

from paper_2109_09772_amd import workloads as W

KC = W.COULOMB_K
BETA = W.beta()
KAPPA = W.debye_kappa()
ETA = W.ETA
DIEL = W.DIELECTRIC
FP32_CAP = 1e30   # FP32 LJ overflows near atoms; such points are compared by kind only


def rel_l2(x, ref, cap=0.0):
    """Relative L2 error over points where both sides are finite (and the
    reference is below ``cap``); returns (err, n_excluded, n_kind_mismatch)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    okx = np.isfinite(x) & ((cap <= 0) | (np.abs(x) <= cap))
    okr = np.isfinite(ref) & ((cap <= 0) | (np.abs(ref) <= cap))
    ok = okx & okr
    den = np.sqrt((ref[ok] ** 2).sum())
    num = np.sqrt(((x[ok] - ref[ok]) ** 2).sum())
    err = num / den if den > 0 else num
    return err, int((~ok).sum()), int((okx != okr).sum())


def assert_close_grid(x, ref, tol, cap=0.0, what=""):
    x = np.asarray(x)
    ref = np.asarray(ref)
    assert x.shape == ref.shape, (what, x.shape, ref.shape)
    for s in range(x.shape[0]):
        err, excl, mism = rel_l2(x[s], ref[s], cap)
        assert mism == 0, f"{what}[{s}]: {mism} points differ in kind (finite vs inf/over cap)"
        if cap <= 0:
            # infinities must sit at the same places with the same sign
            np.testing.assert_array_equal(np.isposinf(x[s]), np.isposinf(ref[s]))
        assert err <= tol, f"{what}[{s}]: rel-L2 {err:.3e} > {tol:.1e} (excluded {excl})"


def oracle_rcut(oracle, wl, lj_cutoff=0.0, lj_tol=0.0):
    if lj_cutoff <= 0 and lj_tol <= 0:
        return None
    return oracle.rcut_table(wl.solute.sigma, wl.solute.eps, wl.sites.sigma, wl.sites.eps,
                             rcut=lj_cutoff, tol=lj_tol)
