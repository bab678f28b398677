"""Pins of the oracle's Taylor-recurrence treecode (Secs. 2.3 and 2.4).

The recurrences are checked against 30-digit derivatives that mpmath takes
of the kernels themselves, so a wrong constant, sign or index in a
recurrence (or a printed form taken literally) fails; the treecode is
checked against the oracle's direct sums where it must reduce to them and
for the geometric decay of its error with the order p."""
import itertools
import math

import mpmath as mp
import numpy as np
import pytest

from paper_2109_09772_amd import workloads as W

KC = W.COULOMB_K
BETA = W.beta()
ETA = 1.0
KAPPA = W.debye_kappa()
DIEL = W.DIELECTRIC


def _mp_coeffs(kind, v, p, eta, kappa):
    """(1/k!) d^k/dx^k phi(|x - y|) at x = 0, y = v, by mpmath differentiation."""
    mp.mp.dps = 30
    y = [mp.mpf(c) for c in v]
    f = {"coulomb": lambda r: 1 / r,
         "dcf": lambda r: mp.erf(r / eta) / r,
         "screened": lambda r: 2 * mp.exp(-kappa * r) / r}[kind]
    out = {}
    for k in itertools.product(range(p + 1), repeat=3):
        if sum(k) > p:
            continue
        g = lambda a, b, c: f(mp.sqrt((a - y[0]) ** 2 + (b - y[1]) ** 2 + (c - y[2]) ** 2))
        d = mp.diff(g, (0, 0, 0), k)
        out[k] = float(d / (math.factorial(k[0]) * math.factorial(k[1]) * math.factorial(k[2])))
    return out


@pytest.mark.parametrize("kind", ["coulomb", "dcf", "screened"])
@pytest.mark.parametrize("v", [(1.3, -0.4, 2.2), (-3.1, 0.2, 0.9)])
def test_taylor_coefficients_match_kernel_derivatives(oracle, kind, v):
    """Sec. 2.3.2 (1/R), Sec. 2.4.1 (erf(R/eta)/R with the Gaussian
    auxiliary term -(eta/sqrt(pi)) exp(-R^2/eta^2)) and Sec. 2.4.2
    (2 exp(-kappa R)/R with the kappa/|k| term): every coefficient up to
    order 6 equals the mpmath derivative of the kernel."""
    p, eta, kappa = 6, 1.1, 0.37
    t = oracle.taylor_coeffs(kind, v, p, eta, kappa)
    ref = _mp_coeffs(kind, v, p, eta, kappa)
    scale = max(abs(x) for x in ref.values())
    for (k1, k2, k3), r in ref.items():
        assert abs(t[k3, k2, k1] - r) <= 1e-12 * scale + 1e-11 * abs(r), (k1, k2, k3)
    # entries beyond order p stay zero
    for k1, k2, k3 in itertools.product(range(p + 1), repeat=3):
        if k1 + k2 + k3 > p:
            assert t[k3, k2, k1] == 0.0


@pytest.mark.parametrize("kind", ["coulomb", "dcf", "screened"])
def test_taylor_series_converges_to_kernel(oracle, kind):
    """The order-p polynomial about x reproduces phi at x' with an error that
    falls geometrically in p (|x' - x| / |y - x| = 0.3 here)."""
    eta, kappa = 1.0, 0.2
    y = np.array([4.0, -2.0, 3.0])
    rho = np.linalg.norm(y)
    dx = 0.3 * rho * np.array([0.48, 0.6, -0.64])
    r = np.linalg.norm(y - dx)
    exact = {"coulomb": 1 / r, "dcf": math.erf(r / eta) / r,
             "screened": 2 * math.exp(-kappa * r) / r}[kind]
    errs = []
    for p in (2, 4, 8, 14):
        t = oracle.taylor_coeffs(kind, y, p, eta, kappa)
        s = 0.0
        for k1, k2, k3 in itertools.product(range(p + 1), repeat=3):
            if k1 + k2 + k3 <= p:
                s += t[k3, k2, k1] * dx[0] ** k1 * dx[1] ** k2 * dx[2] ** k3
        errs.append(abs(s - exact) / abs(exact))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-7
    assert errs[0] > 1e-4


def _case(seed=5, n=24, dims=(20, 18, 16), spacing=0.5):
    wl = W.tiny(n_atoms=n, dims=dims, seed=seed, spacing=spacing)
    wl.solute.xyz *= 1.6
    return wl


def _direct(oracle, wl, ijk, rc):
    sol, st, g = wl.solute, wl.sites, wl.grid
    pts = g.origin + np.asarray(ijk) * g.spacing
    u = oracle.potential_points(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma, st.eps,
                                pts, KC, rc)
    c, h = oracle.asymptotics_points(sol.xyz, sol.q, st.q, st.ionic, pts, KC, ETA, KAPPA,
                                     BETA, DIEL)
    return u, c, h


def _taylor(oracle, wl, ijk, rc, theta, p, batch=4, variant="paper", guard=None):
    sol, st, g = wl.solute, wl.sites, wl.grid
    args = (sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma, st.eps, st.ionic, g.origin,
            g.spacing, g.dims, ijk, KC, ETA, KAPPA, BETA, DIEL, batch, theta, p, rc)
    if variant == "paper":
        return oracle.taylor_cp_points(*args, guard=guard)
    return oracle.taylor_split_cp_points(*args)


def _ijk(g, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, int(d), n) for d in g.dims], axis=1)


@pytest.mark.parametrize("variant", ["paper", "split"])
def test_taylor_treecode_without_far_field_is_the_direct_sum(oracle, variant):
    """With a MAC no cluster satisfies, every atom is summed directly and the
    treecode returns the direct sums (u, c^lr, h^lr) to rounding."""
    wl = _case()
    ijk = _ijk(wl.grid, 60, 1)
    rc = oracle.rcut_table(wl.solute.sigma, wl.solute.eps, wl.sites.sigma, wl.sites.eps, 6.0)
    ref = _direct(oracle, wl, ijk, rc)
    got = _taylor(oracle, wl, ijk, rc, theta=1e-6, p=3, variant=variant)
    for x, r in zip(got, ref):
        np.testing.assert_allclose(x, r, rtol=1e-12, atol=1e-12 * np.abs(r).max())


@pytest.mark.parametrize("variant", ["paper", "split"])
def test_taylor_treecode_error_falls_with_order(oracle, variant):
    """At theta 0.5 the treecode error against the direct sums falls
    geometrically with the Taylor order (Sec. 3, Fig. 6's behaviour at grid
    level), for u, c^lr and h^lr alike: in the paper's form each output is
    the expansion of its own kernel (1/d, erf(d/eta)/d, 2 exp(-kappa d)/d),
    so each converges to its exact direct sum."""
    wl = _case(seed=8, n=30, dims=(24, 22, 20), spacing=0.5)
    ijk = _ijk(wl.grid, 80, 2)
    rc = oracle.rcut_table(wl.solute.sigma, wl.solute.eps, wl.sites.sigma, wl.sites.eps, 6.0)
    ref = _direct(oracle, wl, ijk, rc)
    prev = None
    for p in (1, 3, 5, 7, 9):
        got = _taylor(oracle, wl, ijk, rc, theta=0.5, p=p, variant=variant)
        errs = [np.linalg.norm(x - r) / np.linalg.norm(r) for x, r in zip(got, ref)]
        print(p, errs)
        if prev is not None:
            assert all(e < 0.5 * pe for e, pe in zip(errs, prev))
        prev = errs
    assert max(prev) < 1e-5


def test_taylor_forms_agree_beyond_the_smearing(oracle):
    """Where every accepted atom lies beyond Rs of its cluster's targets, the
    smeared kernels equal their far-field forms to < 1e-16 relative (erf ->
    1, erfc -> 2 and 0), and so do their Taylor coefficients (the Gaussian
    auxiliary of Sec. 2.4.1 is ~exp(-R^2/eta^2)): the paper's form
    (expansions of erf(d/eta)/d and 2 exp(-kappa d)/d) and the split form
    (expansions of 1/d and 2 exp(-kappa d)/d plus exact remainders, none
    reached) give u, c^lr and h^lr equal to rounding.  On this grid the
    smallest (clipped) cluster has a half-diagonal of 2.28 A, so at theta
    0.25 every accepted atom is >= 6.8 A > Rs from every target."""
    wl = _case(seed=8, n=30, dims=(24, 22, 20), spacing=0.5)
    ijk = _ijk(wl.grid, 80, 3)
    rc = oracle.rcut_table(wl.solute.sigma, wl.solute.eps, wl.sites.sigma, wl.sites.eps, 6.0)
    for p in (2, 6):
        a = _taylor(oracle, wl, ijk, rc, theta=0.25, p=p, variant="paper", guard=0.0)
        b = _taylor(oracle, wl, ijk, rc, theta=0.25, p=p, variant="split")
        for x, y in zip(a, b):
            np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-13 * np.abs(y).max())


def test_taylor_guard_bounds_the_tcf_far_field(oracle):
    """Sec. 2.4.2 replaces the TCF kernel by 2 exp(-kappa d)/d wherever an
    atom is well separated; at theta 0.9 the MAC alone accepts atoms a few
    tenths of an angstrom from a cluster's points, where that replacement is
    far off.  With the distance guard the h^lr error falls with the order to
    the level of u's and c^lr's, without it it stalls at the replacement's
    error."""
    wl = _case(seed=8, n=30, dims=(24, 22, 20), spacing=0.5)
    ijk = _ijk(wl.grid, 120, 4)
    rc = oracle.rcut_table(wl.solute.sigma, wl.solute.eps, wl.sites.sigma, wl.sites.eps, 6.0)
    ref = _direct(oracle, wl, ijk, rc)
    rel = lambda x, r: np.linalg.norm(x - r) / np.linalg.norm(r)
    e_no = [rel(_taylor(oracle, wl, ijk, rc, 0.9, p, guard=0.0)[2], ref[2]) for p in (6, 10)]
    e_g = [rel(_taylor(oracle, wl, ijk, rc, 0.9, p)[2], ref[2]) for p in (6, 10)]
    print("no guard", e_no, "guard", e_g)
    assert e_no[1] > 1e-3                   # stalls at the replacement's error
    assert e_g[1] < 0.5 * e_g[0]            # falls with p
    assert e_no[1] > 1e3 * e_g[1]
