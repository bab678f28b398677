"""GPU parity of the direct paths (FP64 reference and FP32 compensated)
against the FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from helpers import BETA, DIEL, ETA, FP32_CAP, KAPPA, KC, assert_close_grid, oracle_rcut, rel_l2
from paper_2109_09772_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"direct_f64": 1e-12, "direct_f32c": 1e-6}


def _api():
    from paper_2109_09772_amd import api
    return api


def _run(wl, method, lj_cutoff=0.0, lj_tol=0.0, out_dtype=None, want=("u", "c", "h"),
         kappa=KAPPA):
    api = _api()
    xyz, q, s, e = api.solute_to_device(wl.solute)
    sites = api.sites_from(wl.sites)
    grid = api.grid_from(wl.grid)
    od = out_dtype or ("f64" if method == "direct_f64" else "f32")
    opts = api.Opts(method=method, out_dtype=od, lj_cutoff=lj_cutoff, lj_tol=lj_tol)
    u, c, h, tail = api.initialize(xyz, q, s, e, sites, grid, opts, ETA, kappa, BETA, DIEL,
                                   want_u="u" in want, want_c="c" in want, want_h="h" in want,
                                   want_tail=True)
    torch.cuda.synchronize()
    f = lambda t: None if t is None else t.double().cpu().numpy()
    return f(u), f(c), f(h), tail


def _oracle_grids(oracle, wl, lj_cutoff=0.0, lj_tol=0.0, kappa=KAPPA):
    sol, st, g = wl.solute, wl.sites, wl.grid
    rc = oracle_rcut(oracle, wl, lj_cutoff, lj_tol)
    u = oracle.potential_grid(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma, st.eps,
                              g.origin, g.spacing, g.dims, KC, rc)
    c, h = oracle.asymptotics_grid(sol.xyz, sol.q, st.q, st.ionic, g.origin, g.spacing, g.dims,
                                   KC, ETA, kappa, BETA, DIEL)
    tail = (oracle.lj_tail(sol.sigma, sol.eps, st.sigma, st.eps, rc) if rc is not None
            else np.zeros(st.n))
    return u, c, (h if st.ionic.sum() else None), tail


def _check(got, ref, method, what):
    f32 = method != "direct_f64"
    tol = TOL[method]
    assert_close_grid(got, ref, tol, cap=FP32_CAP if f32 else 0.0, what=f"{method}:{what}")


@pytest.mark.parametrize("method", ["direct_f64", "direct_f32c"])
def test_small_ball_full_grid(oracle, method):
    """200 atoms in a 20 A ball, 64^3 grid, water sites, no cut-off."""
    wl = W.small_ball()
    u, c, h, _ = _run(wl, method)
    ur, cr, hr, _ = _oracle_grids(oracle, wl)
    assert h is None and hr is None
    _check(u, ur, method, "u")
    _check(c, cr, method, "c")


@pytest.mark.parametrize("method", ["direct_f64", "direct_f32c"])
@pytest.mark.parametrize("cut", [(0.0, 0.0), (9.0, 0.0), (0.0, 1e-4)])
def test_ragged_salt_grid(oracle, method, cut):
    """Ragged 37x29x23 grid (not a multiple of the 16x4x4 brick), non-dyadic
    spacing 0.3 A (FP32 grid coordinates not exact), 4 sites with 2 ionic,
    and the three LJ modes (none, 9 A, per-pair tolerance)."""
    wl = W.tiny(n_atoms=60, dims=(37, 29, 23), seed=7, spacing=0.3)
    wl.solute.xyz *= 1.6
    u, c, h, tail = _run(wl, method, *cut)
    ur, cr, hr, tr = _oracle_grids(oracle, wl, *cut)
    _check(u, ur, method, "u")
    _check(c, cr, method, "c")
    _check(h, hr, method, "h")
    np.testing.assert_allclose(tail, tr, rtol=1e-12)


@pytest.mark.parametrize("method", ["direct_f64", "direct_f32c"])
def test_zero_epsilon_atom_under_tolerance(oracle, method):
    """An atom with eps = 0 (no LJ term with any site) under a tolerance
    cut-off: its pairs are dropped (radius 0) instead of failing the call,
    and the tail constants match the oracle's."""
    wl = W.tiny(n_atoms=40, dims=(23, 19, 17), seed=4, spacing=0.5)
    wl.solute.xyz *= 1.5
    wl.solute.eps[[3, 17]] = 0.0
    u, c, h, tail = _run(wl, method, 0.0, 1e-4)
    ur, cr, hr, tr = _oracle_grids(oracle, wl, 0.0, 1e-4)
    _check(u, ur, method, "u")
    _check(c, cr, method, "c")
    np.testing.assert_allclose(tail, tr, rtol=1e-12)


@pytest.mark.parametrize("method", ["direct_f64", "direct_f32c"])
@pytest.mark.parametrize("cut", [0.0, 9.0])
def test_interior_subgrid_every_point(oracle, method, cut):
    """A 64^3 grid at 0.5 A centred inside the 2,500-atom solute: every point
    lies in or next to the atom cloud, so u is set by the LJ cores of the
    nearest atoms, the hardest case for FP32 pair rounding.  Every point of
    u, c and h against the oracle (no sampling)."""
    base = W.protein_2500()
    wl = W.Workload("ellipsoid2500_grid64", base.solute, base.sites,
                    W.centred_grid([0.0, 0.0, 0.0], 0.5, 64), base.seed)
    u, c, h, tail = _run(wl, method, cut)
    ur, cr, hr, tr = _oracle_grids(oracle, wl, cut)
    for k in range(u.shape[0]):
        print(f"{method} cut={cut} u[{k}] rel-L2 {rel_l2(u[k], ur[k], FP32_CAP)[0]:.3e}")
    _check(u, ur, method, "u")
    _check(c, cr, method, "c")
    _check(h, hr, method, "h")
    np.testing.assert_allclose(tail, tr, rtol=1e-12)


@pytest.mark.parametrize("nsites", [1, 3, 5, 8])
def test_site_counts(oracle, nsites):
    names = (list(W.SITES_SALT) * 2)[:nsites]
    wl = W.tiny(n_atoms=20, dims=(18, 9, 13), seed=3)
    wl.sites = W.make_sites(names)
    for method in ("direct_f64", "direct_f32c"):
        u, c, h, _ = _run(wl, method, 7.0)
        ur, cr, hr, _ = _oracle_grids(oracle, wl, 7.0)
        _check(u, ur, method, "u")
        _check(c, cr, method, "c")
        if hr is not None:
            _check(h, hr, method, "h")


@pytest.mark.parametrize("method", ["direct_f64", "direct_f32c"])
def test_point_on_atom_and_kappa_zero(oracle, method):
    """An atom exactly on a grid point: u = +inf there, c and h take their
    d -> 0 limits; kappa = 0 exercises the unscreened limit."""
    wl = W.tiny(n_atoms=8, dims=(12, 10, 9), seed=5, spacing=0.5)
    g = wl.grid
    wl.solute.xyz[3] = g.origin + g.spacing * np.array([5, 4, 3])
    for kappa in (KAPPA, 0.0):
        u, c, h, _ = _run(wl, method, kappa=kappa)
        ur, cr, hr, _ = _oracle_grids(oracle, wl, kappa=kappa)
        assert np.isposinf(u[:, 3, 4, 5]).all()
        _check(u, ur, method, "u")
        _check(c, cr, method, "c")
        _check(h, hr, method, "h")


@pytest.mark.parametrize("method", ["direct_f64", "direct_f32c", "treecode", "treecode_cp",
                                    "treecode_taylor"])
def test_no_atoms_gives_zero(method):
    api = _api()
    wl = W.tiny(n_atoms=3, dims=(5, 6, 7))
    sites, grid = api.sites_from(wl.sites), api.grid_from(wl.grid)
    z = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    z1 = torch.zeros(0, dtype=torch.float64, device="cuda")
    opts = api.Opts(method=method, lj_cutoff=9.0)
    u, c, h, tail = api.initialize(z, z1, z1, z1, sites, grid, opts, ETA, KAPPA, BETA, DIEL,
                                   want_tail=True)
    torch.cuda.synchronize()
    assert float(u.abs().max()) == 0 and float(c.abs().max()) == 0 and float(h.abs().max()) == 0
    assert (tail == 0).all()


def _gpu_full(wl, method, cut):
    """Device-resident outputs (u, c, h) of one initialisation."""
    api = _api()
    xyz, q, s, e = api.solute_to_device(wl.solute)
    od = "f64" if method == "direct_f64" else "f32"
    opts = api.Opts(method=method, out_dtype=od, lj_cutoff=cut)
    return api.initialize(xyz, q, s, e, api.sites_from(wl.sites), api.grid_from(wl.grid), opts,
                          ETA, KAPPA, BETA, DIEL)


# FP32 far-field floor: away from the atoms a neutral solute's Coulomb sum
# cancels by ~1e3, so the random per-pair FP32 rounding (~1e-7 per term, five
# comparable sources) leaves ~1e-6 relative error there.  The gate of the
# method is the full-grid rel-L2 (1e-6); the far-field sample is held to this.
FAR_FIELD_F32 = 3e-6


@pytest.mark.parametrize("cut", [0.0, 9.0])
def test_protein_2500(oracle, cut):
    """2,500 atoms, 128^3 grid, 4 sites (the benchmark workload).
    1. FP64 direct vs the oracle on 8,192 sampled points: <= 1e-12.
    2. FP32 direct vs the FP64 direct on the full grid (rism_compare): <= 1e-6.
    3. FP32 direct vs the oracle on the samples (far-field diagnostic)."""
    api = _api()
    wl = W.protein_2500()
    idx = W.sample_points(wl.grid, 8192, seed=99)
    sol, st, g = wl.solute, wl.sites, wl.grid
    pts = g.origin + idx * g.spacing
    rc = oracle_rcut(oracle, wl, cut)
    ur = oracle.potential_points(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma, st.eps,
                                 pts, KC, rc)
    cr, hr = oracle.asymptotics_points(sol.xyz, sol.q, st.q, st.ionic, pts, KC, ETA, KAPPA,
                                       BETA, DIEL)
    ref = _gpu_full(wl, "direct_f64", cut)
    got = _gpu_full(wl, "direct_f32c", cut)
    torch.cuda.synchronize()
    ii = torch.as_tensor(idx, device="cuda")
    pick = lambda a: a[:, ii[:, 2], ii[:, 1], ii[:, 0]].double().cpu().numpy()
    for name, r64, x32, orc in zip("uch", ref, got, (ur, cr, hr)):
        assert_close_grid(pick(r64), orc, 1e-12, what=f"f64:{name}")
        for k in range(x32.shape[0]):
            se, sr, mx, excl, mism, _ = api.compare(x32[k], r64[k], ref_cap=FP32_CAP)
            assert mism == 0
            err = (se / sr) ** 0.5
            print(f"cut={cut} {name}[{k}] full-grid rel-L2 {err:.2e} (excluded {int(excl)})")
            assert err <= 1e-6, (name, k, err)
        assert_close_grid(pick(x32), orc, FAR_FIELD_F32, cap=FP32_CAP, what=f"f32 sample:{name}")


def test_f64_output_of_f32_path(oracle):
    """out_dtype only changes the storage type of the FP32 path's results."""
    wl = W.tiny(n_atoms=30, dims=(20, 21, 22), seed=2)
    a = _run(wl, "direct_f32c", 9.0, out_dtype="f64")
    b = _run(wl, "direct_f32c", 9.0, out_dtype="f32")
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_allclose(x.astype(np.float32), y, rtol=0, atol=0)
