"""The C ABI entry by entry: rism_potential (u and the tail constants) and
rism_asymptotics (c^lr, h^lr, either or both) called on their own for every
method against the oracle on a ragged grid, and the error report
(rism_compare, rism_near_mask) against numpy reductions of the same arrays."""
import numpy as np
import pytest
import torch

from helpers import BETA, DIEL, ETA, FP32_CAP, KAPPA, KC, assert_close_grid, oracle_rcut
from paper_2109_09772_amd import workloads as W

pytestmark = pytest.mark.gpu

METHODS = ["direct_f64", "direct_f32c", "treecode", "treecode_cp", "treecode_taylor"]
# (theta, degree) at which each treecode meets 1e-6 on this grid
PARAMS = {"treecode": (0.7, 8), "treecode_cp": (0.6, 10), "treecode_taylor": (0.3, 10)}


def _api():
    from paper_2109_09772_amd import api
    return api


def _ragged():
    wl = W.tiny(n_atoms=60, dims=(37, 29, 23), seed=7, spacing=0.3)
    wl.solute.xyz *= 1.6
    return wl


def _opts(method, cut=9.0, tol=0.0):
    api = _api()
    th, dg = PARAMS.get(method, (0.6, 8))
    return api.Opts(method=method, out_dtype="f64" if method == "direct_f64" else "f32",
                    lj_cutoff=cut, lj_tol=tol, theta=th, degree=dg, leaf_size=16)


def _tol(method):
    return 1e-12 if method == "direct_f64" else 1e-6


def _np(t):
    return None if t is None else t.double().cpu().numpy()


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("cut", [(9.0, 0.0), (0.0, 1e-4), (0.0, 0.0)])
def test_potential_alone(oracle, method, cut):
    """rism_potential: u for every site and the tail constants T_g, against
    the oracle's u (same cut-off rule) and its closed-form tail."""
    api = _api()
    wl = _ragged()
    sol, st, g = wl.solute, wl.sites, wl.grid
    xyz, q, s, e = api.solute_to_device(sol)
    if method.startswith("treecode") and cut == (0.0, 0.0):
        # the treecodes find the LJ pairs through the cut-off's neighbour lists
        with pytest.raises(api.RismError) as ei:
            api.potential(xyz, q, s, e, api.sites_from(st), api.grid_from(g), _opts(method, *cut))
        assert ei.value.code == api.RISM_E_UNSUPPORTED
        return
    u, tail = api.potential(xyz, q, s, e, api.sites_from(st), api.grid_from(g),
                            _opts(method, *cut), want_tail=True)
    torch.cuda.synchronize()
    rc = oracle_rcut(oracle, wl, *cut)
    ur = oracle.potential_grid(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma, st.eps,
                               g.origin, g.spacing, g.dims, KC, rc)
    tr = (oracle.lj_tail(sol.sigma, sol.eps, st.sigma, st.eps, rc) if rc is not None
          else np.zeros(st.n))
    f32 = method != "direct_f64"
    assert_close_grid(_np(u), ur, _tol(method), cap=FP32_CAP if f32 else 0.0, what=f"{method} u")
    np.testing.assert_allclose(tail, tr, rtol=1e-12)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("want", ["ch", "c", "h"])
def test_asymptotics_alone(oracle, method, want):
    """rism_asymptotics: c^lr for every site and h^lr for the ionic sites,
    together or one at a time, against the oracle's Eqs. 4 and 6."""
    api = _api()
    wl = _ragged()
    sol, st, g = wl.solute, wl.sites, wl.grid
    xyz, q, s, e = api.solute_to_device(sol)
    c, h = api.asymptotics(xyz, q, api.sites_from(st), api.grid_from(g), _opts(method), ETA,
                           KAPPA, BETA, DIEL, want_c="c" in want, want_h="h" in want, sigma=s,
                           eps=e)
    torch.cuda.synchronize()
    cr, hr = oracle.asymptotics_grid(sol.xyz, sol.q, st.q, st.ionic, g.origin, g.spacing, g.dims,
                                     KC, ETA, KAPPA, BETA, DIEL)
    f32 = method != "direct_f64"
    cap = FP32_CAP if f32 else 0.0
    if "c" in want:
        assert_close_grid(_np(c), cr, _tol(method), cap=cap, what=f"{method} c")
    else:
        assert c is None
    if "h" in want:
        assert_close_grid(_np(h), hr, _tol(method), cap=cap, what=f"{method} h")
    else:
        assert h is None


def _np_report(x, ref, cap, mask=None):
    x = np.asarray(x, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    keep = np.ones(x.shape, bool) if mask is None else mask.ravel() != 0
    okx = np.isfinite(x) & ((cap <= 0) | (np.abs(x) <= cap))
    okr = np.isfinite(ref) & ((cap <= 0) | (np.abs(ref) <= cap))
    ok = keep & okx & okr
    d = x[ok] - ref[ok]
    return ((d * d).sum(), (ref[ok] ** 2).sum(), np.abs(d).max() if ok.any() else 0.0,
            int((keep & ~ok).sum()), int((keep & (okx != okr)).sum()), int(ok.sum()))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("cap", [0.0, 1e3])
@pytest.mark.parametrize("masked", [False, True])
def test_compare_matches_numpy(dtype, cap, masked):
    """rism_compare against the same reduction in numpy, on arrays holding
    +inf, -inf and NaN on either side, values over the cap on either side,
    both at once, and (masked) a random byte mask."""
    api = _api()
    rng = np.random.default_rng(3)
    n = 1_000_003   # not a multiple of the launch width
    ref = rng.normal(size=n) * 100.0
    x = ref + rng.normal(size=n) * 1e-3
    for arr, k0 in ((x, 0), (ref, 5)):
        idx = rng.choice(n, 40, replace=False)
        arr[idx[:10]] = np.inf
        arr[idx[10:20]] = -np.inf
        arr[idx[20:30]] = np.nan
        arr[idx[30:40]] = 5e3 * (1 + k0)
    both = rng.choice(n, 7, replace=False)
    x[both] = np.nan
    ref[both] = np.inf
    mask = (rng.random(n) < 0.7).astype(np.uint8) if masked else None
    xt = torch.as_tensor(x, dtype=dtype, device="cuda")
    rt = torch.as_tensor(ref, dtype=torch.float64, device="cuda")
    mt = None if mask is None else torch.as_tensor(mask, device="cuda")
    got = api.compare(xt, rt, ref_cap=cap, mask=mt)
    exp = _np_report(xt.double().cpu().numpy(), ref, cap, mask)
    print(got, exp)
    assert got[0] == pytest.approx(exp[0], rel=1e-11)
    assert got[1] == pytest.approx(exp[1], rel=1e-12)
    assert got[2] == exp[2]
    assert (got[3], got[4], got[5]) == exp[3:]


@pytest.mark.parametrize("radius", [1.0, 2.3])
def test_near_mask_matches_numpy(radius):
    """rism_near_mask: 1 exactly where the nearest atom is at least `radius`
    away, on a ragged grid with atoms inside, near the faces and outside."""
    api = _api()
    wl = W.tiny(n_atoms=50, dims=(31, 26, 19), seed=13, spacing=0.45)
    wl.solute.xyz *= 2.4
    g = wl.grid
    xyz = torch.as_tensor(wl.solute.xyz, dtype=torch.float64, device="cuda")
    m = api.near_mask(xyz, api.grid_from(g), radius).cpu().numpy()
    nx, ny, nz = (int(v) for v in g.dims)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([i, j, k], axis=-1) * g.spacing + g.origin
    dmin = np.full(pts.shape[:3], np.inf)
    for y in wl.solute.xyz:
        dmin = np.minimum(dmin, np.sqrt(((pts - y) ** 2).sum(-1)))
    exp = (dmin >= radius).astype(np.uint8)
    assert 0 < exp.sum() < exp.size
    np.testing.assert_array_equal(m, exp)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("bad", ["nan_xyz", "inf_q", "neg_eps"])
def test_invalid_atom_input_is_reported(method, bad):
    """A non-finite coordinate or charge, or a negative eps, is caught by the
    device-side input check: RISM_E_INVALID from every method (the
    cluster-particle treecodes read the check with their end-of-call read-back),
    and a later valid call on the same stream works."""
    api = _api()
    wl = _ragged()
    sol, st, g = wl.solute, wl.sites, wl.grid
    sites, grid = api.sites_from(st), api.grid_from(g)
    xyz, q, s, e = api.solute_to_device(sol)
    if bad == "nan_xyz":
        xyz[7, 1] = float("nan")
    elif bad == "inf_q":
        q[3] = float("inf")
    else:
        e[11] = -0.01
    with pytest.raises(api.RismError) as ei:
        api.initialize(xyz, q, s, e, sites, grid, _opts(method), ETA, KAPPA, BETA, DIEL)
    assert ei.value.code == api.RISM_E_INVALID
    xyz, q, s, e = api.solute_to_device(sol)
    u, c, h = api.initialize(xyz, q, s, e, sites, grid, _opts(method), ETA, KAPPA, BETA, DIEL)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(c).all()) and bool(torch.isfinite(h).all())


@pytest.mark.parametrize("method", ["direct_f32c", "treecode_cp"])
def test_invalid_atom_in_a_later_staging_workgroup(method):
    """700 atoms span three staging workgroups, each writing its own check
    words: a NaN charge on atom 650 (the third workgroup) is reported by the
    synchronous check (direct) and by the deferred one read with the
    cluster-particle pass's flags, and a valid call after it on the same
    stream (whose words replace the old ones) passes."""
    api = _api()
    wl = W.tiny(n_atoms=5, dims=(40, 36, 32), seed=13, spacing=0.5)
    wl.solute = W.ball_solute(700, 12.0, 13)
    wl.solute.xyz += wl.grid.origin + 0.5 * wl.grid.spacing * (np.asarray(wl.grid.dims) - 1)
    sol, st, g = wl.solute, wl.sites, wl.grid
    sites, grid = api.sites_from(st), api.grid_from(g)
    xyz, q, s, e = api.solute_to_device(sol)
    q[650] = float("nan")
    with pytest.raises(api.RismError) as ei:
        api.initialize(xyz, q, s, e, sites, grid, _opts(method), ETA, KAPPA, BETA, DIEL)
    assert ei.value.code == api.RISM_E_INVALID
    xyz, q, s, e = api.solute_to_device(sol)
    u, c, h = api.initialize(xyz, q, s, e, sites, grid, _opts(method), ETA, KAPPA, BETA, DIEL)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(c).all()) and bool(torch.isfinite(h).all())
