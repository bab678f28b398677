"""GPU parity at the two largest workloads.

* 14,000 atoms in a 45x45x80 A ellipsoid on a 256^3 grid: the GPU FP64
  direct sum against the oracle on sampled points (<= 1e-12), and the
  cluster-particle treecode (theta 0.6, degree 8, 9 A LJ cut-off) against the
  GPU FP64 direct sum on the full grid (<= 1e-6 per output grid).
* 1.2 M atoms in a hollow cylinder, one 512x512x384 block of the grid: the
  treecode forward against the oracle on 10^4 sampled points, and the
  treecode adjoint against the oracle's FP64 gradient of 20 sampled atoms
  (the oracle sums those atoms over the whole block).
"""
import numpy as np
import pytest
import torch

from helpers import BETA, DIEL, ETA, FP32_CAP, KAPPA, KC, oracle_rcut
from paper_2109_09772_amd import workloads as W

pytestmark = pytest.mark.gpu


def _api():
    from paper_2109_09772_amd import api
    return api


def _sampled(x, flat):
    """Values of a [S][nz][ny][nx] device grid at flat point indices."""
    ft = torch.as_tensor(flat, device=x.device)
    return x.reshape(x.shape[0], -1)[:, ft].double().cpu().numpy()


def _oracle_points(oracle, wl, pts, cut):
    sol, st = wl.solute, wl.sites
    rc = oracle_rcut(oracle, wl, cut)
    u = oracle.potential_points(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma, st.eps, pts,
                                KC, rc)
    c, h = oracle.asymptotics_points(sol.xyz, sol.q, st.q, st.ionic, pts, KC, ETA, KAPPA, BETA,
                                     DIEL)
    return [np.asarray(v).reshape(len(st.q) if k < 2 else -1, len(pts))
            for k, v in enumerate((u, c, h))]


def _samples(g, n, seed):
    idx = W.sample_points(g, n, seed)
    flat = (idx[:, 2] * g.dims[1] + idx[:, 1]) * g.dims[0] + idx[:, 0]
    return g.origin + idx * g.spacing, flat


def _rel(x, r):
    return float(np.linalg.norm(x - r) / np.linalg.norm(r))


def test_tubulin_14000(oracle):
    api = _api()
    wl = W.tubulin_14000()
    g = wl.grid
    xyz, q, s, e = api.solute_to_device(wl.solute)
    sites, grid = api.sites_from(wl.sites), api.grid_from(g)
    o64 = api.Opts(method="direct_f64", out_dtype="f64", lj_cutoff=9.0)
    ref = api.initialize(xyz, q, s, e, sites, grid, o64, ETA, KAPPA, BETA, DIEL)
    torch.cuda.synchronize()

    pts, flat = _samples(g, 64, 31)
    for name, x, r in zip("uch", ref, _oracle_points(oracle, wl, pts, 9.0)):
        xs = _sampled(x, flat)
        for k in range(xs.shape[0]):
            err = _rel(xs[k], r[k])
            print(f"f64 {name}[{k}] sampled rel-L2 {err:.2e}")
            assert err <= 1e-12

    ot = api.Opts(method="treecode_cp", out_dtype="f32", lj_cutoff=9.0, theta=0.6, degree=8,
                  stats=True)
    out = api.initialize(xyz, q, s, e, sites, grid, ot, ETA, KAPPA, BETA, DIEL)
    torch.cuda.synchronize()
    print("stats", api.last_stats())
    for name, x, r in zip("uch", out, ref):
        for k in range(x.shape[0]):
            se, sr, mx, excl, mism, _ = api.compare(x[k], r[k], ref_cap=FP32_CAP)
            err = (se / sr) ** 0.5
            print(f"treecode {name}[{k}] rel-L2 {err:.2e}")
            assert mism == 0 and err <= 1e-6


@pytest.fixture(scope="module")
def cylinder():
    return W.microtubule_block()


def test_cylinder_block_forward(oracle, cylinder):
    api = _api()
    wl = cylinder
    xyz, q, s, e = api.solute_to_device(wl.solute)
    opts = api.Opts(method="treecode_cp", out_dtype="f32", lj_cutoff=9.0, theta=0.6, degree=8,
                    stats=True)
    out = api.initialize(xyz, q, s, e, api.sites_from(wl.sites), api.grid_from(wl.grid), opts,
                         ETA, KAPPA, BETA, DIEL)
    torch.cuda.synchronize()
    print("stats", api.last_stats())
    pts, flat = _samples(wl.grid, 10_000, 51)
    for name, x, r in zip("uch", out, _oracle_points(oracle, wl, pts, 9.0)):
        xs = _sampled(x, flat)
        assert np.all(np.isfinite(xs))
        for k in range(xs.shape[0]):
            err = _rel(xs[k], r[k])
            print(f"{name}[{k}] sampled rel-L2 {err:.2e}")
            assert err <= 1e-6
    del out
    torch.cuda.empty_cache()


def test_cylinder_block_adjoint(oracle, cylinder):
    api = _api()
    wl = cylinder
    sol, st, g = wl.solute, wl.sites, wl.grid
    xyz, q, s, e = api.solute_to_device(sol)
    w = W.analytic_upstream(g, st, seed=5)
    wt = torch.as_tensor(w, device="cuda")
    opts = api.Opts(method="treecode_cp", out_dtype="f32", lj_cutoff=9.0, theta=0.6, degree=8)
    grads = api.potential_backward(xyz, q, s, e, api.sites_from(st), api.grid_from(g), opts, wt)
    torch.cuda.synchronize()
    del wt
    torch.cuda.empty_cache()
    pick = np.random.default_rng(55).choice(sol.n, 20, replace=False)
    rc = oracle.rcut_table(sol.sigma[pick], sol.eps[pick], st.sigma, st.eps, rcut=9.0)
    ref = oracle.backward_points(sol.xyz[pick], sol.q[pick], sol.sigma[pick], sol.eps[pick],
                                 st.q, st.sigma, st.eps,
                                 oracle.grid_points(g.origin, g.spacing, g.dims),
                                 w.reshape(st.n, -1), KC, rc)
    for name, x, r in zip(("dxyz", "dq", "deps", "dsigma"), grads, ref):
        err = _rel(x.cpu().numpy()[pick], r)
        print(f"{name} rel {err:.2e}")
        assert err <= 1e-5
