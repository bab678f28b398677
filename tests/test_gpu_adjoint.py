"""GPU parity of the hand-written adjoint against the oracle's FP64 gradient
(itself pinned to finite differences), and the autograd wrapper."""
import numpy as np
import pytest
import torch

from helpers import KC, oracle_rcut
from paper_2109_09772_amd import workloads as W

pytestmark = pytest.mark.gpu


def _grad_case(seed=4, n=40, dims=(26, 22, 19), spacing=0.5):
    wl = W.tiny(n_atoms=n, dims=dims, seed=seed, spacing=spacing)
    wl.solute.xyz *= 1.7
    w = W.smooth_upstream(wl.grid, wl.sites, seed=seed + 100)
    return wl, w


def _gpu_grad(wl, w, method, cut=0.0, tol=0.0):
    from paper_2109_09772_amd import api
    xyz, q, s, e = api.solute_to_device(wl.solute)
    od = "f64" if method == "direct_f64" else "f32"
    opts = api.Opts(method=method, out_dtype=od, lj_cutoff=cut, lj_tol=tol)
    wt = torch.as_tensor(w, device="cuda").to(opts.torch_dtype).contiguous()
    out = api.potential_backward(xyz, q, s, e, api.sites_from(wl.sites), api.grid_from(wl.grid),
                                 opts, wt)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out], wt.double().cpu().numpy()


def _rel(x, r):
    return np.linalg.norm(x - r) / np.linalg.norm(r)


@pytest.mark.parametrize("method,tol", [("direct_f64", 1e-11), ("direct_f32c", 1e-5)])
@pytest.mark.parametrize("cut", [0.0, 6.0])
def test_adjoint_vs_oracle(oracle, method, tol, cut):
    wl, w = _grad_case()
    (dx, dq, de, ds), wq = _gpu_grad(wl, w, method, cut)
    sol, st, g = wl.solute, wl.sites, wl.grid
    rc = oracle_rcut(oracle, wl, cut)
    rx, rq, re_, rs = oracle.backward_grid(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma,
                                           st.eps, g.origin, g.spacing, g.dims, wq, KC, rc)
    assert _rel(dx, rx) < tol
    assert _rel(dq, rq) < tol
    assert _rel(de, re_) < tol
    assert _rel(ds, rs) < tol


def test_autograd_function_matches_backward(oracle):
    from paper_2109_09772_amd import api
    wl, w = _grad_case(seed=9, n=25, dims=(20, 18, 16))
    xyz, q, s, e = api.solute_to_device(wl.solute)
    for t in (xyz, q, s, e):
        t.requires_grad_(True)
    opts = api.Opts(method="direct_f32c", out_dtype="f32", lj_cutoff=0.0)
    u = api.RismPotential.apply(xyz, q, s, e, api.sites_from(wl.sites), api.grid_from(wl.grid),
                                opts)
    wt = torch.as_tensor(w, device="cuda", dtype=torch.float32)
    (u * wt).sum().backward()
    sol, st, g = wl.solute, wl.sites, wl.grid
    rx, rq, re_, rs = oracle.backward_grid(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma,
                                           st.eps, g.origin, g.spacing, g.dims,
                                           wt.double().cpu().numpy(), KC)
    assert _rel(xyz.grad.cpu().numpy(), rx) < 1e-5
    assert _rel(q.grad.cpu().numpy(), rq) < 1e-5
    assert _rel(e.grad.cpu().numpy(), re_) < 1e-5
    assert _rel(s.grad.cpu().numpy(), rs) < 1e-5


def test_adjoint_protein_2500_sampled_atoms(oracle):
    """The 2,500-atom solute on its 128^3 grid: FP32 adjoint vs the oracle's
    FP64 gradient on 20 seeded atoms (the oracle evaluates those atoms' full
    grid sums one by one)."""
    wl = W.protein_2500()
    w = W.smooth_upstream(wl.grid, wl.sites, seed=4)
    (dx, dq, de, ds), wq = _gpu_grad(wl, w, "direct_f32c")
    sol, st, g = wl.solute, wl.sites, wl.grid
    pick = np.random.default_rng(20).choice(sol.n, 20, replace=False)
    pts = oracle.grid_points(g.origin, g.spacing, g.dims)
    rx, rq, re_, rs = oracle.backward_points(sol.xyz[pick], sol.q[pick], sol.sigma[pick],
                                             sol.eps[pick], st.q, st.sigma, st.eps, pts,
                                             wq.reshape(st.n, -1), KC)
    assert _rel(dx[pick], rx) < 1e-5
    assert _rel(dq[pick], rq) < 1e-5
    assert _rel(de[pick], re_) < 1e-5
    assert _rel(ds[pick], rs) < 1e-5
