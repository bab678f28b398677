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


def test_fp64_adjoint_vs_central_differences_protein_2500():
    """The 2,500-atom / 128^3 workload with its smooth upstream rho g(r): the
    FP64 direct adjoint against central differences of the GPU FP64 direct
    forward (no cut-off) on 20 seeded atoms, h = 1e-4 A with one Richardson
    step (r^-12 at grid points a few tenths of an angstrom away makes the
    plain difference's O(h^2) term visible).  Each atom is differenced alone
    (a one-atom solute), so the other atoms' terms do not cancel in the
    difference; L is linear in Q, so its difference is exact."""
    from paper_2109_09772_amd import api
    wl = W.protein_2500()
    sol, st, g = wl.solute, wl.sites, wl.grid
    w = W.smooth_upstream(g, st, seed=4)
    wt = torch.as_tensor(w, device="cuda", dtype=torch.float64)
    sites, grid = api.sites_from(st), api.grid_from(g)
    o64 = api.Opts(method="direct_f64", out_dtype="f64", lj_cutoff=0.0)
    xyz, q, s, e = api.solute_to_device(sol)
    dx, dq, de, ds = (t.cpu().numpy() for t in
                      api.potential_backward(xyz, q, s, e, sites, grid, o64, wt))
    out = torch.empty((st.n,) + tuple(int(v) for v in g.dims[::-1]), dtype=torch.float64,
                      device="cuda")

    # the charge and LJ-parameter differences take the Coulomb-only (site
    # eps 0) and LJ-only (site q 0) functionals: each is the part that
    # depends on the parameter, without the other part's much larger values
    # cancelling in the difference
    coul = api.make_sites(st.q, st.sigma, np.zeros(st.n), st.ionic)
    lj = api.make_sites(np.zeros(st.n), st.sigma, st.eps, st.ionic)

    def L(x1, q1, s1, e1, sp=sites):
        f = lambda a: torch.as_tensor(np.atleast_1d(a), dtype=torch.float64,
                                      device="cuda").contiguous()
        api.potential(f(x1).reshape(1, 3), f(q1), f(s1), f(e1), sp, grid, o64, out=out)
        return float((out * wt).sum())

    pick = np.random.default_rng(44).choice(sol.n, 20, replace=False)
    h = 1e-4
    fx, fq, fe, fs = [], [], [], []
    for a in pick:
        x0, q0, s0, e0 = sol.xyz[a].copy(), sol.q[a], sol.sigma[a], sol.eps[a]
        row = []
        for k in range(3):
            def Lk(hh):
                x1 = x0.copy()
                x1[k] += hh
                return L(x1, q0, s0, e0)
            d1 = (Lk(h) - Lk(-h)) / (2 * h)
            d2 = (Lk(h / 2) - Lk(-h / 2)) / h
            row.append((4 * d2 - d1) / 3)
        fx.append(row)
        fq.append(L(x0, q0 + 0.5, s0, e0, coul) - L(x0, q0 - 0.5, s0, e0, coul))
        he, hs = 1e-6 * e0, 1e-6 * s0
        fe.append((L(x0, q0, s0, e0 + he, lj) - L(x0, q0, s0, e0 - he, lj)) / (2 * he))
        fs.append((L(x0, q0, s0 + hs, e0, lj) - L(x0, q0, s0 - hs, e0, lj)) / (2 * hs))
    for name, g_, fd in (("dxyz", dx[pick], np.array(fx)), ("dq", dq[pick], np.array(fq)),
                         ("deps", de[pick], np.array(fe)), ("dsigma", ds[pick], np.array(fs))):
        err = _rel(g_, fd)
        print(f"{name} FP64 adjoint vs central differences {err:.2e}")
        assert err < 1e-6, (name, err)


def test_autograd_non_contiguous_inputs(oracle):
    """Column views of a larger array as xyz (non-contiguous): forward and
    backward both take contiguous copies."""
    from paper_2109_09772_amd import api
    wl, w = _grad_case(seed=5, n=20, dims=(16, 15, 14))
    big = torch.as_tensor(np.concatenate([wl.solute.xyz, np.zeros((wl.solute.n, 2))], axis=1),
                          dtype=torch.float64, device="cuda").requires_grad_(True)
    xyz = big[:, :3]
    assert not xyz.is_contiguous()
    _, q, s, e = api.solute_to_device(wl.solute)
    opts = api.Opts(method="direct_f64", out_dtype="f64", lj_cutoff=0.0)
    u = api.RismPotential.apply(xyz, q, s, e, api.sites_from(wl.sites), api.grid_from(wl.grid),
                                opts)
    wt = torch.as_tensor(w, device="cuda", dtype=torch.float64)
    (u * wt).sum().backward()
    sol, st, g = wl.solute, wl.sites, wl.grid
    rx, _, _, _ = oracle.backward_grid(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma,
                                       st.eps, g.origin, g.spacing, g.dims, w, KC)
    assert _rel(big.grad[:, :3].cpu().numpy(), rx) < 1e-11
    assert float(big.grad[:, 3:].abs().max()) == 0.0


# ------------------------------------------------------------------ tree adjoint

def _tree_opts(method="treecode_cp", theta=0.6, degree=10, cut=6.0, batch=8):
    from paper_2109_09772_amd import api
    return api.Opts(method=method, out_dtype="f32", lj_cutoff=cut, theta=theta, degree=degree,
                    batch_edge=batch, leaf_size=16)


@pytest.mark.parametrize("batch", [4, 8])
def test_tree_adjoint_is_transpose_of_tree_forward(batch):
    """With LJ switched off (site eps = 0), L = sum w u_tree(Q) is linear in Q,
    so sum_a Q_a dL/dQ_a from the tree adjoint must equal L from the tree
    forward (same assignment of atoms to target clusters) to FP32 rounding,
    while the exact L differs from both by the treecode error."""
    from paper_2109_09772_amd import api
    wl, w = _grad_case(seed=6, n=70, dims=(40, 36, 30), spacing=0.5)
    wl.solute.xyz *= 2.0
    wl.sites.eps[:] = 0.0
    xyz, q, s, e = api.solute_to_device(wl.solute)
    sites, grid = api.sites_from(wl.sites), api.grid_from(wl.grid)
    o = _tree_opts(theta=0.7, degree=4, batch=batch)   # coarse on purpose: large tree error
    u = api.potential(xyz, q, s, e, sites, grid, o)
    wt = torch.as_tensor(w, device="cuda", dtype=torch.float32)
    L_tree = float((u.double() * wt.double()).sum())
    _, dq, _, _ = api.potential_backward(xyz, q, s, e, sites, grid, o, wt)
    L_adj = float((q * dq).sum())
    o_ex = api.Opts(method="direct_f64", out_dtype="f64", lj_cutoff=6.0)
    L_exact = float((api.potential(xyz, q, s, e, sites, grid, o_ex) * wt.double()).sum())
    print("L tree", L_tree, "adjoint", L_adj, "exact", L_exact)
    assert abs(L_adj - L_tree) <= 2e-6 * abs(L_tree)
    assert abs(L_exact - L_tree) > 10 * abs(L_adj - L_tree)


@pytest.mark.parametrize("method,dtype", [("treecode", "f32"), ("treecode_cp", "f32"),
                                          ("treecode_cp", "f64")])
def test_tree_adjoint_vs_oracle(oracle, method, dtype):
    """Both treecodes' adjoints, with the upstream gradient in FP32 and (for
    the cluster-particle one) in FP64."""
    wl, w = _grad_case(seed=4, n=60, dims=(37, 29, 23), spacing=0.4)
    wl.solute.xyz *= 2.0
    from paper_2109_09772_amd import api
    xyz, q, s, e = api.solute_to_device(wl.solute)
    o = _tree_opts(method=method)
    o.out_dtype = dtype
    wt = torch.as_tensor(w, device="cuda", dtype=o.torch_dtype)
    dx, dq, de, ds = api.potential_backward(xyz, q, s, e, api.sites_from(wl.sites),
                                            api.grid_from(wl.grid), o, wt)
    sol, st, g = wl.solute, wl.sites, wl.grid
    rc = oracle_rcut(oracle, wl, 6.0)
    rx, rq, re_, rs = oracle.backward_grid(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma,
                                           st.eps, g.origin, g.spacing, g.dims,
                                           wt.double().cpu().numpy(), KC, rc)
    for name, x, r in (("dxyz", dx, rx), ("dq", dq, rq), ("deps", de, re_), ("dsigma", ds, rs)):
        err = _rel(x.cpu().numpy(), r)
        print(method, name, f"{err:.2e}")
        assert err < 1e-5, (name, err)


def test_tree_adjoint_protein_2500():
    """The 2,500-atom / 128^3 workload with the 9 A cut-off: cluster-particle
    tree adjoint against the GPU FP64 direct adjoint, per gradient <= 1e-5."""
    from paper_2109_09772_amd import api
    wl = W.protein_2500()
    w = W.smooth_upstream(wl.grid, wl.sites, seed=4)
    xyz, q, s, e = api.solute_to_device(wl.solute)
    sites, grid = api.sites_from(wl.sites), api.grid_from(wl.grid)
    wt = torch.as_tensor(w, device="cuda", dtype=torch.float32)
    o = _tree_opts(theta=0.6, degree=8, cut=9.0)
    got = api.potential_backward(xyz, q, s, e, sites, grid, o, wt)
    o64 = api.Opts(method="direct_f64", out_dtype="f64", lj_cutoff=9.0)
    ref = api.potential_backward(xyz, q, s, e, sites, grid, o64, wt.double())
    for name, x, r in zip(("dxyz", "dq", "deps", "dsigma"), got, ref):
        err = _rel(x.cpu().numpy(), r.cpu().numpy())
        print(name, f"{err:.2e}")
        assert err < 1e-5, (name, err)


def test_tree_adjoint_per_pair_cutoff_anisotropic(oracle):
    """Per-pair LJ cut-offs from lj_tol (radii differ by site and atom) on a
    grid with a different spacing per axis and atoms beyond its faces: the
    LJ gather's per-plane bounds and the walk's direct blocks against the
    oracle's FP64 gradient."""
    from paper_2109_09772_amd import api
    wl, w = _grad_case(seed=12, n=55, dims=(41, 30, 27), spacing=0.5)
    wl.grid = W.centred_grid([0.4, -0.3, 0.2], [0.42, 0.55, 0.61], (41, 30, 27))
    wl.solute.xyz *= 2.2
    w = W.smooth_upstream(wl.grid, wl.sites, seed=112)
    xyz, q, s, e = api.solute_to_device(wl.solute)
    o = api.Opts(method="treecode_cp", out_dtype="f32", lj_tol=1e-4, theta=0.5, degree=10,
                 batch_edge=8, leaf_size=16)
    wt = torch.as_tensor(w, device="cuda", dtype=torch.float32)
    dx, dq, de, ds = api.potential_backward(xyz, q, s, e, api.sites_from(wl.sites),
                                            api.grid_from(wl.grid), o, wt)
    sol, st, g = wl.solute, wl.sites, wl.grid
    rc = oracle_rcut(oracle, wl, lj_tol=1e-4)
    assert np.ptp(rc) > 1.0
    rx, rq, re_, rs = oracle.backward_grid(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma,
                                           st.eps, g.origin, g.spacing, g.dims,
                                           wt.double().cpu().numpy(), KC, rc)
    for name, x, r in (("dxyz", dx, rx), ("dq", dq, rq), ("deps", de, re_), ("dsigma", ds, rs)):
        err = _rel(x.cpu().numpy(), r)
        print(name, f"{err:.2e}")
        assert err < 1e-5, (name, err)
