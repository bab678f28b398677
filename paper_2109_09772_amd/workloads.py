"""Seeded synthetic solutes, solvent sites and grids.

This module only draws inputs; it holds none of the method's arithmetic
(no mixing rule, no kernel, no cut-off).  Both the HIP path and the FP64
oracle are fed from it, so that they see bit-identical inputs.

The paper's solutes (phenol, CB7, adhiron, tubulin, microtubule; Table 1)
are not available here.  Each configuration below is a synthetic stand-in of
the same atom count and a similar shape, with Amber-like parameter ranges:

* positions: random sequential addition (minimum separation 1.0 A) inside the
  named body, drawn with ``numpy.random.default_rng(seed)``;
* charges ``Q ~ U(-0.8, 0.8)``, then the mean is subtracted (net charge 0);
* ``sigma ~ U(1.5, 4.0)`` A, ``eps ~ U(0.02, 0.2)`` kcal/mol;
* draws happen in the order positions, Q, sigma, eps.

Solvent: SPC/E-like water sites O and H plus Na+ and Cl- for 0.1 M NaCl at
298.15 K in a dielectric of 78.44 (the solvent of Sec. 3.2).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Physical constants of the solvent model (Sec. 3.2 gives T, the dielectric
# constant, and the water / salt concentrations).
COULOMB_K = 332.0522173          # kcal*A/(mol*e^2), Amber's 18.2223^2
BOLTZMANN_K = 0.00198720426      # kcal/(mol*K)
TEMPERATURE = 298.15             # K
DIELECTRIC = 78.44
ETA = 1.0                        # A, charge-smearing length of the asymptotics
AVOGADRO = 6.02214076e23
WATER_MOLAR = 55.2               # mol/L
SALT_MOLAR = 0.1                 # mol/L


def beta() -> float:
    """1/(k_B T) in (kcal/mol)^-1."""
    return 1.0 / (BOLTZMANN_K * TEMPERATURE)


def molar_to_number_density(c_molar: float) -> float:
    """mol/L -> particles per cubic angstrom (1 L = 1e27 A^3)."""
    return c_molar * AVOGADRO / 1e27


def debye_kappa(salt_molar: float = SALT_MOLAR) -> float:
    """Inverse Debye length (1/A) of a 1:1 salt in the model dielectric."""
    rho = molar_to_number_density(salt_molar)
    s = 2.0 * rho * 1.0  # Na+ and Cl-, |q| = 1
    return math.sqrt(4.0 * math.pi * beta() * COULOMB_K * s / DIELECTRIC)


@dataclasses.dataclass
class Sites:
    names: list
    q: np.ndarray
    sigma: np.ndarray
    eps: np.ndarray
    ionic: np.ndarray
    rho: np.ndarray   # bulk number density per site (1/A^3)

    @property
    def n(self) -> int:
        return len(self.names)


_SITE_TABLE = {
    # name: (q, sigma, eps, ionic, density in mol/L of the carrying species)
    "O": (-0.834, 3.15, 0.152, 0, WATER_MOLAR),
    "H": (0.417, 0.4, 0.046, 0, 2.0 * WATER_MOLAR),
    "Na+": (1.0, 2.4, 0.09, 1, SALT_MOLAR),
    "Cl-": (-1.0, 4.4, 0.1, 1, SALT_MOLAR),
}


def make_sites(names) -> Sites:
    rows = [_SITE_TABLE[n] for n in names]
    return Sites(
        names=list(names),
        q=np.array([r[0] for r in rows], dtype=np.float64),
        sigma=np.array([r[1] for r in rows], dtype=np.float64),
        eps=np.array([r[2] for r in rows], dtype=np.float64),
        ionic=np.array([r[3] for r in rows], dtype=np.int32),
        rho=np.array([molar_to_number_density(r[4]) for r in rows]),
    )


@dataclasses.dataclass
class Grid:
    origin: np.ndarray   # (3,) float64, position of grid point (0,0,0)
    spacing: np.ndarray  # (3,) float64
    dims: np.ndarray     # (3,) int32, (nx, ny, nz); storage is [z][y][x]

    @property
    def npoints(self) -> int:
        return int(np.prod(self.dims.astype(np.int64)))

    def axis(self, a: int) -> np.ndarray:
        return self.origin[a] + self.spacing[a] * np.arange(self.dims[a])


def centred_grid(centre, spacing, dims) -> Grid:
    spacing = np.broadcast_to(np.asarray(spacing, dtype=np.float64), (3,)).copy()
    dims = np.broadcast_to(np.asarray(dims, dtype=np.int32), (3,)).copy()
    centre = np.asarray(centre, dtype=np.float64)
    origin = centre - spacing * (dims - 1) / 2.0
    return Grid(origin=origin, spacing=spacing, dims=dims)


@dataclasses.dataclass
class Solute:
    xyz: np.ndarray    # (n, 3) float64
    q: np.ndarray
    sigma: np.ndarray
    eps: np.ndarray

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    solute: Solute
    sites: Sites
    grid: Grid
    seed: int


# ----------------------------------------------------------------------------
# position samplers
# ----------------------------------------------------------------------------

def _rsa_filter(cand: np.ndarray, dmin: float, kept: np.ndarray | None):
    """Random sequential addition: accept candidates in order, rejecting any
    closer than ``dmin`` to an already accepted point."""
    from scipy.spatial import cKDTree

    out_mask = np.ones(len(cand), dtype=bool)
    if kept is not None and len(kept):
        d, _ = cKDTree(kept).query(cand, k=1, distance_upper_bound=dmin)
        out_mask &= ~(d < dmin)
    idx = np.nonzero(out_mask)[0]
    sub = cand[idx]
    pairs = cKDTree(sub).query_pairs(dmin, output_type="ndarray")
    if len(pairs):
        # pairs (i, j) with i < j in candidate order; j dies if i survives
        order = np.argsort(pairs[:, 1], kind="stable")
        pairs = pairs[order]
        alive = np.ones(len(sub), dtype=bool)
        starts = np.searchsorted(pairs[:, 1], np.arange(len(sub)), side="left")
        ends = np.searchsorted(pairs[:, 1], np.arange(len(sub)), side="right")
        has = np.nonzero(ends > starts)[0]
        for j in has:
            lo = pairs[starts[j]:ends[j], 0]
            if alive[lo].any():
                alive[j] = False
        idx = idx[alive]
    return cand[idx]


def _sample_body(rng, n, inside, lo, hi, dmin=1.0):
    """Draw ``n`` points uniformly inside a body (``inside`` predicate on a
    bounding box ``lo..hi``) with minimum separation ``dmin``."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    kept = np.zeros((0, 3))
    while len(kept) < n:
        need = n - len(kept)
        m = max(int(need * 1.6) + 64, 256)
        cand = lo + (hi - lo) * rng.random((m, 3))
        cand = cand[inside(cand)]
        acc = _rsa_filter(cand, dmin, kept)
        kept = np.concatenate([kept, acc[:need]], axis=0)
    return kept[:n]


def _params(rng, n):
    q = rng.uniform(-0.8, 0.8, n)
    q = q - q.mean()
    sigma = rng.uniform(1.5, 4.0, n)
    eps = rng.uniform(0.02, 0.2, n)
    return q, sigma, eps


def ball_solute(n, radius, seed, dmin=1.0) -> Solute:
    rng = np.random.default_rng(seed)
    r2 = radius * radius
    xyz = _sample_body(rng, n, lambda p: (p * p).sum(1) <= r2,
                       [-radius] * 3, [radius] * 3, dmin)
    q, s, e = _params(rng, n)
    return Solute(xyz, q, s, e)


def ellipsoid_solute(n, semi_axes, seed, dmin=1.0) -> Solute:
    rng = np.random.default_rng(seed)
    ax = np.asarray(semi_axes, dtype=np.float64)
    xyz = _sample_body(rng, n, lambda p: ((p / ax) ** 2).sum(1) <= 1.0,
                       -ax, ax, dmin)
    q, s, e = _params(rng, n)
    return Solute(xyz, q, s, e)


def cylinder_shell_solute(n, r_in, r_out, half_len, seed, dmin=1.0) -> Solute:
    rng = np.random.default_rng(seed)

    def inside(p):
        rr = p[:, 0] ** 2 + p[:, 1] ** 2
        return (rr >= r_in * r_in) & (rr <= r_out * r_out)

    xyz = _sample_body(rng, n, inside, [-r_out, -r_out, -half_len],
                       [r_out, r_out, half_len], dmin)
    q, s, e = _params(rng, n)
    return Solute(xyz, q, s, e)


# ----------------------------------------------------------------------------
# named configurations
# ----------------------------------------------------------------------------

SITES_WATER = ("O", "H")
SITES_SALT = ("O", "H", "Na+", "Cl-")


def ellipsoid_semi_axes_for_density(n, density, ratios=(1.0, 1.5, 2.0)):
    """Semi-axes a*ratios of an ellipsoid holding ``n`` atoms at ``density``."""
    vol = n / density
    r = np.asarray(ratios, dtype=np.float64)
    a = (vol / (4.0 / 3.0 * math.pi * r.prod())) ** (1.0 / 3.0)
    return a * r


def small_ball(seed=1) -> Workload:
    """200 atoms in a 20 A ball, 2 water sites, 64^3 grid at 0.5 A."""
    sol = ball_solute(200, 10.0, seed)
    return Workload("ball200_grid64", sol, make_sites(SITES_WATER),
                    centred_grid([0.0, 0.0, 0.0], 0.5, 64), seed)


def protein_2500(seed=2) -> Workload:
    """2,500 atoms at 0.1 /A^3 in a 1:1.5:2 ellipsoid, 4 sites, 128^3 grid."""
    ax = ellipsoid_semi_axes_for_density(2500, 0.1)
    sol = ellipsoid_solute(2500, ax, seed)
    return Workload("ellipsoid2500_grid128", sol, make_sites(SITES_SALT),
                    centred_grid([0.0, 0.0, 0.0], 0.5, 128), seed)


def tubulin_14000(seed=3) -> Workload:
    """14,000 atoms in a 45x45x80 A ellipsoid (0.165 /A^3: the stated atom
    count and box do not fit 0.1 /A^3, so the count and box are kept), 4
    sites, 256^3 grid."""
    sol = ellipsoid_solute(14000, [22.5, 22.5, 40.0], seed)
    return Workload("ellipsoid14000_grid256", sol, make_sites(SITES_SALT),
                    centred_grid([0.0, 0.0, 0.0], 0.5, 256), seed)


def microtubule_block(seed=5, n=1_200_000) -> Workload:
    """1.2 M atoms in a hollow cylinder (r 85..125 A, length 400 A); one
    512x512x384 sub-block of the grid at 0.5 A, centred on the axis."""
    sol = cylinder_shell_solute(n, 85.0, 125.0, 200.0, seed)
    g = Grid(origin=np.array([-127.75, -127.75, -95.75]),
             spacing=np.full(3, 0.5), dims=np.array([512, 512, 384], np.int32))
    return Workload("cylinder1.2M_block512x512x384", sol, make_sites(SITES_SALT), g, seed)


def tiny(n_atoms=5, dims=(4, 5, 6), seed=11, spacing=0.7, sites=SITES_SALT) -> Workload:
    """A handful of atoms and a small non-cubic grid for brute-force checks."""
    sol = ball_solute(n_atoms, 3.0, seed)
    return Workload(f"tiny{n_atoms}", sol, make_sites(sites),
                    centred_grid([0.1, -0.2, 0.3], spacing, dims), seed)


def smooth_upstream(grid: Grid, sites: Sites, seed: int, filt_sigma=2.0) -> np.ndarray:
    """Upstream dL/du_gamma(r) = rho_gamma * g_gamma(r), g a smooth random
    field with U(0, 3) marginals: white noise Gaussian-filtered (2 A),
    standardised, mapped through the normal CDF and scaled by 3."""
    from scipy.ndimage import gaussian_filter
    from scipy.special import ndtr

    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in grid.dims)
    out = np.empty((sites.n, nz, ny, nx), dtype=np.float64)
    for s in range(sites.n):
        z = rng.standard_normal((nz, ny, nx))
        z = gaussian_filter(z, sigma=filt_sigma / np.asarray(grid.spacing)[::-1], mode="wrap")
        z = (z - z.mean()) / z.std()
        out[s] = sites.rho[s] * 3.0 * ndtr(z)
    return out


def analytic_upstream(grid: Grid, sites: Sites, seed: int, wavelength=(12.0, 20.0)) -> np.ndarray:
    """A smooth seeded upstream for grids too large to filter white noise:
    dL/du_gamma = rho_gamma * g_gamma, g_gamma = 1.5 + 1.5 fx(x) fy(y) fz(z)
    with fa = sin(2 pi a / L_a + phi_a), wavelengths and phases drawn per site
    and axis, so that g lies in [0, 3].  FP32, shape [S][nz][ny][nx]."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in grid.dims)
    out = np.empty((sites.n, nz, ny, nx), dtype=np.float32)
    for s in range(sites.n):
        f = []
        for ax, n in enumerate((nx, ny, nz)):
            lam = rng.uniform(*wavelength)
            phi = rng.uniform(0.0, 2.0 * np.pi)
            a = grid.origin[ax] + grid.spacing[ax] * np.arange(n)
            f.append(np.sin(2.0 * np.pi * a / lam + phi).astype(np.float32))
        g = f[2][:, None, None] * f[1][None, :, None]
        out[s] = f[0][None, None, :] * g
        out[s] *= np.float32(1.5 * sites.rho[s])
        out[s] += np.float32(1.5 * sites.rho[s])
    return out


def sample_points(grid: Grid, n: int, seed: int) -> np.ndarray:
    """Indices (n, 3) as (i, j, k) of distinct random grid points."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(grid.npoints, size=n, replace=False)
    nx, ny = int(grid.dims[0]), int(grid.dims[1])
    i = flat % nx
    j = (flat // nx) % ny
    k = flat // (nx * ny)
    return np.stack([i, j, k], axis=1).astype(np.int64)
