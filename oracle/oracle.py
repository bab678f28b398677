"""Python face of the FP64 CPU oracle (``rism_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the library.  It does not
import the package under test; callers pass plain numpy arrays.

Each function is a thin ctypes call into the C direct sums; see the C file
for the definitions and the paper passages they follow.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rism_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math).  sanitize:
    instrument it with AddressSanitizer and UndefinedBehaviorSanitizer (load
    the process with gcc's libasan preloaded to run it)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g",
               "-fno-sanitize-recover=undefined"] if sanitize else []
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", *san,
                               "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        i64, i32, d = C.c_int64, C.c_int32, C.c_double
        lib.oracle_potential_points.argtypes = [i64, _P, _P, _P, _P, i32, _P, _P, _P,
                                                d, _P, C.c_int, i64, _P, _P]
        lib.oracle_potential_grid.argtypes = [i64, _P, _P, _P, _P, i32, _P, _P, _P,
                                              d, _P, C.c_int, _P, _P, _PI, _P]
        lib.oracle_asymptotics_points.argtypes = [i64, _P, _P, i32, _P, _PI, d, d, d, d, d,
                                                  i64, _P, _P, _P]
        lib.oracle_asymptotics_grid.argtypes = [i64, _P, _P, i32, _P, _PI, d, d, d, d, d,
                                                _P, _P, _PI, _P, _P]
        lib.oracle_lj_rcut_from_tol.argtypes = [d, d, d]
        lib.oracle_lj_rcut_from_tol.restype = d
        lib.oracle_lj_rcut_table.argtypes = [i64, _P, _P, i32, _P, _P, d, d, _P]
        lib.oracle_lj_tail.argtypes = [i64, _P, _P, i32, _P, _P, _P, _P]
        lib.oracle_backward_points.argtypes = [i64, _P, _P, _P, _P, i32, _P, _P, _P, d, _P,
                                               i64, _P, _P, _P, _P, _P, _P]
        lib.oracle_grid_points.argtypes = [_P, _P, _PI, _P]
        lib.oracle_asymptotics_k.argtypes = [i64, _P, _P, i32, _P, _PI, d, d, d, d, d,
                                             _P, _P, _PI, d, d, _P, _P]
        lib.oracle_asymptotics_k_entries.argtypes = [i64, _P, _P, i32, _P, _PI, d, d, d, d, d,
                                                     _P, _P, _PI, d, d, i64,
                                                     C.POINTER(C.c_int64), _P, _P]
        lib.oracle_kcut.argtypes = [C.c_int, d, d, d, d, d, d, d, d]
        lib.oracle_kcut.restype = d
        lib.oracle_num_threads.restype = C.c_int
        lib.oracle_set_num_threads.argtypes = [C.c_int]
        lib.oracle_set_num_threads.restype = None
        lib.oracle_taylor_coeffs.argtypes = [C.c_int, _P, C.c_int, d, d, _P]
        lib.oracle_taylor_cp_points.argtypes = [i64, _P, _P, _P, _P, i32, _P, _P, _P, _PI, d,
                                                _P, d, d, d, d, _P, _P, _PI, i32, d, i32, d,
                                                i64, _PI, _P, _P, _P]
        lib.oracle_taylor_split_cp_points.argtypes = [i64, _P, _P, _P, _P, i32, _P, _P, _P,
                                                      _PI, d, _P, d, d, d, d, _P, _P, _PI, i32,
                                                      d, i32, i64, _PI, _P, _P, _P]
        _lib = lib
    return _lib


def _d(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a, t=_P):
    return None if a is None else a.ctypes.data_as(t)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the later oracle sums (n <= 0: every processor)."""
    _load().oracle_set_num_threads(int(n))


def _atoms(xyz, q, sigma, eps):
    return (_d(np.asarray(xyz).reshape(-1, 3)), _d(q), _d(sigma), _d(eps))


def rcut_table(sigma, eps, site_sigma, site_eps, rcut=0.0, tol=0.0):
    """[S][N] cut-off radii: ``rcut`` for all pairs, or per pair from ``tol``."""
    lib = _load()
    sigma, eps, ss, se = _d(sigma), _d(eps), _d(site_sigma), _d(site_eps)
    out = np.empty((len(ss), len(sigma)))
    rc = lib.oracle_lj_rcut_table(len(sigma), _ptr(sigma), _ptr(eps), len(ss), _ptr(ss),
                                  _ptr(se), float(rcut), float(tol), _ptr(out))
    if rc != 0:
        raise ValueError("no LJ cut-off radius for this tolerance")
    return out


def lj_rcut_from_tol(sigma_pair, eps_pair, tol):
    return float(_load().oracle_lj_rcut_from_tol(sigma_pair, eps_pair, tol))


def lj_tail(sigma, eps, site_sigma, site_eps, rcut_tab):
    lib = _load()
    sigma, eps, ss, se = _d(sigma), _d(eps), _d(site_sigma), _d(site_eps)
    rct = _d(rcut_tab)
    out = np.empty(len(ss))
    lib.oracle_lj_tail(len(sigma), _ptr(sigma), _ptr(eps), len(ss), _ptr(ss), _ptr(se),
                       _ptr(rct), _ptr(out))
    return out


def potential_points(xyz, q, sigma, eps, site_q, site_sigma, site_eps, pts,
                     kc, rcut_tab=None, terms=3):
    """u[S][npts] at arbitrary points (npts, 3)."""
    lib = _load()
    xyz, q, sigma, eps = _atoms(xyz, q, sigma, eps)
    sq, ss, se = _d(site_q), _d(site_sigma), _d(site_eps)
    pts = _d(np.asarray(pts).reshape(-1, 3))
    rct = _d(rcut_tab)
    out = np.empty((len(sq), len(pts)))
    rc = lib.oracle_potential_points(len(q), _ptr(xyz), _ptr(q), _ptr(sigma), _ptr(eps),
                                     len(sq), _ptr(sq), _ptr(ss), _ptr(se), float(kc),
                                     _ptr(rct), int(terms), len(pts), _ptr(pts), _ptr(out))
    assert rc == 0
    return out


def potential_grid(xyz, q, sigma, eps, site_q, site_sigma, site_eps, origin, spacing,
                   dims, kc, rcut_tab=None, terms=3):
    """u[S][nz][ny][nx] on the grid origin + (i, j, k) * spacing."""
    lib = _load()
    xyz, q, sigma, eps = _atoms(xyz, q, sigma, eps)
    sq, ss, se = _d(site_q), _d(site_sigma), _d(site_eps)
    o, h = _d(origin), _d(spacing)
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    rct = _d(rcut_tab)
    out = np.empty((len(sq), int(dm[2]), int(dm[1]), int(dm[0])))
    rc = lib.oracle_potential_grid(len(q), _ptr(xyz), _ptr(q), _ptr(sigma), _ptr(eps),
                                   len(sq), _ptr(sq), _ptr(ss), _ptr(se), float(kc),
                                   _ptr(rct), int(terms), _ptr(o), _ptr(h), _ptr(dm, _PI),
                                   _ptr(out))
    assert rc == 0
    return out


def asymptotics_points(xyz, q, site_q, ionic, pts, kc, eta, kappa, beta, diel,
                       want_c=True, want_h=True):
    lib = _load()
    xyz = _d(np.asarray(xyz).reshape(-1, 3))
    q, sq = _d(q), _d(site_q)
    ion = np.ascontiguousarray(ionic, dtype=np.int32)
    pts = _d(np.asarray(pts).reshape(-1, 3))
    c = np.empty((len(sq), len(pts))) if want_c else None
    h = np.empty((int(ion.sum()), len(pts))) if want_h else None
    rc = lib.oracle_asymptotics_points(len(q), _ptr(xyz), _ptr(q), len(sq), _ptr(sq),
                                       _ptr(ion, _PI), float(kc), float(eta), float(kappa),
                                       float(beta), float(diel), len(pts), _ptr(pts),
                                       _ptr(c), _ptr(h))
    assert rc == 0
    return c, h


def asymptotics_grid(xyz, q, site_q, ionic, origin, spacing, dims, kc, eta, kappa,
                     beta, diel, want_c=True, want_h=True):
    lib = _load()
    xyz = _d(np.asarray(xyz).reshape(-1, 3))
    q, sq = _d(q), _d(site_q)
    ion = np.ascontiguousarray(ionic, dtype=np.int32)
    o, h_ = _d(origin), _d(spacing)
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    shp = (int(dm[2]), int(dm[1]), int(dm[0]))
    c = np.empty((len(sq),) + shp) if want_c else None
    h = np.empty((int(ion.sum()),) + shp) if want_h else None
    rc = lib.oracle_asymptotics_grid(len(q), _ptr(xyz), _ptr(q), len(sq), _ptr(sq),
                                     _ptr(ion, _PI), float(kc), float(eta), float(kappa),
                                     float(beta), float(diel), _ptr(o), _ptr(h_),
                                     _ptr(dm, _PI), _ptr(c), _ptr(h))
    assert rc == 0
    return c, h


def asymptotics_k(xyz, q, site_q, ionic, origin, spacing, dims, kc, eta, kappa, beta,
                  diel, kcut_c=0.0, kcut_h=0.0, want_c=True, want_h=True):
    """c^lr(k) [S][nz][ny][nx//2+1] and h^lr(k) [n_ionic][...] as complex128
    (Sec. 2.2, Eqs. 5 and 7; transform-order frequencies, see the C file)."""
    lib = _load()
    xyz = _d(np.asarray(xyz).reshape(-1, 3))
    q, sq = _d(q), _d(site_q)
    ion = np.ascontiguousarray(ionic, dtype=np.int32)
    o, h_ = _d(origin), _d(spacing)
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    shp = (int(dm[2]), int(dm[1]), int(dm[0]) // 2 + 1)
    c = np.empty((len(sq),) + shp + (2,)) if want_c else None
    h = np.empty((int(ion.sum()),) + shp + (2,)) if want_h else None
    rc = lib.oracle_asymptotics_k(len(q), _ptr(xyz), _ptr(q), len(sq), _ptr(sq),
                                  _ptr(ion, _PI), float(kc), float(eta), float(kappa),
                                  float(beta), float(diel), _ptr(o), _ptr(h_), _ptr(dm, _PI),
                                  float(kcut_c), float(kcut_h), _ptr(c), _ptr(h))
    assert rc == 0
    cz = None if c is None else c[..., 0] + 1j * c[..., 1]
    hz = None if h is None else h[..., 0] + 1j * h[..., 1]
    return cz, hz


def asymptotics_k_entries(xyz, q, site_q, ionic, origin, spacing, dims, entries, kc, eta,
                          kappa, beta, diel, kcut_c=0.0, kcut_h=0.0):
    """The same quantities at listed flat indices of the half grid:
    c [S][len(entries)], h [n_ionic][len(entries)], complex128."""
    lib = _load()
    xyz = _d(np.asarray(xyz).reshape(-1, 3))
    q, sq = _d(q), _d(site_q)
    ion = np.ascontiguousarray(ionic, dtype=np.int32)
    o, h_ = _d(origin), _d(spacing)
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    ent = np.ascontiguousarray(entries, dtype=np.int64)
    c = np.empty((len(sq), len(ent), 2))
    h = np.empty((int(ion.sum()), len(ent), 2))
    rc = lib.oracle_asymptotics_k_entries(len(q), _ptr(xyz), _ptr(q), len(sq), _ptr(sq),
                                          _ptr(ion, _PI), float(kc), float(eta), float(kappa),
                                          float(beta), float(diel), _ptr(o), _ptr(h_),
                                          _ptr(dm, _PI), float(kcut_c), float(kcut_h), len(ent),
                                          ent.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(c),
                                          _ptr(h))
    assert rc == 0
    return c[..., 0] + 1j * c[..., 1], h[..., 0] + 1j * h[..., 1]


def kcut(which, tol, qmax, qabs_sum, kc, eta, kappa, beta, diel):
    """Frequency cut-off of the c^lr ('c') or h^lr ('h') bound of Sec. 2.5."""
    return float(_load().oracle_kcut(0 if which == "c" else 1, float(tol), float(qmax),
                                     float(qabs_sum), float(kc), float(eta), float(kappa),
                                     float(beta), float(diel)))


def grid_points(origin, spacing, dims):
    lib = _load()
    o, h = _d(origin), _d(spacing)
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    m = int(np.prod(dm.astype(np.int64)))
    out = np.empty((m, 3))
    lib.oracle_grid_points(_ptr(o), _ptr(h), _ptr(dm, _PI), _ptr(out))
    return out


def backward_points(xyz, q, sigma, eps, site_q, site_sigma, site_eps, pts, w, kc,
                    rcut_tab=None):
    """Gradients of L = sum w[S][npts] * u[S][npts] w.r.t. (xyz, q, eps, sigma)."""
    lib = _load()
    xyz, q, sigma, eps = _atoms(xyz, q, sigma, eps)
    sq, ss, se = _d(site_q), _d(site_sigma), _d(site_eps)
    pts = _d(np.asarray(pts).reshape(-1, 3))
    w = _d(np.asarray(w).reshape(len(sq), -1))
    rct = _d(rcut_tab)
    n = len(q)
    dxyz = np.empty((n, 3))
    dq, de, ds = np.empty(n), np.empty(n), np.empty(n)
    rc = lib.oracle_backward_points(n, _ptr(xyz), _ptr(q), _ptr(sigma), _ptr(eps), len(sq),
                                    _ptr(sq), _ptr(ss), _ptr(se), float(kc), _ptr(rct),
                                    len(pts), _ptr(pts), _ptr(w), _ptr(dxyz), _ptr(dq),
                                    _ptr(de), _ptr(ds))
    assert rc == 0
    return dxyz, dq, de, ds


def backward_grid(xyz, q, sigma, eps, site_q, site_sigma, site_eps, origin, spacing,
                  dims, w, kc, rcut_tab=None):
    pts = grid_points(origin, spacing, dims)
    return backward_points(xyz, q, sigma, eps, site_q, site_sigma, site_eps, pts,
                           np.asarray(w).reshape(len(site_q), -1), kc, rcut_tab)


TAYLOR_KINDS = {"coulomb": 0, "dcf": 1, "screened": 2}


def taylor_coeffs(kind, v, p, eta=1.0, kappa=0.0):
    """Order-p Taylor coefficients t[k3][k2][k1] = (1/k!) d^k phi/dx^k of the
    kernel ``kind`` ('coulomb' 1/R, 'dcf' erf(R/eta)/R, 'screened'
    2 exp(-kappa R)/R) at a centre x with v = y - x, by the paper's
    recurrences (zero where |k| > p)."""
    out = np.empty((p + 1, p + 1, p + 1))
    vv = _d(np.asarray(v, dtype=np.float64).reshape(3))
    rc = _load().oracle_taylor_coeffs(TAYLOR_KINDS[kind], _ptr(vv), int(p), float(eta),
                                      float(kappa), _ptr(out))
    assert rc == 0
    return out


def taylor_guard(eta, kappa):
    """Distance guard of the paper's Taylor treecode when h^lr is expanded:
    eta (6 + kappa eta / 2), where the erfc -> 2/0 step of Sec. 2.4.2 is off
    by about erfc(6) ~ 2e-17 (see the C file)."""
    return eta * (6.0 + 0.5 * kappa * eta)


def _taylor_call(fn, guard, xyz, q, sigma, eps, site_q, site_sigma, site_eps, ionic, origin,
                 spacing, dims, ijk, kc, eta, kappa, beta, diel, batch_edge, theta, p,
                 rcut_tab):
    xyz, q, sigma, eps = _atoms(xyz, q, sigma, eps)
    sq, ss, se = _d(site_q), _d(site_sigma), _d(site_eps)
    ion = np.ascontiguousarray(ionic, dtype=np.int32)
    o, h_ = _d(origin), _d(spacing)
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    g = np.ascontiguousarray(np.asarray(ijk).reshape(-1, 3), dtype=np.int32)
    rct = _d(rcut_tab)
    u = np.empty((len(sq), len(g)))
    c = np.empty((len(sq), len(g)))
    h = np.empty((int(ion.sum()), len(g)))
    args = [len(q), _ptr(xyz), _ptr(q), _ptr(sigma), _ptr(eps), len(sq), _ptr(sq), _ptr(ss),
            _ptr(se), _ptr(ion, _PI), float(kc), _ptr(rct), float(eta), float(kappa),
            float(beta), float(diel), _ptr(o), _ptr(h_), _ptr(dm, _PI), int(batch_edge),
            float(theta), int(p)]
    if guard is not None:
        args.append(float(guard))
    args += [len(g), _ptr(g, _PI), _ptr(u), _ptr(c), _ptr(h)]
    rc = fn(*args)
    assert rc == 0
    return u, c, h


def taylor_cp_points(xyz, q, sigma, eps, site_q, site_sigma, site_eps, ionic, origin,
                     spacing, dims, ijk, kc, eta, kappa, beta, diel, batch_edge, theta, p,
                     rcut_tab=None, guard=None):
    """The paper's Taylor cluster-particle treecode (far fields: Taylor
    polynomials of 1/d, erf(d/eta)/d and 2 exp(-kappa d)/d) at grid points
    ijk (npts, 3): u [S][npts], c [S][npts], h [n_ionic][npts].  ``guard``:
    the MAC's distance condition (default taylor_guard(eta, kappa); 0 = the
    MAC alone)."""
    if guard is None:
        guard = taylor_guard(eta, kappa)
    return _taylor_call(_load().oracle_taylor_cp_points, guard, xyz, q, sigma, eps, site_q,
                        site_sigma, site_eps, ionic, origin, spacing, dims, ijk, kc, eta, kappa,
                        beta, diel, batch_edge, theta, p, rcut_tab)


def taylor_split_cp_points(xyz, q, sigma, eps, site_q, site_sigma, site_eps, ionic, origin,
                           spacing, dims, ijk, kc, eta, kappa, beta, diel, batch_edge, theta, p,
                           rcut_tab=None):
    """The exact-split variant: far fields 1/d and 2 exp(-kappa d)/d only, the
    smeared kernels' remainders added exactly within Rs (see the C file)."""
    return _taylor_call(_load().oracle_taylor_split_cp_points, None, xyz, q, sigma, eps, site_q,
                        site_sigma, site_eps, ionic, origin, spacing, dims, ijk, kc, eta, kappa,
                        beta, diel, batch_edge, theta, p, rcut_tab)
