"""Thin Python binding of librism.so (ctypes).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  torch provides device memory and the current HIP
stream.  The library must be built (``paper_2109_09772_amd.build``); there is
no fallback of any kind, and every entry point raises if the library or the
GPU is missing.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

from . import workloads as _wl

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librism.so")

RISM_OK = 0
RISM_E_INVALID = -1
RISM_E_NOMEM = -2
RISM_E_HIP = -3
RISM_E_UNSUPPORTED = -4

METHODS = {"direct_f64": 0, "direct_f32c": 1, "treecode": 2, "treecode_cp": 3,
           "treecode_taylor": 4}
DTYPES = {"f32": 0, "f64": 1}
FLAG_NO_DEVICE_CHECK = 1
FLAG_PHASE_EVENTS = 2
FLAG_STATS = 4
FLAG_TAYLOR_SPLIT = 8
MAX_SITES = 8
PHASES = ["stage", "direct_f64", "direct_f32", "tree_build", "upward", "lists", "eval",
          "downward", "adjoint", "adjoint_reduce", "other", "recip"]


class RismError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librism error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("spacing", C.c_double * 3), ("dims", C.c_int32 * 3)]


class Solute(C.Structure):
    _fields_ = [("n", C.c_int64), ("xyz", C.c_void_p), ("q", C.c_void_p),
                ("sigma", C.c_void_p), ("eps", C.c_void_p)]


class Sites(C.Structure):
    _fields_ = [("n", C.c_int32), ("q", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)),
                ("eps", C.POINTER(C.c_double)), ("ionic", C.POINTER(C.c_int32))]


class OptsC(C.Structure):
    _fields_ = [("method", C.c_int32), ("out_dtype", C.c_int32), ("coulomb_k", C.c_double),
                ("lj_cutoff", C.c_double), ("lj_tol", C.c_double), ("theta", C.c_double),
                ("degree", C.c_int32), ("leaf_size", C.c_int32), ("batch_edge", C.c_int32),
                ("flags", C.c_uint32), ("max_workspace_bytes", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [("pairs_direct", C.c_double), ("pairs_far", C.c_double),
                ("pairs_short", C.c_double), ("upward_flops", C.c_double),
                ("n_nodes", C.c_int64), ("n_batches", C.c_int64),
                ("workspace_bytes", C.c_int64)]


_lib = None


def lib():
    """Loads librism.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2109_09772_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        d = C.c_double
        L.rism_default_opts.argtypes = [P(OptsC)]
        L.rism_default_opts.restype = None
        common = [P(Solute), P(Sites), P(Grid), P(OptsC)]
        L.rism_potential.argtypes = common + [vp, P(C.c_double), vp]
        L.rism_asymptotics.argtypes = common + [d, d, d, d, vp, vp, vp]
        L.rism_initialize.argtypes = common + [d, d, d, d, vp, P(C.c_double), vp, vp, vp]
        L.rism_asymptotics_k.argtypes = common + [d, d, d, d, d, vp, vp, vp]
        L.rism_initialize_noalloc.argtypes = common + [d, d, d, d, vp, P(C.c_double), vp, vp,
                                                       vp]
        L.rism_potential_backward.argtypes = common + [vp, vp, vp, vp, vp, vp]
        L.rism_compare.argtypes = [vp, C.c_int32, vp, C.c_int64, d, vp, P(C.c_double), vp]
        L.rism_near_mask.argtypes = [P(Solute), P(Grid), d, vp, vp]
        L.rism_last_stats.argtypes = [P(Stats)]
        L.rism_last_error.restype = C.c_char_p
        L.rism_phase_times.argtypes = [P(C.c_double), P(C.c_int64)]
        L.rism_phase_times.restype = C.c_int
        for f in ("rism_potential", "rism_asymptotics", "rism_initialize",
                  "rism_potential_backward", "rism_compare", "rism_last_stats",
                  "rism_asymptotics_k", "rism_initialize_noalloc", "rism_near_mask"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != RISM_OK:
        raise RismError(rc, lib().rism_last_error().decode())


@dataclasses.dataclass
class Opts:
    method: str = "treecode_cp"
    out_dtype: str = "f32"
    coulomb_k: float = _wl.COULOMB_K
    lj_cutoff: float = 9.0
    lj_tol: float = 0.0
    theta: float = 0.6
    degree: int = 8
    leaf_size: int = 64
    batch_edge: int = 8
    device_check: bool = True
    phase_events: bool = False
    stats: bool = False
    taylor_split: bool = False
    max_workspace_bytes: int = 0

    def to_c(self) -> OptsC:
        o = OptsC()
        lib().rism_default_opts(C.byref(o))
        o.method = METHODS[self.method]
        o.out_dtype = DTYPES[self.out_dtype]
        o.coulomb_k = self.coulomb_k
        o.lj_cutoff = self.lj_cutoff
        o.lj_tol = self.lj_tol
        o.theta = self.theta
        o.degree = self.degree
        o.leaf_size = self.leaf_size
        o.batch_edge = self.batch_edge
        o.flags = (0 if self.device_check else FLAG_NO_DEVICE_CHECK) | \
            (FLAG_PHASE_EVENTS if self.phase_events else 0) | \
            (FLAG_STATS if self.stats else 0) | (FLAG_TAYLOR_SPLIT if self.taylor_split else 0)
        o.max_workspace_bytes = self.max_workspace_bytes
        return o

    @property
    def torch_dtype(self):
        return torch.float64 if self.out_dtype == "f64" else torch.float32


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class _Keep:
    """Keeps host arrays referenced by the C structs alive."""


def make_sites(q, sigma, eps, ionic=None):
    k = _Keep()
    k.q = np.ascontiguousarray(q, dtype=np.float64)
    k.s = np.ascontiguousarray(sigma, dtype=np.float64)
    k.e = np.ascontiguousarray(eps, dtype=np.float64)
    n = len(k.q)
    k.i = np.ascontiguousarray(np.zeros(n) if ionic is None else ionic, dtype=np.int32)
    st = Sites(n, k.q.ctypes.data_as(C.POINTER(C.c_double)),
               k.s.ctypes.data_as(C.POINTER(C.c_double)),
               k.e.ctypes.data_as(C.POINTER(C.c_double)),
               k.i.ctypes.data_as(C.POINTER(C.c_int32)))
    st._keep = k
    return st


def make_grid(origin, spacing, dims):
    g = Grid()
    sp = np.broadcast_to(np.asarray(spacing, dtype=np.float64), (3,))
    dm = np.broadcast_to(np.asarray(dims, dtype=np.int64), (3,))
    for a in range(3):
        g.origin[a] = float(origin[a])
        g.spacing[a] = float(sp[a])
        g.dims[a] = int(dm[a])
    return g


def make_solute(xyz, q, sigma, eps):
    """All four must be contiguous FP64 CUDA tensors (xyz shaped (n, 3))."""
    for t in (xyz, q, sigma, eps):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("solute arrays must be contiguous float64 device tensors")
    s = Solute(int(q.shape[0]), xyz.data_ptr(), q.data_ptr(), sigma.data_ptr(), eps.data_ptr())
    s._keep = (xyz, q, sigma, eps)
    return s


def n_ionic(ionic):
    return int(np.count_nonzero(np.asarray(ionic))) if ionic is not None else 0


def _grid_shape(grid):
    return (int(grid.dims[2]), int(grid.dims[1]), int(grid.dims[0]))


def potential(xyz, q, sigma, eps, sites, grid, opts: Opts, want_tail=False, out=None):
    """u[S][nz][ny][nx] (and the LJ tail constants if requested)."""
    L = lib()
    so = make_solute(xyz, q, sigma, eps)
    oc = opts.to_c()
    if out is None:
        out = torch.empty((sites.n,) + _grid_shape(grid), dtype=opts.torch_dtype, device=xyz.device)
    tail = (C.c_double * MAX_SITES)() if want_tail else None
    _check(L.rism_potential(C.byref(so), C.byref(sites), C.byref(grid), C.byref(oc), _ptr(out),
                            tail, _stream()))
    if want_tail:
        return out, np.array(tail[:sites.n])
    return out


def asymptotics(xyz, q, sites, grid, opts: Opts, eta, kappa, beta, dielectric, want_c=True,
                want_h=True, sigma=None, eps=None, c_out=None, h_out=None):
    L = lib()
    z = torch.zeros_like(q)
    so = make_solute(xyz, q, z if sigma is None else sigma, z if eps is None else eps)
    oc = opts.to_c()
    shp = _grid_shape(grid)
    ni = n_ionic(np.ctypeslib.as_array(sites.ionic, shape=(sites.n,)))
    c = c_out if (c_out is not None or not want_c) else torch.empty((sites.n,) + shp, dtype=opts.torch_dtype, device=xyz.device)
    h = None
    if want_h and ni > 0:
        h = h_out if h_out is not None else torch.empty((ni,) + shp, dtype=opts.torch_dtype, device=xyz.device)
    _check(L.rism_asymptotics(C.byref(so), C.byref(sites), C.byref(grid), C.byref(oc), eta, kappa,
                              beta, dielectric, _ptr(c), _ptr(h), _stream()))
    return c, h


def asymptotics_k(xyz, q, sigma, eps, sites, grid, opts: Opts, eta, kappa, beta, dielectric,
                  tol=0.0, want_c=True, want_h=True, outs=None):
    """Reciprocal-space c^lr(k) [S][nz][ny][nx//2+1] and h^lr(k) [n_ionic][...]
    as complex tensors (views of interleaved real buffers); ``tol`` > 0
    applies the frequency cut-off.  ``outs`` may supply the real (c, h)
    buffers of shape [...][2]."""
    L = lib()
    so = make_solute(xyz, q, sigma, eps)
    oc = opts.to_c()
    nz, ny, nx = _grid_shape(grid)
    shp = (nz, ny, nx // 2 + 1, 2)
    ni = n_ionic(np.ctypeslib.as_array(sites.ionic, shape=(sites.n,)))
    if outs is None:
        dt, dev = opts.torch_dtype, xyz.device
        c = torch.empty((sites.n,) + shp, dtype=dt, device=dev) if want_c else None
        h = torch.empty((ni,) + shp, dtype=dt, device=dev) if (want_h and ni) else None
    else:
        c, h = outs
    _check(L.rism_asymptotics_k(C.byref(so), C.byref(sites), C.byref(grid), C.byref(oc), eta,
                                kappa, beta, dielectric, float(tol), _ptr(c), _ptr(h), _stream()))
    cz = None if c is None else torch.view_as_complex(c)
    hz = None if h is None else torch.view_as_complex(h)
    return cz, hz


def initialize(xyz, q, sigma, eps, sites, grid, opts: Opts, eta, kappa, beta, dielectric,
               want_u=True, want_c=True, want_h=True, want_tail=False, outs=None,
               noalloc=False):
    """Fused u, c^lr, h^lr.  ``outs`` may supply preallocated (u, c, h).
    ``noalloc``: call rism_initialize_noalloc (direct methods; the library
    allocates nothing, its scratch is a fixed device array)."""
    L = lib()
    so = make_solute(xyz, q, sigma, eps)
    oc = opts.to_c()
    shp = _grid_shape(grid)
    ni = n_ionic(np.ctypeslib.as_array(sites.ionic, shape=(sites.n,)))
    if outs is None:
        dt, dev = opts.torch_dtype, xyz.device
        u = torch.empty((sites.n,) + shp, dtype=dt, device=dev) if want_u else None
        c = torch.empty((sites.n,) + shp, dtype=dt, device=dev) if want_c else None
        h = torch.empty((ni,) + shp, dtype=dt, device=dev) if (want_h and ni) else None
    else:
        u, c, h = outs
    tail = (C.c_double * MAX_SITES)() if want_tail else None
    fn = L.rism_initialize_noalloc if noalloc else L.rism_initialize
    _check(fn(C.byref(so), C.byref(sites), C.byref(grid), C.byref(oc), eta, kappa, beta,
              dielectric, _ptr(u), tail, _ptr(c), _ptr(h), _stream()))
    if want_tail:
        return u, c, h, np.array(tail[:sites.n])
    return u, c, h


def potential_backward(xyz, q, sigma, eps, sites, grid, opts: Opts, dL_du, need=(True,) * 4):
    """(dL/dxyz, dL/dq, dL/deps, dL/dsigma) as FP64 device tensors (None where
    not requested)."""
    L = lib()
    so = make_solute(xyz, q, sigma, eps)
    oc = opts.to_c()
    n = q.shape[0]
    dev = xyz.device
    if not dL_du.is_contiguous() or dL_du.dtype != opts.torch_dtype:
        raise ValueError("dL_du must be contiguous with the dtype of opts.out_dtype")
    dx = torch.empty((n, 3), dtype=torch.float64, device=dev) if need[0] else None
    dq = torch.empty(n, dtype=torch.float64, device=dev) if need[1] else None
    de = torch.empty(n, dtype=torch.float64, device=dev) if need[2] else None
    ds = torch.empty(n, dtype=torch.float64, device=dev) if need[3] else None
    _check(L.rism_potential_backward(C.byref(so), C.byref(sites), C.byref(grid), C.byref(oc),
                                     _ptr(dL_du), _ptr(dx), _ptr(dq), _ptr(de), _ptr(ds),
                                     _stream()))
    return dx, dq, de, ds


def compare(x, ref, ref_cap=0.0, mask=None):
    """(sum sq err, sum sq ref, max abs err, excluded, kind mismatches,
    compared) over the points where ``mask`` (uint8 device tensor, or None)
    is nonzero."""
    if ref.dtype != torch.float64 or x.numel() != ref.numel():
        raise ValueError("ref must be float64 with as many elements as x")
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != x.numel()):
        raise ValueError("mask must be uint8 with as many elements as x")
    out = (C.c_double * 6)()
    dt = DTYPES["f64"] if x.dtype == torch.float64 else DTYPES["f32"]
    _check(lib().rism_compare(_ptr(x.contiguous()), dt, _ptr(ref.contiguous()), x.numel(),
                              ref_cap, _ptr(None if mask is None else mask.contiguous()), out,
                              _stream()))
    return tuple(out)


def near_mask(xyz, grid, radius=1.0):
    """uint8 [nz][ny][nx] device tensor: 1 where every atom is >= radius away."""
    z = torch.zeros(xyz.shape[0], dtype=torch.float64, device=xyz.device)
    so = make_solute(xyz, z, z, z)
    m = torch.empty(_grid_shape(grid), dtype=torch.uint8, device=xyz.device)
    _check(lib().rism_near_mask(C.byref(so), C.byref(grid), float(radius), _ptr(m), _stream()))
    return m


def phase_times() -> dict:
    """{phase: (total ms, launches)} since the previous call (phase_events)."""
    ms = (C.c_double * len(PHASES))()
    cnt = (C.c_int64 * len(PHASES))()
    _check(lib().rism_phase_times(ms, cnt))
    return {p: (ms[i], cnt[i]) for i, p in enumerate(PHASES) if cnt[i]}


def last_stats() -> dict:
    s = Stats()
    _check(lib().rism_last_stats(C.byref(s)))
    return {k: getattr(s, k) for k, _ in Stats._fields_}


class RismPotential(torch.autograd.Function):
    """u = RismPotential.apply(xyz, q, sigma, eps, sites, grid, opts).

    forward saves only the inputs; backward calls the hand-written adjoint
    (rism_potential_backward), which recomputes the pair terms."""

    @staticmethod
    def forward(ctx, xyz, q, sigma, eps, sites, grid, opts):
        ctx.save_for_backward(xyz, q, sigma, eps)
        ctx.sites, ctx.grid, ctx.opts = sites, grid, opts
        return potential(xyz.detach().contiguous(), q.detach().contiguous(),
                         sigma.detach().contiguous(), eps.detach().contiguous(), sites, grid, opts)

    @staticmethod
    def backward(ctx, g):
        xyz, q, sigma, eps = ctx.saved_tensors
        need = ctx.needs_input_grad[:4]
        dx, dq, ds_, de = None, None, None, None
        if any(need):
            w = g.detach().to(ctx.opts.torch_dtype).contiguous()
            dx, dq, de, ds_ = potential_backward(xyz.detach().contiguous(),
                                                 q.detach().contiguous(),
                                                 sigma.detach().contiguous(),
                                                 eps.detach().contiguous(), ctx.sites, ctx.grid,
                                                 ctx.opts, w,
                                                 need=(need[0], need[1], need[3], need[2]))
        return dx, dq, ds_, de, None, None, None


def sites_from(ws: "_wl.Sites"):
    return make_sites(ws.q, ws.sigma, ws.eps, ws.ionic)


def grid_from(g: "_wl.Grid"):
    return make_grid(g.origin, g.spacing, g.dims)


def solute_to_device(sol: "_wl.Solute", device="cuda"):
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
    return f(sol.xyz.reshape(-1, 3)), f(sol.q), f(sol.sigma), f(sol.eps)
