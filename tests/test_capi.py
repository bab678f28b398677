"""The C ABI loads, exports every entry point include/rism.h declares, and
rejects invalid arguments on the host before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rism.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rism_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("rism_potential", "rism_asymptotics", "rism_potential_backward", "rism_last_error",
              "rism_initialize", "rism_default_opts", "rism_compare", "rism_last_stats",
              "rism_asymptotics_k"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2109_09772_amd import api
    L = api.lib()
    for n in _declared():
        assert hasattr(L, n), n
    out = C.create_string_buffer(b"")
    assert L.rism_last_error() is not None


def test_default_opts():
    from paper_2109_09772_amd import api
    o = api.OptsC()
    api.lib().rism_default_opts(C.byref(o))
    assert o.method == api.METHODS["treecode_cp"] and o.out_dtype == 0 and o.degree == 8
    assert o.theta == pytest.approx(0.6) and o.lj_cutoff == 9.0
    assert o.coulomb_k == pytest.approx(332.0522173)


def _call_potential(solute, sites, grid, opts, u=C.c_void_p(16)):
    from paper_2109_09772_amd import api
    L = api.lib()
    return L.rism_potential(C.byref(solute) if solute is not None else None,
                            C.byref(sites) if sites is not None else None,
                            C.byref(grid) if grid is not None else None,
                            C.byref(opts) if opts is not None else None, u, None, None)


def _valid():
    from paper_2109_09772_amd import api
    so = api.Solute(4, 16, 16, 16, 16)       # fake device pointers: never dereferenced
    si = api.make_sites([-0.834, 0.417], [3.15, 0.4], [0.152, 0.046])
    g = api.make_grid([0, 0, 0], 0.5, 8)
    o = api.OptsC()
    api.lib().rism_default_opts(C.byref(o))
    return so, si, g, o


@pytest.mark.parametrize("mutate, frag", [
    (lambda so, si, g, o: setattr(so, "n", -1), "n < 0"),
    (lambda so, si, g, o: setattr(so, "xyz", None), "null solute"),
    (lambda so, si, g, o: setattr(si, "n", 0), "sites"),
    (lambda so, si, g, o: setattr(si, "n", 9), "sites"),
    (lambda so, si, g, o: g.dims.__setitem__(1, 0), "dims"),
    (lambda so, si, g, o: g.spacing.__setitem__(2, -0.5), "spacing"),
    (lambda so, si, g, o: g.spacing.__setitem__(0, float("nan")), "spacing"),
    (lambda so, si, g, o: g.origin.__setitem__(0, float("inf")), "origin"),
    (lambda so, si, g, o: setattr(o, "method", 7), "method"),
    (lambda so, si, g, o: setattr(o, "out_dtype", 3), "out_dtype"),
    (lambda so, si, g, o: setattr(o, "theta", 1.0), "theta"),
    (lambda so, si, g, o: setattr(o, "theta", 0.0), "theta"),
    (lambda so, si, g, o: setattr(o, "degree", 0), "degree"),
    (lambda so, si, g, o: setattr(o, "degree", 17), "degree"),
    (lambda so, si, g, o: setattr(o, "leaf_size", 0), "leaf"),
    (lambda so, si, g, o: setattr(o, "batch_edge", 6), "batch"),
    (lambda so, si, g, o: setattr(o, "lj_tol", -1.0), "lj_tol"),
    (lambda so, si, g, o: setattr(o, "coulomb_k", float("nan")), "coulomb"),
    (lambda so, si, g, o: (setattr(o, "method", 4), setattr(o, "degree", 13)), "Taylor order"),
])
def test_host_validation(mutate, frag):
    from paper_2109_09772_amd import api
    so, si, g, o = _valid()
    mutate(so, si, g, o)
    rc = _call_potential(so, si, g, o)
    assert rc == api.RISM_E_INVALID
    assert frag in api.lib().rism_last_error().decode()


def test_null_structs_and_outputs():
    from paper_2109_09772_amd import api
    so, si, g, o = _valid()
    assert _call_potential(None, si, g, o) == api.RISM_E_INVALID
    assert _call_potential(so, si, g, None) == api.RISM_E_INVALID
    L = api.lib()
    assert L.rism_potential(C.byref(so), C.byref(si), C.byref(g), C.byref(o), None, None,
                            None) == api.RISM_E_INVALID
    assert L.rism_asymptotics(C.byref(so), C.byref(si), C.byref(g), C.byref(o), 1.0, 0.1, 1.0,
                              78.0, None, None, None) == api.RISM_E_INVALID
    assert L.rism_compare(None, 0, None, 5, 0.0, None, None, None) == api.RISM_E_INVALID
    assert L.rism_near_mask(C.byref(so), C.byref(g), 1.0, None, None) == api.RISM_E_INVALID
    assert L.rism_near_mask(C.byref(so), C.byref(g), -1.0, C.c_void_p(16),
                            None) == api.RISM_E_INVALID
    assert L.rism_initialize_noalloc(None, C.byref(si), C.byref(g), C.byref(o), 1.0, 0.1, 1.0,
                                     78.0, None, None, None, None, None) == api.RISM_E_INVALID


def test_site_parameter_validation():
    from paper_2109_09772_amd import api
    so, _, g, o = _valid()
    si = api.make_sites([-0.834, 0.417], [3.15, -0.4], [0.152, 0.046])
    assert _call_potential(so, si, g, o) == api.RISM_E_INVALID
    si = api.make_sites([-0.834, float("nan")], [3.15, 0.4], [0.152, 0.046])
    assert _call_potential(so, si, g, o) == api.RISM_E_INVALID


def test_reciprocal_asymptotics_validation():
    from paper_2109_09772_amd import api
    so, si, g, o = _valid()
    L = api.lib()
    args = (C.byref(so), C.byref(si), C.byref(g), C.byref(o))
    fake = C.c_void_p(16)
    assert L.rism_asymptotics_k(*args, 1.0, 0.1, 1.0, 78.0, 0.0, None, None,
                                None) == api.RISM_E_INVALID
    assert "no output" in L.rism_last_error().decode()
    assert L.rism_asymptotics_k(*args, 0.0, 0.1, 1.0, 78.0, 0.0, fake, None,
                                None) == api.RISM_E_INVALID
    assert "eta" in L.rism_last_error().decode()
    assert L.rism_asymptotics_k(*args, 1.0, -0.1, 1.0, 78.0, 0.0, fake, None,
                                None) == api.RISM_E_INVALID
    assert L.rism_asymptotics_k(*args, 1.0, 0.1, 1.0, 78.0, float("nan"), fake, None,
                                None) == api.RISM_E_INVALID
    assert "tol" in L.rism_last_error().decode()


def test_taylor_treecode_has_no_adjoint():
    """The Taylor-recurrence treecode is forward only: its backward call
    fails before touching any device memory."""
    from paper_2109_09772_amd import api
    so, si, g, o = _valid()
    o.method = 4
    o.degree = 6
    L = api.lib()
    rc = L.rism_potential_backward(C.byref(so), C.byref(si), C.byref(g), C.byref(o),
                                   C.c_void_p(16), C.c_void_p(16), None, None, None, None)
    assert rc == api.RISM_E_UNSUPPORTED
    assert "Taylor" in L.rism_last_error().decode()
