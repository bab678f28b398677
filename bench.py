"""Benchmark of the 3D-RISM initialisation hot path on one MI355X.

A step is one initialisation of the 2,500-atom / 128^3-grid / 4-site
workload (u for all sites with a 9 A LJ cut-off, c^lr for all sites, h^lr for
the two ionic sites), computed by the FP32 path selected with --method
(default: the particle-cluster treecode, theta 0.7, degree 8).  Inputs are
resident in HBM before the timed region.

Also measured (outside the timed steps, reported in the same JSON line):
the GPU FP64 direct sum of the same quantities (the comparison of the
metric), the error of the FP32 path against it, the adjoint, the dominant
kernel's duration from HIP events recorded by the library on the call's
stream (roofline), and the FP64 CPU oracle on a bounded sample of grid points
(cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3D-RISM init time (s) & Gpair-interactions/s, FP32 treecode vs FP64 direct @1e-6"
UNIT = "Gpair-interactions/s"

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.  Packed FP32 instructions are
# disabled in this build, so an FP32 VALU lane retires one op per clock:
# 256*64*2.4e9 = 39.3e12 lane-ops/s, 78.6 TFLOP/s counting an FMA as 2.
VALU_LANE_OPS = 256 * 64 * 2.4e9
FP32_VALU_PEAK_TFLOPS = 2 * VALU_LANE_OPS / 1e12       # 78.6 (non-packed)
FP32_VALU_PUBLISHED_TFLOPS = 157.3                     # with packed FP32
HBM_PEAK_GBS = 8000.0


def flops_per_pair_direct_f32(ns, asym, lj):
    """Algorithmic FP32 work of one (grid point, atom) pair in the long-range
    loop (FMA = 2 flops, rsqrt/exp2 = 1 each): hi/lo differences 6, d^2 5,
    1/d 1, Coulomb 2; Yukawa: d 1, scale 1, exp2 1, accumulate 2; LJ: 1/d^2,
    1/d^6 3, per site (A r6 - B) r6 accumulated 4."""
    f = 6 + 5 + 1 + 2
    if asym:
        f += 5
    if lj:
        f += 3 + 4 * ns
    return f


def issue_slots_per_pair_direct_f32(ns, asym, lj):
    """Ideal VALU issue slots of the same pair (a transcendental takes 4)."""
    s = 6 + 3 + 4 + 2 + 2 + 2   # diffs, d^2, rsq, select, Coulomb, hit flag
    if asym:
        s += 2 + 4 + 1 + 1      # d, scale, exp2, fma, branch test
    if lj:
        s += 3 + 4 * ns
    return s


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--method", default="treecode_cp",
                    choices=["treecode", "treecode_cp", "direct_f32c"])
    ap.add_argument("--theta", type=float, default=0.6)
    ap.add_argument("--degree", type=int, default=8)
    ap.add_argument("--lj-cutoff", type=float, default=9.0)
    ap.add_argument("--workload", default="protein_2500",
                    choices=["protein_2500", "small_ball", "tubulin_14000"])
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 direct comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a device buffer of this size (MiB) once: a "
                         "kernel of known traffic for scaling HBM byte counters")
    return ap.parse_args()


def cpu_baseline(wl, lj_cutoff, target_s):
    """The FP64 oracle (plain direct sum, OpenMP) on seeded random grid points
    of the same workload: u (cut-off as in the GPU run), c^lr and h^lr."""
    from oracle import oracle
    from paper_2109_09772_amd import workloads as W
    oracle.build(force=False)
    sol, st, g = wl.solute, wl.sites, wl.grid
    rc = oracle.rcut_table(sol.sigma, sol.eps, st.sigma, st.eps, rcut=lj_cutoff)

    def run(npts, seed):
        idx = W.sample_points(g, npts, seed)
        pts = g.origin + idx * g.spacing
        t0 = time.perf_counter()
        oracle.potential_points(sol.xyz, sol.q, sol.sigma, sol.eps, st.q, st.sigma, st.eps, pts,
                                W.COULOMB_K, rc)
        oracle.asymptotics_points(sol.xyz, sol.q, st.q, st.ionic, pts, W.COULOMB_K, W.ETA,
                                  W.debye_kappa(), W.beta(), W.DIELECTRIC)
        return time.perf_counter() - t0

    n0 = 2000
    t0 = run(n0, 1)
    npts = int(min(g.npoints, max(n0, n0 * target_s / max(t0, 1e-3))))
    t = run(npts, 2)
    return {"value": sol.n * npts / t / 1e9, "unit": UNIT, "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{npts} seeded random grid points of the {g.dims.tolist()} grid, all "
                      f"{sol.n} atoms, u ({st.n} sites, {lj_cutoff} A LJ cut-off) + c^lr + h^lr, "
                      f"FP64, {t:.1f} s",
            "seconds": t}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the initialisation shards the grid with no "
              "communication, and this build measures one GPU's share (see DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2109_09772_amd import api
    from paper_2109_09772_amd import workloads as W

    wl = getattr(W, args.workload)()
    sol, st, g = wl.solute, wl.sites, wl.grid
    eta, kap, beta, diel = W.ETA, W.debye_kappa(), W.beta(), W.DIELECTRIC
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    xyz, q, s, e = api.solute_to_device(sol, dev)
    sites, grid = api.sites_from(st), api.grid_from(g)
    shp = (int(g.dims[2]), int(g.dims[1]), int(g.dims[0]))
    ni = int(st.ionic.sum())
    n, m = sol.n, g.npoints

    opts = api.Opts(method=args.method, out_dtype="f32", lj_cutoff=args.lj_cutoff,
                    theta=args.theta, degree=args.degree, device_check=False)
    outs = (torch.empty((st.n,) + shp, device=dev), torch.empty((st.n,) + shp, device=dev),
            torch.empty((ni,) + shp, device=dev) if ni else None)

    def step(o):
        api.initialize(xyz, q, s, e, sites, grid, o, eta, kap, beta, diel, outs=outs)

    for _ in range(args.warmup):
        step(opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(opts)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_per_step = 1e3 * t_total / args.steps
    stats = api.last_stats()

    # per-kernel durations from the library's own HIP events (same stream)
    ev_opts = api.Opts(**{**opts.__dict__, "phase_events": True})
    api.phase_times()
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step(ev_opts)
    torch.cuda.synchronize()
    phases = {k: (v[0] / v[1], v[1] / args.steps) for k, v in api.phase_times().items()}
    dominant = max(phases, key=lambda k: phases[k][0] * phases[k][1])

    result = {
        "metric": METRIC,
        "value": n * m / (ms_per_step * 1e-3) / 1e9,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "atoms": n, "grid": [int(v) for v in g.dims],
                   "spacing_A": float(g.spacing[0]), "sites": st.names,
                   "outputs": f"u x{st.n} (LJ cut-off {args.lj_cutoff} A), c_lr x{st.n}, "
                              f"h_lr x{ni}",
                   "method": args.method, "theta": args.theta, "degree": args.degree,
                   "eta_A": eta, "kappa_per_A": kap},
        "init_time_s": ms_per_step * 1e-3,
        "phases_ms": {k: round(v[0], 4) for k, v in phases.items()},
        "stats": {k: stats[k] for k in ("pairs_direct", "pairs_far", "pairs_short", "n_nodes",
                                        "n_batches")},
    }

    # roofline of the dominant kernel
    ms_dom, per_step = phases[dominant]
    if dominant == "direct_f32":
        fl = flops_per_pair_direct_f32(st.n, True, True) * n * m
        slots = issue_slots_per_pair_direct_f32(st.n, True, True) * n * m
        achieved = fl / (ms_dom * 1e-3) / 1e12
        result["roofline"] = {
            "kernel": "k_direct_f32", "bound": "alu", "achieved": achieved,
            "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_VALU_PEAK_TFLOPS,
            "traffic": None, "issue_frac": slots / (ms_dom * 1e-3) / VALU_LANE_OPS,
            "peak_published_packed": FP32_VALU_PUBLISHED_TFLOPS, "kernel_ms": ms_dom}
    else:
        result["roofline"] = {"kernel": dominant, "bound": "alu", "achieved": None,
                              "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                              "traffic": None, "kernel_ms": ms_dom}

    # FP64 direct: the comparison of the metric, and the accuracy reference
    if not args.no_f64:
        o64 = api.Opts(method="direct_f64", out_dtype="f64", lj_cutoff=args.lj_cutoff,
                       device_check=False)
        refs = (torch.empty((st.n,) + shp, device=dev, dtype=torch.float64),
                torch.empty((st.n,) + shp, device=dev, dtype=torch.float64),
                torch.empty((ni,) + shp, device=dev, dtype=torch.float64) if ni else None)
        api.initialize(xyz, q, s, e, sites, grid, o64, eta, kap, beta, diel, outs=refs)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            api.initialize(xyz, q, s, e, sites, grid, o64, eta, kap, beta, diel, outs=refs)
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - t0) / reps
        step(opts)
        torch.cuda.synchronize()
        errs = {}
        for name, x, r in zip("uch", outs, refs):
            if x is None:
                continue
            worst = 0.0
            for k in range(x.shape[0]):
                se, sr, mx, excl, mism = api.compare(x[k], r[k], ref_cap=1e30)
                worst = max(worst, (se / sr) ** 0.5 if sr > 0 else 0.0)
                if mism:
                    worst = float("inf")
            errs[name] = worst
        result["fp64_direct"] = {"init_time_s": t64, "gpair_per_s": n * m / t64 / 1e9}
        result["speedup_vs_fp64_direct"] = t64 / (ms_per_step * 1e-3)
        result["rel_l2_vs_fp64_direct"] = errs
        del refs

    if not args.no_adjoint:
        w = torch.rand((st.n,) + shp, device=dev, generator=torch.Generator(dev).manual_seed(4))
        w *= torch.as_tensor(st.rho, device=dev, dtype=torch.float32).view(-1, 1, 1, 1) * 3.0
        ao = api.Opts(**{**opts.__dict__})
        try:
            api.potential_backward(xyz, q, s, e, sites, grid, ao, w)
        except api.RismError as err:
            if err.code != api.RISM_E_UNSUPPORTED:
                raise
            ao = api.Opts(**{**opts.__dict__, "method": "direct_f32c"})
            api.potential_backward(xyz, q, s, e, sites, grid, ao, w)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            api.potential_backward(xyz, q, s, e, sites, grid, ao, w)
        torch.cuda.synchronize()
        result["adjoint"] = {"method": ao.method, "time_s": (time.perf_counter() - t0) / reps}

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, args.lj_cutoff, args.cpu_seconds)

    if args.copy_probe_mb > 0:
        nel = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(nel, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_probe_bytes"] = {"read": nel * 4, "write": nel * 4}

    print(json.dumps(result))


if __name__ == "__main__":
    main()
