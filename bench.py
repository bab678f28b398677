"""Benchmark of the 3D-RISM initialisation hot path on one MI355X.

A step is one initialisation of the 2,500-atom / 128^3-grid / 4-site
workload (u for all sites with a 9 A LJ cut-off, c^lr for all sites, h^lr for
the two ionic sites), computed by the FP32 path selected with --method
(default: the cluster-particle treecode, theta 0.6, degree 8).  Inputs are
resident in HBM before the timed region.

Also measured (outside the timed steps, reported in the same JSON line):
the GPU FP64 direct sum of the same quantities (the comparison of the
metric), the error of the FP32 path against it, the adjoint, the per-phase
durations from HIP events recorded by the library on the call's stream
(roofline of the dominant kernel), and the FP64 CPU oracle on a bounded
sample of grid points (cpu_baseline).
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

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.  One wave64 VALU instruction
# per SIMD every 4 clocks is 39.3e12 lane-ops/s (78.6 TFLOP/s counting an FMA
# as 2); the SIMD can issue a second VALU instruction in the same cycle (dual
# issue, counted by SQ_ACTIVE_INST_VALU2), which doubles that to the
# published FP32 vector peak of 157.3 TFLOP/s, the roofline used here.
VALU_LANE_OPS = 256 * 64 * 2.4e9
FP32_VALU_PEAK_TFLOPS = 157.3
FP32_VALU_SINGLE_ISSUE_TFLOPS = 2 * VALU_LANE_OPS / 1e12   # 78.6
# dense FP32 matrix-core (MFMA) peak, published: the same 157.3 TFLOP/s
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
ROOT_PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")


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


def flops_per_pair_short_f32(ns, asym, lj):
    """A short-range pair of the treecode leaf kernel (the atom's far field
    comes from proxies): hi/lo differences 6, d^2 5, 1/d 1; LJ as above; the
    smeared kernels' range test and exp2 of the Yukawa term: d 1, scale 1,
    exp2 1 (the table lookup of the pairs within R_s is not counted)."""
    f = 6 + 5 + 1
    if asym:
        f += 3
    if lj:
        f += 3 + 4 * ns
    return f


def flops_per_far_pair(asym):
    """One (atom, proxy) pair of the far-field sweep: differences 3, d^2 5,
    1/d 1, Coulomb 2; Yukawa: d 1, scale 1, exp2 1, accumulate 2."""
    return 11 + (5 if asym else 0)


def leaf_interp_flops(points, blocks, degree, batch, ncomp):
    """FP64 interpolation of the level-1 proxy values onto the grid: per
    component the two block-level contractions and the per-point one."""
    n1 = degree + 1
    per_block = 2 * (n1 ** 3 * batch + n1 ** 2 * batch ** 2)
    return ncomp * (2 * n1 * points + per_block * blocks)


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/<kernel>_<workload>_counters.txt, or None when it is absent or
    was taken from other kernel sources than the ones in the tree."""
    path = os.path.join(ROOT_PROFILES, f"{kernel}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    files = kv.get("sources", "").split()
    if not files or source_hash(files) != kv.get("sources_sha256"):
        return None
    return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
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
    ap.add_argument("--no-recip", action="store_true",
                    help="skip the reciprocal-space asymptotics timing")
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
        print("bench.py runs on exactly one GPU: the initialisation shards the grid into "
              "blocks that need no communication, and the benchmark measures one GPU's share.",
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
    # interaction counts (opt-in device counters, outside the timed steps)
    step(api.Opts(**{**opts.__dict__, "stats": True}))
    torch.cuda.synchronize()
    stats = api.last_stats()

    # per-kernel durations from the library's own HIP events (same stream)
    ev_opts = api.Opts(**{**opts.__dict__, "phase_events": True})
    api.phase_times()
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step(ev_opts)
    torch.cuda.synchronize()
    # per phase: (ms per timed launch, launches per step, ms per step)
    phases = {k: (v[0] / v[1], v[1] / args.steps, v[0] / args.steps)
              for k, v in api.phase_times().items()}
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
        "phases_ms": {k: round(v[2], 4) for k, v in phases.items()},
        "stats": {k: stats[k] for k in ("pairs_direct", "pairs_far", "pairs_short", "n_nodes",
                                        "n_batches")},
    }

    # roofline of the dominant kernel: algorithmic flops of each modelled
    # phase (from the library's interaction counts) over its measured time
    ni_asym = True
    work = {}
    if "direct_f32" in phases:
        work["direct_f32"] = ("k_direct_f32",
                              flops_per_pair_direct_f32(st.n, ni_asym, True) * n * m)
    if args.method == "treecode_cp":
        B = 8
        blocks = -(-int(g.dims[0]) // B) * -(-int(g.dims[1]) // B) * -(-int(g.dims[2]) // B)
        work["eval"] = ("k_cp_leaf",
                        flops_per_pair_direct_f32(st.n, True, True) * stats["pairs_direct"]
                        + flops_per_pair_short_f32(st.n, True, True) * stats["pairs_short"]
                        + leaf_interp_flops(m, blocks, args.degree, B, 2))
        # the far sweep runs along proxy x-lines for 8, 9 and 11 nodes per axis
        sweep = "k_cp_sweep_lines" if args.degree + 1 in (8, 9, 11) else "k_cp_sweep"
        work["upward"] = (sweep, flops_per_far_pair(True) * stats["pairs_far"])
    elif args.method == "treecode":
        work["eval"] = ("k_tree_eval",
                        flops_per_pair_direct_f32(st.n, True, True) * stats["pairs_direct"]
                        + flops_per_far_pair(True) * stats["pairs_far"])
    rl = {}
    for ph, (kern, fl) in work.items():
        if ph not in phases:
            continue
        ms_ph = phases[ph][0]
        ach = fl / (ms_ph * 1e-3) / 1e12
        rl[ph] = {"kernel": kern, "flops": fl, "ms": ms_ph, "achieved": ach,
                  "frac": ach / FP32_VALU_PEAK_TFLOPS}
    dom = max(rl, key=lambda k: rl[k]["ms"]) if rl else None
    if dom is not None:
        d = rl[dom]
        traffic = counter_traffic(d["kernel"], wl.name)
        result["roofline"] = {
            "kernel": d["kernel"], "phase": dom, "bound": "alu", "achieved": d["achieved"],
            "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": d["frac"],
            "traffic": traffic, "kernel_ms": d["ms"],
            "peak_single_issue": FP32_VALU_SINGLE_ISSUE_TFLOPS,
            "note": "algorithmic flops (FMA 2, rsqrt/exp2 1) over the kernel time; the kernel "
                    "issues VALU instructions at the SIMDs' single-issue rate (rocprofv3 "
                    "instruction counters in profiles/), so the remaining gap to the peak is the "
                    "flop model against instruction count and the dual issue or packed FP32 the "
                    "peak assumes",
            "other_phases": {k: {kk: v[kk] for kk in ("kernel", "achieved", "frac", "ms")}
                             for k, v in rl.items() if k != dom}}
    else:
        result["roofline"] = {"kernel": dominant, "bound": "alu", "achieved": None,
                              "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                              "traffic": None}

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

    # reciprocal-space asymptotics (the next row after the real-space path):
    # c^lr(k) and h^lr(k) on the half grid, frequency cut-off at tol 1e-6
    if not args.no_recip:
        ck = (torch.empty((st.n, shp[0], shp[1], shp[2] // 2 + 1, 2), device=dev),
              torch.empty((ni, shp[0], shp[1], shp[2] // 2 + 1, 2), device=dev) if ni else None)
        ok = api.Opts(**{**opts.__dict__})
        api.asymptotics_k(xyz, q, s, e, sites, grid, ok, eta, kap, beta, diel, tol=1e-6, outs=ck)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            api.asymptotics_k(xyz, q, s, e, sites, grid, ok, eta, kap, beta, diel, tol=1e-6,
                              outs=ck)
        torch.cuda.synchronize()
        tk = (time.perf_counter() - t0) / reps
        terms = n * shp[0] * shp[1] * (shp[2] // 2 + 1)
        # the matrix-core kernel's own duration (HIP events on the call's stream):
        # it sums the full 32-column tiles of the half grid, 8 flops per
        # (atom, k-point) term (complex multiply-add as 4 FP32 MFMA products)
        ok.phase_events = True
        api.phase_times()
        api.asymptotics_k(xyz, q, s, e, sites, grid, ok, eta, kap, beta, diel, tol=1e-6, outs=ck)
        ph = api.phase_times()
        ok.phase_events = False
        nxm = (shp[2] // 2 + 1) // 32 * 32
        mf_ms = ph["recip"][0] / ph["recip"][1]
        mf_tf = 8.0 * n * nxm * shp[1] * shp[0] / (mf_ms * 1e-3) / 1e12
        result["asymptotics_k"] = {"time_s": tk, "tol": 1e-6,
                                   "gterm_per_s": terms / tk / 1e9,
                                   "note": "structure-factor terms (atom, k-point) per second "
                                           "over the whole half grid",
                                   "roofline": {"kernel": "k_asym_k_mfma", "bound": "mfma",
                                                "achieved": mf_tf, "peak": FP32_MFMA_PEAK_TFLOPS,
                                                "unit": "TFLOP/s",
                                                "frac": mf_tf / FP32_MFMA_PEAK_TFLOPS,
                                                "kernel_ms": mf_ms}}
        del ck

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
