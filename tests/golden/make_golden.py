"""Writes oracle_tiny.json: oracle outputs for a fixed hand-placed input.

Calls only the oracle.  Rerun (python tests/golden/make_golden.py) only when
a change to the oracle's arithmetic is justified by a passage of the paper;
the regression test then flags every other change."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import oracle  # noqa: E402

CASE = {
    "xyz": [[0.1, 0.2, -0.3], [1.4, -0.7, 0.9], [-1.1, 1.3, 0.4]],
    "q": [0.5, -0.8, 0.3],
    "sigma": [3.0, 1.8, 2.6],
    "eps": [0.1, 0.05, 0.15],
    "site_q": [-0.834, 0.417, 1.0, -1.0],
    "site_sigma": [3.15, 0.4, 2.4, 4.4],
    "site_eps": [0.152, 0.046, 0.09, 0.1],
    "site_ionic": [0, 0, 1, 1],
    "points": [[2.0, 0.0, 0.0], [0.0, -2.5, 1.0], [3.0, 3.0, 3.0], [0.6, 0.1, 0.2], [9.5, -1.0, 0.5]],
    "kc": 332.0522173, "eta": 1.0, "kappa": 0.10399, "beta": 1.6878066, "diel": 78.44,
    "rcut": 9.0,
}


def compute(case):
    rc = oracle.rcut_table(case["sigma"], case["eps"], case["site_sigma"], case["site_eps"],
                           rcut=case["rcut"])
    args = (case["xyz"], case["q"], case["sigma"], case["eps"], case["site_q"],
            case["site_sigma"], case["site_eps"])
    u = oracle.potential_points(*args, case["points"], case["kc"])
    ucut = oracle.potential_points(*args, case["points"], case["kc"], rc)
    c, h = oracle.asymptotics_points(case["xyz"], case["q"], case["site_q"], case["site_ionic"],
                                     case["points"], case["kc"], case["eta"], case["kappa"],
                                     case["beta"], case["diel"])
    tail = oracle.lj_tail(case["sigma"], case["eps"], case["site_sigma"], case["site_eps"], rc)
    w = np.linspace(0.1, 1.0, 4 * len(case["points"])).reshape(4, -1)
    g = oracle.backward_points(*args, case["points"], w, case["kc"])
    return {"u": u.tolist(), "u_cut9": ucut.tolist(), "c_lr": c.tolist(), "h_lr": h.tolist(),
            "lj_tail_cut9": tail.tolist(), "grad_xyz": g[0].tolist(), "grad_q": g[1].tolist(),
            "grad_eps": g[2].tolist(), "grad_sigma": g[3].tolist()}


if __name__ == "__main__":
    oracle.build(force=False)
    out = {"case": CASE, "values": compute(CASE)}
    with open(os.path.join(HERE, "oracle_tiny.json"), "w") as f:
        json.dump(out, f, indent=1)
