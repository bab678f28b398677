"""Golden fixtures: the paper's printed solvent model and an oracle
regression file written by tests/golden/make_golden.py (oracle only)."""
import importlib.util
import json
import os

import numpy as np

from paper_2109_09772_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_solvent_model_matches_paper():
    g = json.load(open(os.path.join(GOLD, "solvent_model.json")))
    assert W.TEMPERATURE == g["temperature_K"]
    assert W.DIELECTRIC == g["dielectric"]
    assert W.WATER_MOLAR == g["water_molar"]
    assert W.SALT_MOLAR == g["nacl_molar"]
    # Debye kappa of 0.1 M 1:1 salt at the paper's T and dielectric
    assert abs(W.debye_kappa() - 0.10399) < 5e-6
    assert abs(W.beta() - 1.6878066) < 1e-6


def test_oracle_regression(oracle):
    spec = importlib.util.spec_from_file_location("mk", os.path.join(GOLD, "make_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    ref = json.load(open(os.path.join(GOLD, "oracle_tiny.json")))
    now = mk.compute(ref["case"])
    for k, v in ref["values"].items():
        np.testing.assert_allclose(np.array(now[k]), np.array(v), rtol=1e-13, atol=0, err_msg=k)
