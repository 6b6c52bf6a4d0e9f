import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def golden_problem(name):
    """Structured arrays of a hand-derived fixture as float64 numpy arrays."""
    g = load_golden(name)
    p = {}
    N = g["nx"] * g["ny"]
    m = g["L"] + 3
    p["s_diag"] = np.array(g["s_diag"], dtype=np.float64).reshape(N, m)
    p["s_sub"] = np.array(g["s_sub"], dtype=np.float64).reshape(N, g["L"] - 1)
    p["s_sup"] = np.array(g["s_sup"], dtype=np.float64).reshape(N, g["L"] - 1)
    p["s_flow"] = np.array(g["s_flow"], dtype=np.float64).reshape(N, 6)
    p["s_nbr"] = np.array(g["s_nbr"], dtype=np.float64).reshape(N, 4, m)
    p["u"] = np.array(g["u"], dtype=np.float64).reshape(N, 5, m)
    p["v"] = np.array(g["v"], dtype=np.float64).reshape(N, 5, m)
    return g, p


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
