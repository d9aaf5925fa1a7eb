"""Helpers shared by the tests: starting points and comparisons."""
import numpy as np

from synth.grids import power_flow_start
from oracle import acopf


def start_point(g, pi_scale=0.0, seed=0):
    s = power_flow_start(g)
    x = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    rng = np.random.default_rng(seed)
    pi = rng.standard_normal((g.n_line, 4)) * pi_scale
    pi[:, 2:] = -np.abs(pi[:, 2:])
    return x, pi


def rel_err(a, b):
    """max |a - b| / max |b| (norm-wise relative error of an array)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(float(np.abs(b).max(initial=0.0)), 1e-300)
    return float(np.abs(a - b).max(initial=0.0)) / scale
