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


# Columns whose largest magnitude is below COL_FLOOR times the array's are
# compared against that floor (a column of zeros is checked in absolute terms
# at the array's scale).
COL_FLOOR = 1e-6


def rel_err_cols(a, b):
    """Largest over the columns of a 2-D array (each coupling or field on
    its own scale) of max |a - b| / max |b| in the column, the column scale
    floored at COL_FLOOR x the array's largest magnitude; 1-D arrays are one
    column."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        a, b = a[:, None], b[:, None]
    top = max(float(np.abs(b).max(initial=0.0)), 1e-300)
    scale = np.maximum(np.abs(b).max(axis=0, initial=0.0), COL_FLOOR * top)
    return float((np.abs(a - b).max(axis=0, initial=0.0) / scale).max(initial=0.0))
