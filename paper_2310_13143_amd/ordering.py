"""Locality order of a grid's components for the sweep kernels.

The bus phase gathers each line end's coupling values and the line phase
reads the bus values of both ends, so a sweep runs fastest when buses that
share lines sit close in memory and lines are stored in the order of their
end buses.  The library keeps the caller's numbering; a grid given in an
arbitrary order can be renumbered once, before setup, with the permutations
returned here: buses in reverse Cuthill-McKee order of the network graph
(bandwidth-reducing), lines sorted by (lower, higher) end bus, generators by
bus.  Results are mapped back with the same permutations.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

BUS_FIELDS = ("vmin", "vmax", "pd", "qd", "gsh", "bsh")
LINE_FIELDS = ("gii", "bii", "gij", "bij", "gji", "bji", "gjj", "bjj", "smax_ij", "smax_ji", "r", "x", "bc", "tap")
GEN_FIELDS = ("pmin", "pmax", "qmin", "qmax", "cost2", "cost1")


def locality_order(n_bus: int, f: np.ndarray, t: np.ndarray, gen_bus: np.ndarray):
    """(bus_perm, line_perm, gen_perm): new component k is old component
    perm[k]."""
    f, t = np.asarray(f), np.asarray(t)
    a = sp.coo_matrix((np.ones(2 * f.size), (np.r_[f, t], np.r_[t, f])), shape=(n_bus, n_bus)).tocsr()
    bus_perm = np.asarray(reverse_cuthill_mckee(a, symmetric_mode=True), dtype=np.int64)
    inv = np.empty(n_bus, dtype=np.int64)
    inv[bus_perm] = np.arange(n_bus)
    fn, tn = inv[f], inv[t]
    line_perm = np.lexsort((np.maximum(fn, tn), np.minimum(fn, tn)))
    gen_perm = np.argsort(inv[np.asarray(gen_bus)], kind="stable")
    return bus_perm, line_perm, gen_perm


def reorder(grid, bus_perm, line_perm, gen_perm):
    """A copy of a grid description (a dataclass with the fields of
    DeviceGrid's input) renumbered by the permutations."""
    inv = np.empty(grid.n_bus, dtype=np.int64)
    inv[bus_perm] = np.arange(grid.n_bus)
    kw = {}
    for n in BUS_FIELDS:
        kw[n] = np.asarray(getattr(grid, n))[bus_perm]
    for n in LINE_FIELDS:
        v = getattr(grid, n, None)
        if v is not None:
            kw[n] = np.asarray(v)[line_perm]
    for n in GEN_FIELDS:
        kw[n] = np.asarray(getattr(grid, n))[gen_perm]
    kw["f"] = inv[np.asarray(grid.f)[line_perm]]
    kw["t"] = inv[np.asarray(grid.t)[line_perm]]
    kw["gbus"] = inv[np.asarray(grid.gbus)[gen_perm]]
    kw["ref"] = int(inv[grid.ref])
    return dataclasses.replace(grid, **kw)
