"""Seeded synthetic power grids (input generation only).

This module draws the network data the ACOPF model of Section III-A takes as
parameters: bus demands and voltage limits, branch admittances in the
per-branch pi-model, thermal limits, generator limits and costs.  It holds no
arithmetic of the SQP/ADMM method itself; both the CPU oracle and the GPU path
take its output as input.

Recipes (all quantities per unit on a 100 MVA base):

* branch series impedance ``r ~ U[0.005, 0.05]``, ``x = r * U[3, 10]``, line
  charging ``b ~ U[0, 0.05]``; optional off-nominal tap ``tau ~ U[0.95, 1.05]``
  on a fraction of branches (from side), no phase shifters;
* every bus carries a load ``P ~ U[0.1, 0.5]`` with power factor
  ``U[0.9, 0.98]``; voltage magnitude limits ``[0.94, 1.06]``; no shunts
  unless ``shunt_scale`` is given (test grids use it to exercise the shunt
  terms of the balance constraints);
* generators on distinct random buses, the reference bus always among them;
  ``P_max`` = demand of the generator's graph-Voronoi cell (the buses closer
  to it than to any other generator, in hops) divided by ``load_factor``
  (default 0.6), so total demand is 60% of capacity; ``P_min = 0``,
  ``Q in [-0.5, 0.5] * P_max``; MATPOWER-style costs ``c2 ~ U[0.001, 0.05]``
  $/MW^2h, ``c1 ~ U[10, 40]`` $/MWh converted to per-unit coefficients
  ``cost2 = c2 * 100^2`` and ``cost1 = c1 * 100`` so that
  ``f(p) = cost2 p^2 + cost1 p`` with ``p`` in per unit;
* thermal limits ``s_max = max(2 |f_DC|, 0.1)`` from a DC power flow of the
  cell dispatch (each generator serves the demand of its cell).

Topologies: ``ring`` (a ring plus random distinct chords) and ``rgg``
(spatially clustered random geometric graph: Gaussian clusters in the unit
square, Euclidean minimum spanning tree plus the shortest non-tree k-nearest-
neighbour edges up to the requested branch count).  Buses of an ``rgg`` grid
are renumbered along a Morton curve and branches sorted by end buses, so
components that are close in the network are close in memory.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import numpy as np

BASE_MVA = 100.0


@dataclass
class Grid:
    """Network data in the paper's notation (Section III-A)."""

    n_bus: int
    n_line: int
    n_gen: int
    ref: int
    # buses
    vmin: np.ndarray
    vmax: np.ndarray
    pd: np.ndarray
    qd: np.ndarray
    gsh: np.ndarray
    bsh: np.ndarray
    # branches (i = from, j = to); admittance tuple of the branch pi-model
    f: np.ndarray
    t: np.ndarray
    gii: np.ndarray
    bii: np.ndarray
    gij: np.ndarray
    bij: np.ndarray
    gji: np.ndarray
    bji: np.ndarray
    gjj: np.ndarray
    bjj: np.ndarray
    smax_ij: np.ndarray
    smax_ji: np.ndarray
    # generators
    gbus: np.ndarray
    pmin: np.ndarray
    pmax: np.ndarray
    qmin: np.ndarray
    qmax: np.ndarray
    cost2: np.ndarray
    cost1: np.ndarray
    # raw branch data kept for tests of the admittance tuple
    r: np.ndarray = field(repr=False, default=None)
    x: np.ndarray = field(repr=False, default=None)
    bc: np.ndarray = field(repr=False, default=None)
    tap: np.ndarray = field(repr=False, default=None)
    name: str = ""

    def with_loads(self, pd: np.ndarray, qd: np.ndarray) -> "Grid":
        return replace(self, pd=np.ascontiguousarray(pd, dtype=np.float64),
                       qd=np.ascontiguousarray(qd, dtype=np.float64))


def pi_model(r, x, bc, tap):
    """Per-branch pi-model admittances (Y_ff, Y_ft, Y_tf, Y_tt).

    The paper's flow definitions use, for branch (i, j), the from-end self
    term g_ii + j b_ii, the transfer terms g_ij + j b_ij and g_ji + j b_ji and
    the to-end self term g_jj + j b_jj of the branch's own 2x2 admittance
    matrix (tap on the from side, no phase shift).
    """
    y = 1.0 / (r + 1j * x)
    yff = (y + 0.5j * bc) / (tap * tap)
    yft = -y / tap
    ytf = -y / tap
    ytt = y + 0.5j * bc
    return yff, yft, ytf, ytt


def _morton_order(xy: np.ndarray) -> np.ndarray:
    q = np.clip((xy - xy.min(0)) / max(np.ptp(xy, 0).max(), 1e-12), 0, 1)
    qi = (q * 65535).astype(np.uint64)

    def spread(v):
        v = v & np.uint64(0xFFFF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v

    code = spread(qi[:, 0]) | (spread(qi[:, 1]) << np.uint64(1))
    return np.argsort(code, kind="stable")


def _ring_topology(n_bus, n_line, rng):
    edges = {(i, (i + 1) % n_bus) for i in range(n_bus)}
    edges = {(min(a, b), max(a, b)) for a, b in edges}
    while len(edges) < n_line:
        a, b = rng.choice(n_bus, size=2, replace=False)
        e = (int(min(a, b)), int(max(a, b)))
        edges.add(e)
    ring = [(i, (i + 1) % n_bus) for i in range(n_bus)]
    chords = sorted(edges - {(min(a, b), max(a, b)) for a, b in ring})
    el = ring + chords
    return np.array([e[0] for e in el]), np.array([e[1] for e in el]), None


def _star_topology(n_bus, n_line, rng):
    """Bus 0 joined to every other bus, plus random chords between the others
    (a bus of very high degree)."""
    spokes = [(0, i) for i in range(1, n_bus)]
    edges = set(spokes)
    while len(edges) < n_line:
        a, b = rng.choice(np.arange(1, n_bus), size=2, replace=False)
        edges.add((int(min(a, b)), int(max(a, b))))
    el = spokes + sorted(edges - set(spokes))
    return np.array([e[0] for e in el]), np.array([e[1] for e in el]), None


def _rgg_topology(n_bus, n_line, n_clusters, sigma, knn, rng):
    from scipy.spatial import Delaunay, cKDTree
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree

    centers = rng.uniform(0.0, 1.0, size=(n_clusters, 2))
    lab = rng.integers(0, n_clusters, size=n_bus)
    xy = centers[lab] + rng.normal(0.0, sigma, size=(n_bus, 2))
    # Euclidean MST (a subgraph of the Delaunay triangulation)
    tri = Delaunay(xy)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    w = np.linalg.norm(xy[e[:, 0]] - xy[e[:, 1]], axis=1) + 1e-15
    g = coo_matrix((w, (e[:, 0], e[:, 1])), shape=(n_bus, n_bus)).tocsr()
    mst = minimum_spanning_tree(g).tocoo()
    tree = np.sort(np.stack([mst.row, mst.col], 1), axis=1)
    if len(tree) != n_bus - 1:
        raise RuntimeError("synthetic grid: spanning tree is not connected")
    have = set(map(tuple, tree.tolist()))
    extra_needed = n_line - len(tree)
    if extra_needed < 0:
        raise ValueError("n_line smaller than a spanning tree")
    kd = cKDTree(xy)
    d, nb = kd.query(xy, k=knn + 1)
    cand = []
    for i in range(n_bus):
        for kk in range(1, knn + 1):
            j = int(nb[i, kk])
            a, b = (i, j) if i < j else (j, i)
            cand.append((float(d[i, kk]), a, b))
    cand.sort()
    extra = []
    for dist, a, b in cand:
        if len(extra) >= extra_needed:
            break
        if (a, b) in have:
            continue
        have.add((a, b))
        extra.append((a, b))
    if len(extra) < extra_needed:
        raise RuntimeError("synthetic grid: not enough kNN candidate edges")
    el = np.concatenate([tree, np.array(extra, dtype=np.int64).reshape(-1, 2)])
    # random orientation of each branch (the tap sits on the from side)
    flip = rng.random(len(el)) < 0.5
    f = np.where(flip, el[:, 1], el[:, 0])
    t = np.where(flip, el[:, 0], el[:, 1])
    return f, t, xy


def _nearest_source(n_bus, f, t, sources):
    """Index (into ``sources``) of the nearest source of every bus in hops
    (multi-source breadth-first search; ties go to the source reached first
    in source order)."""
    from collections import deque
    adj = [[] for _ in range(n_bus)]
    for a, b in zip(np.asarray(f).tolist(), np.asarray(t).tolist()):
        adj[a].append(b)
        adj[b].append(a)
    owner = np.full(n_bus, -1, dtype=np.int64)
    dq = deque()
    for k, sbus in enumerate(np.asarray(sources).tolist()):
        owner[sbus] = k
        dq.append(sbus)
    while dq:
        u = dq.popleft()
        for v in adj[u]:
            if owner[v] < 0:
                owner[v] = owner[u]
                dq.append(v)
    return owner


def _dc_limits(n_bus, f, t, x, tap, pinj, ref):
    """Branch flows of a DC power flow B theta = P_inj with theta_ref = 0."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    bser = 1.0 / (x * tap)
    nl = len(f)
    rows = np.concatenate([f, t, f, t])
    cols = np.concatenate([f, t, t, f])
    vals = np.concatenate([bser, bser, -bser, -bser])
    B = sp.coo_matrix((vals, (rows, cols)), shape=(n_bus, n_bus)).tocsr()
    keep = np.array([i for i in range(n_bus) if i != ref])
    Bred = B[keep][:, keep].tocsc()
    th = np.zeros(n_bus)
    th[keep] = spla.spsolve(Bred, pinj[keep])
    flow = bser * (th[f] - th[t])
    resid = B @ th - pinj
    resid[ref] = 0.0
    return flow, th, float(np.abs(resid).max())


def make_grid(n_bus: int, n_line: int, n_gen: int, seed: int, topology: str = "rgg",
              n_clusters: int | None = None, sigma: float = 0.03, knn: int = 8,
              tap_fraction: float = 0.0, load_factor: float = 0.6,
              shunt_scale: float = 0.0, name: str = "") -> Grid:
    """Draw a seeded synthetic grid following the recipe in the module doc."""
    rng = np.random.default_rng(seed)
    if topology == "ring":
        f, t, xy = _ring_topology(n_bus, n_line, rng)
    elif topology == "star":
        f, t, xy = _star_topology(n_bus, n_line, rng)
    elif topology == "rgg":
        nc = n_clusters if n_clusters is not None else max(1, n_bus // 100)
        f, t, xy = _rgg_topology(n_bus, n_line, nc, sigma, knn, rng)
    else:
        raise ValueError(topology)
    nl = len(f)
    assert nl == n_line
    # generators: original bus 0 is the reference and always has one
    others = rng.choice(np.arange(1, n_bus), size=n_gen - 1, replace=False)
    gbus = np.concatenate([[0], others]).astype(np.int64)

    # renumber buses spatially (ring grids keep their natural order)
    if xy is not None:
        order = _morton_order(xy)           # new -> old
        inv = np.empty(n_bus, dtype=np.int64)
        inv[order] = np.arange(n_bus)       # old -> new
        f, t, gbus = inv[f], inv[t], inv[gbus]
        ref = int(inv[0])
    else:
        ref = 0

    r = rng.uniform(0.005, 0.05, nl)
    x = r * rng.uniform(3.0, 10.0, nl)
    bc = rng.uniform(0.0, 0.05, nl)
    tap = np.ones(nl)
    if tap_fraction > 0:
        m = rng.random(nl) < tap_fraction
        tap[m] = rng.uniform(0.95, 1.05, int(m.sum()))

    P = rng.uniform(0.1, 0.5, n_bus)
    pf = rng.uniform(0.9, 0.98, n_bus)
    Q = P * np.tan(np.arccos(pf))
    vmin = np.full(n_bus, 0.94)
    vmax = np.full(n_bus, 1.06)
    gsh = np.zeros(n_bus)
    bsh = np.zeros(n_bus)
    if shunt_scale > 0:
        gsh = rng.uniform(0.0, shunt_scale, n_bus)
        bsh = rng.uniform(-shunt_scale, shunt_scale, n_bus)

    # capacity: demand of each generator's graph-Voronoi cell (the buses
    # nearest to it in hops) divided by the load factor
    cell = _nearest_source(n_bus, f, t, gbus)
    cell_load = np.bincount(cell, P, n_gen)
    cap = cell_load / load_factor
    pmin = np.zeros(n_gen)
    pmax = cap
    qmin = -0.5 * cap
    qmax = 0.5 * cap
    c2 = rng.uniform(0.001, 0.05, n_gen)
    c1 = rng.uniform(10.0, 40.0, n_gen)

    # thermal limits from a DC flow of the cell dispatch (each generator
    # serves the demand of its cell)
    pg_dc = cell_load
    pinj = -P.copy()
    np.add.at(pinj, gbus, pg_dc)
    flow, _, _ = _dc_limits(n_bus, f, t, x, tap, pinj, ref)
    smax = np.maximum(2.0 * np.abs(flow), 0.1)

    # sort generators by bus and branches by (from, to)
    go = np.lexsort((np.arange(n_gen), gbus))
    lo = np.lexsort((t, f)) if xy is not None else np.arange(nl)
    f, t, r, x, bc, tap, smax = f[lo], t[lo], r[lo], x[lo], bc[lo], tap[lo], smax[lo]
    gbus, pmin, pmax, qmin, qmax, c2, c1 = (a[go] for a in (gbus, pmin, pmax, qmin, qmax, c2, c1))

    yff, yft, ytf, ytt = pi_model(r, x, bc, tap)
    as_i = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    as_d = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    return Grid(
        n_bus=n_bus, n_line=nl, n_gen=n_gen, ref=ref,
        vmin=as_d(vmin), vmax=as_d(vmax), pd=as_d(P), qd=as_d(Q), gsh=as_d(gsh), bsh=as_d(bsh),
        f=as_i(f), t=as_i(t),
        gii=as_d(yff.real), bii=as_d(yff.imag), gij=as_d(yft.real), bij=as_d(yft.imag),
        gji=as_d(ytf.real), bji=as_d(ytf.imag), gjj=as_d(ytt.real), bjj=as_d(ytt.imag),
        smax_ij=as_d(smax), smax_ji=as_d(smax.copy()),
        gbus=as_i(gbus), pmin=as_d(pmin), pmax=as_d(pmax), qmin=as_d(qmin), qmax=as_d(qmax),
        cost2=as_d(c2 * BASE_MVA ** 2), cost1=as_d(c1 * BASE_MVA),
        r=as_d(r), x=as_d(x), bc=as_d(bc), tap=as_d(tap), name=name,
    )


def perturb_loads(grid: Grid, seed: int, sd: float = 0.1) -> Grid:
    """Scenario: multiplicative per-bus load factor N(1, sd) clipped to [0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    fac = np.clip(rng.normal(1.0, sd, grid.n_bus), 0.5, 1.5)
    return grid.with_loads(grid.pd * fac, grid.qd * fac)


# Named workloads -------------------------------------------------------------

def grid_14(**kw) -> Grid:
    """14 buses: ring plus 6 random distinct chords (20 branches), 5 gens, seed 14."""
    return make_grid(14, 20, 5, seed=14, topology="ring", name="ring14", **kw)


def grid_300() -> Grid:
    return make_grid(300, 405, 60, seed=300, topology="rgg", tap_fraction=0.2, name="rgg300")


def grid_2000() -> Grid:
    """2,000-bus clustered RGG, 2,700 branches, 400 gens, 20% taps, seed 2000."""
    return make_grid(2000, 2700, 400, seed=2000, topology="rgg", n_clusters=20,
                     tap_fraction=0.2, name="rgg2000")


def grid_10000() -> Grid:
    return make_grid(10000, 13500, 2000, seed=10000, topology="rgg", tap_fraction=0.2,
                     name="rgg10000")


def grid_70000() -> Grid:
    """70,000-bus clustered RGG (700 clusters), 88,000 branches, 10,000 gens, seed 70000."""
    return make_grid(70000, 88000, 10000, seed=70000, topology="rgg", n_clusters=700,
                     tap_fraction=0.2, name="rgg70000")


def tiny_grid(seed: int = 1, n_bus: int = 4, n_line: int = 5, n_gen: int = 2,
              shunt_scale: float = 0.02) -> Grid:
    """Small ring grids with shunts for unit tests."""
    return make_grid(n_bus, n_line, n_gen, seed=seed, topology="ring",
                     shunt_scale=shunt_scale, name=f"tiny{n_bus}_{seed}")


WORKLOADS = {
    "ring14": grid_14,
    "rgg300": grid_300,
    "rgg2000": grid_2000,
    "rgg10000": grid_10000,
    "rgg70000": grid_70000,
}


# Starting operating point ------------------------------------------------------

def ybus(grid: Grid):
    """Complex bus admittance matrix from the per-branch pi-model tuples and shunts."""
    import scipy.sparse as sp
    nb = grid.n_bus
    yff = grid.gii + 1j * grid.bii
    yft = grid.gij + 1j * grid.bij
    ytf = grid.gji + 1j * grid.bji
    ytt = grid.gjj + 1j * grid.bjj
    rows = np.concatenate([grid.f, grid.f, grid.t, grid.t, np.arange(nb)])
    cols = np.concatenate([grid.f, grid.t, grid.f, grid.t, np.arange(nb)])
    vals = np.concatenate([yff, yft, ytf, ytt, grid.gsh + 1j * grid.bsh])
    return sp.coo_matrix((vals, (rows, cols)), shape=(nb, nb)).tocsr()


def power_flow_start(grid: Grid, vset: float = 1.0, tol: float = 1e-10, max_iter: int = 30):
    """Operating point the SQP starts from, the analogue of the solved power
    flow that published test cases carry: generator buses voltage-controlled
    at ``vset``, all other buses at their demand, generators at the
    proportional dispatch ``P_max * sum(P_d) / sum(P_max)`` scaled by a
    common factor that covers the losses (distributed slack), reference
    angle 0 (polar Newton-Raphson).  Reactive output of a bus is split among
    its generators in proportion to capacity.  Returns a dict with pg, qg, w,
    th, wR, wI and a ``converged`` flag; if Newton fails, the flat start with
    DC angles is returned instead (flag False).
    """
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    nb = grid.n_bus
    Y = ybus(grid)
    pg0 = np.clip(grid.pmax * (grid.pd.sum() / grid.pmax.sum()), grid.pmin, grid.pmax)
    isgen = np.zeros(nb, dtype=bool)
    isgen[grid.gbus] = True
    pq = np.nonzero(~isgen)[0]
    nonref = np.nonzero(np.arange(nb) != grid.ref)[0]
    gen_at = np.bincount(grid.gbus, pg0, nb)
    x = grid.x if grid.x is not None else np.ones(grid.n_line)
    tap = grid.tap if grid.tap is not None else np.ones(grid.n_line)
    _, th0, _ = _dc_limits(nb, grid.f, grid.t, x, tap, gen_at - grid.pd, grid.ref)
    vm = np.ones(nb)
    vm[isgen] = vset
    va = th0.copy()
    kappa = 0.0
    converged = False
    for _ in range(max_iter):
        V = vm * np.exp(1j * va)
        I = Y @ V
        S = V * np.conj(I)
        mis = S - ((1.0 + kappa) * gen_at - grid.pd - 1j * grid.qd)
        F = np.concatenate([mis.real, mis.imag[pq]])
        if np.abs(F).max() < tol:
            converged = True
            break
        dV = sp.diags(V)
        dS_dVa = 1j * dV @ np.conj(sp.diags(I) - Y @ dV)
        dS_dVm = dV @ np.conj(Y @ sp.diags(V / vm)) + np.conj(sp.diags(I)) @ sp.diags(V / vm)
        kcol = sp.csr_matrix(np.concatenate([-gen_at, np.zeros(pq.size)])[:, None])
        J = sp.hstack([sp.vstack([dS_dVa.real[:, nonref], dS_dVa.imag[pq][:, nonref]]),
                       sp.vstack([dS_dVm.real[:, pq], dS_dVm.imag[pq][:, pq]]),
                       kcol]).tocsc()
        dx = spla.spsolve(J, -F)
        va[nonref] += dx[:nonref.size]
        vm[pq] += dx[nonref.size:nonref.size + pq.size]
        kappa += dx[-1]
        if not (np.all(np.isfinite(vm)) and vm.min() > 0.3 and np.isfinite(kappa)):
            break
    if converged:
        V = vm * np.exp(1j * va)
        S = V * np.conj(Y @ V) + grid.pd + 1j * grid.qd
        capbus = np.bincount(grid.gbus, grid.pmax, nb)
        qg = S.imag[grid.gbus] * grid.pmax / capbus[grid.gbus]
        pg = pg0 * (1.0 + kappa)
        w, th = vm ** 2, va
    else:
        pg, qg = pg0, np.zeros(grid.n_gen)
        w, th = np.ones(nb), th0
    ph = th[grid.f] - th[grid.t]
    vv = np.sqrt(w[grid.f] * w[grid.t])
    return {"pg": pg, "qg": qg, "w": w, "th": th, "wR": vv * np.cos(ph), "wI": vv * np.sin(ph),
            "converged": converged}
