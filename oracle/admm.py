"""Serial two-block ADMM for the QP subproblem (Section IV, Algorithm 2).

Coupling constraints (eq. cpl): every generator output and every line flow
has a bus-side copy, and every line holds copies of the voltage variables
(d_w, d_th) of its two end buses.  For a coupling c we write x_c for the
generator/line-side value, xbar_c for the bus-side value, lam_c for its
multiplier and rho_c > 0 for its penalty; the augmented Lagrangian term is
lam_c (x_c - xbar_c) + rho_c/2 (x_c - xbar_c)^2.

Per line the 8 couplings are ordered (p_ij, q_ij, p_ji, q_ji, w_i, th_i,
w_j, th_j); the bus-side value of the last four is the end bus's (d_w, d_th).
Per generator the 2 couplings are (p, q).

One sweep (Algorithm 2): generator update (eq. gen_kernel, closed form
clamp), line update (eq. line_kernel, exact minimiser from ``lineqp``), bus
update (eq. bus_kernel, closed form of eq. bus_kernel_simp), multiplier
update (eq. multiplier), residuals r = x - xbar and s = rho (xbar_new -
xbar_old) (Section IV-B5) with stop when ||r||_2 <= eps_pri and
||s||_2 <= eps_dual.  Generators and lines form the first block (both use
the previous bus values); buses form the second block.

Start (the paper leaves d0 and lam0 open): x = xbar = 0 and lam = 0 unless a
warm-start lam is given.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

from .lineqp import solve_line_qps


@dataclass
class AdmmState:
    xg: np.ndarray       # (G, 2)
    xbar_g: np.ndarray   # (G, 2)
    lam_g: np.ndarray    # (G, 2)
    xl: np.ndarray       # (L, 8)
    xbar_f: np.ndarray   # (L, 4) bus-side copies of the four flows
    lam_l: np.ndarray    # (L, 8)
    dw: np.ndarray       # (B,)
    dth: np.ndarray      # (B,)
    mu: np.ndarray       # (L, 2) multipliers of the limit rows in the last line solve
    nu: np.ndarray       # (B, 2) balance multipliers of the last bus update

    def copy(self):
        return AdmmState(*(a.copy() for a in (self.xg, self.xbar_g, self.lam_g, self.xl,
                                               self.xbar_f, self.lam_l, self.dw, self.dth, self.mu,
                                               self.nu)))


@dataclass
class Rho:
    g: np.ndarray  # (G, 2)
    l: np.ndarray  # (L, 8)

    @staticmethod
    def scalar(grid, rho: float) -> "Rho":
        return Rho(np.full((grid.n_gen, 2), float(rho)), np.full((grid.n_line, 8), float(rho)))


@dataclass
class AdmmResult:
    state: AdmmState
    sweeps: int
    r: float
    s: float
    converged: bool
    infeasible_lines: int
    history: list = field(default_factory=list)


def cold_state(grid) -> AdmmState:
    G, L, B = grid.n_gen, grid.n_line, grid.n_bus
    z = np.zeros
    return AdmmState(z((G, 2)), z((G, 2)), z((G, 2)), z((L, 8)), z((L, 4)), z((L, 8)),
                     z(B), z(B), z((L, 2)), z((B, 2)))


def warm_state(grid, lam_g, lam_l) -> AdmmState:
    """Previous-iterate warm start: multipliers carried over, primal values zero."""
    st = cold_state(grid)
    st.lam_g = np.array(lam_g, dtype=np.float64, copy=True)
    st.lam_l = np.array(lam_l, dtype=np.float64, copy=True)
    return st


def gen_update(qp, st: AdmmState, rho: Rho):
    """Closed form of (eq. gen_kernel): x* = clamp(Q^{-1} c, l, u) per coordinate."""
    g = qp.gen
    rp, rq = rho.g[:, 0], rho.g[:, 1]
    xp = (rp * st.xbar_g[:, 0] - st.lam_g[:, 0] - g.fp) / (g.fpp + rp)
    fq = 0.0 if g.fq is None else g.fq
    fqq = 0.0 if g.fqq is None else g.fqq
    xq = (rq * st.xbar_g[:, 1] - st.lam_g[:, 1] - fq) / (fqq + rq)
    xp = np.minimum(np.maximum(xp, g.lo[:, 0]), g.hi[:, 0])
    xq = np.minimum(np.maximum(xq, g.lo[:, 1]), g.hi[:, 1])
    return np.stack([xp, xq], 1)


def line_matrices(qp, rho: Rho):
    """Q = M + sum_f rho_f F_f^T F_f + diag(rho_v) of the line subproblem."""
    L = qp.line
    rf = rho.l[:, :4]
    Q = L.M + np.einsum("lf,lfi,lfj->lij", rf, L.F, L.F)
    Q = Q + np.einsum("li,ij->lij", rho.l[:, 4:], np.eye(4))
    return Q


def line_update(grid, qp, st: AdmmState, rho: Rho, Q=None, solver: str = "exact"):
    """Solve of (eq. line_kernel) for every line: exact (enumeration), or
    "alm": the paper's local method (ALM + TRON, ``alm.solve_line``) from the
    previous sweep's solution and limit-row multipliers.  Returns
    (x (L,8), mu, solved)."""
    L = qp.line
    if Q is None:
        Q = line_matrices(qp, rho)
    rf, rv = rho.l[:, :4], rho.l[:, 4:]
    lam_f, lam_v = st.lam_l[:, :4], st.lam_l[:, 4:]
    xbar_v = np.stack([st.dw[grid.f], st.dth[grid.f], st.dw[grid.t], st.dth[grid.t]], 1)
    c = L.q + np.einsum("lf,lfi->li", lam_f + rf * (L.f0 - st.xbar_f), L.F) + lam_v - rv * xbar_v
    if solver == "alm":
        from . import alm
        n = Q.shape[0]
        z, mu, feas = np.zeros((n, 4)), np.zeros((n, 2)), np.zeros(n, dtype=bool)
        for l in range(n):
            r = alm.solve_line(Q[l], c[l], L.lo[l], L.hi[l], L.G[l], L.h[l], z0=st.xl[l, 4:8], u0=st.mu[l])
            z[l], mu[l], feas[l] = r.z, r.u, r.converged
    elif solver == "exact":
        z, mu, _, feas = solve_line_qps(Q, c, L.lo, L.hi, L.G, L.h)
    else:
        raise ValueError(solver)
    flows = np.einsum("lfi,li->lf", L.F, z) + L.f0
    return np.concatenate([flows, z], 1), mu, feas


def bus_update(grid, qp, xg, xl, st: AdmmState, rho: Rho):
    """Closed form of (eq. bus_kernel_simp) per bus with diagonal Q:
    nu = (A Q^-1 A^T)^-1 (A Q^-1 c - b), xbar = Q^-1 (c - A^T nu).

    Unknowns at bus i: the bus-side copies of its generators' (p, q) and of
    the flows at its line ends, plus (d_w, d_th).  The objective terms
    -lam xbar + rho/2 (x - xbar)^2 give Q_c = rho_c and c_c = rho_c x_c +
    lam_c; d_w collects every w coupling at the bus.  Rows of A: active and
    reactive balance (+1 on generator copies, -1 on flow copies, -g_sh and
    +b_sh on d_w), right-hand side (p^{d,(k)}, q^{d,(k)}).  d_th enters no
    constraint and is the rho-weighted mean of its copies (0 at the
    reference bus).  Returns (xbar_g, xbar_f, dw, dth, nu)."""
    nb = grid.n_bus
    f, t, gb = grid.f, grid.t, grid.gbus
    S = np.zeros((nb, 2, 2))
    R = np.zeros((nb, 2))

    def add(bus, a, Qc, cc):
        a = np.asarray(a, dtype=np.float64)
        for i in range(2):
            R[:, i] += np.bincount(bus, a[..., i] * cc / Qc, nb)
            for j in range(2):
                S[:, i, j] += np.bincount(bus, a[..., i] * a[..., j] / Qc, nb)

    ones = lambda n: np.ones(n)
    zeros = lambda n: np.zeros(n)
    # generator copies
    cg = rho.g * xg + st.lam_g
    add(gb, np.stack([ones(grid.n_gen), zeros(grid.n_gen)], 1), rho.g[:, 0], cg[:, 0])
    add(gb, np.stack([zeros(grid.n_gen), ones(grid.n_gen)], 1), rho.g[:, 1], cg[:, 1])
    # flow copies: p_ij, q_ij at the from bus; p_ji, q_ji at the to bus
    cl = rho.l * xl + st.lam_l
    nl = grid.n_line
    for k, bus, a in ((0, f, (-1.0, 0.0)), (1, f, (0.0, -1.0)), (2, t, (-1.0, 0.0)), (3, t, (0.0, -1.0))):
        add(bus, np.tile(np.array(a), (nl, 1)), rho.l[:, k], cl[:, k])
    # voltage magnitude variable d_w
    Qw = np.bincount(f, rho.l[:, 4], nb) + np.bincount(t, rho.l[:, 6], nb)
    cw = np.bincount(f, cl[:, 4], nb) + np.bincount(t, cl[:, 6], nb)
    aw = np.stack([-grid.gsh, grid.bsh], 1)
    add(np.arange(nb), aw, Qw, cw)
    b = np.stack([qp.bus.pdk, qp.bus.qdk], 1)
    nu = np.linalg.solve(S, (R - b)[:, :, None])[:, :, 0]

    xbar_g = np.stack([(cg[:, 0] - nu[gb, 0]) / rho.g[:, 0],
                       (cg[:, 1] - nu[gb, 1]) / rho.g[:, 1]], 1)
    xbar_f = np.stack([(cl[:, 0] + nu[f, 0]) / rho.l[:, 0],
                       (cl[:, 1] + nu[f, 1]) / rho.l[:, 1],
                       (cl[:, 2] + nu[t, 0]) / rho.l[:, 2],
                       (cl[:, 3] + nu[t, 1]) / rho.l[:, 3]], 1)
    dw = (cw - (aw[:, 0] * nu[:, 0] + aw[:, 1] * nu[:, 1])) / Qw
    Qt = np.bincount(f, rho.l[:, 5], nb) + np.bincount(t, rho.l[:, 7], nb)
    ct = np.bincount(f, cl[:, 5], nb) + np.bincount(t, cl[:, 7], nb)
    dth = ct / Qt
    dth[grid.ref] = 0.0
    return xbar_g, xbar_f, dw, dth, nu


def sweep(grid, qp, st: AdmmState, rho: Rho, Q=None, line_solver: str = "exact", norm: str = "2"):
    """One ADMM iteration of Algorithm 2; returns (new state, r, s, feasible)
    with r, s the Euclidean norms of the primal and dual residuals over all
    couplings, or their infinity norms (norm "inf")."""
    xg = gen_update(qp, st, rho)
    xl, mu, feas = line_update(grid, qp, st, rho, Q, line_solver)
    xbar_g, xbar_f, dw, dth, nu = bus_update(grid, qp, xg, xl, st, rho)
    f, t = grid.f, grid.t
    xbar_l = np.concatenate([xbar_f, np.stack([dw[f], dth[f], dw[t], dth[t]], 1)], 1)
    xbar_l_old = np.concatenate([st.xbar_f, np.stack([st.dw[f], st.dth[f], st.dw[t], st.dth[t]], 1)], 1)
    lam_g = st.lam_g + rho.g * (xg - xbar_g)
    lam_l = st.lam_l + rho.l * (xl - xbar_l)
    if norm == "inf":
        r2 = max(np.max((xg - xbar_g) ** 2, initial=0.0), np.max((xl - xbar_l) ** 2, initial=0.0))
        s2 = max(np.max((rho.g * (xbar_g - st.xbar_g)) ** 2, initial=0.0),
                 np.max((rho.l * (xbar_l - xbar_l_old)) ** 2, initial=0.0))
    elif norm == "2":
        r2 = np.sum((xg - xbar_g) ** 2) + np.sum((xl - xbar_l) ** 2)
        s2 = np.sum((rho.g * (xbar_g - st.xbar_g)) ** 2) + np.sum((rho.l * (xbar_l - xbar_l_old)) ** 2)
    else:
        raise ValueError(norm)
    new = AdmmState(xg, xbar_g, lam_g, xl, xbar_f, lam_l, dw, dth, mu, nu)
    return new, float(np.sqrt(r2)), float(np.sqrt(s2)), feas


@dataclass
class Balance:
    """Residual balancing of the penalties (the heuristic the paper names,
    in a commented passage beside its ADMM termination rule, for better
    convergence; Section V lists the heuristic ADMM tuning as a limitation).
    After every `every`-th sweep that does not stop the solve, all penalties
    are multiplied by tau when ||r|| > mu ||s||, divided by tau when
    ||s|| > mu ||r||, and kept otherwise; the multipliers lam are not
    scaled (the unscaled form)."""
    mu: float = 10.0
    tau: float = 2.0
    every: int = 64


def balance_factor(r: float, s: float, b: Balance) -> float:
    if r > b.mu * s:
        return b.tau
    if s > b.mu * r:
        return 1.0 / b.tau
    return 1.0


def solve(grid, qp, rho: Rho, max_sweeps: int, eps_pri: float, eps_dual: float,
          state: AdmmState | None = None, record: bool = False, record_states: bool = False,
          balance: Balance | None = None, line_solver: str = "exact", norm: str = "2"):
    """Algorithm 2 until ||r|| <= eps_pri and ||s|| <= eps_dual (Euclidean
    norms, or infinity norms with norm "inf") or max_sweeps;
    with ``balance``, residual balancing of the penalties between sweeps
    (the result's ``rho`` holds the final penalties)."""
    st = cold_state(grid) if state is None else state.copy()
    rho = Rho(rho.g.copy(), rho.l.copy())
    Q = line_matrices(qp, rho)
    hist = []
    r = s = np.inf
    bad = 0
    k = 0
    for k in range(1, max_sweeps + 1):
        st, r, s, feas = sweep(grid, qp, st, rho, Q, line_solver, norm)
        bad = int((~feas).sum())
        if record:
            hist.append((r, s))
        if record_states:
            hist.append(st.copy())
        if r <= eps_pri and s <= eps_dual:
            res = AdmmResult(st, k, r, s, True, bad, hist)
            res.rho = rho
            return res
        if balance is not None and k % balance.every == 0 and k < max_sweeps:
            f = balance_factor(r, s, balance)
            if f != 1.0:
                rho = Rho(rho.g * f, rho.l * f)
                Q = line_matrices(qp, rho)
    res = AdmmResult(st, k, r, s, False, bad, hist)
    res.rho = rho
    return res
