"""ACOPF model in rectangular form (Section III-A, eqs. acopf and acopf_pf).

Variables: generator outputs ``pg, qg``; per bus ``w = v^2`` and angle ``th``;
per line ``wR, wI`` (physically v_i v_j cos and v_i v_j sin of the angle
difference).  The Lagrangian uses the paper's sign (f + sum of multiplier
times constraint, Section II), so multipliers of the inequality
constraints c >= 0 are <= 0 at a KKT point.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np


@dataclass
class Iterate:
    pg: np.ndarray
    qg: np.ndarray
    w: np.ndarray
    th: np.ndarray
    wR: np.ndarray
    wI: np.ndarray

    def copy(self) -> "Iterate":
        return Iterate(*(a.copy() for a in (self.pg, self.qg, self.w, self.th, self.wR, self.wI)))

    def plus(self, d: "Iterate") -> "Iterate":
        return Iterate(self.pg + d.pg, self.qg + d.qg, self.w + d.w, self.th + d.th,
                       self.wR + d.wR, self.wI + d.wI)


def flat_start(grid) -> Iterate:
    """Flat start: w = 1, th = 0, wR = 1, wI = 0; generators at the proportional
    dispatch pmax * sum(pd)/sum(pmax) and qg = 0, clipped to their bounds."""
    share = grid.pd.sum() / grid.pmax.sum()
    pg = np.clip(grid.pmax * share, grid.pmin, grid.pmax)
    qg = np.clip(np.zeros(grid.n_gen), grid.qmin, grid.qmax)
    return Iterate(pg, qg, np.ones(grid.n_bus), np.zeros(grid.n_bus),
                   np.ones(grid.n_line), np.zeros(grid.n_line))


def flows(grid, w, wR, wI):
    """Branch flows (eq. acopf_pf): p_ij, q_ij at the from end, p_ji, q_ji at
    the to end, linear in (w_i, w_j, wR, wI)."""
    wi, wj = w[grid.f], w[grid.t]
    pij = grid.gii * wi + grid.gij * wR + grid.bij * wI
    qij = -grid.bii * wi - grid.bij * wR + grid.gij * wI
    pji = grid.gjj * wj + grid.gji * wR - grid.bji * wI
    qji = -grid.bjj * wj - grid.bji * wR - grid.gji * wI
    return pij, qij, pji, qji


def objective(grid, pg):
    """Sum of generator costs f_g(p) = cost2 p^2 + cost1 p."""
    return float(np.sum(grid.cost2 * pg * pg + grid.cost1 * pg))


def balance(grid, x: Iterate):
    """Residuals of the power balance (opfc5, opfc6), written as
    sum p_g - p_d - sum_j p_ij - g_sh w (and the reactive analogue + b_sh w)."""
    pij, qij, pji, qji = flows(grid, x.w, x.wR, x.wI)
    rp = -grid.pd - grid.gsh * x.w
    rq = -grid.qd + grid.bsh * x.w
    rp = rp + np.bincount(grid.gbus, x.pg, grid.n_bus)
    rq = rq + np.bincount(grid.gbus, x.qg, grid.n_bus)
    rp -= np.bincount(grid.f, pij, grid.n_bus) + np.bincount(grid.t, pji, grid.n_bus)
    rq -= np.bincount(grid.f, qij, grid.n_bus) + np.bincount(grid.t, qji, grid.n_bus)
    return rp, rq


def nonlinear_constraints(grid, x: Iterate):
    """c11 = wR^2 + wI^2 - w_i w_j (opfc11), c12 = wR sin - wI cos (opfc12),
    c13 = s_ij^2 - p_ij^2 - q_ij^2 (opfc13), c14 likewise at the to end."""
    wi, wj = x.w[grid.f], x.w[grid.t]
    ph = x.th[grid.f] - x.th[grid.t]
    c11 = x.wR ** 2 + x.wI ** 2 - wi * wj
    c12 = x.wR * np.sin(ph) - x.wI * np.cos(ph)
    pij, qij, pji, qji = flows(grid, x.w, x.wR, x.wI)
    c13 = grid.smax_ij ** 2 - pij ** 2 - qij ** 2
    c14 = grid.smax_ji ** 2 - pji ** 2 - qji ** 2
    return c11, c12, c13, c14


def infeas_h(grid, x: Iterate) -> float:
    """h(x) of the l1 merit (Section II-C): sum |c_E| + sum [c_I]^- over the
    nonlinear constraints (opfc11-14) only."""
    c11, c12, c13, c14 = nonlinear_constraints(grid, x)
    neg = lambda c: np.maximum(0.0, -c)
    return float(np.abs(c11).sum() + np.abs(c12).sum() + neg(c13).sum() + neg(c14).sum())


def merit(grid, x: Iterate, mu: float) -> float:
    """phi_1(x; mu) = f(x) + mu h(x)."""
    return objective(grid, x.pg) + mu * infeas_h(grid, x)


def line_hessian(grid, x: Iterate, pi: np.ndarray) -> np.ndarray:
    """Hessian of the line Lagrangian L_ij (eq. lag) in the lifted order
    u = (w_i, th_i, wR, wI, w_j, th_j); returns (n_line, 6, 6).

    pi[:, 0..3] multiply (opfc11)..(opfc14) with the paper's plus sign.
    """
    n = grid.n_line
    wR, wI = x.wR, x.wI
    ph = x.th[grid.f] - x.th[grid.t]
    s, c = np.sin(ph), np.cos(ph)
    H = np.zeros((n, 6, 6))
    W_I, T_I, R, I, W_J, T_J = range(6)
    p11, p12, p13, p14 = pi[:, 0], pi[:, 1], pi[:, 2], pi[:, 3]
    # pi11 [wR^2 + wI^2 - w_i w_j]
    H[:, R, R] += 2 * p11
    H[:, I, I] += 2 * p11
    H[:, W_I, W_J] -= p11
    H[:, W_J, W_I] -= p11
    # pi12 [wR sin(th_i - th_j) - wI cos(th_i - th_j)]
    T = -wR * s + wI * c  # second derivative in the angle difference
    H[:, T_I, T_I] += p12 * T
    H[:, T_J, T_J] += p12 * T
    H[:, T_I, T_J] -= p12 * T
    H[:, T_J, T_I] -= p12 * T
    for (a, b, v) in ((R, T_I, c), (R, T_J, -c), (I, T_I, s), (I, T_J, -s)):
        H[:, a, b] += p12 * v
        H[:, b, a] += p12 * v
    # pi13 (s^2 - p_ij^2 - q_ij^2), pi14 (s^2 - p_ji^2 - q_ji^2): flows are linear
    z = np.zeros(n)
    gp_ij = np.stack([grid.gii, z, grid.gij, grid.bij, z, z], 1)
    gq_ij = np.stack([-grid.bii, z, -grid.bij, grid.gij, z, z], 1)
    gp_ji = np.stack([z, z, grid.gji, -grid.bji, grid.gjj, z], 1)
    gq_ji = np.stack([z, z, -grid.bji, -grid.gji, -grid.bjj, z], 1)
    outer = lambda g: g[:, :, None] * g[:, None, :]
    H -= 2 * p13[:, None, None] * (outer(gp_ij) + outer(gq_ij))
    H -= 2 * p14[:, None, None] * (outer(gp_ji) + outer(gq_ji))
    return H


def line_lagrangian(grid, u: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """L_ij of (eq. lag) evaluated at lifted points u (n_line, 6); used by the
    finite-difference checks of ``line_hessian``."""
    wi, thi, wR, wI, wj, thj = (u[:, k] for k in range(6))
    ph = thi - thj
    pij = grid.gii * wi + grid.gij * wR + grid.bij * wI
    qij = -grid.bii * wi - grid.bij * wR + grid.gij * wI
    pji = grid.gjj * wj + grid.gji * wR - grid.bji * wI
    qji = -grid.bjj * wj - grid.bji * wR - grid.gji * wI
    return (pi[:, 0] * (wR ** 2 + wI ** 2 - wi * wj)
            + pi[:, 1] * (wR * np.sin(ph) - wI * np.cos(ph))
            + pi[:, 2] * (grid.smax_ij ** 2 - pij ** 2 - qij ** 2)
            + pi[:, 3] * (grid.smax_ji ** 2 - pji ** 2 - qji ** 2))


def primal_infeasibility(grid, x: Iterate) -> dict:
    """Infinity norms of the constraint violations of (eq. acopf) at x:
    power balance, opfc11, opfc12, line limits, variable bounds."""
    rp, rq = balance(grid, x)
    c11, c12, c13, c14 = nonlinear_constraints(grid, x)
    neg = lambda c: np.maximum(0.0, -c)
    bnd = np.concatenate([
        neg(x.pg - grid.pmin), neg(grid.pmax - x.pg),
        neg(x.qg - grid.qmin), neg(grid.qmax - x.qg),
        neg(x.w - grid.vmin ** 2), neg(grid.vmax ** 2 - x.w),
        neg(x.th + 2 * np.pi), neg(2 * np.pi - x.th),
    ])
    parts = {
        "balance": float(max(np.abs(rp).max(initial=0), np.abs(rq).max(initial=0))),
        "c11": float(np.abs(c11).max(initial=0)),
        "c12": float(np.abs(c12).max(initial=0)),
        "limit": float(max(neg(c13).max(initial=0), neg(c14).max(initial=0))),
        "bounds": float(bnd.max(initial=0)),
    }
    parts["primal"] = max(parts.values())
    return parts


def lagrangian_gradient(grid, x: Iterate, yp, yq, pi):
    """Gradient of the ACOPF Lagrangian f + y_p c_P + y_q c_Q + sum pi c_nl
    (bounds excluded) with respect to (pg, qg, w, th, wR, wI)."""
    gpg = 2 * grid.cost2 * x.pg + grid.cost1 + yp[grid.gbus]
    gqg = yq[grid.gbus].copy()
    f, t = grid.f, grid.t
    wi, wj = x.w[f], x.w[t]
    ph = x.th[f] - x.th[t]
    s, c = np.sin(ph), np.cos(ph)
    pij, qij, pji, qji = flows(grid, x.w, x.wR, x.wI)
    p11, p12, p13, p14 = pi[:, 0], pi[:, 1], pi[:, 2], pi[:, 3]
    ypf, yqf, ypt, yqt = yp[f], yq[f], yp[t], yq[t]
    # balance terms: c_P = ... - sum flows - gsh w ; c_Q = ... - sum flows + bsh w
    gw = -grid.gsh * yp + grid.bsh * yq
    dwi = -ypf * grid.gii - yqf * (-grid.bii) + p11 * (-wj) + p13 * (-2 * pij * grid.gii + 2 * qij * grid.bii)
    dwj = -ypt * grid.gjj - yqt * (-grid.bjj) + p11 * (-wi) + p14 * (-2 * pji * grid.gjj + 2 * qji * grid.bjj)
    gw = gw + np.bincount(f, dwi, grid.n_bus) + np.bincount(t, dwj, grid.n_bus)
    K = x.wR * c + x.wI * s
    gth = np.bincount(f, p12 * K, grid.n_bus) - np.bincount(t, p12 * K, grid.n_bus)
    gwR = (-ypf * grid.gij - yqf * (-grid.bij) - ypt * grid.gji - yqt * (-grid.bji)
           + p11 * 2 * x.wR + p12 * s
           + p13 * (-2 * pij * grid.gij + 2 * qij * grid.bij)
           + p14 * (-2 * pji * grid.gji + 2 * qji * grid.bji))
    gwI = (-ypf * grid.bij - yqf * grid.gij - ypt * (-grid.bji) - yqt * (-grid.gji)
           + p11 * 2 * x.wI - p12 * c
           + p13 * (-2 * pij * grid.bij - 2 * qij * grid.gij)
           + p14 * (2 * pji * grid.bji + 2 * qji * grid.gji))
    return gpg, gqg, gw, gth, gwR, gwI


def dual_infeasibility(grid, x: Iterate, yp, yq, pi, active_tol: float = 1e-6) -> float:
    """Infinity norm of the projected Lagrangian gradient: at a variable that
    sits on a bound only the sign that a bound multiplier cannot absorb
    counts; the reference angle is fixed and excluded.  Scaled by
    max(1, ||grad f||_inf) so the figure is unitless."""
    gpg, gqg, gw, gth, gwR, gwI = lagrangian_gradient(grid, x, yp, yq, pi)

    def proj(g, v, lo, hi):
        atlo = v <= lo + active_tol
        athi = v >= hi - active_tol
        r = np.abs(g)
        r = np.where(atlo, np.maximum(-g, 0.0), r)
        r = np.where(athi, np.maximum(g, 0.0), r)
        r = np.where(atlo & athi, 0.0, r)
        return r

    gth = gth.copy()
    gth[grid.ref] = 0.0
    parts = [proj(gpg, x.pg, grid.pmin, grid.pmax), proj(gqg, x.qg, grid.qmin, grid.qmax),
             proj(gw, x.w, grid.vmin ** 2, grid.vmax ** 2), np.abs(gth), np.abs(gwR), np.abs(gwI)]
    scale = max(1.0, float(np.abs(2 * grid.cost2 * x.pg + grid.cost1).max(initial=0)))
    return float(max(p.max(initial=0) for p in parts)) / scale
