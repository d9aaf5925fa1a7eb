"""QP subproblem of one SQP iteration (Section III-B, eq. QPsub) with the
elimination of Section III-C (eq. elim) and the line-subproblem data of
Section IV-B2 (eq. line_kernel: A_ij, b_ij, H_ij and the flow substitution).

Per line the independent step variables are z = (d_w_i, d_th_i, d_w_j, d_th_j)
(the ordering of A_ij); the lifted step is u = A z + b in the order
(w_i, th_i, wR, wI, w_j, th_j).

Readings where the paper is silent (also listed in the design notes):
* the trust region bounds pg, qg, w, th only; wR, wI are eliminated (III-C);
* d_th at the reference bus is fixed to 0 (theta_ref = 0 convention);
* "psd" Hessian mode replaces each reduced line Hessian M = A^T H A by its
  projection onto the PSD cone (negative eigenvalues clipped to 0); "raw"
  keeps M as is;
* a box whose lower end exceeds its upper end (an iterate outside a variable
  bound by more than the trust radius) is collapsed to its upper end.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from .acopf import Iterate, flows, line_hessian
from .lineqp import limit_relaxation

TWO_PI = 2.0 * np.pi


@dataclass
class LineQP:
    aR: np.ndarray   # (L, 4)
    bR: np.ndarray   # (L,)
    aI: np.ndarray
    bI: np.ndarray
    H: np.ndarray    # (L, 6, 6) raw Lagrangian Hessian
    M: np.ndarray    # (L, 4, 4) reduced Hessian used by the QP
    q: np.ndarray    # (L, 4)  A^T H b
    F: np.ndarray    # (L, 4, 4) rows d_p_ij, d_q_ij, d_p_ji, d_q_ji over z
    f0: np.ndarray   # (L, 4)
    lo: np.ndarray   # (L, 4)
    hi: np.ndarray   # (L, 4)
    G: np.ndarray    # (L, 2, 4) linearised line limits G z <= h
    h: np.ndarray    # (L, 2)
    pk: np.ndarray   # (L, 4) flows at the iterate
    c0: np.ndarray   # (L,) 0.5 b^T H b
    relax: np.ndarray  # (L, 2) shift already added to h (lineqp.limit_relaxation)


@dataclass
class GenQP:
    fp: np.ndarray   # f'(p^k)
    fpp: np.ndarray  # f''(p^k)
    lo: np.ndarray   # (G, 2)
    hi: np.ndarray   # (G, 2)
    fq: np.ndarray = None   # reactive power's f', f'' (None: zero, the cost has no reactive term)
    fqq: np.ndarray = None


@dataclass
class BusQP:
    pdk: np.ndarray  # p_i^{d,(k)}
    qdk: np.ndarray  # q_i^{d,(k)}
    lo: np.ndarray   # (B, 2) box of (d_w, d_th) (shared by every line copy)
    hi: np.ndarray


@dataclass
class QP:
    line: LineQP
    gen: GenQP
    bus: BusQP
    delta: float
    ref: int


def elimination(grid, x: Iterate, rhs_shift=None):
    """Solve the linearised (opfc11) and (opfc12) of (QPsub) for d_wR, d_wI
    as affine functions of z = (d_w_i, d_th_i, d_w_j, d_th_j) (eq. elim):
    returns a^R, b^R, a^I, b^I.  ``rhs_shift`` (n_line, 2) adds to the
    right-hand sides of the two linearised constraints (sensitivity tests)."""
    f, t = grid.f, grid.t
    wi, wj = x.w[f], x.w[t]
    ph = x.th[f] - x.th[t]
    s, c = np.sin(ph), np.cos(ph)
    wR, wI = x.wR, x.wI
    # linear system in (d_wR, d_wI):
    #   [2wR  2wI] [d_wR]   [r1 + wj d_wi + wi d_wj            ]
    #   [ s   -c ] [d_wI] = [r2 - K d_thi + K d_thj            ]
    # with r1 = wi wj - wR^2 - wI^2, r2 = -wR s + wI c, K = wR c + wI s.
    K = wR * c + wI * s
    r1 = wi * wj - wR ** 2 - wI ** 2
    r2 = -wR * s + wI * c
    if rhs_shift is not None:
        r1 = r1 + rhs_shift[:, 0]
        r2 = r2 + rhs_shift[:, 1]
    if np.any(np.abs(K) < 1e-8):
        raise FloatingPointError("elimination: wR cos + wI sin vanishes")
    det = -2.0 * K
    # inverse of [[2wR, 2wI], [s, -c]] = (1/det) [[-c, -2wI], [-s, 2wR]]
    i00, i01, i10, i11 = -c / det, -2 * wI / det, -s / det, 2 * wR / det
    # right-hand side as (coefficients on z, constant)
    rhs1 = np.stack([wj, np.zeros_like(wj), wi, np.zeros_like(wj)], 1)
    rhs2 = np.stack([np.zeros_like(K), -K, np.zeros_like(K), K], 1)
    aR = i00[:, None] * rhs1 + i01[:, None] * rhs2
    aI = i10[:, None] * rhs1 + i11[:, None] * rhs2
    bR = i00 * r1 + i01 * r2
    bI = i10 * r1 + i11 * r2
    return aR, bR, aI, bI


def lift_matrix(aR, bR, aI, bI):
    """A_ij (6x4) and b_ij (6) of Section IV-B2 (rows in u order)."""
    n = aR.shape[0]
    A = np.zeros((n, 6, 4))
    A[:, 0, 0] = 1.0
    A[:, 1, 1] = 1.0
    A[:, 2, :] = aR
    A[:, 3, :] = aI
    A[:, 4, 2] = 1.0
    A[:, 5, 3] = 1.0
    b = np.zeros((n, 6))
    b[:, 2] = bR
    b[:, 3] = bI
    return A, b


def psd_project(M):
    """Nearest PSD matrix in Frobenius norm: clip negative eigenvalues to 0."""
    lam, V = np.linalg.eigh(M)
    lam = np.maximum(lam, 0.0)
    P = (V * lam[:, None, :]) @ np.swapaxes(V, 1, 2)
    return 0.5 * (P + np.swapaxes(P, 1, 2))


def restoration_hessian(grid):
    """Per-line Hessian of the restoration QP's objective 0.5 ||d||^2 in
    u = (w_i, th_i, wR, wI, w_j, th_j): each bus variable's term shared
    among its incident lines (1 / degree), so that the shares add up to
    0.5 (d_w^2 + d_th^2) per bus."""
    deg = np.bincount(grid.f, minlength=grid.n_bus) + np.bincount(grid.t, minlength=grid.n_bus)
    wf, wt = 1.0 / deg[grid.f], 1.0 / deg[grid.t]
    one = np.ones(grid.n_line)
    diag = np.stack([wf, wf, one, one, wt, wt], 1)
    return np.einsum("li,ij->lij", diag, np.eye(6))


def build_qp(grid, x: Iterate, pi: np.ndarray, delta: float, hessian_mode: str = "psd",
             rhs_shift=None, c_shift=None) -> QP:
    """Data of (QPsub) at iterate x with line multipliers pi and trust radius delta.

    ``hessian_mode`` "restore": the QP of a feasibility restoration step, the
    same linearised constraints with the objective 0.5 ||d||^2 (lines:
    ``restoration_hessian``; generators 0.5 (d_p^2 + d_q^2); pi unused).

    ``c_shift`` (n_line, 4), if given, is added to the constraint values
    c11..c14 of (opfc11-14) at x in their linearisations (opfqpc11-14): the
    QP of a second-order correction, whose linearised constraints then read
    c(x) + e + grad c(x)^T d with e the second-order error of a trial step."""
    f, t = grid.f, grid.t
    n = grid.n_line
    if c_shift is not None:
        # the elimination's right-hand sides are -c11 and -c12
        cs = -np.asarray(c_shift, dtype=np.float64)[:, :2]
        rhs_shift = cs if rhs_shift is None else rhs_shift + cs
    aR, bR, aI, bI = elimination(grid, x, rhs_shift)
    if hessian_mode == "restore":
        H = restoration_hessian(grid)
    else:
        H = line_hessian(grid, x, pi)
    A, b = lift_matrix(aR, bR, aI, bI)
    At = np.swapaxes(A, 1, 2)
    M = At @ H @ A
    M = 0.5 * (M + np.swapaxes(M, 1, 2))
    if hessian_mode == "psd":
        M = psd_project(M)
    elif hessian_mode not in ("raw", "restore"):
        raise ValueError(hessian_mode)
    q = (At @ (H @ b[:, :, None]))[:, :, 0]
    c0 = 0.5 * np.einsum("li,lij,lj->l", b, H, b)

    # flow substitution (Section IV-B2): d_flow = F z + f0
    F = np.zeros((n, 4, 4))
    e0 = np.zeros((n, 4)); e0[:, 0] = 1.0
    e2 = np.zeros((n, 4)); e2[:, 2] = 1.0
    col = lambda v: v[:, None]
    F[:, 0] = col(grid.gii) * e0 + col(grid.gij) * aR + col(grid.bij) * aI
    F[:, 1] = -col(grid.bii) * e0 - col(grid.bij) * aR + col(grid.gij) * aI
    F[:, 2] = col(grid.gjj) * e2 + col(grid.gji) * aR - col(grid.bji) * aI
    F[:, 3] = -col(grid.bjj) * e2 - col(grid.bji) * aR - col(grid.gji) * aI
    f0 = np.stack([grid.gij * bR + grid.bij * bI,
                   -grid.bij * bR + grid.gij * bI,
                   grid.gji * bR - grid.bji * bI,
                   -grid.bji * bR - grid.gji * bI], 1)

    # bus box of (d_w, d_th): bounds (opfc3, opfc4) shifted to the iterate, intersected with the TR
    wlo = np.maximum(-delta, grid.vmin ** 2 - x.w)
    whi = np.minimum(delta, grid.vmax ** 2 - x.w)
    tlo = np.maximum(-delta, -TWO_PI - x.th)
    thi = np.minimum(delta, TWO_PI - x.th)
    tlo[grid.ref] = 0.0
    thi[grid.ref] = 0.0
    wlo = np.minimum(wlo, whi)
    tlo = np.minimum(tlo, thi)
    blo = np.stack([wlo, tlo], 1)
    bhi = np.stack([whi, thi], 1)
    lo = np.concatenate([blo[f], blo[t]], 1)
    hi = np.concatenate([bhi[f], bhi[t]], 1)

    pij, qij, pji, qji = flows(grid, x.w, x.wR, x.wI)
    pk = np.stack([pij, qij, pji, qji], 1)
    # linearised limits (opfqpc13, opfqpc14) in z
    G = np.zeros((n, 2, 4))
    G[:, 0] = 2 * col(pij) * F[:, 0] + 2 * col(qij) * F[:, 1]
    G[:, 1] = 2 * col(pji) * F[:, 2] + 2 * col(qji) * F[:, 3]
    h = np.stack([grid.smax_ij ** 2 - pij ** 2 - qij ** 2 - 2 * pij * f0[:, 0] - 2 * qij * f0[:, 1],
                  grid.smax_ji ** 2 - pji ** 2 - qji ** 2 - 2 * pji * f0[:, 2] - 2 * qji * f0[:, 3]], 1)
    if c_shift is not None:
        # c13 + e13 - 2 p_ij dp_ij - 2 q_ij dq_ij >= 0  <=>  G z <= h + e13
        h = h + np.asarray(c_shift, dtype=np.float64)[:, 2:4]
    # a line whose box and limit rows do not intersect gets its rows relaxed
    # by its least-squares violation (plus a rounding guard): the QP's line
    # minimiser is then the limit of the paper's line solver on that line
    relax = limit_relaxation(lo, hi, G, h)
    h = h + relax

    # generators (eq. gen_kernel bounds)
    fp = 2 * grid.cost2 * x.pg + grid.cost1
    fpp = 2 * grid.cost2
    plo = np.maximum(-delta, grid.pmin - x.pg)
    phi = np.minimum(delta, grid.pmax - x.pg)
    qlo = np.maximum(-delta, grid.qmin - x.qg)
    qhi = np.minimum(delta, grid.qmax - x.qg)
    plo, qlo = np.minimum(plo, phi), np.minimum(qlo, qhi)

    # buses: p_i^{d,(k)}, q_i^{d,(k)} (constants after eq. acopf_qppf)
    nb = grid.n_bus
    pdk = (grid.pd - np.bincount(grid.gbus, x.pg, nb)
           + np.bincount(f, pij, nb) + np.bincount(t, pji, nb) + grid.gsh * x.w)
    qdk = (grid.qd - np.bincount(grid.gbus, x.qg, nb)
           + np.bincount(f, qij, nb) + np.bincount(t, qji, nb) - grid.bsh * x.w)

    return QP(
        line=LineQP(aR, bR, aI, bI, H, M, q, F, f0, lo, hi, G, h, pk, c0, relax),
        gen=(GenQP(np.zeros(grid.n_gen), np.ones(grid.n_gen), np.stack([plo, qlo], 1), np.stack([phi, qhi], 1),
                   np.zeros(grid.n_gen), np.ones(grid.n_gen)) if hessian_mode == "restore"
             else GenQP(fp, fpp, np.stack([plo, qlo], 1), np.stack([phi, qhi], 1))),
        bus=BusQP(pdk, qdk, blo, bhi),
        delta=float(delta), ref=int(grid.ref),
    )


def qp_objective(qp: QP, dpg, zline):
    """Model objective of (QPsub) in eliminated form: generator quadratic terms
    plus, per line, 0.5 z^T M z + q^T z + 0.5 b^T H b (the constant keeps
    the value equal to the unreduced 0.5 u^T H u when M is not projected)."""
    g = qp.gen
    L = qp.line
    val = np.sum(g.fp * dpg + 0.5 * g.fpp * dpg * dpg)
    val += np.sum(0.5 * np.einsum("li,lij,lj->l", zline, L.M, zline)
                  + np.einsum("li,li->l", L.q, zline) + L.c0)
    return float(val)
