"""Trust-region SQP around the ADMM QP solver (Section II, Algorithm 1), with
the multiplier recovery and step return of Section IV-B5.

Readings where the paper is silent (also listed in the design notes):
* start: flat start (``acopf.flat_start``), pi = 0, Delta0 = 1; the linear
  feasibility projection (eq. linfeas) is not run: the power balance is
  linear, so the first QP restores it;
* the step: d_pg, d_qg from the generator side, d_w, d_th from the bus side,
  d_wR, d_wI by the elimination (eq. elim) applied to the bus-side values,
  so the linearised (opfc11, opfc12) hold exactly;
* multipliers pi (eq. lag): pi13, pi14 = -mu of the line-limit rows of the
  last line solve (the paper's plus-sign Lagrangian makes them <= 0);
  pi11, pi12 from the stationarity of the line subproblem in (d_wR, d_wI)
  before elimination, a 2x2 system with determinant -2(wR cos + wI sin);
* acceptance: ared > 0 and pred > 0 (then ared/pred > 0); the trust radius
  doubles (up to Delta_max) after an accepted step that reached it with
  ared >= 0.75 pred, stays put after other accepted steps, and becomes
  0.5 min(Delta, ||d||_inf) after a rejection;
* the model q(d; mu) of Section II-C takes the full step: its quadratic
  term is 0.5 u^T H u over the lifted line steps u = A z + b of eq. elim
  (d_wR, d_wI included), which in eliminated form is 0.5 z^T M z + q^T z +
  0.5 b^T H b per line.  With the PSD projection the Hessian is the one
  whose reduction is the projected M (H plus the change of M on the z
  block), so the same three terms hold with the projected M;
* pi and the ADMM multipliers are carried to the next iteration (warm
  start); pi is replaced only on acceptance;
* second-order correction (``soc``): a rejected step with pred > 0 gets a
  second QP whose linearised (opfc11-14) carry the step's second-order
  error e = c(x + d) - c(x) - grad c(x)^T d; it starts from the rejected
  solve's multipliers, its step is accepted iff its actual reduction is
  positive (against the first step's pred), and the radius then grows as
  after any accepted step that reached it.  The next solve starts from the
  correction solve's multipliers whether or not its step was taken;
* optional safeguard (``pi_if_converged``, off by default): pi is replaced
  only if the solve also met its stop test (eps > 0).  On a QP without a
  feasible point the ADMM multipliers grow with every sweep; their
  estimates scale the next line Hessians without bound, until the line
  matrices cannot be factored in FP64.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

from . import acopf, admm, qp as qpmod
from .acopf import Iterate


@dataclass
class SqpParams:
    rho: float = 2e4
    max_sweeps: int = 20000
    eps_pri: float = 1e-4
    eps_dual: float = 1e-4
    mu_merit: float = 1e5
    delta0: float = 1.0
    delta_max: float = 10.0
    delta_min: float = 1e-8
    tol_primal: float = 1e-4
    tol_dual: float = 1e-4
    tol_step: float = 1e-6
    max_iter: int = 30
    hessian_mode: str = "psd"
    # "admm": the QP is solved by the serial ADMM of Algorithm 2 (the method);
    # "direct": by the interior-point solve of the same eliminated QP
    # (``direct.solve``), which gives the SQP iterates of exact QP solutions
    qp_solver: str = "admm"
    # line subproblems of the ADMM: "exact" (enumeration; needs a positive
    # definite line matrix, so hessian_mode "psd" or a convex "raw"), or
    # "alm": the paper's local method (Section IV-B2) on the unmodified
    # Hessians (hessian_mode "raw")
    line_solver: str = "exact"
    # an accepted step that reached the radius doubles it when
    # ared >= grow_ratio * pred
    grow_ratio: float = 0.75
    # second-order correction of a rejected step (the remedy the paper names
    # as future work at the end of Section II-D): re-solve the QP with the
    # second-order error of the step added to the linearised constraints
    soc: bool = False
    # Algorithm 1 before the loop: a start that violates the linear
    # constraints (balance, bounds) by more than linfeas_tol is first
    # projected onto them (eq. linfeas)
    linfeas: bool = False
    linfeas_tol: float = 1e-8
    # False: an accepted step always takes the new multiplier estimates
    # (Algorithm 1).  True: only when the ADMM solve met its stop test (a
    # safeguard for QPs without a feasible point; see the module docstring).
    pi_if_converged: bool = False
    # feasibility restoration (named by the paper as missing, Section V):
    # when the radius falls below delta_min, up to max_restore times a
    # restoration step is taken instead of stopping: the QP with the same
    # linearised constraints and the objective 0.5 ||d||^2 (hessian mode
    # "restore") within radius restore_delta (0: delta0), solved cold; it is
    # accepted iff it lowers the constraint violation h of the merit
    # function, and then the radius restarts at delta0 and the next QP solve
    # starts cold; pi is kept.  A rejected restoration step ends the run
    # (TR_COLLAPSED).
    restore: bool = False
    max_restore: int = 3
    restore_delta: float = 0.0


@dataclass
class SqpRecord:
    k: int
    accepted: bool
    ared: float
    pred: float
    delta: float
    step_inf: float
    sweeps: int
    r: float
    s: float
    objective: float
    primal: float
    dual: float
    soc: bool = False
    restore: bool = False


@dataclass
class SqpResult:
    x: Iterate
    pi: np.ndarray
    outcome: str
    iterations: int
    records: list = field(default_factory=list)


def step_from_bus_values(grid, qp, pg, qg, dw, dth) -> Iterate:
    """Full step d from generator-side (d_pg, d_qg) and bus-side (d_w, d_th):
    d_wR, d_wI by the elimination (eq. elim) of each line's end values."""
    z = np.stack([dw[grid.f], dth[grid.f], dw[grid.t], dth[grid.t]], 1)
    L = qp.line
    dwR = np.einsum("li,li->l", L.aR, z) + L.bR
    dwI = np.einsum("li,li->l", L.aI, z) + L.bI
    return Iterate(np.array(pg, copy=True), np.array(qg, copy=True), np.array(dw, copy=True),
                   np.array(dth, copy=True), dwR, dwI)


def assemble_step(grid, qp, st: admm.AdmmState) -> Iterate:
    """Trial step d returned to SQP after the ADMM solve."""
    return step_from_bus_values(grid, qp, st.xg[:, 0], st.xg[:, 1], st.dw, st.dth)


def pi_from_line_kkt(grid, x: Iterate, qp, z, lam_f, mu) -> np.ndarray:
    """Multipliers pi of (opfc11-14) from the stationarity of a line's QP in
    (d_wR, d_wI) before elimination, given the line's voltage step z (n, 4),
    the multipliers lam_f (n, 4) of its four flow terms and mu (n, 2) >= 0 of
    its two linearised limit rows G z <= h."""
    L = qp.line
    A, b = qpmod.lift_matrix(L.aR, L.bR, L.aI, L.bI)
    u = (A @ z[:, :, None])[:, :, 0] + b
    Hu = (L.H @ u[:, :, None])[:, :, 0]
    lam = lam_f
    pij, qij, pji, qji = L.pk[:, 0], L.pk[:, 1], L.pk[:, 2], L.pk[:, 3]
    dfR = np.stack([grid.gij, -grid.bij, grid.gji, -grid.bji], 1)
    dfI = np.stack([grid.bij, grid.gij, -grid.bji, -grid.gji], 1)
    llR = np.stack([2 * pij * grid.gij - 2 * qij * grid.bij, 2 * pji * grid.gji - 2 * qji * grid.bji], 1)
    llI = np.stack([2 * pij * grid.bij + 2 * qij * grid.gij, -2 * pji * grid.bji - 2 * qji * grid.gji], 1)
    gR = Hu[:, 2] + np.sum(lam * dfR, 1) + np.sum(mu * llR, 1)
    gI = Hu[:, 3] + np.sum(lam * dfI, 1) + np.sum(mu * llI, 1)
    ph = x.th[grid.f] - x.th[grid.t]
    s, c = np.sin(ph), np.cos(ph)
    # [2wR  s] [pi11]     [gR]
    # [2wI -c] [pi12] = - [gI]
    det = -2 * x.wR * c - 2 * x.wI * s
    p11 = (-gR * (-c) - s * (-gI)) / det
    p12 = (2 * x.wR * (-gI) - 2 * x.wI * (-gR)) / det
    return np.stack([p11, p12, -mu[:, 0], -mu[:, 1]], 1)


def recover_pi(grid, x: Iterate, qp, st: admm.AdmmState) -> np.ndarray:
    """Multipliers pi of (opfc11-14) from the KKT conditions of the line
    subproblems (eq. line_kernel) at the line-side solution."""
    return pi_from_line_kkt(grid, x, qp, st.xl[:, 4:8], st.lam_l[:, :4], st.mu)


def direct_qp_step(grid, x: Iterate, qp):
    """Step, pi and balance multipliers from the interior-point solve of the
    eliminated QP.  The flow multipliers of a line are minus the balance
    multipliers of the bus the flow leaves (a flow enters its bus's balance
    with coefficient -1)."""
    from . import direct
    sol = direct.solve(grid, qp)
    ix = direct.var_index(grid)
    y = sol.y
    d = step_from_bus_values(grid, qp, y[ix["pg"]], y[ix["qg"]], y[ix["w"]], y[ix["th"]])
    B = grid.n_bus
    nup, nuq = sol.nu[:B], sol.nu[B:]
    f, t = grid.f, grid.t
    lam_f = -np.stack([nup[f], nuq[f], nup[t], nuq[t]], 1)
    mu = sol.mu.reshape(grid.n_line, 2)
    pi = pi_from_line_kkt(grid, x, qp, np.stack([d.w[f], d.th[f], d.w[t], d.th[t]], 1), lam_f, mu)
    return d, pi, nup, nuq


def linearised_constraints(grid, x: Iterate, qp, d: Iterate):
    """c_i(x) + grad c_i(x)^T d for (opfc11-14)."""
    f, t = grid.f, grid.t
    wi, wj = x.w[f], x.w[t]
    ph = x.th[f] - x.th[t]
    s, c = np.sin(ph), np.cos(ph)
    c11, c12, c13, c14 = acopf.nonlinear_constraints(grid, x)
    K = x.wR * c + x.wI * s
    l11 = c11 + 2 * x.wR * d.wR + 2 * x.wI * d.wI - wj * d.w[f] - wi * d.w[t]
    l12 = c12 + s * d.wR - c * d.wI + K * (d.th[f] - d.th[t])
    dp = acopf.flows(grid, d.w, d.wR, d.wI)
    pk = qp.line.pk
    l13 = c13 - 2 * pk[:, 0] * dp[0] - 2 * pk[:, 1] * dp[1]
    l14 = c14 - 2 * pk[:, 2] * dp[2] - 2 * pk[:, 3] * dp[3]
    return l11, l12, l13, l14


def model_m(grid, x: Iterate, qp, d: Iterate) -> float:
    """m(d) of Section II-C: l1 violation of the linearised nonlinear constraints."""
    l11, l12, l13, l14 = linearised_constraints(grid, x, qp, d)
    neg = lambda v: np.maximum(0.0, -v)
    return float(np.abs(l11).sum() + np.abs(l12).sum() + neg(l13).sum() + neg(l14).sum())


def second_order_error(grid, x: Iterate, qp, d: Iterate) -> np.ndarray:
    """e = c(x + d) - c(x) - grad c(x)^T d of (opfc11-14) per line (n, 4):
    the shift of the second-order correction QP."""
    lin = linearised_constraints(grid, x, qp, d)
    cn = acopf.nonlinear_constraints(grid, x.plus(d))
    return np.stack([a - b for a, b in zip(cn, lin)], 1)


def predicted_reduction(grid, x: Iterate, qp, d: Iterate, mu_merit: float) -> float:
    """q(0; mu) - q(d; mu) of Section II-C: q(d) = grad f^T d + 0.5 d^T H d
    + mu m(d) with the full step d (the line quadratic in eliminated form
    is 0.5 z^T M z + q^T z + 0.5 b^T H b, ``qp.qp_objective``)."""
    z = np.stack([d.w[grid.f], d.th[grid.f], d.w[grid.t], d.th[grid.t]], 1)
    quad = qpmod.qp_objective(qp, d.pg, z)
    return float(-quad + mu_merit * (acopf.infeas_h(grid, x) - model_m(grid, x, qp, d)))


def step_norm(d: Iterate) -> float:
    return float(max(np.abs(d.pg).max(initial=0), np.abs(d.qg).max(initial=0),
                     np.abs(d.w).max(initial=0), np.abs(d.th).max(initial=0)))


def solve(grid, params: SqpParams = SqpParams(), x0: Iterate | None = None, time_fn=None) -> SqpResult:
    """Algorithm 1 with the ADMM QP solver."""
    x = acopf.flat_start(grid) if x0 is None else x0.copy()
    if params.linfeas:
        from . import linfeas
        if linfeas.violation(grid, x) > params.linfeas_tol:
            x = linfeas.project(grid, x).x
    pi = np.zeros((grid.n_line, 4))
    delta = params.delta0
    rho = admm.Rho.scalar(grid, params.rho)
    lam_g = lam_l = None
    recs = []
    outcome = "MAX_ITER"
    restores = 0
    restoring = False

    def qp_solve(qp, lam_g, lam_l):
        if params.qp_solver == "direct":
            d, pi_new, nup, nuq = direct_qp_step(grid, x, qp)
            return d, pi_new, nup, nuq, admm.AdmmResult(None, 0, 0.0, 0.0, True, 0), lam_g, lam_l
        if params.qp_solver != "admm":
            raise ValueError(params.qp_solver)
        start = admm.cold_state(grid) if lam_g is None else admm.warm_state(grid, lam_g, lam_l)
        res = admm.solve(grid, qp, rho, params.max_sweeps, params.eps_pri, params.eps_dual, start,
                         line_solver=params.line_solver)
        st = res.state
        return (assemble_step(grid, qp, st), recover_pi(grid, x, qp, st), st.nu[:, 0], st.nu[:, 1], res,
                st.lam_g, st.lam_l)

    for k in range(params.max_iter):
        if restoring:
            # feasibility restoration step (see SqpParams.restore)
            restoring = False
            restores += 1
            dr = params.restore_delta if params.restore_delta > 0 else params.delta0
            qp = qpmod.build_qp(grid, x, pi, dr, "restore")
            d, _, nup, nuq, res, _, _ = qp_solve(qp, None, None)
            xt = x.plus(d)
            h0, h1 = acopf.infeas_h(grid, x), acopf.infeas_h(grid, xt)
            accepted = h1 < h0
            if accepted:
                x = xt
                delta = params.delta0
            lam_g = lam_l = None
            pr = acopf.primal_infeasibility(grid, x)["primal"]
            du = acopf.dual_infeasibility(grid, x, nup, nuq, pi)
            recs.append(SqpRecord(k, accepted, h0 - h1, 0.0, dr, step_norm(d), res.sweeps, res.r, res.s,
                                  acopf.objective(grid, x.pg), pr, du, False, True))
            if not accepted:
                outcome = "TR_COLLAPSED"
                break
            continue
        qp = qpmod.build_qp(grid, x, pi, delta, params.hessian_mode)
        d, pi_new, nup, nuq, res, lam_g, lam_l = qp_solve(qp, lam_g, lam_l)
        xt = x.plus(d)
        phi0 = acopf.merit(grid, x, params.mu_merit)
        ared = phi0 - acopf.merit(grid, xt, params.mu_merit)
        pred = predicted_reduction(grid, x, qp, d, params.mu_merit)
        dn = step_norm(d)
        accepted = ared > 0 and pred > 0
        soc_used = False
        if not accepted and params.soc and pred > 0:
            # second-order correction: same model, constraints shifted by the
            # step's second-order error; judged against the first model's pred
            e = second_order_error(grid, x, qp, d)
            qp2 = qpmod.build_qp(grid, x, pi, delta, params.hessian_mode, c_shift=e)
            try:
                d2, pi2, nup2, nuq2, res2, lg2, ll2 = qp_solve(qp2, lam_g, lam_l)
                xt2 = x.plus(d2)
                ared2 = phi0 - acopf.merit(grid, xt2, params.mu_merit)
                # the next solve starts from the last solve's multipliers and
                # the residual report uses its bus update, taken or not
                lam_g, lam_l, nup, nuq = lg2, ll2, nup2, nuq2
            except (RuntimeError, np.linalg.LinAlgError, FloatingPointError):
                ared2 = -np.inf  # the correction QP has no solution: the step stays rejected
            if ared2 > 0:
                d, pi_new, res = d2, pi2, res2
                xt, ared, accepted, soc_used = xt2, ared2, True, True
        if accepted:
            x = xt
            stop_set = params.eps_pri > 0 or params.eps_dual > 0
            if not params.pi_if_converged or (stop_set and res.converged):
                pi = pi_new
            if dn >= 0.99 * delta and ared >= params.grow_ratio * pred:
                delta = min(2 * delta, params.delta_max)
        else:
            delta = 0.5 * min(delta, dn)
        pr = acopf.primal_infeasibility(grid, x)["primal"]
        du = acopf.dual_infeasibility(grid, x, nup, nuq, pi)
        recs.append(SqpRecord(k, accepted, ared, pred, delta, dn, res.sweeps, res.r, res.s,
                              acopf.objective(grid, x.pg), pr, du, soc_used))
        if accepted and pr <= params.tol_primal and du <= params.tol_dual:
            outcome = "CONVERGED"
            break
        if accepted and dn < params.tol_step:
            outcome = "SMALL_STEP"
            break
        if delta < params.delta_min:
            if params.restore and restores < params.max_restore:
                restoring = True
                continue
            outcome = "TR_COLLAPSED"
            break
    return SqpResult(x, pi, outcome, len(recs), recs)
