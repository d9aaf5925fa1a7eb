"""Pins of the oracle's SQP-level functions (Section II: the l1 merit, its
model q(d; mu), Algorithm 1) and of the residual report, against finite
differences, hand-computed cases and an independent solve of the full
ACOPF (eq. acopf) by SciPy."""
import numpy as np
import pytest
from scipy.optimize import minimize

from synth.grids import Grid, grid_14, tiny_grid, power_flow_start
from oracle import acopf, qp as qpm, sqp


def _random_iterate(g, rng, spread=0.05):
    w = rng.uniform(0.9, 1.1, g.n_bus)
    th = rng.uniform(-0.3, 0.3, g.n_bus)
    th[g.ref] = 0.0
    ph = th[g.f] - th[g.t]
    vv = np.sqrt(w[g.f] * w[g.t])
    wR = vv * np.cos(ph) * (1 + spread * rng.standard_normal(g.n_line))
    wI = vv * np.sin(ph) + spread * rng.standard_normal(g.n_line)
    return acopf.Iterate(rng.uniform(0, 1, g.n_gen), rng.uniform(-0.5, 0.5, g.n_gen), w, th, wR, wI)


def _vec(x):
    return np.concatenate([x.pg, x.qg, x.w, x.th, x.wR, x.wI])


def _unvec(g, v):
    out, o = [], 0
    for n in (g.n_gen, g.n_gen, g.n_bus, g.n_bus, g.n_line, g.n_line):
        out.append(v[o:o + n])
        o += n
    return acopf.Iterate(*out)


def test_lagrangian_gradient_matches_central_differences():
    """grad of f + y_p c_P + y_q c_Q + sum pi c_nl, assembled here from
    ``objective``, ``balance`` and ``nonlinear_constraints`` only."""
    g = tiny_grid(seed=5, n_bus=6, n_line=9, n_gen=3)
    rng = np.random.default_rng(1)
    x = _random_iterate(g, rng)
    yp, yq = rng.standard_normal(g.n_bus) * 50, rng.standard_normal(g.n_bus) * 50
    pi = rng.standard_normal((g.n_line, 4)) * 30

    def lag(v):
        xv = _unvec(g, v)
        rp, rq = acopf.balance(g, xv)
        cs = acopf.nonlinear_constraints(g, xv)
        return acopf.objective(g, xv.pg) + yp @ rp + yq @ rq + sum(pi[:, k] @ cs[k] for k in range(4))

    v0 = _vec(x)
    eps = 1e-6
    fd = np.array([(lag(v0 + eps * e) - lag(v0 - eps * e)) / (2 * eps) for e in np.eye(v0.size)])
    got = np.concatenate(acopf.lagrangian_gradient(g, x, yp, yq, pi))
    assert np.abs(got - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_linearised_constraints_and_model_m_are_first_order_taylor():
    """c(x) + grad c(x)^T d of (opfc11-14) against central differences of
    ``nonlinear_constraints`` along d, and m(d) as the l1 violation of them."""
    g = tiny_grid(seed=7, n_bus=6, n_line=9, n_gen=3)
    rng = np.random.default_rng(2)
    x = _random_iterate(g, rng)
    pi = np.zeros((g.n_line, 4))
    Q = qpm.build_qp(g, x, pi, 0.1)
    d = _unvec(g, 0.05 * rng.standard_normal(_vec(x).size))
    eps = 1e-6
    cp = acopf.nonlinear_constraints(g, _unvec(g, _vec(x) + eps * _vec(d)))
    cm = acopf.nonlinear_constraints(g, _unvec(g, _vec(x) - eps * _vec(d)))
    c0 = acopf.nonlinear_constraints(g, x)
    lin_fd = [c0[k] + (cp[k] - cm[k]) / (2 * eps) for k in range(4)]
    lin = sqp.linearised_constraints(g, x, Q, d)
    for k in range(4):
        assert np.abs(lin[k] - lin_fd[k]).max() <= 1e-8 * (1 + np.abs(lin_fd[k]).max())
    m_fd = (np.abs(lin_fd[0]).sum() + np.abs(lin_fd[1]).sum() + np.maximum(0, -lin_fd[2]).sum()
            + np.maximum(0, -lin_fd[3]).sum())
    assert sqp.model_m(g, x, Q, d) == pytest.approx(m_fd, rel=1e-8)
    # the second-order error is what the linearisation leaves of c(x + d)
    e = sqp.second_order_error(g, x, Q, d)
    cn = acopf.nonlinear_constraints(g, x.plus(d))
    for k in range(4):
        np.testing.assert_allclose(e[:, k], cn[k] - lin_fd[k], atol=1e-8)


@pytest.mark.parametrize("mode", ["raw", "psd"])
def test_predicted_reduction_is_q0_minus_qd_on_the_full_step(mode):
    """pred = q(0; mu) - q(d; mu) of Section II-C evaluated without the
    elimination's algebra: grad f^T d + 0.5 d^T H d over the full step
    (d_wR, d_wI included) with the line Hessian of eq. lag; in PSD mode the
    Hessian whose reduction is the projected M (H plus the projection's
    change on the z block)."""
    g = tiny_grid(seed=9, n_bus=6, n_line=9, n_gen=3)
    rng = np.random.default_rng(3)
    x = _random_iterate(g, rng, spread=0.1)   # c11, c12 != 0: b of eq. elim is nonzero
    pi = rng.standard_normal((g.n_line, 4)) * 40
    pi[:, 2:] = -np.abs(pi[:, 2:])
    pi[:, 0] -= 60.0  # an indefinite line Hessian somewhere (PSD projection acts)
    Q = qpm.build_qp(g, x, pi, 0.2, mode)
    dw, dth = 0.05 * rng.standard_normal(g.n_bus), 0.05 * rng.standard_normal(g.n_bus)
    dth[g.ref] = 0.0
    d = sqp.step_from_bus_values(g, Q, 0.1 * rng.standard_normal(g.n_gen), 0.1 * rng.standard_normal(g.n_gen),
                                 dw, dth)
    H = acopf.line_hessian(g, x, pi)
    if mode == "psd":
        Mraw = qpm.build_qp(g, x, pi, 0.2, "raw").line.M
        sel = [0, 1, 4, 5]
        H = H.copy()
        for a, i in enumerate(sel):
            for b, j in enumerate(sel):
                H[:, i, j] += Q.line.M[:, a, b] - Mraw[:, a, b]
        assert np.abs(Q.line.M - Mraw).max() > 1e-3
    u = np.stack([d.w[g.f], d.th[g.f], d.wR, d.wI, d.w[g.t], d.th[g.t]], 1)
    fgrad = 2 * g.cost2 * x.pg + g.cost1
    quad = fgrad @ d.pg + (g.cost2 * d.pg ** 2).sum() + 0.5 * np.einsum("li,lij,lj->", u, H, u)
    mu = 1e3
    q0 = mu * acopf.infeas_h(g, x)
    qd = quad + mu * sqp.model_m(g, x, Q, d)
    assert abs(np.einsum("li,lij,lj->", u, H, u)) > 1e-3
    assert sqp.predicted_reduction(g, x, Q, d, mu) == pytest.approx(q0 - qd, rel=1e-10, abs=1e-9)


def _hand_grid():
    """Two buses, one line, one generator; numbers chosen so that every
    quantity below is exact in a few decimal places."""
    one = lambda v: np.array([v], dtype=np.float64)
    two = lambda a, b: np.array([a, b], dtype=np.float64)
    return Grid(n_bus=2, n_line=1, n_gen=1, ref=0,
                vmin=two(0.94, 0.94), vmax=two(1.06, 1.06), pd=two(0.1, 0.2), qd=two(0.1, 0.05),
                gsh=two(0.0, 0.0), bsh=two(0.0, 0.0),
                f=np.array([0]), t=np.array([1]),
                gii=one(2.0), bii=one(-4.9), gij=one(-2.0), bij=one(5.0),
                gji=one(-2.0), bji=one(5.0), gjj=one(2.0), bjj=one(-4.9),
                smax_ij=one(1.0), smax_ji=one(2.0),
                gbus=np.array([0]), pmin=one(0.0), pmax=one(1.0), qmin=one(-0.25), qmax=one(0.25),
                cost2=one(2.0), cost1=one(3.0), name="hand2")


def test_merit_and_residuals_hand_case():
    """At w = (1, 1), th = (0, 0), wR = 1.1, wI = 0.2, pg = 0.5, qg = 0.3:
    c11 = 1.21 + 0.04 - 1 = 0.25, c12 = -wI = -0.2; p_ij = 2 - 2.2 + 1 =
    0.8, q_ij = 4.9 - 5.5 - 0.4 = -1, c13 = 1 - 0.64 - 1 = -0.64; p_ji =
    2 - 2.2 - 1 = -1.2, q_ji = 4.9 - 5.5 + 0.4 = -0.2, c14 = 4 - 1.44 - 0.04
    = 2.52; h = 0.25 + 0.2 + 0.64 = 1.09; f = 2 * 0.25 + 3 * 0.5 = 2.
    Balance: bus 0 p 0.5 - 0.1 - 0.8 = -0.4, q 0.3 - 0.1 + 1 = 1.2; bus 1
    p -0.2 + 1.2 = 1.0, q -0.05 + 0.2 = 0.15.  qg exceeds qmax by 0.05."""
    g = _hand_grid()
    x = acopf.Iterate(np.array([0.5]), np.array([0.3]), np.array([1.0, 1.0]), np.array([0.0, 0.0]),
                      np.array([1.1]), np.array([0.2]))
    c11, c12, c13, c14 = acopf.nonlinear_constraints(g, x)
    assert (c11[0], c12[0], c13[0], c14[0]) == pytest.approx((0.25, -0.2, -0.64, 2.52), abs=1e-14)
    assert acopf.infeas_h(g, x) == pytest.approx(1.09, abs=1e-14)
    assert acopf.objective(g, x.pg) == pytest.approx(2.0, abs=1e-14)
    assert acopf.merit(g, x, 10.0) == pytest.approx(2.0 + 10.9, abs=1e-13)
    rp, rq = acopf.balance(g, x)
    np.testing.assert_allclose(rp, [-0.4, 1.0], atol=1e-14)
    np.testing.assert_allclose(rq, [1.2, 0.15], atol=1e-14)
    pr = acopf.primal_infeasibility(g, x)
    assert pr["balance"] == pytest.approx(1.2, abs=1e-14)
    assert pr["c11"] == pytest.approx(0.25, abs=1e-14)
    assert pr["c12"] == pytest.approx(0.2, abs=1e-14)
    assert pr["limit"] == pytest.approx(0.64, abs=1e-14)
    assert pr["bounds"] == pytest.approx(0.05, abs=1e-14)
    assert pr["primal"] == pytest.approx(1.2, abs=1e-14)


def test_dual_infeasibility_hand_cases():
    """With zero multipliers the Lagrangian gradient is f'(pg) = 2 * 2 pg + 3
    on pg and 0 elsewhere.  An interior pg counts |f'|; at the lower bound a
    positive f' is absorbed by the bound's multiplier (0); at the upper bound
    it is not.  The figure is divided by max(1, |f'|)."""
    g = _hand_grid()
    z = lambda n: np.zeros(n)
    for pg, pmin, pmax, want in ((0.5, 0.0, 1.0, 1.0), (0.5, 0.5, 1.0, 0.0), (0.5, 0.0, 0.5, 1.0)):
        gg = Grid(**{**g.__dict__, "pmin": np.array([pmin]), "pmax": np.array([pmax])})
        x = acopf.Iterate(np.array([pg]), np.array([0.0]), np.array([1.0, 1.0]), np.array([0.0, 0.0]),
                          np.array([1.0]), np.array([0.0]))
        assert acopf.dual_infeasibility(gg, x, z(2), z(2), np.zeros((1, 4))) == pytest.approx(want, abs=1e-14)
    gg = Grid(**{**g.__dict__, "cost1": np.array([0.5]), "cost2": np.array([0.1])})
    x = acopf.Iterate(np.array([0.5]), np.array([0.0]), np.array([1.0, 1.0]), np.array([0.0, 0.0]),
                      np.array([1.0]), np.array([0.0]))
    # f' = 0.2 * 0.5 + 0.5 = 0.6: the scale is max(1, 0.6) = 1
    assert acopf.dual_infeasibility(gg, x, z(2), z(2), np.zeros((1, 4))) == pytest.approx(0.6, abs=1e-14)


def _full_acopf_slsqp(g, s):
    """The full ACOPF (eq. acopf) by SciPy's SLSQP from the power-flow start:
    variables (pg, qg, w, th, wR, wI), balance and (opfc11, opfc12) as
    equalities, (opfc13, opfc14) as inequalities, variable bounds, theta_ref
    = 0; derivatives by SciPy's own finite differences."""
    G, B, L = g.n_gen, g.n_bus, g.n_line
    v0 = np.concatenate([s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"]])

    def eq(v):
        xv = _unvec(g, v)
        rp, rq = acopf.balance(g, xv)
        c11, c12, _, _ = acopf.nonlinear_constraints(g, xv)
        return np.concatenate([rp, rq, c11, c12])

    def ineq(v):
        _, _, c13, c14 = acopf.nonlinear_constraints(g, _unvec(g, v))
        return np.concatenate([c13, c14])

    thlo, thhi = np.full(B, -2 * np.pi), np.full(B, 2 * np.pi)
    thlo[g.ref] = thhi[g.ref] = 0.0
    lo = np.concatenate([g.pmin, g.qmin, g.vmin ** 2, thlo, np.full(2 * L, -np.inf)])
    hi = np.concatenate([g.pmax, g.qmax, g.vmax ** 2, thhi, np.full(2 * L, np.inf)])
    r = minimize(lambda v: acopf.objective(g, v[:G]), v0, method="SLSQP", bounds=list(zip(lo, hi)),
                 constraints=[{"type": "eq", "fun": eq}, {"type": "ineq", "fun": ineq}],
                 options={"maxiter": 500, "ftol": 1e-12})
    viol = max(np.abs(eq(r.x)).max(), max(0.0, -ineq(r.x).min()),
               np.maximum(lo - r.x, 0).max(), np.maximum(r.x - hi, 0).max())
    return float(r.fun), float(viol)


@pytest.mark.parametrize("mode", ["psd", "raw"])
def test_sqp_reaches_kkt_point_of_full_acopf(mode):
    """Algorithm 1 (exact QP solves by the interior-point method, l1 merit
    with mu = 1e5, second-order correction of rejected steps) on the 14-bus
    grid ends at primal and dual infeasibility <= 1e-4, and its objective is
    within 1e-4 (relative) of an independent SLSQP solve of the full ACOPF."""
    g = grid_14()
    s = power_flow_start(g)
    x0 = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    res = sqp.solve(g, sqp.SqpParams(qp_solver="direct", hessian_mode=mode, soc=True, max_iter=40), x0)
    assert res.outcome == "CONVERGED", [(r.accepted, r.primal, r.dual) for r in res.records]
    last = res.records[-1]
    assert last.primal <= 1e-4 and last.dual <= 1e-4
    ref, viol = _full_acopf_slsqp(g, s)
    assert viol < 1e-8
    assert abs(last.objective - ref) <= 1e-4 * abs(ref)
    assert any(r.soc for r in res.records)


def test_sqp_without_correction_is_held_back_by_the_merit():
    """Without the second-order correction the same run takes steps far
    below the trust radius the correction reaches: the l1 merit's curvature
    term (mu = 1e5 times the second-order error of (opfc11-14)) rejects
    larger steps (the Maratos effect)."""
    g = grid_14()
    s = power_flow_start(g)
    x0 = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    plain = sqp.solve(g, sqp.SqpParams(qp_solver="direct", soc=False, max_iter=20), x0)
    assert plain.outcome == "MAX_ITER"
    assert max(r.step_inf for r in plain.records if r.accepted) < 0.02


def test_sqp_from_the_flat_start_with_the_linear_feasibility_projection():
    """Algorithm 1 from the flat start: the start violates the power balance,
    so it is first projected onto the linear constraints (eq. linfeas); the
    run then ends at the same KKT point as from the power-flow start (primal
    and dual <= 1e-4, objective within 1e-4 of SLSQP on the full ACOPF)."""
    g = grid_14()
    res = sqp.solve(g, sqp.SqpParams(qp_solver="direct", soc=True, linfeas=True, max_iter=40))
    assert res.outcome == "CONVERGED"
    last = res.records[-1]
    assert last.primal <= 1e-4 and last.dual <= 1e-4
    ref, viol = _full_acopf_slsqp(g, power_flow_start(g))
    assert viol < 1e-8 and abs(last.objective - ref) <= 1e-4 * abs(ref)


def test_restoration_qp_objective_is_half_the_squared_step():
    """The restoration QP (hessian mode "restore") has the same linearised
    constraints and the objective 0.5 ||d||^2: for any bus-side (d_w, d_th),
    the line terms 0.5 z^T M z + q^T z + c0 over all lines add up to
    0.5 (sum_bus (d_w^2 + d_th^2) + sum_line (d_wR^2 + d_wI^2)) with d_wR,
    d_wI from the elimination, and the generator terms are 0.5 (d_p^2 +
    d_q^2); its constraints are those of the ordinary QP."""
    g = grid_14()
    rng = np.random.default_rng(31)
    x = _random_iterate(g, rng)
    pi = rng.standard_normal((g.n_line, 4))
    Q = qpm.build_qp(g, x, pi, 0.05, "restore")
    Q0 = qpm.build_qp(g, x, pi, 0.05, "psd")
    for f in ("F", "f0", "G", "h", "lo", "hi", "aR", "bR", "aI", "bI"):
        np.testing.assert_array_equal(getattr(Q.line, f), getattr(Q0.line, f))
    np.testing.assert_array_equal(Q.bus.pdk, Q0.bus.pdk)
    for _ in range(3):
        dw, dth = rng.standard_normal(g.n_bus) * 0.01, rng.standard_normal(g.n_bus) * 0.01
        z = np.stack([dw[g.f], dth[g.f], dw[g.t], dth[g.t]], 1)
        L = Q.line
        line = float(np.sum(0.5 * np.einsum("li,lij,lj->l", z, L.M, z) + (L.q * z).sum(1) + L.c0))
        dwR = np.einsum("li,li->l", L.aR, z) + L.bR
        dwI = np.einsum("li,li->l", L.aI, z) + L.bI
        ref = 0.5 * (np.sum(dw ** 2) + np.sum(dth ** 2) + np.sum(dwR ** 2) + np.sum(dwI ** 2))
        assert abs(line - ref) <= 1e-12 * (1 + ref)
    np.testing.assert_array_equal(Q.gen.fp, 0.0)
    np.testing.assert_array_equal(Q.gen.fpp, 1.0)
    np.testing.assert_array_equal(Q.gen.fq, 0.0)
    np.testing.assert_array_equal(Q.gen.fqq, 1.0)


def _tight_ring14():
    import dataclasses
    g = grid_14()
    return dataclasses.replace(g, smax_ij=0.5 * g.smax_ij, smax_ji=0.5 * g.smax_ji)


def test_restoration_lowers_the_violation_after_a_collapse():
    """With line limits halved the 14-bus SQP (exact QP solves, second-order
    correction) collapses its radius after one step.  With restoration the
    run takes restoration steps instead of stopping: the first is accepted,
    lowers the constraint violation h (by the amount its step gives when
    recomputed from the collapsed iterate) and restarts the radius; the run
    ends with less than half the h of the run without restoration."""
    g = _tight_ring14()
    s = power_flow_start(g)
    x0 = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    base = dict(max_iter=30, qp_solver="direct", soc=True, delta0=0.05, delta_min=1e-3)
    r0 = sqp.solve(g, sqp.SqpParams(**base), x0=x0)
    assert r0.outcome == "TR_COLLAPSED" and not any(q.restore for q in r0.records)
    r1 = sqp.solve(g, sqp.SqpParams(restore=True, **base), x0=x0)
    k = next(i for i, q in enumerate(r1.records) if q.restore)
    assert [q.accepted for q in r1.records[:k]] == [q.accepted for q in r0.records[:k]]
    rec = r1.records[k]
    assert rec.accepted and rec.ared > 0 and rec.delta == base["delta0"]
    h_final0 = acopf.infeas_h(g, r0.x)
    h_final1 = acopf.infeas_h(g, r1.x)
    assert h_final1 < 0.5 * h_final0
    # replay up to the restoration to check its step
    x = r0.x  # the collapsed iterate (no step was accepted after the first)
    qp = qpm.build_qp(g, x, r0.pi, base["delta0"], "restore")
    d = sqp.direct_qp_step(g, x, qp)[0]
    xt = x.plus(d)
    assert acopf.infeas_h(g, x) - acopf.infeas_h(g, xt) == pytest.approx(rec.ared, rel=1e-9)
