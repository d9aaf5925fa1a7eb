"""Pins of the oracle's subproblem solvers, direct QP solve, ADMM and
multiplier recovery against independent solvers, dense KKT systems, brute
force and sensitivity analysis."""
import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from synth.grids import tiny_grid, grid_14, power_flow_start
from oracle import acopf, qp as qpm, admm, direct, lineqp, sqp


def _random_line_qps(n, seed, row_scale=1.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, 4, 4))
    Q = A @ np.swapaxes(A, 1, 2) + 0.5 * np.eye(4)
    c = rng.standard_normal((n, 4)) * 3
    lo = -rng.uniform(0.05, 1.0, (n, 4))
    hi = rng.uniform(0.05, 1.0, (n, 4))
    G = rng.standard_normal((n, 2, 4)) * row_scale
    h = rng.uniform(0.05, 0.5, (n, 2))
    # some fixed variables (the reference-angle case)
    fx = rng.random(n) < 0.2
    lo[fx, 1] = 0.0
    hi[fx, 1] = 0.0
    return Q, c, lo, hi, G, h


def test_line_qp_matches_slsqp_and_kkt():
    Q, c, lo, hi, G, h = _random_line_qps(60, 0)
    z, mu, bm, feas = lineqp.solve_line_qps(Q, c, lo, hi, G, h)
    assert feas.all()
    for k in range(Q.shape[0]):
        cons = [{"type": "ineq", "fun": lambda v, k=k: h[k] - G[k] @ v, "jac": lambda v, k=k: -G[k]}]
        r = minimize(lambda v: 0.5 * v @ Q[k] @ v + c[k] @ v, np.clip(np.zeros(4), lo[k], hi[k]),
                     jac=lambda v: Q[k] @ v + c[k], bounds=list(zip(lo[k], hi[k])),
                     constraints=cons, method="SLSQP", options={"ftol": 1e-15, "maxiter": 500})
        fz = 0.5 * z[k] @ Q[k] @ z[k] + c[k] @ z[k]
        assert fz <= r.fun + 1e-9 * (1 + abs(r.fun))
        np.testing.assert_allclose(z[k], r.x, atol=1e-6)
        # KKT certificate: stationarity, signs, complementarity
        gr = Q[k] @ z[k] + c[k] + G[k].T @ mu[k] + bm[k]
        assert np.abs(gr).max() < 1e-9
        assert mu[k].min() > -1e-9
        slack = h[k] - G[k] @ z[k]
        assert np.abs(mu[k] * slack).max() < 1e-9
        free = (lo[k] < hi[k])
        atlo = free & (np.abs(z[k] - lo[k]) < 1e-12)
        athi = free & (np.abs(z[k] - hi[k]) < 1e-12)
        assert np.all(bm[k][atlo] <= 1e-9) and np.all(bm[k][athi] >= -1e-9)
        inner = free & ~atlo & ~athi
        assert np.abs(bm[k][inner]).max(initial=0) < 1e-9


def test_line_qp_unconstrained_and_infeasible():
    Q, c, lo, hi, G, h = _random_line_qps(10, 1)
    lo[:] = -1e6; hi[:] = 1e6; h[:] = 1e9
    z, mu, _, feas = lineqp.solve_line_qps(Q, c, lo, hi, G, h)
    np.testing.assert_allclose(z, -np.linalg.solve(Q, c[:, :, None])[:, :, 0], atol=1e-12)
    assert np.all(mu == 0)
    # box [0, 1]^4 with a row requiring sum(z) <= -1: no feasible point
    Q, c, lo, hi, G, h = _random_line_qps(3, 2)
    lo[:] = 0; hi[:] = 1
    G[:] = 0; G[:, 0, :] = 1.0; h[:, 0] = -1.0; h[:, 1] = 1.0
    _, _, _, feas = lineqp.solve_line_qps(Q, c, lo, hi, G, h)
    assert not feas.any()


def _relax_cases(n, seed):
    rng = np.random.default_rng(seed)
    lo = -rng.uniform(0, 0.1, (n, 4)); hi = rng.uniform(0, 0.1, (n, 4))
    lo[::7, 1] = 0.0; hi[::7, 1] = 0.0
    G = rng.standard_normal((n, 2, 4)); h = rng.uniform(-0.3, 0.1, (n, 2))
    G[::11, 1] = 0.0
    return lo, hi, G, h


def test_min_max_violation_against_linprog():
    """t* = min over the box of the larger row violation (the test for a
    common point of box and rows): the oracle's vertex and edge enumeration
    against SciPy's LP solver."""
    from scipy.optimize import linprog
    lo, hi, G, h = _relax_cases(200, 0)
    t = lineqp.min_max_violation(lo, hi, G, h)
    for k in range(lo.shape[0]):
        r = linprog(np.r_[np.zeros(4), 1.0], A_ub=np.hstack([G[k], -np.ones((2, 1))]), b_ub=h[k],
                    bounds=[(lo[k, i], hi[k, i]) for i in range(4)] + [(None, None)], method="highs")
        assert r.status == 0 and abs(t[k] - r.fun) < 1e-12
    assert 0.2 < (t > 0).mean() < 0.9


def test_min_violation_against_a_qp_solver():
    """v* = (G z* - h)^+ at the least-squares violation over the box: the
    oracle's minimum over the segments of the polygon G [lo, hi] against
    SciPy's SLSQP on the equivalent QP min 0.5 |s|^2 s.t. s >= G z - h,
    s >= 0, lo <= z <= hi (s is unique)."""
    from scipy.optimize import minimize
    lo, hi, G, h = _relax_cases(120, 5)
    v = lineqp.min_violation(lo, hi, G, h)
    t = lineqp.min_max_violation(lo, hi, G, h)
    assert np.all(v[t <= 0] == 0.0) and np.all(v[t > 0].max(1) > 0)
    n_both = 0
    for k in np.nonzero(t > 0)[0]:
        cons = [{"type": "ineq", "fun": lambda u, k=k: u[4:] - (G[k] @ u[:4] - h[k]), "jac":
                 lambda u, k=k: np.hstack([-G[k], np.eye(2)])}]
        best = None
        for s0 in range(3):
            z0 = lo[k] + np.random.default_rng(s0).uniform(0, 1, 4) * (hi[k] - lo[k])
            u0 = np.r_[z0, np.maximum(G[k] @ z0 - h[k], 0) + 0.1]
            r = minimize(lambda u: 0.5 * u[4:] @ u[4:], u0, jac=lambda u: np.r_[np.zeros(4), u[4:]],
                         bounds=[(lo[k, i], hi[k, i]) for i in range(4)] + [(0, None)] * 2,
                         constraints=cons, method="SLSQP", options={"ftol": 1e-15, "maxiter": 500})
            if best is None or r.fun < best.fun:
                best = r
        s = np.maximum(best.x[4:], 0)
        assert np.abs(v[k] - s).max() <= 1e-6 * (1 + np.abs(s).max()), (k, v[k], s)
        n_both += int((v[k] > 0).all())
    assert n_both >= 10


def test_limit_relaxation_hand_cases():
    """Hand cases of the relaxation.  (1) Box [0, 1]^4, rows sum(z) <= -1
    and 0 <= 1: z = 0 violates the first row by 1, v* = (1, 0).  (2) One
    variable on [-2, 2] (the others fixed at 0), rows 2 z <= -2 and -z <=
    -0.5: for z in [-1, 0.5] both rows are violated, 0.5 ((2z + 2)^2 +
    (0.5 - z)^2) has derivative 5 z + 3.5 and is least at z = -0.7,
    v* = (0.6, 1.2), while the smallest common violation is t* = 1 at
    z = -0.5.  The shifted rows then admit the
    box's points of least violation only."""
    lo1, hi1 = np.zeros((1, 4)), np.ones((1, 4))
    G1 = np.zeros((1, 2, 4)); G1[0, 0] = 1.0
    h1 = np.array([[-1.0, 1.0]])
    assert lineqp.min_max_violation(lo1, hi1, G1, h1)[0] == 1.0
    np.testing.assert_allclose(lineqp.min_violation(lo1, hi1, G1, h1)[0], [1.0, 0.0], atol=1e-15)
    guard = 1e-9 * (1 + 2 + 4)
    np.testing.assert_allclose(lineqp.limit_relaxation(lo1, hi1, G1, h1)[0], [1.0 + guard, guard], rtol=1e-14)
    lo2, hi2 = np.array([[-2.0, 0, 0, 0]]), np.array([[2.0, 0, 0, 0]])
    G2 = np.zeros((1, 2, 4)); G2[0, 0, 0] = 2.0; G2[0, 1, 0] = -1.0
    h2 = np.array([[-2.0, -0.5]])
    assert lineqp.min_max_violation(lo2, hi2, G2, h2)[0] == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(lineqp.min_violation(lo2, hi2, G2, h2)[0], [0.6, 1.2], atol=1e-14)
    shift = lineqp.limit_relaxation(lo2, hi2, G2, h2)
    # on the relaxed rows only z = -0.7 (up to the guard) is left
    Q = np.eye(4)[None]
    for c0 in (-5.0, 5.0):
        z, _, _, feas = lineqp.solve_line_qps(Q, np.array([[c0, 0, 0, 0]]), lo2, hi2, G2, h2 + shift)
        assert feas[0] and abs(z[0, 0] + 0.7) < 1e-7


def test_relaxed_rows_admit_only_points_of_least_violation():
    """On random infeasible lines the QP on the relaxed rows is feasible,
    and its minimisers (of random objectives) have the least squared
    violation psi* = 0.5 |v*|^2 of the original rows up to the guard: each
    row is violated by at most v*_r + guard, so psi <= 0.5 |v* + guard|^2,
    and no point of the box has psi < psi*."""
    lo, hi, G, h = _relax_cases(200, 0)
    shift = lineqp.limit_relaxation(lo, hi, G, h)
    t = lineqp.min_max_violation(lo, hi, G, h)
    assert np.all(shift[t <= 0] == 0.0) and np.all(shift[t > 0] > 0.0)
    v = lineqp.min_violation(lo, hi, G, h)
    guard = lineqp.relax_guard(lo, hi, G, h)
    bad = t > 0
    psi_star = 0.5 * (v ** 2).sum(1)
    rng = np.random.default_rng(9)
    for _ in range(3):
        Q = np.broadcast_to(np.eye(4), (lo.shape[0], 4, 4)).copy()
        c = rng.standard_normal((lo.shape[0], 4))
        z, _, _, feas = lineqp.solve_line_qps(Q, c, lo, hi, G, h + shift)
        assert feas.all()
        viol = np.maximum(np.einsum("nrj,nj->nr", G, z) - h, 0.0)
        psi = 0.5 * (viol ** 2).sum(1)
        # the enumeration accepts rows met to FEAS_TOL times their scale
        tol = lineqp.FEAS_TOL * (1 + np.abs(h) + np.einsum("nrj,nj->nr", np.abs(G), np.abs(z)))
        slack = guard[:, None] + tol
        assert np.all(viol[bad] <= v[bad] + slack[bad])
        assert np.all(psi[bad] <= 0.5 * ((v[bad] + slack[bad]) ** 2).sum(1))
        assert np.all(psi[bad] >= psi_star[bad] * (1 - 1e-12))


def test_gen_update_matches_scalar_minimisation():
    g = tiny_grid(seed=2, n_bus=8, n_line=10, n_gen=5)
    rng = np.random.default_rng(3)
    x = acopf.Iterate(rng.uniform(0, 0.5, g.n_gen), rng.uniform(-0.2, 0.2, g.n_gen),
                      np.ones(g.n_bus), np.zeros(g.n_bus), np.ones(g.n_line), np.zeros(g.n_line))
    Q = qpm.build_qp(g, x, np.zeros((g.n_line, 4)), 0.3)
    st = admm.cold_state(g)
    st.xbar_g = rng.standard_normal((g.n_gen, 2)) * 0.3
    st.lam_g = rng.standard_normal((g.n_gen, 2)) * 1e3
    rho = admm.Rho(rng.uniform(1e3, 3e4, (g.n_gen, 2)), np.full((g.n_line, 8), 1e4))
    xg = admm.gen_update(Q, st, rho)
    for k in range(g.n_gen):
        fp = lambda d: (Q.gen.fp[k] * d + 0.5 * Q.gen.fpp[k] * d * d + st.lam_g[k, 0] * d
                        + 0.5 * rho.g[k, 0] * (d - st.xbar_g[k, 0]) ** 2)
        fq = lambda d: st.lam_g[k, 1] * d + 0.5 * rho.g[k, 1] * (d - st.xbar_g[k, 1]) ** 2
        rp = minimize_scalar(fp, bounds=(Q.gen.lo[k, 0], Q.gen.hi[k, 0]), method="bounded",
                             options={"xatol": 1e-12})
        rq = minimize_scalar(fq, bounds=(Q.gen.lo[k, 1], Q.gen.hi[k, 1]), method="bounded",
                             options={"xatol": 1e-12})
        assert abs(xg[k, 0] - rp.x) < 1e-8 and abs(xg[k, 1] - rq.x) < 1e-8


def test_bus_update_matches_dense_kkt():
    """Closed form of (eq. bus_kernel) against the KKT system of the bus QP
    assembled densely, bus by bus."""
    g = tiny_grid(seed=4, n_bus=7, n_line=11, n_gen=3, shunt_scale=0.05)
    rng = np.random.default_rng(5)
    x = acopf.Iterate(rng.uniform(0, 0.5, g.n_gen), np.zeros(g.n_gen), np.ones(g.n_bus),
                      np.zeros(g.n_bus), np.ones(g.n_line), np.zeros(g.n_line))
    Q = qpm.build_qp(g, x, np.zeros((g.n_line, 4)), 0.3)
    st = admm.cold_state(g)
    st.lam_g = rng.standard_normal((g.n_gen, 2)) * 100
    st.lam_l = rng.standard_normal((g.n_line, 8)) * 100
    xg = rng.standard_normal((g.n_gen, 2)) * 0.1
    xl = rng.standard_normal((g.n_line, 8)) * 0.1
    rho = admm.Rho(rng.uniform(1e3, 3e4, (g.n_gen, 2)), rng.uniform(1e3, 3e4, (g.n_line, 8)))
    xbar_g, xbar_f, dw, dth, nu = admm.bus_update(g, Q, xg, xl, st, rho)
    for i in range(g.n_bus):
        # unknowns: gen copies (p, q) per gen at i, flow copies (p, q) per line end at i, d_w
        terms = []  # (rho, x, lam, aP, aQ, kind, idx)
        for k in np.nonzero(g.gbus == i)[0]:
            terms.append((rho.g[k, 0], xg[k, 0], st.lam_g[k, 0], 1.0, 0.0, "g", (k, 0)))
            terms.append((rho.g[k, 1], xg[k, 1], st.lam_g[k, 1], 0.0, 1.0, "g", (k, 1)))
        for l in np.nonzero(g.f == i)[0]:
            terms.append((rho.l[l, 0], xl[l, 0], st.lam_l[l, 0], -1.0, 0.0, "f", (l, 0)))
            terms.append((rho.l[l, 1], xl[l, 1], st.lam_l[l, 1], 0.0, -1.0, "f", (l, 1)))
        for l in np.nonzero(g.t == i)[0]:
            terms.append((rho.l[l, 2], xl[l, 2], st.lam_l[l, 2], -1.0, 0.0, "f", (l, 2)))
            terms.append((rho.l[l, 3], xl[l, 3], st.lam_l[l, 3], 0.0, -1.0, "f", (l, 3)))
        wl = [(rho.l[l, 4], xl[l, 4], st.lam_l[l, 4]) for l in np.nonzero(g.f == i)[0]] + \
             [(rho.l[l, 6], xl[l, 6], st.lam_l[l, 6]) for l in np.nonzero(g.t == i)[0]]
        n = len(terms) + 1
        H = np.zeros((n, n)); lin = np.zeros(n); A = np.zeros((2, n))
        for a, (r, xv, lv, ap, aq, _, _) in enumerate(terms):
            H[a, a] = r; lin[a] = -lv - r * xv; A[0, a] = ap; A[1, a] = aq
        H[-1, -1] = sum(r for r, _, _ in wl)
        lin[-1] = sum(-lv - r * xv for r, xv, lv in wl)
        A[0, -1] = -g.gsh[i]; A[1, -1] = g.bsh[i]
        K = np.block([[H, A.T], [A, np.zeros((2, 2))]])
        sol = np.linalg.solve(K, np.concatenate([-lin, [Q.bus.pdk[i], Q.bus.qdk[i]]]))
        for a, (_, _, _, _, _, kind, (k, j)) in enumerate(terms):
            got = xbar_g[k, j] if kind == "g" else xbar_f[k, j]
            assert abs(got - sol[a]) < 1e-10 * (1 + abs(sol[a]))
        assert abs(dw[i] - sol[n - 1]) < 1e-10
        np.testing.assert_allclose(nu[i], sol[n:], rtol=1e-9, atol=1e-7)
        th = [(rho.l[l, 5], xl[l, 5], st.lam_l[l, 5]) for l in np.nonzero(g.f == i)[0]] + \
             [(rho.l[l, 7], xl[l, 7], st.lam_l[l, 7]) for l in np.nonzero(g.t == i)[0]]
        ref_th = 0.0 if i == g.ref else sum(r * xv + lv for r, xv, lv in th) / sum(r for r, _, _ in th)
        assert abs(dth[i] - ref_th) < 1e-12


def _qp_at_power_flow(g, delta=0.3, seed=0, pi_scale=0.0):
    s = power_flow_start(g)
    x = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    rng = np.random.default_rng(seed)
    pi = rng.standard_normal((g.n_line, 4)) * pi_scale
    pi[:, 2:] = -np.abs(pi[:, 2:])
    return x, pi, qpm.build_qp(g, x, pi, delta)


def test_direct_solution_kkt_and_against_slsqp():
    g = tiny_grid(seed=6, n_bus=4, n_line=5, n_gen=2)
    x, pi, Q = _qp_at_power_flow(g, pi_scale=20.0)
    ds = direct.solve(g, Q)
    assert ds.kkt["stationarity"] < 1e-7 and ds.kkt["primal"] < 1e-9
    assert ds.kkt["dual"] < 1e-9 and ds.kkt["complementarity"] < 1e-7
    m = direct.assemble(g, Q)
    # independent solve with SciPy's trust-region constrained method; the
    # fixed reference angle is substituted out first
    from scipy.optimize import LinearConstraint, Bounds
    free = m.lo < m.hi
    P = m.P.toarray()[np.ix_(free, free)]
    A = m.A.toarray()[:, free]
    Gl = m.Gl.toarray()[:, free]
    cons = [LinearConstraint(A, m.b, m.b), LinearConstraint(Gl, -np.inf, m.hl)]
    r = minimize(lambda y: 0.5 * y @ P @ y + m.q[free] @ y, np.zeros(free.sum()),
                 jac=lambda y: P @ y + m.q[free], hess=lambda y: P,
                 bounds=Bounds(m.lo[free], m.hi[free]), constraints=cons, method="trust-constr",
                 options={"gtol": 1e-12, "xtol": 1e-14, "maxiter": 20000})
    assert r.constr_violation < 1e-8
    assert abs(ds.objective - (r.fun + m.const)) < 1e-6 * (1 + abs(ds.objective))


@pytest.mark.parametrize("rho", [3e3, 1e3])
def test_admm_limit_equals_direct_solve(rho):
    """On a convex QP the ADMM limit is the QP minimiser: objective within 1e-6
    relative and constraint violation within 1e-5 of the direct solve; the
    limit does not depend on rho."""
    g = tiny_grid(seed=8, n_bus=5, n_line=6, n_gen=2, shunt_scale=0.03)
    x, pi, Q = _qp_at_power_flow(g, delta=0.2, pi_scale=30.0)
    ds = direct.solve(g, Q)
    res = admm.solve(g, Q, admm.Rho.scalar(g, rho), 40000, 1e-9, 1e-9)
    assert res.converged
    d = sqp.assemble_step(g, Q, res.state)
    z = np.stack([d.w[g.f], d.th[g.f], d.w[g.t], d.th[g.t]], 1)
    obj = qpm.qp_objective(Q, d.pg, z)
    assert abs(obj - ds.objective) <= 1e-6 * abs(ds.objective)
    assert direct.max_violation(g, Q, np.concatenate([d.pg, d.qg, d.w, d.th])) < 1e-5
    # balance multipliers agree with the direct solve
    nb = g.n_bus
    np.testing.assert_allclose(res.state.nu[:, 0], ds.nu[:nb], rtol=1e-4, atol=1e-3)


def test_pi_recovery_equals_sensitivity_of_optimal_value():
    """Multipliers of the linearised (opfc11, opfc12): the recovered pi11,
    pi12 equal minus the derivative of the QP optimal value with respect to
    the constraint's right-hand side (central differences of direct solves);
    pi13, pi14 equal minus the line-limit multipliers."""
    g = tiny_grid(seed=10, n_bus=4, n_line=5, n_gen=2)
    x, pi, Q = _qp_at_power_flow(g, delta=0.2, pi_scale=10.0)
    ds = direct.solve(g, Q, tol=1e-13)
    ix = direct.var_index(g)
    nb = g.n_bus
    st = admm.cold_state(g)
    st.dw, st.dth = ds.y[ix["w"]], ds.y[ix["th"]]
    st.xl[:, 4:] = np.stack([st.dw[g.f], st.dth[g.f], st.dw[g.t], st.dth[g.t]], 1)
    nuP, nuQ = ds.nu[:nb], ds.nu[nb:]
    st.lam_l[:, :4] = np.stack([-nuP[g.f], -nuQ[g.f], -nuP[g.t], -nuQ[g.t]], 1)
    st.mu = ds.mu.reshape(-1, 2)
    pir = sqp.recover_pi(g, x, Q, st)
    eps = 1e-5
    for line in range(g.n_line):
        for k in range(2):
            sh = np.zeros((g.n_line, 2)); sh[line, k] = eps
            vp = direct.solve(g, qpm.build_qp(g, x, pi, 0.2, rhs_shift=sh), tol=1e-13).objective
            vm = direct.solve(g, qpm.build_qp(g, x, pi, 0.2, rhs_shift=-sh), tol=1e-13).objective
            slope = (vp - vm) / (2 * eps)
            assert abs(pir[line, k] + slope) < 1e-4 * (1 + abs(slope)), (line, k, pir[line, k], slope)
    np.testing.assert_allclose(pir[:, 2:], -st.mu)


def test_infinity_norm_stop_test_bounds_the_euclidean_one():
    """One sweep from the same state with both residual norms: the infinity
    norm of r is the largest coupling residual |x_c - xbar_c| rebuilt here
    from the new state (generators; flows against their bus-side copies;
    voltage copies against the end buses' values), ||.||_inf <= ||.||_2 <=
    sqrt(couplings) ||.||_inf, and the state is the same."""
    from oracle import admm, qp as qpm
    from synth.grids import grid_14, power_flow_start
    from oracle import acopf
    g = grid_14()
    s = power_flow_start(g)
    x = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    rng = np.random.default_rng(2)
    pi = rng.standard_normal((g.n_line, 4)) * 20
    Q = qpm.build_qp(g, x, pi, 0.05)
    rho = admm.Rho.scalar(g, 2e4)
    st = admm.warm_state(g, rng.standard_normal((g.n_gen, 2)) * 100, rng.standard_normal((g.n_line, 8)) * 100)
    n = 2 * g.n_gen + 8 * g.n_line
    for _ in range(3):
        s2, r2, q2, _ = admm.sweep(g, Q, st, rho)
        si, ri, qi, _ = admm.sweep(g, Q, st, rho, norm="inf")
        np.testing.assert_array_equal(s2.xl, si.xl)
        f, t = np.asarray(g.f), np.asarray(g.t)
        bus_side = np.column_stack([si.xbar_f, si.dw[f], si.dth[f], si.dw[t], si.dth[t]])
        r_direct = max(np.abs(si.xg - si.xbar_g).max(), np.abs(si.xl - bus_side).max())
        assert abs(ri - r_direct) <= 1e-15 * r_direct
        assert ri <= r2 * (1 + 1e-15) and r2 <= np.sqrt(n) * ri * (1 + 1e-15)
        assert qi <= q2 * (1 + 1e-15) and q2 <= np.sqrt(n) * qi * (1 + 1e-15)
        st = s2
    res = admm.solve(g, Q, rho, 400, 1e-3, 1e-3, norm="inf")
    res2 = admm.solve(g, Q, rho, 400, 1e-3, 1e-3)
    assert res.sweeps <= res2.sweeps
