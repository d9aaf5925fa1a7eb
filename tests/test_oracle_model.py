"""Pins of the ACOPF model and QP construction of the oracle against
identities that do not depend on the oracle's own formulas."""
import numpy as np
import pytest

from synth.grids import grid_14, tiny_grid, pi_model, power_flow_start, ybus
from oracle import acopf, qp as qpm


def _random_iterate(g, rng, spread=0.05):
    w = rng.uniform(0.9, 1.1, g.n_bus)
    th = rng.uniform(-0.3, 0.3, g.n_bus)
    th[g.ref] = 0.0
    ph = th[g.f] - th[g.t]
    vv = np.sqrt(w[g.f] * w[g.t])
    wR = vv * np.cos(ph) * (1 + spread * rng.standard_normal(g.n_line))
    wI = vv * np.sin(ph) + spread * rng.standard_normal(g.n_line)
    return acopf.Iterate(rng.uniform(0, 1, g.n_gen), rng.uniform(-0.5, 0.5, g.n_gen), w, th, wR, wI)


def test_flows_equal_complex_power_of_pi_model():
    """Flow definitions (eq. acopf_pf) equal S_ij = V_i conj(Y_ff V_i + Y_ft V_j)
    at wR = v_i v_j cos, wI = v_i v_j sin (textbook branch model)."""
    g = tiny_grid(seed=3, n_bus=6, n_line=8, n_gen=2)
    rng = np.random.default_rng(0)
    tap = rng.uniform(0.95, 1.05, g.n_line)
    yff, yft, ytf, ytt = pi_model(g.r, g.x, g.bc, tap)
    g2 = type(g)(**{**g.__dict__, "gii": yff.real, "bii": yff.imag, "gij": yft.real, "bij": yft.imag,
                    "gji": ytf.real, "bji": ytf.imag, "gjj": ytt.real, "bjj": ytt.imag, "tap": tap})
    vm = rng.uniform(0.9, 1.1, g.n_bus)
    va = rng.uniform(-0.5, 0.5, g.n_bus)
    V = vm * np.exp(1j * va)
    Sij = V[g.f] * np.conj(yff * V[g.f] + yft * V[g.t])
    Sji = V[g.t] * np.conj(ytf * V[g.f] + ytt * V[g.t])
    ph = va[g.f] - va[g.t]
    w = vm ** 2
    wR = vm[g.f] * vm[g.t] * np.cos(ph)
    wI = vm[g.f] * vm[g.t] * np.sin(ph)
    pij, qij, pji, qji = acopf.flows(g2, w, wR, wI)
    np.testing.assert_allclose(pij, Sij.real, atol=1e-13)
    np.testing.assert_allclose(qij, Sij.imag, atol=1e-13)
    np.testing.assert_allclose(pji, Sji.real, atol=1e-13)
    np.testing.assert_allclose(qji, Sji.imag, atol=1e-13)


def test_balance_zero_at_solved_power_flow():
    """A Newton power flow solved on the bus admittance matrix satisfies the
    balance constraints (opfc5, opfc6) and the consistency constraints."""
    g = grid_14()
    s = power_flow_start(g)
    assert s["converged"]
    x = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    rp, rq = acopf.balance(g, x)
    assert np.abs(rp).max() < 1e-9 and np.abs(rq).max() < 1e-9
    c11, c12, _, _ = acopf.nonlinear_constraints(g, x)
    assert np.abs(c11).max() < 1e-12 and np.abs(c12).max() < 1e-12


def test_line_hessian_matches_finite_differences():
    """Hessian of L_ij (eq. lag) against central differences of the
    constraint functions evaluated through ``nonlinear_constraints``."""
    g = tiny_grid(seed=5, n_bus=5, n_line=7, n_gen=2)
    rng = np.random.default_rng(1)
    x = _random_iterate(g, rng)
    pi = rng.standard_normal((g.n_line, 4)) * 10

    def lag_at(u, line):
        xx = x.copy()
        f, t = g.f[line], g.t[line]
        xx.w[f], xx.th[f], xx.wR[line], xx.wI[line], xx.w[t], xx.th[t] = u
        c = acopf.nonlinear_constraints(g, xx)
        return sum(pi[line, k] * c[k][line] for k in range(4))

    H = acopf.line_hessian(g, x, pi)
    h = 1e-4
    for line in range(g.n_line):
        f, t = g.f[line], g.t[line]
        u0 = np.array([x.w[f], x.th[f], x.wR[line], x.wI[line], x.w[t], x.th[t]])
        Hfd = np.zeros((6, 6))
        for a in range(6):
            for b in range(6):
                ea = np.eye(6)[a] * h
                eb = np.eye(6)[b] * h
                Hfd[a, b] = (lag_at(u0 + ea + eb, line) - lag_at(u0 + ea - eb, line)
                             - lag_at(u0 - ea + eb, line) + lag_at(u0 - ea - eb, line)) / (4 * h * h)
        np.testing.assert_allclose(H[line], Hfd, atol=2e-5 * (1 + np.abs(Hfd).max()))
        np.testing.assert_allclose(H[line], H[line].T, atol=0)


def test_elimination_satisfies_linearised_consistency():
    """d_wR, d_wI of (eq. elim) make the linearised (opfc11, opfc12) of
    (QPsub) hold for any z."""
    g = tiny_grid(seed=7, n_bus=6, n_line=9, n_gen=2)
    rng = np.random.default_rng(2)
    x = _random_iterate(g, rng)
    aR, bR, aI, bI = qpm.elimination(g, x)
    z = rng.standard_normal((g.n_line, 4)) * 0.1
    dwR = np.sum(aR * z, 1) + bR
    dwI = np.sum(aI * z, 1) + bI
    wi, wj = x.w[g.f], x.w[g.t]
    ph = x.th[g.f] - x.th[g.t]
    s, c = np.sin(ph), np.cos(ph)
    r11 = 2 * x.wR * dwR + 2 * x.wI * dwI - wj * z[:, 0] - wi * z[:, 2] - (wi * wj - x.wR ** 2 - x.wI ** 2)
    r12 = s * dwR - c * dwI + (x.wR * c + x.wI * s) * (z[:, 1] - z[:, 3]) - (-x.wR * s + x.wI * c)
    assert np.abs(r11).max() < 1e-14 and np.abs(r12).max() < 1e-14


def test_elimination_is_gradient_at_consistent_point():
    """At a point where opfc11 and opfc12 hold, wR = sqrt(w_i w_j) cos and
    wI = sqrt(w_i w_j) sin of the angle difference, so a^R, a^I are their
    gradients in z and b^R = b^I = 0 (central differences)."""
    g = tiny_grid(seed=9, n_bus=5, n_line=7, n_gen=2)
    rng = np.random.default_rng(3)
    x = _random_iterate(g, rng, spread=0.0)
    aR, bR, aI, bI = qpm.elimination(g, x)
    assert np.abs(bR).max() < 1e-14 and np.abs(bI).max() < 1e-14

    def wr_wi(z4):
        wi, thi, wj, thj = z4
        return np.sqrt(wi * wj) * np.cos(thi - thj), np.sqrt(wi * wj) * np.sin(thi - thj)

    h = 1e-6
    for line in range(g.n_line):
        z0 = np.array([x.w[g.f[line]], x.th[g.f[line]], x.w[g.t[line]], x.th[g.t[line]]])
        for k in range(4):
            e = np.eye(4)[k] * h
            (r1, i1), (r0, i0) = wr_wi(z0 + e), wr_wi(z0 - e)
            assert abs((r1 - r0) / (2 * h) - aR[line, k]) < 1e-8
            assert abs((i1 - i0) / (2 * h) - aI[line, k]) < 1e-8


def test_reduced_objective_and_flow_map():
    """0.5 (Az+b)^T H (Az+b) = 0.5 z^T M z + q^T z + c0 (raw mode), and
    F z + f0 equals the change of the flows (eq. acopf_pf) under the step
    (z, d_wR, d_wI); G z <= h is the first-order Taylor expansion of
    (opfc13, opfc14) (central differences)."""
    g = tiny_grid(seed=11, n_bus=6, n_line=9, n_gen=3)
    rng = np.random.default_rng(4)
    x = _random_iterate(g, rng)
    pi = rng.standard_normal((g.n_line, 4)) * 5
    Q = qpm.build_qp(g, x, pi, 0.5, "raw")
    L = Q.line
    z = rng.standard_normal((g.n_line, 4)) * 0.1
    dwR = np.sum(L.aR * z, 1) + L.bR
    dwI = np.sum(L.aI * z, 1) + L.bI
    u = np.stack([z[:, 0], z[:, 1], dwR, dwI, z[:, 2], z[:, 3]], 1)
    full = 0.5 * np.einsum("li,lij,lj->l", u, L.H, u)
    red = 0.5 * np.einsum("li,lij,lj->l", z, L.M, z) + np.sum(L.q * z, 1) + L.c0
    np.testing.assert_allclose(red, full, rtol=1e-12, atol=1e-12)
    # flows, one line at a time (buses are shared between lines)
    for line in range(g.n_line):
        f, t = g.f[line], g.t[line]
        w = x.w.copy(); w[f] += z[line, 0]; w[t] += z[line, 2]
        wR = x.wR.copy(); wR[line] += dwR[line]
        wI = x.wI.copy(); wI[line] += dwI[line]
        new = np.array(acopf.flows(g, w, wR, wI))[:, line]
        old = np.array(acopf.flows(g, x.w, x.wR, x.wI))[:, line]
        np.testing.assert_allclose(L.F[line] @ z[line] + L.f0[line], new - old, atol=1e-12)
        # linearised line limits in terms of the flow change
        c13 = g.smax_ij[line] ** 2 - old[0] ** 2 - old[1] ** 2
        c14 = g.smax_ji[line] ** 2 - old[2] ** 2 - old[3] ** 2
        d = L.F[line] @ z[line] + L.f0[line]
        lin13 = c13 - 2 * old[0] * d[0] - 2 * old[1] * d[1]
        lin14 = c14 - 2 * old[2] * d[2] - 2 * old[3] * d[3]
        np.testing.assert_allclose(L.h[line] - L.G[line] @ z[line], [lin13, lin14], atol=1e-12)


def test_gradient_of_flow_limits_is_taylor():
    """G_ij rows are the gradients of -(p^2 + q^2) in z through the flow map."""
    g = tiny_grid(seed=13, n_bus=5, n_line=6, n_gen=2)
    rng = np.random.default_rng(5)
    x = _random_iterate(g, rng)
    Q = qpm.build_qp(g, x, np.zeros((g.n_line, 4)), 0.5)
    L = Q.line
    h = 1e-6
    for line in range(g.n_line):
        def s2(z4):
            d = L.F[line] @ z4 + L.f0[line] - L.f0[line]
            p = L.pk[line] + d
            return np.array([p[0] ** 2 + p[1] ** 2, p[2] ** 2 + p[3] ** 2])
        for k in range(4):
            e = np.eye(4)[k] * h
            fd = (s2(e) - s2(-e)) / (2 * h)
            np.testing.assert_allclose(L.G[line][:, k], fd, rtol=1e-6, atol=1e-9)


def test_psd_projection_against_matrix_square_root():
    """PSD projection equals (M + sqrt(M^2)) / 2 (polar decomposition)."""
    from scipy.linalg import sqrtm
    rng = np.random.default_rng(6)
    A = rng.standard_normal((20, 4, 4))
    M = A + np.swapaxes(A, 1, 2)
    P = qpm.psd_project(M)
    for k in range(M.shape[0]):
        ref = 0.5 * (M[k] + np.real(sqrtm(M[k] @ M[k])))
        np.testing.assert_allclose(P[k], ref, atol=1e-10)
        assert np.linalg.eigvalsh(P[k]).min() > -1e-12
    S = A @ np.swapaxes(A, 1, 2)
    np.testing.assert_allclose(qpm.psd_project(S), S, atol=1e-12)


def test_qp_constants_match_linearised_balance():
    """p^{d,(k)} makes the linearised balance of (QPsub) equivalent to a zero
    balance residual at x + d (the balance is linear in the variables)."""
    g = tiny_grid(seed=15, n_bus=6, n_line=8, n_gen=3)
    rng = np.random.default_rng(7)
    x = _random_iterate(g, rng)
    Q = qpm.build_qp(g, x, np.zeros((g.n_line, 4)), 0.5)
    rp, rq = acopf.balance(g, x)
    np.testing.assert_allclose(Q.bus.pdk, -rp, atol=1e-13)
    np.testing.assert_allclose(Q.bus.qdk, -rq, atol=1e-13)
