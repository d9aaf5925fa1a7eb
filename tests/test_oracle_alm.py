"""Pins of the local line solver (ALM + TRON, Section IV-B2): on convex line
subproblems it reaches the exact minimiser of the enumeration; on
nonconvex ones it ends at a point that satisfies the first- and
second-order conditions of a local minimiser; a hand case with negative
curvature ends at the local minimiser its descent path leads to."""
import numpy as np
import pytest

from oracle import alm, lineqp


def _random_lines(rng, n, convex=True):
    A = rng.standard_normal((n, 4, 4))
    Q = A @ np.swapaxes(A, 1, 2) + 0.3 * np.eye(4)
    if not convex:
        Q = Q - rng.uniform(1.0, 4.0, (n, 1, 1)) * np.eye(4)
    Q[: n // 2] *= rng.uniform(1e2, 1e6, (n // 2, 1, 1))
    c = rng.standard_normal((n, 4)) * np.abs(Q).max(axis=(1, 2))[:, None] * rng.uniform(0.01, 2, (n, 1))
    lo = -rng.uniform(0.01, 0.3, (n, 4))
    hi = rng.uniform(0.01, 0.3, (n, 4))
    G = rng.standard_normal((n, 2, 4))
    h = rng.uniform(0.01, 0.2, (n, 2))
    return Q, c, lo, hi, G, h


def test_alm_reaches_the_exact_minimiser_of_convex_lines():
    rng = np.random.default_rng(11)
    Q, c, lo, hi, G, h = _random_lines(rng, 200)
    zr, mur, _, feas = lineqp.solve_line_qps(Q, c, lo, hi, G, h)
    assert feas.all()
    for k in range(Q.shape[0]):
        r = alm.solve_line(Q[k], c[k], lo[k], hi[k], G[k], h[k])
        assert r.converged, k
        assert np.abs(r.z - zr[k]).max() <= 1e-7 * (1 + np.abs(zr[k]).max()), k
        assert np.abs(r.u - mur[k]).max() <= 1e-5 * (1 + np.abs(mur[k]).max()), k


def _kkt(Q, c, lo, hi, G, h, z, u, tol=1e-7):
    """First- and second-order conditions of a local minimiser of
    0.5 z^T Q z + c^T z on the box with G z <= h, multipliers u of the rows."""
    zs = 1 + np.abs(lo).max() + np.abs(hi).max()
    gs = 1 + np.abs(Q).max() * zs + np.abs(c).max()
    g = G @ z - h
    assert (z >= lo - tol * zs).all() and (z <= hi + tol * zs).all()
    assert (g <= tol * (1 + np.abs(G).sum(1) * zs + np.abs(h))).all()
    assert (u >= 0).all()
    assert np.all(np.abs(u * g) <= tol * gs * zs)
    grad = Q @ z + c + G.T @ u           # = bound multipliers' share: lower bounds push up, upper down
    atlo = z <= lo + tol * zs
    athi = z >= hi - tol * zs
    free = ~atlo & ~athi
    assert np.all(np.abs(grad[free]) <= tol * gs)
    assert np.all(grad[atlo & ~athi] >= -tol * gs) and np.all(grad[athi & ~atlo] <= tol * gs)
    # second order: Q on the free variables, restricted to directions that keep the active rows
    act = (u > tol * gs) | (np.abs(g) <= tol * (1 + np.abs(h)))
    Nf = G[act][:, free]
    if free.sum() > 0:
        if Nf.shape[0] > 0:
            _, sv, vt = np.linalg.svd(Nf)
            rank = int((sv > 1e-12 * max(1.0, sv.max(initial=0))).sum())
            Z = vt[rank:].T
        else:
            Z = np.eye(int(free.sum()))
        if Z.shape[1] > 0:
            Hr = Z.T @ Q[np.ix_(free, free)] @ Z
            assert np.linalg.eigvalsh(Hr).min() >= -tol * np.abs(Q).max()


def test_alm_ends_at_local_minimisers_of_nonconvex_lines():
    rng = np.random.default_rng(12)
    Q, c, lo, hi, G, h = _random_lines(rng, 200, convex=False)
    assert (np.linalg.eigvalsh(Q).min(axis=1) < 0).sum() > 150
    n_conv = 0
    for k in range(Q.shape[0]):
        r = alm.solve_line(Q[k], c[k], lo[k], hi[k], G[k], h[k])
        if not r.converged:
            continue
        n_conv += 1
        _kkt(Q[k], c[k], lo[k], hi[k], G[k], h[k], r.z, r.u)
        # no better feasible point nearby (random small moves inside the box and rows)
        phi = lambda z: 0.5 * z @ Q[k] @ z + c[k] @ z
        for _ in range(20):
            d = rng.standard_normal(4) * 1e-4 * (hi[k] - lo[k])
            zn = np.clip(r.z + d, lo[k], hi[k])
            if np.all(G[k] @ zn <= h[k]):
                assert phi(zn) >= phi(r.z) - 1e-9 * (1 + abs(phi(r.z)))
    assert n_conv >= 190


def test_negative_curvature_hand_case():
    """phi(z) = -0.5 z0^2 + 0.1 z0 + 0.5 (z1^2 + z2^2 + z3^2) on [-1, 2]^4
    with rows that never bind: from z = 0 the descent direction is -z0, so
    the solver ends at the local minimiser z0 = -1 (phi = -0.6; the other
    local minimiser z0 = 2 has phi = -1.8), the others at 0."""
    Q = np.diag([-1.0, 1.0, 1.0, 1.0])
    c = np.array([0.1, 0.0, 0.0, 0.0])
    lo, hi = np.full(4, -1.0), np.full(4, 2.0)
    G = np.array([[1.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 1.0]])
    h = np.array([10.0, 10.0])
    r = alm.solve_line(Q, c, lo, hi, G, h)
    assert r.converged
    np.testing.assert_allclose(r.z, [-1.0, 0.0, 0.0, 0.0], atol=1e-9)
    np.testing.assert_allclose(r.u, [0.0, 0.0], atol=1e-12)


def test_relaxed_rows_give_the_local_solvers_point_on_lines_without_a_feasible_point():
    """The QP build relaxes the limit rows of lines whose box and rows have
    no common point (Section V: the paper's ADMM keeps progressing on such
    QPs).  Pin of that reading: on the lines of the 2,000-bus grid without a
    feasible point at trust radius 0.00625, the exact minimiser on the
    relaxed rows is the point the paper's local method (ALM + TRON on the
    original rows) runs to; the penalty parameter then falls to zero and the
    iterates approach the minimiser over the points of least violation."""
    from oracle import admm, qp as qpm
    from synth.grids import grid_2000
    from tests._util import start_point
    g = grid_2000()
    x, pi = start_point(g, pi_scale=20.0, seed=2)
    Q = qpm.build_qp(g, x, pi, 0.00625, "psd")
    L = Q.line
    idx = np.nonzero((L.relax > 0).any(1))[0]
    assert idx.size > 50
    rho = admm.Rho.scalar(g, 2e4)
    QL = admm.line_matrices(Q, rho)[idx]
    # the line data of a first sweep from zero multipliers and bus values
    c = (L.q + np.einsum("lf,lfi->li", rho.l[:, :4] * L.f0, L.F))[idx]
    h0 = (L.h - L.relax)[idx]
    lo, hi, G = L.lo[idx], L.hi[idx], L.G[idx]
    assert (lineqp.min_max_violation(lo, hi, G, h0) > 0).all()
    z, _, _, feas = lineqp.solve_line_qps(QL, c, lo, hi, G, L.h[idx])
    assert feas.all()
    # the other candidate reading: both rows shifted by the smallest common
    # violation t* (plus 10%), the minimiser over the box's points whose
    # larger violation is least
    t = lineqp.min_max_violation(lo, hi, G, h0)
    z_mm, _, _, feas_mm = lineqp.solve_line_qps(QL, c, lo, hi, G, h0 + 1.1 * t[:, None])
    assert feas_mm.all()
    err, err_mm = [], []
    for k in range(idx.size):
        r = alm.solve_line(QL[k], c[k], lo[k], hi[k], G[k], h0[k])
        assert not r.converged          # no feasible point: the penalty runs down
        width = np.abs(hi[k] - lo[k]).max()
        err.append(np.abs(r.z - z[k]).max() / width)
        err_mm.append(np.abs(r.z - z_mm[k]).max() / width)
    err, err_mm = np.array(err), np.array(err_mm)
    # the local method stalls near the limit once its penalty parameter is
    # tiny (the subproblems are then ill-conditioned), a few parts in 1e7 of
    # the box width at the median; the min-max reading is tens of percent away
    assert np.median(err) < 1e-6 and np.percentile(err, 90) < 1e-4 and err.max() < 1e-3, \
        (np.median(err), np.percentile(err, 90), err.max())
    assert np.median(err_mm) > 1e-2


def test_psi_change_equals_the_difference_of_values():
    rng = np.random.default_rng(13)
    Q, c, lo, hi, G, h = _random_lines(rng, 50, convex=False)
    for k in range(50):
        z = rng.uniform(lo[k], hi[k])
        s = rng.standard_normal(4) * 0.05
        u = np.abs(rng.standard_normal(2))
        mu = 10.0 ** rng.uniform(-3, 1)
        ref = alm.psi(z + s, Q[k], c[k], G[k], h[k], u, mu) - alm.psi(z, Q[k], c[k], G[k], h[k], u, mu)
        got = alm.psi_change(z, s, Q[k], c[k], G[k], h[k], u, mu)
        scale = abs(alm.psi(z, Q[k], c[k], G[k], h[k], u, mu)) + abs(ref) + 1.0
        assert abs(got - ref) <= 1e-12 * scale


def test_alm_converges_from_a_start_at_the_minimiser_of_stiff_lines():
    """Strictly convex, stiff lines (line matrices with eigenvalues from 2e4
    to 7e6 on a box of half-width 0.05, as penalties of 2e4 give on large
    grids), rows far from binding, started a hair away from their minimiser
    (the previous sweep's solution): the ratio test must see the model's
    decrease although psi itself is large, and the method converges to the
    exact minimiser."""
    rng = np.random.default_rng(14)
    n = 60
    ok = 0
    for k in range(n):
        qm, _ = np.linalg.qr(rng.standard_normal((4, 4)))
        Q = qm @ np.diag([2e4, 1e5, 1e6, 7e6]) @ qm.T
        lo, hi = np.full(4, -0.05), np.full(4, 0.05)
        c = rng.standard_normal(4) * 2e5
        G = rng.standard_normal((2, 4))
        h = np.full(2, 5.0)
        zr, _, _, feas = lineqp.solve_line_qps(Q[None], c[None], lo[None], hi[None], G[None], h[None])
        r = alm.solve_line(Q, c, lo, hi, G, h, z0=zr[0] + 1e-9 * rng.standard_normal(4), u0=np.zeros(2))
        assert r.converged, k
        assert np.abs(r.z - zr[0]).max() <= 1e-8, k
        ok += 1
    assert ok == n
