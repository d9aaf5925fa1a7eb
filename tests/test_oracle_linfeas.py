"""Pins of the linear feasibility projection (Section II-A, eq. linfeas)."""
import numpy as np
import pytest

from synth.grids import grid_14, tiny_grid, power_flow_start
from oracle import acopf, linfeas


def _pf(g):
    s = power_flow_start(g)
    return acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])


def test_balance_matrix_reproduces_the_balance_residuals():
    """A x - b equals the model's balance residuals at random points (the
    matrix is read off the model at unit vectors, so this checks that the
    residuals are affine and the reading is complete)."""
    g = tiny_grid(seed=4, n_bus=6, n_line=9, n_gen=3)
    A, b = linfeas.balance_matrix(g)
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = acopf.Iterate(*(rng.standard_normal(n) for n in (g.n_gen, g.n_gen, g.n_bus, g.n_bus, g.n_line,
                                                               g.n_line)))
        rp, rq = acopf.balance(g, x)
        np.testing.assert_allclose(A @ linfeas._vec(x) - b, np.concatenate([rp, rq]), atol=1e-12)


def test_a_linearly_feasible_start_is_its_own_projection():
    """A point that meets every linear constraint (here: a projection of the
    power-flow start, which is below some voltage bounds) projects onto
    itself with objective 0."""
    g = grid_14()
    x0 = _pf(g)
    assert linfeas.violation(g, x0) > 1e-3
    x1 = linfeas.project(g, x0).x
    assert linfeas.violation(g, x1) < 1e-8
    p = linfeas.project(g, x1)
    assert p.objective < 1e-12
    np.testing.assert_allclose(linfeas._vec(p.x), linfeas._vec(x1), atol=1e-6)


def test_projection_kkt_and_nearest_feasible_point():
    """From the flat start (which violates the balance): the result meets the
    linear constraints, satisfies the KKT conditions of the projection (the
    step x - x0 plus A^T nu is absorbed by bound multipliers of the right
    sign at active bounds only), and no other feasible point found here is
    closer to x0 (projections of perturbed starts are feasible points)."""
    g = grid_14()
    x0 = acopf.flat_start(g)
    assert linfeas.violation(g, x0) > 1e-3
    p = linfeas.project(g, x0)
    assert linfeas.violation(g, p.x) < 1e-8
    A, b = linfeas.balance_matrix(g)
    lo, hi = linfeas.bounds(g)
    v, v0 = linfeas._vec(p.x), linfeas._vec(x0)
    grad = (v - v0) + A.T @ p.nu
    atlo, athi = v <= lo + 1e-7, v >= hi - 1e-7
    free = ~atlo & ~athi
    assert np.abs(grad[free]).max() < 1e-7
    assert (grad[atlo & ~athi] >= -1e-7).all() and (grad[athi & ~atlo] <= 1e-7).all()
    assert p.objective > 0.0  # the start was not linearly feasible
    rng = np.random.default_rng(1)
    for _ in range(5):
        xs = linfeas._unvec(g, v0 + 0.05 * rng.standard_normal(v0.size))
        y = linfeas._vec(linfeas.project(g, xs).x)
        assert linfeas.violation(g, linfeas._unvec(g, y)) < 1e-8
        assert np.sum((y - v0) ** 2) >= p.objective - 1e-9


@pytest.mark.parametrize("case", ["ring14", "tiny_shunt"])
def test_decomposed_projection_reaches_the_projection(case):
    """The projection run through the ADMM decomposition of the QP
    subproblems (identity Hessian: generators, lines with free wR, wI and a
    1/degree share of each bus's w term, buses with their balance rows)
    converges to the interior-point projection: the same point to 1e-7, the
    linear constraints met."""
    g = grid_14() if case == "ring14" else tiny_grid(seed=21, n_bus=7, n_line=10, n_gen=3, shunt_scale=0.04)
    x0 = acopf.flat_start(g)
    assert linfeas.violation(g, x0) > 1e-3
    p = linfeas.project(g, x0)
    a = linfeas.admm_project(g, x0, 1.0, 20000, 1e-10, 1e-10)
    assert a.converged
    assert linfeas.violation(g, a.x) < 1e-8
    np.testing.assert_allclose(linfeas._vec(a.x), linfeas._vec(p.x), atol=1e-7)
    # the angles are not moved (theta_ref of the start is 0 and no other
    # linear constraint involves them)
    assert np.array_equal(a.x.th, x0.th)
