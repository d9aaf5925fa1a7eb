"""Pins of the learned warm start's oracle (network, training step, targets,
decoding) against calculus, hand-computed values and the ADMM solver's own
residual history."""
import numpy as np
import pytest

from oracle import mlp, admm, qp as qpm
from synth.grids import tiny_grid
from tests._util import start_point


def _random_net(rng, n_in=16, n_h=64, n_out=16, scale=0.3):
    v = rng.standard_normal(mlp.n_params(n_in, n_h, n_out)) * scale
    return mlp.Params.unflat(v, n_in, n_h, n_out)


def test_forward_hand_case():
    # y = relu(x) + relu(-x) + 0.5 = |x| + 0.5 through two hidden units
    p = mlp.Params(W1=np.array([[1.0], [-1.0]]), b1=np.zeros(2), W2=np.eye(2), b2=np.zeros(2),
                   W3=np.array([[1.0, 1.0]]), b3=np.array([0.5]))
    y, _ = mlp.forward(p, np.array([[-3.0], [2.0], [0.0]]))
    assert np.allclose(y[:, 0], [3.5, 2.5, 0.5], rtol=0, atol=0)
    # the second ReLU acts: a negative pre-activation of layer 2 is cut
    p.b2 = np.array([-1.0, 0.0])
    y, _ = mlp.forward(p, np.array([[0.5], [3.0]]))
    assert np.allclose(y[:, 0], [0.5 + 0.0, 0.5 + 2.0], rtol=0, atol=0)


def test_loss_of_zero_network_is_mean_square_target():
    rng = np.random.default_rng(1)
    p = mlp.Params.unflat(np.zeros(mlp.n_params(8, 64, 4)), 8, 64, 4)
    X, T = rng.standard_normal((30, 8)), rng.standard_normal((30, 4))
    assert mlp.loss(p, X, T) == pytest.approx(np.mean(T ** 2), rel=1e-15)


@pytest.mark.parametrize("n_in,n_out", [(16, 16), (8, 4)])
def test_gradients_match_central_differences(n_in, n_out):
    rng = np.random.default_rng(n_in)
    p = _random_net(rng, n_in, 64, n_out)
    X, T = rng.standard_normal((40, n_in)), rng.standard_normal((40, n_out))
    g = mlp.gradients(p, X, T).flat()
    th = p.flat()
    h = 1e-6
    idx = rng.choice(th.size, 300, replace=False)
    fd = np.empty(idx.size)
    for j, i in enumerate(idx):
        a, b = th.copy(), th.copy()
        a[i] += h
        b[i] -= h
        fd[j] = (mlp.loss(mlp.Params.unflat(a, n_in, 64, n_out), X, T)
                 - mlp.loss(mlp.Params.unflat(b, n_in, 64, n_out), X, T)) / (2 * h)
    err = np.linalg.norm(fd - g[idx]) / np.linalg.norm(g[idx])
    assert err < 1e-7, err


def test_adam_first_step_is_lr_times_sign():
    # with m = v = 0 the bias-corrected moments are g and g^2
    g = np.array([3.0, -0.02, 1e-3, -50.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-15, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_fits_a_teacher_network():
    rng = np.random.default_rng(7)
    teacher = _random_net(rng, 8, 64, 4, scale=0.4)
    X = rng.standard_normal((256, 8))
    T, _ = mlp.forward(teacher, X)
    p = _random_net(rng, 8, 64, 4, scale=0.1)
    th = p.flat()
    m, v = np.zeros_like(th), np.zeros_like(th)
    l0 = mlp.loss(p, X, T)
    for t in range(1, 1501):
        p = mlp.Params.unflat(th, 8, 64, 4)
        th, m, v = mlp.adam_step(th, mlp.gradients(p, X, T).flat(), m, v, t, lr=3e-3)
    l1 = mlp.loss(mlp.Params.unflat(th, 8, 64, 4), X, T)
    assert l1 < 1e-2 * l0, (l0, l1)


def test_trace_sums_reproduce_the_solver_residual_norms():
    """Summed per coupling, the squared residuals recomputed from recorded
    states equal the residual norms the ADMM solver reports every sweep (a
    wrong coupling index or a missed copy breaks the equality)."""
    g = tiny_grid(3)
    x, pi = start_point(g, pi_scale=50.0)
    Q = qpm.build_qp(g, x, pi, 0.05)
    rng = np.random.default_rng(3)
    rho = admm.Rho(rng.uniform(1e3, 5e4, (g.n_gen, 2)), rng.uniform(1e3, 5e4, (g.n_line, 8)))
    st0 = admm.cold_state(g)
    norms = admm.solve(g, Q, rho, 12, 0.0, 0.0, state=st0, record=True).history
    states = admm.solve(g, Q, rho, 12, 0.0, 0.0, state=st0, record_states=True).history
    prev = st0
    for k, st in enumerate(states):
        # one-sweep sums of squares from the same function on |.|^2 pieces
        rg, sg, rl, sl = mlp.trace_sums(g, rho, prev, [st])
        r2 = np.sum(rg ** 2) + np.sum(rl ** 2)
        s2 = np.sum(sg ** 2) + np.sum(sl ** 2)
        assert np.sqrt(r2) == pytest.approx(norms[k][0], rel=1e-12)
        assert np.sqrt(s2) == pytest.approx(norms[k][1], rel=1e-12, abs=1e-300)
        prev = st
    # additivity over sweeps
    tot = mlp.trace_sums(g, rho, st0, states)
    parts = [mlp.trace_sums(g, rho, a, [b]) for a, b in zip([st0] + states[:-1], states)]
    for j in range(4):
        assert np.allclose(tot[j], sum(p[j] for p in parts), rtol=1e-13, atol=0)


def test_log_rho_factor_cases():
    rho = np.array([2.0, 2.0, 2.0, 2.0, 2.0, 2.0, 2e4])
    sr = np.array([1.0, 1.0, 1.0, 0.0, 1.0, 4.0, 1e-17])
    ss = np.array([2.0, 2e6, 2e-6, 0.0, 0.0, 2.0, 0.0])
    got = mlp.log_rho_factor(rho, sr, ss)
    # balanced -> 1; far off -> clipped; 0/0 -> 1; r/0 -> upper clip; sqrt(4);
    # rounding noise on a coupling that never moves -> 1
    assert np.allclose(np.exp(got), [1.0, 0.1, 10.0, 1.0, 10.0, 2.0, 1.0], rtol=1e-6)


def test_decode_applies_scales_clip_and_guard():
    out_l = np.zeros((2, 16))
    out_l[0, :8] = np.arange(8) * 0.5
    out_l[0, 8:] = [0.0, 1.0, -1.0, 5.0, -5.0, np.log(2.0), np.nan, 0.0]
    out_l[1, 3] = np.inf
    out_g = np.array([[1.0, np.nan, 0.5, np.nan]])
    prev_l = np.full((2, 8), -7.0)
    prev_g = np.full((1, 2), 9.0)
    lam_l, lam_g, rho_l, rho_g = mlp.decode(out_l, out_g, 100.0, 50.0, prev_l, prev_g, True, True)
    # multipliers: the plain start plus the scaled correction
    assert np.allclose(lam_l[0], -7.0 + np.arange(8) * 500.0)
    assert lam_l[1, 3] == -7.0 and np.all(lam_l[1, [0, 1, 2, 4, 5, 6, 7]] == -7.0)
    assert np.allclose(rho_l[0], 100.0 * np.array([1.0, np.e, 1 / np.e, 10.0, 0.1, 2.0, 1.0, 1.0]))
    assert lam_g[0, 0] == 1009.0 and lam_g[0, 1] == 9.0
    assert rho_g[0, 0] == pytest.approx(50.0 * np.exp(0.5)) and rho_g[0, 1] == 50.0
    lam_l2, lam_g2, rho_l2, rho_g2 = mlp.decode(out_l, out_g, 100.0, 50.0, prev_l, prev_g, False, False)
    assert np.all(lam_l2 == -7.0) and np.all(lam_g2 == 9.0)
    assert np.all(rho_l2 == 100.0) and np.all(rho_g2 == 50.0)


def test_targets_are_the_scaled_change_of_the_multipliers():
    rho = admm.Rho(np.full((1, 2), 4.0), np.full((1, 8), 4.0))
    lam0_l, lam_l = np.arange(8.0)[None] * 100, np.arange(8.0)[None] * 300
    lam0_g, lam_g = np.array([[5.0, -5.0]]), np.array([[2005.0, 995.0]])
    sums = (np.ones((1, 2)), np.full((1, 2), 4.0), np.ones((1, 8)), np.full((1, 8), 16.0))
    tl, tg = mlp.targets(rho, lam_g, lam_l, lam0_g, lam0_l, sums)
    assert np.allclose(tl[0, :8], np.arange(8) * 0.2) and np.allclose(tg[0, :2], [2.0, 1.0])
    # log factors: sqrt(4 * 1 / 4) = 1, sqrt(4 * 1 / 16) = 1/2
    assert np.allclose(tg[0, 2:], 0.0, atol=1e-6) and np.allclose(tl[0, 8:], np.log(0.5), atol=1e-6)


def test_column_stats_and_standardize_hand_cases():
    X = np.array([[1.0, 7.0], [2.0, 7.0], [3.0, 7.0], [4.0, 7.0]])
    mean, std = mlp.column_stats(X)
    assert np.allclose(mean, [2.5, 7.0]) and np.allclose(std, [np.sqrt(1.25), mlp.STD_FLOOR])
    Z = mlp.standardize(np.array([[2.5 + 10 * np.sqrt(1.25), 7.0]]), mean, std, clip=5.0)
    assert np.allclose(Z, [[5.0, 0.0]])
    assert np.allclose(mlp.standardize(X, mean, std)[:, 0], (X[:, 0] - 2.5) / np.sqrt(1.25))


def test_fold_equals_the_standardised_network():
    """Folding the input and output maps into the first and last layers
    gives the same function as applying them around the network."""
    rng = np.random.default_rng(11)
    p = _random_net(rng, 25, 64, 16)
    X = rng.standard_normal((50, 25)) * rng.uniform(0.01, 3, 25) + rng.uniform(-2, 2, 25)
    mi, si = X.mean(0), X.std(0)
    mo, so = rng.uniform(-1, 1, 16), rng.uniform(0.1, 2, 16)
    y_ref, _ = mlp.forward(p, (X - mi) / si)
    y_ref = y_ref * so + mo
    y, _ = mlp.forward(mlp.fold(p, mi, si, mo, so), X)
    assert np.allclose(y, y_ref, rtol=1e-12, atol=1e-12)


def test_features_have_the_documented_columns():
    g = tiny_grid(5)
    x, _ = start_point(g)
    rng = np.random.default_rng(2)
    pl, pg = rng.normal(0, 1e3, (g.n_line, 8)), rng.normal(0, 1e3, (g.n_gen, 2))
    fl, fg = mlp.line_features(g, x, pl, True), mlp.gen_features(g, x, pg, False)
    assert fl.shape == (g.n_line, mlp.N_LINE_FEAT) and fg.shape == (g.n_gen, mlp.N_GEN_FEAT)
    l = g.n_line - 1
    assert fl[l, 0] == g.pd[g.f[l]] and fl[l, 3] == g.qd[g.t[l]] and fl[l, 12] == x.wR[l]
    assert fl[l, 14] == np.sin(x.th[g.f[l]] - x.th[g.t[l]]) and fl[l, 15] == g.smax_ij[l]
    assert np.allclose(fl[:, 16:24], pl / 1e3) and np.all(fl[:, 24] == 1.0)
    k = g.n_gen - 1
    assert fg[k, 0] == g.pd[g.gbus[k]] and fg[k, 4] == x.pg[k] and fg[k, 7] == g.qmax[k]
    assert np.allclose(fg[:, 8:10], pg / 1e3) and np.all(fg[:, 10] == 0.0)
