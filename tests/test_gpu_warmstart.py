"""GPU parity of the learned warm start's kernels against the FP64 oracle:
network forward pass, back-propagated gradient and loss, Adam, component
features, trace sums and training targets of a traced solve, and the
decoding of outputs (with its guard)."""
import numpy as np
import pytest

from oracle import admm, mlp, qp as qpm
from synth.grids import tiny_grid
from tests._util import rel_err, start_point

pytestmark = pytest.mark.gpu

# FP32 products of depth <= 64 against FP64: relative error ~1e-6; the
# norm-wise bound allows for the largest FP32 accumulation error
FP32_TOL = 1e-4


def _torch():
    import torch
    return torch


def _net(n_in, n_out, seed):
    from paper_2310_13143_amd.warmstart import MLP, init_params
    net = MLP(n_in, n_out, "cuda:0", seed)
    rng = np.random.default_rng(seed)
    th = init_params(n_in, n_out, seed) + rng.normal(0, 0.05, net.count).astype(np.float32)
    net.theta.copy_(_torch().as_tensor(th))
    return net, mlp.Params.unflat(th.astype(np.float64), n_in, 64, n_out)


# Least distance of every pre-activation from zero in the parity inputs.  A
# ReLU takes a decision on the sign of its input; FP32 rounding (~1e-7 of the
# terms) would otherwise flip the odd decision against the FP64 oracle and
# move a gradient entry by one sample's whole contribution.
MARGIN = 1e-4


def _samples(n_in, n_out, n, ld, seed, p=None):
    """Seeded samples in columns 0..n-1 of [n_in][ld] / [n_out][ld] arrays;
    with the oracle network p, samples with a pre-activation closer than
    MARGIN to zero are redrawn."""
    torch = _torch()
    rng = np.random.default_rng(seed + 100)
    X = np.zeros((n_in, ld), np.float32)
    T = np.zeros((n_out, ld), np.float32)
    X[:, :n] = rng.standard_normal((n_in, n))
    T[:, :n] = rng.standard_normal((n_out, n))
    for _ in range(50 if p is not None else 0):
        _, (_, z1, _, z2, _) = mlp.forward(p, X[:, :n].T.astype(np.float64))
        bad = np.nonzero((np.abs(z1) < MARGIN).any(1) | (np.abs(z2) < MARGIN).any(1))[0]
        if bad.size == 0:
            break
        X[:, bad] = rng.standard_normal((n_in, bad.size))
    else:
        assert p is None, "could not draw samples away from the ReLU kinks"
    # columns past n hold garbage the kernels must not read
    X[:, n:] = np.nan
    T[:, n:] = np.nan
    return X, T, torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda()


@pytest.mark.parametrize("n_in,n_out,n", [(16, 16, 1000), (8, 4, 70), (5, 3, 64), (16, 16, 65636), (64, 16, 257)])
def test_mlp_forward_gradient_loss_match_oracle(n_in, n_out, n):
    """Ragged tails, sizes that are not multiples of the tiles, more tiles
    than blocks (65,636 samples) and a leading dimension above n."""
    print(f"[gpu] mlp n_in={n_in} n_out={n_out} n={n}", flush=True)
    net, p = _net(n_in, n_out, n_in * 7 + n_out)
    X, T, Xd, Td = _samples(n_in, n_out, n, n + 9, n, p)
    Y = net.forward(Xd, n).cpu().numpy()
    yref, _ = mlp.forward(p, X[:, :n].T.astype(np.float64))
    assert rel_err(Y.T, yref) <= FP32_TOL
    g, loss = net.gradient(Xd, Td, n)
    gref = mlp.gradients(p, X[:, :n].T.astype(np.float64), T[:, :n].T.astype(np.float64)).flat()
    lref = mlp.loss(p, X[:, :n].T.astype(np.float64), T[:, :n].T.astype(np.float64))
    assert rel_err(g.cpu().numpy(), gref) <= FP32_TOL
    assert abs(loss.item() - lref) <= FP32_TOL * lref
    # each layer's share of the gradient on its own (a wrong block would hide in the norm)
    off = np.cumsum([0, 64 * n_in, 64, 64 * 64, 64, n_out * 64, n_out])
    gd = g.cpu().numpy()
    for a, b in zip(off[:-1], off[1:]):
        assert rel_err(gd[a:b], gref[a:b]) <= FP32_TOL, (a, b)


def test_mlp_gradient_is_deterministic():
    net, _ = _net(16, 16, 3)
    _, _, Xd, Td = _samples(16, 16, 5000, 5000, 3)
    g1, l1 = net.gradient(Xd, Td)
    g2, l2 = net.gradient(Xd, Td)
    assert _torch().equal(g1, g2) and _torch().equal(l1, l2)


# The ABI takes Adam's hyperparameters in FP32: 0.999 becomes 0.99900001, so
# 1 - beta2 differs from 0.001 by 1.3e-5 relative.  The oracle gets the same
# rounded values.
F32_ADAM = {k: float(np.float32(v)) for k, v in (("lr", 0.01), ("b1", 0.9), ("b2", 0.999), ("eps", 1e-8))}


def test_mlp_adam_matches_oracle():
    print("[gpu] mlp adam", flush=True)
    torch = _torch()
    net, p = _net(8, 4, 11)
    rng = np.random.default_rng(5)
    th = p.flat()
    m, v = np.zeros_like(th), np.zeros_like(th)
    for t in range(1, 4):
        g = (rng.standard_normal(net.count) * 10.0 ** rng.integers(-3, 2)).astype(np.float32)
        net.adam(torch.as_tensor(g).cuda(), 0.01)
        th, m, v = mlp.adam_step(th, g.astype(np.float64), m, v, t, **F32_ADAM)
    assert rel_err(net.theta.cpu().numpy(), th) <= 1e-6
    assert rel_err(net.m.cpu().numpy(), m) <= 1e-6
    assert rel_err(net.v.cpu().numpy(), v) <= 1e-5


def test_training_lowers_the_loss_like_the_oracle():
    """Twenty device Adam steps track twenty oracle steps from the same start.
    Adam divides each gradient entry by its own running magnitude, so FP32
    rounding in entries near zero moves them by up to a step (lr): the
    parameter tolerance is 1e-3 rather than the gradient's 1e-4."""
    print("[gpu] mlp training", flush=True)
    net, p = _net(16, 16, 21)
    X, T, Xd, Td = _samples(16, 16, 3000, 3000, 21, p)
    Xo, To = X.T.astype(np.float64), T.T.astype(np.float64)
    th = p.flat()
    m, v = np.zeros_like(th), np.zeros_like(th)
    for t in range(1, 21):
        g, _ = net.gradient(Xd, Td)
        net.adam(g, 3e-3)
        gref = mlp.gradients(mlp.Params.unflat(th, 16, 64, 16), Xo, To).flat()
        th, m, v = mlp.adam_step(th, gref, m, v, t, **dict(F32_ADAM, lr=float(np.float32(3e-3))))
    assert rel_err(net.theta.cpu().numpy(), th) <= 1e-3
    l0 = mlp.loss(p, Xo, To)
    l1 = mlp.loss(mlp.Params.unflat(net.theta.cpu().numpy().astype(np.float64), 16, 64, 16), Xo, To)
    assert l1 < l0


def test_features_trace_targets_and_decode_match_oracle():
    print("[gpu] warm-start features / traced solve / targets / decode", flush=True)
    torch = _torch()
    from paper_2310_13143_amd import _abi
    from paper_2310_13143_amd.solver import DeviceGrid
    g = tiny_grid(7)
    G, L = g.n_gen, g.n_line
    x, pi = start_point(g, pi_scale=30.0)
    dg = DeviceGrid(g, "cuda:0")
    xi = dg.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pi)
    fl, fg = dg.features(xi, True)
    zl, zg = np.zeros((L, 8)), np.zeros((G, 2))
    assert rel_err(fl.cpu().numpy().T, mlp.line_features(g, x, zl, True)) <= 1e-7
    assert rel_err(fg.cpu().numpy()[:, :G].T, mlp.gen_features(g, x, zg, True)) <= 1e-7

    rng = np.random.default_rng(9)
    rho = admm.Rho(rng.uniform(5e3, 5e4, (g.n_gen, 2)), rng.uniform(5e3, 5e4, (g.n_line, 8)))
    lam0 = admm.warm_state(g, rng.normal(0, 500, (g.n_gen, 2)), rng.normal(0, 500, (g.n_line, 8)))
    Q = qpm.build_qp(g, x, pi, 0.05)
    dg.qp_build(xi, 0.05)
    dg.admm_init(rho.g.T.ravel(), rho.l.T.ravel(), lam0.lam_g.T.ravel(), lam0.lam_l.T.ravel())
    sweeps = 40
    dg.admm_solve(sweeps, sweep_mode=_abi.SWEEP_LAUNCHES, block_size=64, trace=True)
    ref = admm.solve(g, Q, rho, sweeps, 0.0, 0.0, state=lam0, record_states=True)
    sums = mlp.trace_sums(g, rho, lam0, ref.history)
    st = dg.admm_state()
    got = [st["sum_r_g"].cpu().numpy().reshape(2, G).T, st["sum_s_g"].cpu().numpy().reshape(2, G).T,
           st["sum_r_l"].cpu().numpy().reshape(8, L).T, st["sum_s_l"].cpu().numpy().reshape(8, L).T]
    for a, b in zip(got, sums):
        assert rel_err(a, b) <= 1e-8
    tl, tg = dg.warm_targets()
    rl, rg = mlp.targets(rho, ref.state.lam_g, ref.state.lam_l, lam0.lam_g, lam0.lam_l, sums)
    assert rel_err(tl.cpu().numpy().T, rl) <= 1e-6
    assert rel_err(tg.cpu().numpy()[:, :G].T, rg) <= 1e-6

    # features of a later QP carry the workspace's multipliers
    plain_l, plain_g = st["lam_l"].cpu().numpy().reshape(8, L).T, st["lam_g"].cpu().numpy().reshape(2, G).T
    fl, fg = dg.features(xi, False)
    assert rel_err(fl.cpu().numpy().T, mlp.line_features(g, x, plain_l, False)) <= 1e-7
    assert rel_err(fg.cpu().numpy()[:, :G].T, mlp.gen_features(g, x, plain_g, False)) <= 1e-7

    # decode: network-like outputs with non-finite entries, later and first QP
    yl = rng.normal(0, 1, (16, L)).astype(np.float32)
    yg = rng.normal(0, 1, (4, G)).astype(np.float32)
    yl[3, 1] = np.nan
    yl[10, 2] = np.inf
    yl[9, 0] = 7.0
    yg[1, 0] = np.nan
    for first, use_lam, use_rho in ((False, True, True), (True, True, False), (False, False, True)):
        got = dg.warm_decode(torch.as_tensor(yl).cuda(), torch.as_tensor(yg).cuda(), 2e4, 3e4, first, use_lam,
                             use_rho)
        base_l, base_g = (zl, zg) if first else (plain_l, plain_g)
        el, eg, erl, erg = mlp.decode(yl.T.astype(np.float64), yg.T.astype(np.float64), 2e4, 3e4, base_l, base_g,
                                      use_lam, use_rho)
        lam_g, lam_l, rho_g, rho_l = (t.cpu().numpy() for t in got)
        assert rel_err(lam_l.reshape(8, L).T, el) <= 1e-15
        assert rel_err(lam_g.reshape(2, G).T, eg) <= 1e-15
        assert rel_err(rho_l.reshape(8, L).T, erl) <= 1e-14
        assert rel_err(rho_g.reshape(2, G).T, erg) <= 1e-14


def test_standardize_and_fold_match_oracle():
    """Per-feature statistics, in-place standardisation with clipping, and
    the fold of both maps into the network, against the oracle."""
    print("[gpu] mlp stats / standardize / fold", flush=True)
    torch = _torch()
    from paper_2310_13143_amd import _abi
    lib = _abi.load()
    rng = np.random.default_rng(4)
    n, ld = 5003, 5011
    X = np.zeros((25, ld), np.float32)
    X[:, :n] = rng.standard_normal((25, n)) * rng.uniform(1e-3, 5, (25, 1)) + rng.uniform(-3, 3, (25, 1))
    X[7, :n] = 1.5  # constant feature: deviation floored
    Xd = torch.as_tensor(X).cuda()
    mean = torch.empty(25, dtype=torch.float64, device="cuda")
    std = torch.empty(25, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    _abi.check(lib.acopf_mlp_feature_stats(Xd.data_ptr(), 25, ld, n, mean.data_ptr(), std.data_ptr(), stream))
    m_ref, s_ref = mlp.column_stats(X[:, :n].T.astype(np.float64))
    assert rel_err(mean.cpu().numpy(), m_ref) <= 1e-12 and rel_err(std.cpu().numpy(), s_ref) <= 1e-10
    _abi.check(lib.acopf_mlp_standardize(Xd.data_ptr(), 25, ld, n, mean.data_ptr(), std.data_ptr(), 2.0, stream))
    Z = Xd.cpu().numpy()
    assert rel_err(Z[:, :n].T, mlp.standardize(X[:, :n].T.astype(np.float64), m_ref, s_ref, 2.0)) <= 1e-6
    assert np.array_equal(Z[:, n:], X[:, n:])  # columns past n untouched

    net, p = _net(25, 16, 5)
    mo, so = rng.uniform(-1, 1, 16), rng.uniform(0.1, 3, 16)
    mod, sod = torch.as_tensor(mo).cuda(), torch.as_tensor(so).cuda()
    _abi.check(lib.acopf_mlp_fold(net.theta.data_ptr(), 25, 16, mean.data_ptr(), std.data_ptr(), mod.data_ptr(),
                                  sod.data_ptr(), stream))
    ref = mlp.fold(p, m_ref, s_ref, mo, so).flat()
    assert rel_err(net.theta.cpu().numpy(), ref) <= 1e-6
