"""Parity of the HIP path with the oracle on the GPU.

Iterates of the ADMM sweeps (Algorithm 2) must match the serial oracle
within 1e-8 for fixed sweep counts, relative per column of each state array
(each coupling on its own scale; ``tests._util.rel_err_cols``); the
limit must match the direct solve of the QP within 1e-6 relative objective
and 1e-5 constraint violation.  All calls go through the C ABI."""
import os

import numpy as np
import pytest

from synth.grids import grid_14, grid_2000, grid_70000, make_grid, tiny_grid
from oracle import acopf, admm, direct, qp as qpm, sqp
from tests._util import rel_err, rel_err_cols, start_point

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _dev():
    from paper_2310_13143_amd.solver import DeviceGrid
    return DeviceGrid


def _rho(g, seed, lo=5e3, hi=3e4):
    rng = np.random.default_rng(seed)
    return admm.Rho(rng.uniform(lo, hi, (g.n_gen, 2)), rng.uniform(lo, hi, (g.n_line, 8)))


def _run_gpu(g, x, pi, delta, rho, lam_g, lam_l, sweeps, mode=0, eps=0.0, hessian=0, **kw):
    dg = _dev()(g)
    xi = dg.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pi)
    dg.qp_build(xi, delta, hessian)
    dg.admm_init(rho.g.T.reshape(-1), rho.l.T.reshape(-1),
                 None if lam_g is None else lam_g.T.reshape(-1), None if lam_l is None else lam_l.T.reshape(-1))
    res = dg.admm_solve(sweeps, eps, eps, sweep_mode=mode, **kw)
    st = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    return dg, xi, res, st


def _compare_state(st, ref, tol=TOL):
    G, L, B = ref.xg.shape[0], ref.xl.shape[0], ref.dw.shape[0]
    pairs = {
        "xl": (st["xl"].reshape(8, L).T, ref.xl), "lam_l": (st["lam_l"].reshape(8, L).T, ref.lam_l),
        "xbar_f": (st["xbar_f"].reshape(4, L).T, ref.xbar_f), "xg": (st["xg"].reshape(2, G).T, ref.xg),
        "lam_g": (st["lam_g"].reshape(2, G).T, ref.lam_g), "xbar_g": (st["xbar_g"].reshape(2, G).T, ref.xbar_g),
        "dw": (st["dw"], ref.dw), "dth": (st["dth"], ref.dth), "nu": (st["nu"].reshape(2, B).T, ref.nu),
    }
    for name, (a, b) in pairs.items():
        e = rel_err_cols(a, b)
        assert e <= tol, f"{name}: relative error {e:.3e}"


CASES = {
    "ring14": lambda: grid_14(),
    "tiny_shunt": lambda: tiny_grid(seed=21, n_bus=7, n_line=10, n_gen=3, shunt_scale=0.04),
    # a bus of degree 89, wider than a 64-slot item block: one whole-bus slot
    "star90": lambda: make_grid(90, 100, 6, seed=90, topology="star", name="star90"),
}


@pytest.mark.parametrize("mode", [0, 1], ids=["persistent", "launches"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_sweeps_match_oracle(case, mode):
    print(f"[gpu] sweeps {case} mode={mode}", flush=True)
    g = CASES[case]()
    x, pi = start_point(g, pi_scale=50.0, seed=3)
    delta = 0.05
    rho = _rho(g, 4)
    rng = np.random.default_rng(5)
    lam_g, lam_l = rng.standard_normal((g.n_gen, 2)) * 100, rng.standard_normal((g.n_line, 8)) * 100
    nsw = 60
    Q = qpm.build_qp(g, x, pi, delta, "psd")
    ref = admm.solve(g, Q, rho, nsw, 0.0, 0.0, state=admm.warm_state(g, lam_g, lam_l), record=True)
    dg, xi, res, st = _run_gpu(g, x, pi, delta, rho, lam_g, lam_l, nsw, mode=mode)
    assert res["sweeps"] == nsw and res["infeasible_lines"] == 0
    _compare_state(st, ref.state)
    assert abs(res["r"] - ref.r) <= 1e-7 * ref.r and abs(res["s"] - ref.s) <= 1e-7 * ref.s
    # step and multiplier estimates (Section IV-B5)
    d = {k: v.cpu().numpy() for k, v in dg.step(xi).items()}
    dref = sqp.assemble_step(g, Q, ref.state)
    pref = sqp.recover_pi(g, x, Q, ref.state)
    for k in ("pg", "qg", "w", "th", "wR", "wI"):
        assert rel_err(d[k], getattr(dref, k)) <= TOL, k
    assert rel_err(d["pi"].reshape(4, -1).T, pref) <= 1e-7


def test_raw_hessian_and_cold_start_match_oracle():
    print("[gpu] raw hessian ring14", flush=True)
    g = grid_14()
    x, pi = start_point(g, pi_scale=20.0, seed=8)
    rho = admm.Rho.scalar(g, 2e4)
    Q = qpm.build_qp(g, x, pi, 0.1, "raw")
    ref = admm.solve(g, Q, rho, 50, 0.0, 0.0)
    _, _, res, st = _run_gpu(g, x, pi, 0.1, rho, None, None, 50, hessian=1)
    _compare_state(st, ref.state)


def test_raw_mode_reports_a_nonconvex_line():
    """With the unmodified line Hessian (RAW mode), a line whose QP matrix
    M + sum rho_f F^T F + diag(rho_v) is not positive definite (strong
    negative curvature from pi, small penalties) stops the solve with
    ACOPF_ERR_NONCONVEX_LINE; the oracle's matrices confirm the sign."""
    from paper_2310_13143_amd import AcopfError
    print("[gpu] raw mode nonconvex line", flush=True)
    g = grid_14()
    x, pi = start_point(g)
    pi[3, 0] = -5e4
    rho = admm.Rho.scalar(g, 1.0)
    Q = qpm.build_qp(g, x, pi, 0.1, "raw")
    lam_min = np.linalg.eigvalsh(admm.line_matrices(Q, rho)).min(axis=1)
    assert lam_min[3] < 0 and (np.delete(lam_min, 3) > 0).all()
    dg = _dev()(g)
    xi = dg.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pi)
    dg.qp_build(xi, 0.1, 1)
    with pytest.raises(AcopfError) as e:
        dg.admm_init(*dg.rho_scalar(1.0))
        dg.admm_solve(5)
    assert e.value.code == -3
    # the projected mode solves the same line
    dg.qp_build(xi, 0.1, 0)
    dg.admm_init(*dg.rho_scalar(1.0))
    assert dg.admm_solve(5)["sweeps"] == 5


def test_rgg2000_500_sweeps_match_the_stored_oracle_run():
    """500 sweeps of the 2,000-bus QP against the oracle's run stored by
    tests/golden/make_rgg2000_sweeps.py (sampled lines, all generators and
    buses, after 100 and 500 sweeps; residual norms of every sweep)."""
    from paper_2310_13143_amd import _abi
    print("[gpu] rgg2000 500 sweeps vs stored oracle run", flush=True)
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "rgg2000_500sweeps.npz"))
    g = grid_2000()
    x, pi = start_point(g, pi_scale=20.0, seed=2)
    dg = _dev()(g)
    xi = dg.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pi)
    dg.qp_build(xi, float(ref["delta"]), 0)
    dg.admm_init(*dg.rho_scalar(float(ref["rho"])))
    G, L, B = g.n_gen, g.n_line, g.n_bus
    sample = ref["lines"]
    done = 0
    for k in ref["sweeps"]:
        res = dg.admm_solve(int(k) - done, 0.0, 0.0, sweep_mode=_abi.SWEEP_GRAPH)
        done = int(k)
        st = {n: v.cpu().numpy() for n, v in dg.admm_state().items()}
        got = {"xl": st["xl"].reshape(8, L).T[sample], "lam_l": st["lam_l"].reshape(8, L).T[sample],
               "xbar_f": st["xbar_f"].reshape(4, L).T[sample], "xg": st["xg"].reshape(2, G).T,
               "lam_g": st["lam_g"].reshape(2, G).T, "xbar_g": st["xbar_g"].reshape(2, G).T, "dw": st["dw"],
               "dth": st["dth"], "nu": st["nu"].reshape(2, B).T}
        for name, a in got.items():
            e = rel_err_cols(a, ref[f"{name}_{k}"])
            assert e <= TOL, f"sweep {k} {name}: {e:.3e}"
        r_ref, s_ref = ref["rs"][k - 1]
        assert abs(res["r"] - r_ref) <= 1e-7 * r_ref and abs(res["s"] - s_ref) <= 1e-7 * s_ref


def test_batch_with_large_scenarios_matches_solo_runs_and_oracle():
    """A batch of the 300-bus grid and two 10,000-bus scenarios (27,400
    lines, whose bus phase runs item blocks of several scenarios in one
    launch) in the bench's graph mode:
    the large scenarios reproduce their solo runs bit for bit and the
    300-bus scenario matches the oracle.  A grid below 16,384 lines alone
    runs the line phase's wave search, the batch runs one full solve per
    thread: the same minimisers, found on different paths, so the large
    scenarios match their solo runs to rounding (1e-10 per column), not
    bit for bit."""
    from paper_2310_13143_amd import _abi
    from synth.grids import grid_300, grid_10000, perturb_loads
    print("[gpu] batch 300 + 2 x 10000", flush=True)
    grids = [perturb_loads(grid_300(), 64000), perturb_loads(grid_10000(), 64002), perturb_loads(grid_10000(), 64005)]
    pts = [start_point(g, pi_scale=20.0, seed=k) for k, g in enumerate(grids)]
    DeviceGrid = _dev()
    nsw = 150
    dg = DeviceGrid(grids)
    assert dg.n_line > 16384
    cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
    xb = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), np.concatenate([p[1] for p in pts]))
    dg.qp_build(xb, 0.05)
    dg.admm_init(*dg.rho_scalar(2e4))
    dg.admm_solve(nsw, 0.0, 0.0, sweep_mode=_abi.SWEEP_GRAPH, block_size=64)
    res = dg.admm_results()
    st = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    for k in (1, 2):
        x, pik = pts[k]
        solo = DeviceGrid(grids[k])
        xs = solo.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pik)
        solo.qp_build(xs, 0.05)
        solo.admm_init(*solo.rho_scalar(2e4))
        solo.admm_solve(nsw, 0.0, 0.0, sweep_mode=_abi.SWEEP_GRAPH, block_size=64)
        ss = {k2: v.cpu().numpy() for k2, v in solo.admm_state().items()}
        part = _slice_state(st, dg, k, dg.n_gen, dg.n_line, dg.n_bus)
        for name, a in part.items():
            b = ss[name].reshape(a.shape) if a.ndim == 2 else ss[name]
            assert rel_err_cols(a.T if a.ndim == 2 else a, b.T if b.ndim == 2 else b) <= 1e-10, (k, name)
        assert res[k]["sweeps"] == nsw
    g, (x, pik) = grids[0], pts[0]
    Q = qpm.build_qp(g, x, pik, 0.05)
    ref = admm.solve(g, Q, admm.Rho.scalar(g, 2e4), nsw, 0.0, 0.0)
    part = _slice_state(st, dg, 0, dg.n_gen, dg.n_line, dg.n_bus)
    assert rel_err_cols(part["xl"].T, ref.state.xl) <= TOL and rel_err_cols(part["lam_l"].T, ref.state.lam_l) <= TOL
    assert rel_err_cols(part["dw"], ref.state.dw) <= TOL and rel_err_cols(part["nu"].T, ref.state.nu) <= TOL
    assert rel_err_cols(part["xg"].T, ref.state.xg) <= TOL and rel_err_cols(part["lam_g"].T, ref.state.lam_g) <= TOL


def test_infinity_norms_on_a_large_batch():
    """The infinity-norm residuals of the batch kernels used above 16,384
    lines (four item blocks per bus-phase workgroup): the norm leaves the
    iterates unchanged (bit for bit against the Euclidean run), each
    scenario's reported primal norm is the largest coupling residual
    |x_c - xbar_c| recomputed from the exported state (a maximum does not
    depend on the reduction order), and both norms sit between the
    Euclidean ones divided by sqrt(couplings) and the Euclidean ones."""
    from paper_2310_13143_amd import _abi
    from synth.grids import grid_300, grid_10000, perturb_loads
    print("[gpu] infinity norms, batch 300 + 2 x 10000", flush=True)
    grids = [perturb_loads(grid_300(), 64000), perturb_loads(grid_10000(), 64002), perturb_loads(grid_10000(), 64005)]
    pts = [start_point(g, pi_scale=20.0, seed=k) for k, g in enumerate(grids)]
    dg = _dev()(grids)
    assert dg.n_line > 16384
    cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
    xb = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), np.concatenate([p[1] for p in pts]))
    dg.qp_build(xb, 0.05)
    nsw = 40
    runs = []
    for inf in (False, True):
        dg.admm_init(*dg.rho_scalar(2e4))
        dg.admm_solve(nsw, 0.0, 0.0, sweep_mode=_abi.SWEEP_GRAPH, block_size=64, norm_inf=inf)
        runs.append((dg.admm_results(), {k: v.cpu().numpy() for k, v in dg.admm_state().items()}))
    (res2, st2), (resi, sti) = runs
    for name in ("xl", "lam_l", "xbar_f", "xg", "xbar_g", "lam_g", "dw", "dth", "nu"):
        assert np.array_equal(st2[name], sti[name]), name
    G, L, B = dg.n_gen, dg.n_line, dg.n_bus
    bo, lo, go = dg.offsets["bus"], dg.offsets["line"], dg.offsets["gen"]
    for k, g in enumerate(grids):
        xl = sti["xl"].reshape(8, L)[:, lo[k]:lo[k + 1]]
        xbf = sti["xbar_f"].reshape(4, L)[:, lo[k]:lo[k + 1]]
        dw, dth = sti["dw"][bo[k]:bo[k + 1]], sti["dth"][bo[k]:bo[k + 1]]
        f, t = np.asarray(g.f), np.asarray(g.t)
        r = np.concatenate([
            (sti["xg"].reshape(2, G) - sti["xbar_g"].reshape(2, G))[:, go[k]:go[k + 1]].ravel(),
            (xl[:4] - xbf).ravel(),
            xl[4] - dw[f], xl[5] - dth[f], xl[6] - dw[t], xl[7] - dth[t]])
        n_c = r.size
        assert n_c == 2 * g.n_gen + 8 * g.n_line
        r_max = np.abs(r).max()
        assert resi[k]["sweeps"] == nsw and res2[k]["sweeps"] == nsw
        assert abs(resi[k]["r"] - r_max) <= 1e-14 * r_max, (k, resi[k]["r"], r_max)
        for q in ("r", "s"):
            e, i = res2[k][q], resi[k][q]
            assert 0.0 < i <= e * (1 + 1e-12) and e <= np.sqrt(n_c) * i * (1 + 1e-12), (k, q, e, i)


def test_traced_sweeps_on_a_large_batch():
    """Traced sweeps (the per-coupling sums of |r_c| and |s_c| that the
    learned warm start trains on) in the bus kernel used above 16,384 lines:
    the 300-bus scenario of the batch against the oracle's sums, the two
    10,000-bus scenarios against their solo runs (one-block bus-phase
    workgroups, the line phase's wave search: the same minimisers to
    rounding, hence 1e-9 per column)."""
    from paper_2310_13143_amd import _abi
    from oracle import mlp
    from synth.grids import grid_300, grid_10000, perturb_loads
    print("[gpu] traced sweeps, batch 300 + 2 x 10000", flush=True)
    grids = [perturb_loads(grid_300(), 64000), perturb_loads(grid_10000(), 64002), perturb_loads(grid_10000(), 64005)]
    pts = [start_point(g, pi_scale=20.0, seed=k) for k, g in enumerate(grids)]
    DeviceGrid = _dev()
    nsw = 30
    dg = DeviceGrid(grids)
    assert dg.n_line > 16384
    cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
    xb = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), np.concatenate([p[1] for p in pts]))
    dg.qp_build(xb, 0.05)
    dg.admm_init(*dg.rho_scalar(2e4))
    dg.admm_solve(nsw, 0.0, 0.0, sweep_mode=_abi.SWEEP_LAUNCHES, block_size=64, trace=True)
    st = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    G, L = dg.n_gen, dg.n_line
    lo, go = dg.offsets["line"], dg.offsets["gen"]

    def sums(state, k, G, L, lo, go):
        return [state["sum_r_g"].reshape(2, G)[:, go[k]:go[k + 1]].T, state["sum_s_g"].reshape(2, G)[:, go[k]:go[k + 1]].T,
                state["sum_r_l"].reshape(8, L)[:, lo[k]:lo[k + 1]].T, state["sum_s_l"].reshape(8, L)[:, lo[k]:lo[k + 1]].T]

    g, (x, pik) = grids[0], pts[0]
    rho = admm.Rho.scalar(g, 2e4)
    start = admm.warm_state(g, np.zeros((g.n_gen, 2)), np.zeros((g.n_line, 8)))
    ref = admm.solve(g, qpm.build_qp(g, x, pik, 0.05), rho, nsw, 0.0, 0.0, state=start, record_states=True)
    for a, b in zip(sums(st, 0, G, L, lo, go), mlp.trace_sums(g, rho, start, ref.history)):
        assert rel_err_cols(a, b) <= 1e-8
    for k in (1, 2):
        x, pik = pts[k]
        solo = DeviceGrid(grids[k])
        xs = solo.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pik)
        solo.qp_build(xs, 0.05)
        solo.admm_init(*solo.rho_scalar(2e4))
        solo.admm_solve(nsw, 0.0, 0.0, sweep_mode=_abi.SWEEP_LAUNCHES, block_size=64, trace=True)
        ss = {k2: v.cpu().numpy() for k2, v in solo.admm_state().items()}
        Gs, Ls = solo.n_gen, solo.n_line
        for a, b in zip(sums(st, k, G, L, lo, go), sums(ss, 0, Gs, Ls, [0, Ls], [0, Gs])):
            assert rel_err_cols(a, b) <= 1e-9, k


def test_step_decision_and_residuals_on_a_large_grid():
    """The step decision's merit sums and the residual report on the
    2,000-bus grid, whose reductions run several blocks per scenario,
    against the oracle's merit, model and residual functions at the device's
    own iterate and trial step: ared = phi(x) - phi(x + d), pred = q(0) -
    q(d) on the QP built at x, the step's infinity norm, and the maxima of
    the constraint violations at the new iterate."""
    from paper_2310_13143_amd import _abi
    print("[gpu] step decision and residual report, rgg2000", flush=True)
    g = grid_2000()
    x0, _ = start_point(g)
    dg = _dev()(g)
    assert g.n_line > 2048
    x = dg.iterate(x0.pg, x0.qg, x0.w, x0.th, x0.wR, x0.wI, None)
    rho_g, rho_l = dg.rho_scalar(2e4)
    d = dg.empty_iterate()
    mu = 1e5
    out = dg.sqp_step(x, 0.05, rho_g, rho_l, mu=mu, max_sweeps=200, eps=0.0, d=d, sweep_mode=_abi.SWEEP_GRAPH)
    host = lambda it: acopf.Iterate(*(it[k].cpu().numpy() for k in ("pg", "qg", "w", "th", "wR", "wI")))
    dh = host(d)
    Q = qpm.build_qp(g, x0, np.zeros((g.n_line, 4)), 0.05)
    m0, m1 = acopf.merit(g, x0, mu), acopf.merit(g, x0.plus(dh), mu)
    assert abs(out["ared"] - (m0 - m1)) <= 1e-11 * (abs(m0) + abs(m1)), (out["ared"], m0 - m1)
    pred = sqp.predicted_reduction(g, x0, Q, dh, mu)
    assert abs(out["pred"] - pred) <= 1e-11 * (abs(m0) + abs(pred)), (out["pred"], pred)
    assert out["step_inf"] == pytest.approx(sqp.step_norm(dh), rel=1e-15)
    xn = host(x)
    np.testing.assert_array_equal(xn.pg, (x0.plus(dh) if out["accepted"] else x0).pg)
    res = dg.residuals(x)
    ref = acopf.primal_infeasibility(g, xn)
    for k in ("primal", "balance", "c11", "c12", "limit", "bounds"):
        assert abs(res[k] - ref[k]) <= 1e-10 * (1.0 + ref[k]), (k, res[k], ref[k])


@pytest.mark.parametrize("rho,mu", [(2e4, 10.0), (2e2, 2.0)])
def test_residual_balancing_matches_oracle(rho, mu):
    """Residual balancing of the penalties every 64 sweeps (graph sweeps)
    against the oracle's: the same factors at the same sweeps, so the same
    iterates and final penalties."""
    from paper_2310_13143_amd import _abi
    print(f"[gpu] residual balancing ring14 rho={rho:g}", flush=True)
    g = grid_14()
    x, pi = start_point(g, pi_scale=20.0, seed=3)
    Q = qpm.build_qp(g, x, pi, 0.05, "psd")
    bal = admm.Balance(mu=mu, tau=2.0, every=64)
    nsw = 640
    ref = admm.solve(g, Q, admm.Rho.scalar(g, rho), nsw, 0.0, 0.0, balance=bal)
    assert not np.allclose(ref.rho.l, rho)  # the penalties moved
    _, _, res, st = _run_gpu(g, x, pi, 0.05, admm.Rho.scalar(g, rho), None, None, nsw,
                             mode=_abi.SWEEP_GRAPH, balance=(bal.every, bal.mu, bal.tau))
    assert res["sweeps"] == nsw
    np.testing.assert_array_equal(st["rho_l"].reshape(8, -1).T, ref.rho.l)
    np.testing.assert_array_equal(st["rho_g"].reshape(2, -1).T, ref.rho.g)
    _compare_state(st, ref.state)


def test_stop_rule_and_limit_match_direct_solve():
    """With eps > 0 the GPU stops at the oracle's sweep (ties within 1
    sweep allowed) and its limit solves the QP: objective within 1e-6
    relative and violation within 1e-5 of the direct interior-point solve."""
    print("[gpu] stop rule tiny", flush=True)
    g = tiny_grid(seed=8, n_bus=5, n_line=6, n_gen=2, shunt_scale=0.03)
    x, pi = start_point(g, pi_scale=30.0, seed=0)
    Q = qpm.build_qp(g, x, pi, 0.2, "psd")
    rho = admm.Rho.scalar(g, 1e3)
    ref = admm.solve(g, Q, rho, 40000, 1e-9, 1e-9)
    ds = direct.solve(g, Q)
    for mode in (0, 1):
        dg, xi, res, st = _run_gpu(g, x, pi, 0.2, rho, None, None, 40000, mode=mode, eps=1e-9)
        assert res["converged"] and abs(res["sweeps"] - ref.sweeps) <= 1
        d = {k: v.cpu().numpy() for k, v in dg.step(xi).items()}
        z = np.stack([d["w"][g.f], d["th"][g.f], d["w"][g.t], d["th"][g.t]], 1)
        obj = qpm.qp_objective(Q, d["pg"], z)
        assert abs(obj - ds.objective) <= 1e-6 * abs(ds.objective)
        assert direct.max_violation(g, Q, np.concatenate([d["pg"], d["qg"], d["w"], d["th"]])) <= 1e-5


def test_determinism_bitwise():
    print("[gpu] determinism ring14", flush=True)
    g = grid_14()
    x, pi = start_point(g, pi_scale=10.0, seed=1)
    rho = admm.Rho.scalar(g, 2e4)
    _, _, r1, s1 = _run_gpu(g, x, pi, 0.1, rho, None, None, 200)
    _, _, r2, s2 = _run_gpu(g, x, pi, 0.1, rho, None, None, 200)
    for k in s1:
        assert np.array_equal(s1[k], s2[k]), k
    assert r1["r"] == r2["r"] and r1["s"] == r2["s"]


def test_rgg2000_sweeps_match_oracle():
    print("[gpu] rgg2000 20 sweeps", flush=True)
    g = grid_2000()
    x, pi = start_point(g, pi_scale=20.0, seed=2)
    rho = admm.Rho.scalar(g, 2e4)
    Q = qpm.build_qp(g, x, pi, 0.05, "psd")
    ref = admm.solve(g, Q, rho, 20, 0.0, 0.0)
    for mode in (0, 1):
        _, _, res, st = _run_gpu(g, x, pi, 0.05, rho, None, None, 20, mode=mode)
        _compare_state(st, ref.state)


def test_relaxed_lines_match_oracle():
    """At a trust radius too small for some lines to reach their linearised
    limits, the build relaxes those lines' rows like the oracle (to their
    least-squares violation) and every line subproblem has a solution.  The
    relaxed lines' subproblems are ill-conditioned (their rows bind along
    directions in which their coefficients are tiny, with multipliers up to
    about 1e8), so FP64 solvers with KKT tolerances of 1e-12 to 1e-10 give
    points up to 1e-4 of the box width apart whose objectives agree to a few
    parts in 1e8; the state is compared per column to 1e-4, the bus values
    to 1e-6."""
    print("[gpu] rgg2000 relaxed lines", flush=True)
    g = grid_2000()
    x, pi = start_point(g, pi_scale=20.0, seed=2)
    rho = admm.Rho.scalar(g, 2e4)
    delta = 0.00625
    Q = qpm.build_qp(g, x, pi, delta, "psd")
    n_relaxed = int((Q.line.relax > 0).any(1).sum())
    assert n_relaxed > 10
    ref = admm.solve(g, Q, rho, 6, 0.0, 0.0)
    assert ref.infeasible_lines == 0
    _, _, res, st = _run_gpu(g, x, pi, delta, rho, None, None, 6, mode=1)
    assert res["relaxed_lines"] == n_relaxed and res["infeasible_lines"] == 0
    _compare_state(st, ref.state, tol=1e-4)
    assert rel_err_cols(st["dw"], ref.state.dw) <= 1e-6
    assert rel_err_cols(st["nu"].reshape(2, -1).T, ref.state.nu) <= 1e-6


def test_rgg70000_sampled_line_and_bus_updates():
    """At 70,000 buses (88,000 lines, the bench workload, in the bench's graph
    sweep mode) the oracle checks one sweep of sampled lines and all buses
    from the GPU's own previous state."""
    from paper_2310_13143_amd import _abi
    print("[gpu] rgg70000 sampled", flush=True)
    g = grid_70000()
    x, pi = start_point(g, pi_scale=20.0, seed=2)
    rho = admm.Rho.scalar(g, 2e4)
    Q = qpm.build_qp(g, x, pi, 0.05, "psd")
    dg = _dev()(g)
    xi = dg.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pi)
    dg.qp_build(xi, 0.05, 0)
    dg.admm_init(*dg.rho_scalar(2e4))
    dg.admm_solve(7, 0.0, 0.0, sweep_mode=_abi.SWEEP_GRAPH)
    s0 = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    dg.admm_solve(1, 0.0, 0.0, sweep_mode=_abi.SWEEP_GRAPH)   # continues from the state: one more sweep
    s1 = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    G, L, B = g.n_gen, g.n_line, g.n_bus
    st = admm.cold_state(g)
    st.xg, st.xbar_g, st.lam_g = (s0[k].reshape(2, G).T.copy() for k in ("xg", "xbar_g", "lam_g"))
    st.xl, st.lam_l = (s0[k].reshape(8, L).T.copy() for k in ("xl", "lam_l"))
    st.xbar_f = s0["xbar_f"].reshape(4, L).T.copy()
    st.dw, st.dth = s0["dw"].copy(), s0["dth"].copy()
    # sampled line updates
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(L, 2000, replace=False))
    Qm = admm.line_matrices(Q, rho)
    sub = _subset_lines(Q, sample)
    xl_ref, _, _ = admm.line_update(_subgrid(g, sample), sub, st_sub(st, g, sample), _subrho(rho, sample), Qm[sample])
    assert rel_err(s1["xl"].reshape(8, L).T[sample], xl_ref) <= TOL
    # all generators and buses from the GPU's line values of this sweep
    xg = admm.gen_update(Q, st, rho)
    assert rel_err(s1["xg"].reshape(2, G).T, xg) <= TOL
    xbar_g, xbar_f, dw, dth, nu = admm.bus_update(g, Q, xg, s1["xl"].reshape(8, L).T, st, rho)
    assert rel_err(s1["dw"], dw) <= TOL and rel_err(s1["dth"], dth) <= TOL
    assert rel_err(s1["xbar_f"].reshape(4, L).T, xbar_f) <= TOL
    assert rel_err(s1["nu"].reshape(2, B).T, nu) <= TOL


def _subset_lines(Q, idx):
    import copy
    L = copy.copy(Q.line)
    for f in ("aR", "bR", "aI", "bI", "H", "M", "q", "F", "f0", "lo", "hi", "G", "h", "pk", "c0", "relax"):
        setattr(L, f, getattr(Q.line, f)[idx])
    out = copy.copy(Q)
    out.line = L
    return out


def _subgrid(g, idx):
    import copy
    s = copy.copy(g)
    s.f, s.t = g.f[idx], g.t[idx]
    return s


def st_sub(st, g, idx):
    import copy
    s = copy.copy(st)
    s.lam_l, s.xbar_f = st.lam_l[idx], st.xbar_f[idx]
    return s


def _subrho(rho, idx):
    return admm.Rho(rho.g, rho.l[idx])


def test_error_paths():
    """Invalid arguments and non-finite data are reported as errors."""
    from paper_2310_13143_amd import AcopfError
    print("[gpu] error paths", flush=True)
    g = grid_14()
    x, pi = start_point(g)
    DeviceGrid = _dev()
    dg = DeviceGrid(g)
    w = x.w.copy()
    w[3] = np.nan
    xi = dg.iterate(x.pg, x.qg, w, x.th, x.wR, x.wI, pi)
    dg.qp_build(xi, 0.1)
    dg.admm_init(*dg.rho_scalar(2e4))
    with pytest.raises(AcopfError) as e:
        dg.admm_solve(5)
    assert e.value.code == -4
    with pytest.raises(AcopfError):
        dg.qp_build(xi, -1.0)
    bad = grid_14()
    bad.f = bad.f.copy()
    bad.f[0] = bad.n_bus + 3
    with pytest.raises(AcopfError) as e:
        DeviceGrid(bad)
    assert e.value.code == -1


@pytest.mark.parametrize("pi_rule", [0, 1])
def test_sqp_iterations_match_oracle(pi_rule):
    """Trust-region SQP (Algorithm 1) on the device against the oracle's SQP,
    iteration by iteration, with a fixed sweep budget per QP (no early stop,
    so both sides run the same ADMM iterations): acceptance decisions, trust
    radii, iterates, multipliers and the residual report.  pi_rule 1 (keep
    pi unless the solve met a stop test) keeps pi at zero here."""
    print(f"[gpu] sqp ring14 pi_rule={pi_rule}", flush=True)
    g = grid_14()
    x0, _ = start_point(g)
    params = sqp.SqpParams(max_iter=6, max_sweeps=300, eps_pri=0.0, eps_dual=0.0, delta0=0.05, tol_step=0.0,
                           tol_primal=0.0, tol_dual=0.0, pi_if_converged=bool(pi_rule))
    ref = sqp.solve(g, params, x0=x0)
    dg = _dev()(g)
    x = dg.iterate(x0.pg, x0.qg, x0.w, x0.th, x0.wR, x0.wI, None)
    rho_g, rho_l = dg.rho_scalar(params.rho)
    delta = params.delta0
    for k, rec in enumerate(ref.records):
        out = dg.sqp_step(x, delta, rho_g, rho_l, mu=params.mu_merit, delta_max=params.delta_max,
                          warm_start=k > 0, max_sweeps=params.max_sweeps, eps=0.0, pi_update=pi_rule)
        assert out["admm_sweeps"] == params.max_sweeps
        assert bool(out["accepted"]) == rec.accepted, k
        scale = 1.0 + abs(rec.pred)
        assert abs(out["ared"] - rec.ared) <= 1e-6 * (1.0 + abs(rec.ared)), (k, out["ared"], rec.ared)
        assert abs(out["pred"] - rec.pred) <= 1e-6 * scale, (k, out["pred"], rec.pred)
        assert abs(out["delta"] - rec.delta) <= 1e-12 * rec.delta, k
        delta = out["delta"]
        res = dg.residuals(x)
        assert abs(res["primal"] - rec.primal) <= 1e-6 * (1.0 + rec.primal), (k, res, rec.primal)
        assert abs(res["dual"] - rec.dual) <= 1e-6 * (1.0 + rec.dual), (k, res, rec.dual)
    xf = {k: v.cpu().numpy() for k, v in x.items()}
    for name in ("pg", "qg", "w", "th", "wR", "wI"):
        assert rel_err(xf[name], getattr(ref.x, name)) <= TOL, name
    if pi_rule:
        assert np.all(ref.pi == 0.0) and np.all(xf["pi"] == 0.0)
    else:
        assert rel_err(xf["pi"].reshape(4, -1).T, ref.pi) <= 1e-7


def test_sqp_with_second_order_correction_matches_oracle():
    """Algorithm 1 with the second-order correction of rejected steps on the
    device against the oracle's SQP with the same correction, iteration by
    iteration (fixed sweep budget, no early stop): decisions (corrected
    steps taken where the oracle takes them), merit reductions, radii,
    residuals, final iterate and multipliers."""
    print("[gpu] sqp ring14 with second-order correction", flush=True)
    g = grid_14()
    x0, _ = start_point(g)
    params = sqp.SqpParams(max_iter=6, max_sweeps=300, eps_pri=0.0, eps_dual=0.0, delta0=0.05, tol_step=0.0,
                           tol_primal=0.0, tol_dual=0.0, soc=True)
    ref = sqp.solve(g, params, x0=x0)
    assert sum(r.soc for r in ref.records) >= 2
    dg = _dev()(g)
    x = dg.iterate(x0.pg, x0.qg, x0.w, x0.th, x0.wR, x0.wI, None)
    rho_g, rho_l = dg.rho_scalar(params.rho)
    delta = params.delta0
    for k, rec in enumerate(ref.records):
        out = dg.sqp_step(x, delta, rho_g, rho_l, mu=params.mu_merit, delta_max=params.delta_max,
                          warm_start=k > 0, max_sweeps=params.max_sweeps, eps=0.0, soc=True)
        assert bool(out["accepted"]) == rec.accepted, k
        assert (out["accepted"] and out["soc_sweeps"] > 0) == rec.soc, k
        assert abs(out["ared"] - rec.ared) <= 1e-6 * (1.0 + abs(rec.ared)), (k, out["ared"], rec.ared)
        assert abs(out["pred"] - rec.pred) <= 1e-6 * (1.0 + abs(rec.pred)), (k, out["pred"], rec.pred)
        assert abs(out["delta"] - rec.delta) <= 1e-12 * rec.delta, k
        delta = out["delta"]
        res = dg.residuals(x)
        assert abs(res["primal"] - rec.primal) <= 1e-6 * (1.0 + rec.primal), (k, res, rec.primal)
        assert abs(res["dual"] - rec.dual) <= 1e-6 * (1.0 + rec.dual), (k, res, rec.dual)
    xf = {k: v.cpu().numpy() for k, v in x.items()}
    for name in ("pg", "qg", "w", "th", "wR", "wI"):
        assert rel_err(xf[name], getattr(ref.x, name)) <= TOL, name
    assert rel_err(xf["pi"].reshape(4, -1).T, ref.pi) <= 1e-7


def _batch_cases():
    from synth.grids import perturb_loads
    base = grid_14()
    return [perturb_loads(base, 64000 + k) for k in range(3)] + \
        [tiny_grid(seed=21, n_bus=7, n_line=10, n_gen=3, shunt_scale=0.04)]


def _slice_state(st, dg, k, G, L, B):
    bo, lo, go = dg.offsets["bus"], dg.offsets["line"], dg.offsets["gen"]
    sl = lambda a, n, o, f: a.reshape(f, n)[:, o[k]:o[k + 1]]
    return {"xl": sl(st["xl"], L, lo, 8), "lam_l": sl(st["lam_l"], L, lo, 8), "xbar_f": sl(st["xbar_f"], L, lo, 4),
            "xg": sl(st["xg"], G, go, 2), "lam_g": sl(st["lam_g"], G, go, 2), "dw": st["dw"][bo[k]:bo[k + 1]],
            "dth": st["dth"][bo[k]:bo[k + 1]], "nu": sl(st["nu"], B, bo, 2)}


@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_batch_matches_solo_runs_and_oracle(eps):
    """Scenarios solved together in one batch (block tables per scenario,
    per-scenario stop) reproduce their solo GPU runs bit for bit and the
    oracle within 1e-8; with eps > 0 each scenario stops at its own sweep."""
    print(f"[gpu] batch eps={eps}", flush=True)
    grids = _batch_cases()
    DeviceGrid = _dev()
    pts = [start_point(g, pi_scale=20.0, seed=k) for k, g in enumerate(grids)]
    nsw = 400
    dg = DeviceGrid(grids)
    cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
    pi = np.concatenate([p[1] for p in pts])
    xb = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), pi)
    dg.qp_build(xb, 0.05)
    dg.admm_init(*dg.rho_scalar(2e4))
    dg.admm_solve(nsw, eps, eps, sweep_mode=1, block_size=64)
    res = dg.admm_results()
    st = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    for k, g in enumerate(grids):
        x, pik = pts[k]
        solo = DeviceGrid(g)
        xs = solo.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pik)
        solo.qp_build(xs, 0.05)
        solo.admm_init(*solo.rho_scalar(2e4))
        rs = solo.admm_solve(nsw, eps, eps, sweep_mode=1, block_size=64)
        ss = {k2: v.cpu().numpy() for k2, v in solo.admm_state().items()}
        part = _slice_state(st, dg, k, dg.n_gen, dg.n_line, dg.n_bus)
        for name, a in part.items():
            b = ss[name].reshape(a.shape) if a.ndim == 2 else ss[name]
            assert np.array_equal(a, b), (k, name)
        assert res[k]["sweeps"] == rs["sweeps"] and res[k]["r"] == rs["r"] and res[k]["s"] == rs["s"]
        Q = qpm.build_qp(g, x, pik, 0.05)
        ref = admm.solve(g, Q, admm.Rho.scalar(g, 2e4), nsw, eps, eps)
        assert abs(res[k]["sweeps"] - ref.sweeps) <= 1
        if res[k]["sweeps"] == ref.sweeps:
            G, L = g.n_gen, g.n_line
            assert rel_err(part["xl"].T, ref.state.xl) <= TOL and rel_err(part["dw"], ref.state.dw) <= TOL
            assert rel_err(part["lam_g"].T, ref.state.lam_g) <= TOL


def test_batch_isolates_a_failed_scenario():
    """A scenario whose QP cannot be built (non-finite iterate) is reported
    per scenario and not solved; the others match their solo runs bit for
    bit, in the ADMM solve and in the SQP step (the failed one is rejected
    with its radius halved)."""
    print("[gpu] batch with a failed scenario", flush=True)
    from paper_2310_13143_amd import _abi
    grids = _batch_cases()
    DeviceGrid = _dev()
    pts = [start_point(g, pi_scale=20.0, seed=k) for k, g in enumerate(grids)]
    bad = 1
    pts[bad][0].w = pts[bad][0].w.copy()
    pts[bad][0].w[2] = np.nan
    dg = DeviceGrid(grids)
    cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
    pi = np.concatenate([p[1] for p in pts])
    xb = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), pi)
    dg.qp_build(xb, 0.05)
    dg.admm_init(*dg.rho_scalar(2e4))
    dg.admm_solve(100, 1e-6, 1e-6, sweep_mode=1, block_size=64, sync=False)
    res = dg.admm_results()  # a batch reports failures per scenario, no exception
    assert res[bad]["status"] == -4 and res[bad]["outcome"] == _abi.ADMM_FAILED and res[bad]["sweeps"] == 0
    st = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    for k, g in enumerate(grids):
        if k == bad:
            continue
        assert res[k]["status"] == 0 and res[k]["outcome"] != _abi.ADMM_FAILED
        x, pik = pts[k]
        solo = DeviceGrid(g)
        xs = solo.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pik)
        solo.qp_build(xs, 0.05)
        solo.admm_init(*solo.rho_scalar(2e4))
        rs = solo.admm_solve(100, 1e-6, 1e-6, sweep_mode=1, block_size=64)
        ss = {k2: v.cpu().numpy() for k2, v in solo.admm_state().items()}
        for name, a in _slice_state(st, dg, k, dg.n_gen, dg.n_line, dg.n_bus).items():
            b = ss[name].reshape(a.shape) if a.ndim == 2 else ss[name]
            assert np.array_equal(a, b), (k, name)
        assert res[k]["sweeps"] == rs["sweeps"]
    # SQP step of the batch: the failed scenario is rejected, radius halved
    dg.set_delta(0.05)
    rho_g, rho_l = dg.rho_scalar(2e4)
    outs = dg.sqp_step_batch(xb, rho_g, rho_l, max_sweeps=100, eps=0.0, block_size=64)
    assert outs[bad]["status"] == -4 and outs[bad]["accepted"] == 0 and outs[bad]["delta"] == 0.025
    assert all(outs[k]["status"] == 0 for k in range(len(grids)) if k != bad)
    # a single grid still raises
    from paper_2310_13143_amd import AcopfError
    x, pik = pts[bad]
    solo = DeviceGrid(grids[bad])
    xs = solo.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pik)
    solo.qp_build(xs, 0.05)
    solo.admm_init(*solo.rho_scalar(2e4))
    with pytest.raises(AcopfError) as e:
        solo.admm_solve(10, sweep_mode=1, block_size=64)
    assert e.value.code == -4


@pytest.mark.parametrize("soc", [False, True])
def test_batch_sqp_matches_oracle_per_scenario(soc):
    """Batched SQP iterations: every scenario follows its own oracle SQP (with
    the second-order correction: scenarios that take a correction and
    scenarios that do not share the pass)."""
    print(f"[gpu] batch sqp soc={soc}", flush=True)
    grids = _batch_cases()[:3]
    params = sqp.SqpParams(max_iter=4, max_sweeps=200, eps_pri=0.0, eps_dual=0.0, delta0=0.05, tol_step=0.0,
                           tol_primal=0.0, tol_dual=0.0, soc=soc)
    refs, pts = [], []
    for g in grids:
        x0, _ = start_point(g)
        pts.append(x0)
        refs.append(sqp.solve(g, params, x0=x0))
    dg = _dev()(grids)
    cat = lambda name: np.concatenate([getattr(p, name) for p in pts])
    x = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)
    dg.set_delta(params.delta0)
    rho_g, rho_l = dg.rho_scalar(params.rho)
    for it in range(params.max_iter):
        outs = dg.sqp_step_batch(x, rho_g, rho_l, mu=params.mu_merit, warm_start=it > 0,
                                 max_sweeps=params.max_sweeps, eps=0.0, block_size=64, soc=soc)
        for k, ref in enumerate(refs):
            rec = ref.records[it]
            assert bool(outs[k]["accepted"]) == rec.accepted, (k, it)
            assert (outs[k]["accepted"] and outs[k]["soc_sweeps"] > 0) == rec.soc, (k, it)
            assert abs(outs[k]["delta"] - rec.delta) <= 1e-12 * rec.delta, (k, it)
    xf = {k: v.cpu().numpy() for k, v in x.items()}
    bo = dg.offsets["bus"]
    for k, ref in enumerate(refs):
        assert rel_err(xf["w"][bo[k]:bo[k + 1]], ref.x.w) <= TOL
    if soc:
        assert any(r.soc for ref in refs for r in ref.records)
        assert any(not r.soc and not r.accepted for ref in refs for r in ref.records) or \
            any(r.accepted and not r.soc for ref in refs for r in ref.records)


@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_graph_sweeps_match_launches(eps):
    """Sweeps replayed from cached HIP graphs give bit for bit the state,
    sweep count and residuals of plain launches (single grid and batch, two
    solves each so that the second replays a cached graph)."""
    print(f"[gpu] graph sweep mode eps={eps}", flush=True)
    from paper_2310_13143_amd import _abi
    DeviceGrid = _dev()
    for grids in ([grid_14()], _batch_cases()):
        pts = [start_point(g, pi_scale=20.0, seed=k) for k, g in enumerate(grids)]
        cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
        pi = np.concatenate([p[1] for p in pts])
        out = {}
        for mode in (_abi.SWEEP_LAUNCHES, _abi.SWEEP_GRAPH):
            dg = DeviceGrid(grids if len(grids) > 1 else grids[0])
            xb = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), pi)
            dg.qp_build(xb, 0.05)
            runs = []
            for rep in range(2):
                dg.admm_init(*dg.rho_scalar(2e4))
                dg.admm_solve(150, eps, eps, sweep_mode=mode, block_size=64, sync=False)
                res = dg.admm_results()
                st = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
                runs.append((res, st))
            out[mode] = runs
        for (ra, sa), (rb, sb) in zip(out[_abi.SWEEP_LAUNCHES], out[_abi.SWEEP_GRAPH]):
            for k in range(len(grids)):
                assert ra[k]["sweeps"] == rb[k]["sweeps"] and ra[k]["r"] == rb[k]["r"] and ra[k]["s"] == rb[k]["s"]
            for name in sa:
                assert np.array_equal(sa[name], sb[name]), name


def test_captured_sqp_iteration_replays_like_eager():
    """One batched SQP iteration (fixed sweep count, no host results)
    recorded under stream capture and replayed three times, with eager work
    between the replays, gives bit for bit the iterates of three eager
    iterations after every replay."""
    print("[gpu] captured batched SQP iteration", flush=True)
    import torch
    from paper_2310_13143_amd import _abi
    DeviceGrid = _dev()
    grids = _batch_cases()
    pts = [start_point(g) for g in grids]
    cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
    kw = dict(mu=1e5, warm_start=_abi.START_PREVIOUS, max_sweeps=120, eps=0.0, block_size=64, sync=False)

    def fresh():
        dg = DeviceGrid(grids)
        x = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)
        dg.set_delta(0.05)
        rho_g, rho_l = (t.cuda() for t in dg.rho_scalar(2e4))
        return dg, x, rho_g, rho_l, dg.empty_iterate()

    dg_e, x_e, rg_e, rl_e, d_e = fresh()
    eager = []
    for it in range(3):
        dg_e.sqp_step_batch(x_e, rg_e, rl_e, d=d_e, **kw)
        eager.append({k: v.cpu().numpy() for k, v in x_e.items()})
    dg_c, x_c, rg_c, rl_c, d_c = fresh()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        dg_c.sqp_step_batch(x_c, rg_c, rl_c, d=d_c, **kw)
    # capture records without executing: the iterate is still the start point
    assert np.array_equal(x_c["w"].cpu().numpy(), cat("w"))
    for it in range(3):
        graph.replay()
        dg_c.residuals_batch(x_c)  # eager work and a synchronisation between replays
        got = {k: v.cpu().numpy() for k, v in x_c.items()}
        for name in got:
            assert np.array_equal(got[name], eager[it][name]), (it, name)


def test_captured_sqp_loop_with_device_stops_replays_like_eager():
    """A whole batched SQP run (six iterations, ADMM stop test at eps = 1e-4
    and per-scenario SQP stop rule on the device) recorded under stream
    capture: every replay, with eager work and a new start between replays,
    reproduces the eager run's iterates, stop reasons and iteration counts
    bit for bit; stopped scenarios keep their iterate; the oracle's SQP with
    the same stop rule takes the same number of iterations per scenario."""
    print("[gpu] captured SQP loop with device stops", flush=True)
    import torch
    from paper_2310_13143_amd import _abi
    DeviceGrid = _dev()
    grids = _batch_cases()[:3]
    pts = [start_point(g) for g in grids]
    cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
    iters, sweeps = 6, 640
    stop = (1e-4, 1e9, 1e-9, 1e-8)  # primal infeasibility <= 1e-4 (the time-to-1e-4 rule)
    kw = dict(mu=1e5, max_sweeps=sweeps, eps=1e-4, block_size=64, sync=False, stop=stop)

    def fresh():
        dg = DeviceGrid(grids)
        x = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)
        rho_g, rho_l = (t.cuda() for t in dg.rho_scalar(1e3))
        return dg, x, rho_g, rho_l, dg.empty_iterate()

    def run(dg, x, rg, rl, d):
        for it in range(iters):
            dg.sqp_step_batch(x, rg, rl, d=d, warm_start=_abi.START_ZERO if it == 0 else _abi.START_PREVIOUS, **kw)

    dg_e, x_e, rg_e, rl_e, d_e = fresh()
    dg_e.set_delta(0.05)
    run(dg_e, x_e, rg_e, rl_e, d_e)
    eager = {k: v.cpu().numpy() for k, v in x_e.items()}
    out_e = dg_e.sqp_outcomes()
    assert any(o["done"] for o in out_e)
    # the oracle's run with the same stop rule and ADMM settings
    params = sqp.SqpParams(max_iter=iters, rho=1e3, max_sweeps=sweeps, eps_pri=1e-4, eps_dual=1e-4, delta0=0.05,
                           tol_primal=stop[0], tol_dual=stop[1], tol_step=stop[2], delta_min=stop[3])
    k = next(i for i, o in enumerate(out_e) if o["done"])
    ref = sqp.solve(grids[k], params, x0=pts[k][0])
    assert ref.outcome == "CONVERGED" and ref.iterations == out_e[k]["iterations"], (k, ref.outcome)
    assert out_e[k]["reason"] == 1 and out_e[k]["seconds"] > 0.0
    dg_c, x_c, rg_c, rl_c, d_c = fresh()
    x0c = {k: v.clone() for k, v in x_c.items()}
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run(dg_c, x_c, rg_c, rl_c, d_c)
    for rep in range(3):
        for k in x_c:
            x_c[k].copy_(x0c[k])
        dg_c.set_delta(0.05)
        graph.replay()
        dg_c.residuals_batch(x_c)  # eager work and a synchronisation between replays
        got = {k: v.cpu().numpy() for k, v in x_c.items()}
        for name in got:
            assert np.array_equal(got[name], eager[name]), (rep, name)
        out_c = dg_c.sqp_outcomes()
        for a, b in zip(out_c, out_e):
            assert (a["done"], a["reason"], a["iterations"]) == (b["done"], b["reason"], b["iterations"]), rep


LOCAL_CASES = {"convex": (300.0, 2e4), "nonconvex": (3000.0, 30.0)}


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["persistent", "launches", "graph"])
@pytest.mark.parametrize("case", sorted(LOCAL_CASES))
def test_local_line_solver_matches_oracle(case, mode):
    """Sweeps with the paper's local line solver (ALM + TRON on the
    unmodified line Hessians, hessian mode RAW_LOCAL) against the oracle's
    ADMM with the same solver.  In the nonconvex case (line multipliers of
    scale 3000, penalties 30) most line matrices are indefinite: the exact
    solver's RAW mode refuses them, the local solver proceeds."""
    from paper_2310_13143_amd import AcopfError
    print(f"[gpu] local line solver {case} mode={mode}", flush=True)
    pi_scale, rho_v = LOCAL_CASES[case]
    g = grid_14()
    x, pi = start_point(g, pi_scale=pi_scale, seed=5)
    delta = 0.05
    rho = admm.Rho.scalar(g, rho_v)
    Q = qpm.build_qp(g, x, pi, delta, "raw")
    lam_min = np.linalg.eigvalsh(admm.line_matrices(Q, rho)).min(axis=1)
    assert ((lam_min < 0).sum() >= 5) == (case == "nonconvex")
    nsw = 20
    ref = admm.solve(g, Q, rho, nsw, 0.0, 0.0, record=True, line_solver="alm")
    dg, xi, res, st = _run_gpu(g, x, pi, delta, rho, None, None, nsw, mode=mode, hessian=2)
    assert res["sweeps"] == nsw
    assert res["infeasible_lines"] == ref.infeasible_lines
    _compare_state(st, ref.state, tol=1e-7)
    assert abs(res["r"] - ref.r) <= 1e-6 * ref.r and abs(res["s"] - ref.s) <= 1e-6 * ref.s
    if case == "nonconvex":
        # the same QP with the exact solver's mode stops at the first line
        dg.qp_build(xi, delta, 1)
        with pytest.raises(AcopfError) as e:
            dg.admm_init(*dg.rho_scalar(rho_v))
            dg.admm_solve(2)
        assert e.value.code == -3
        # and a fresh setup goes back to the exact solver's kernels
        dg2, _, _, st2 = _run_gpu(g, x, pi, delta, admm.Rho.scalar(g, 2e4), None, None, 10, mode=mode, hessian=0)
        ref2 = admm.solve(g, qpm.build_qp(g, x, pi, delta, "psd"), admm.Rho.scalar(g, 2e4), 10, 0.0, 0.0)
        _compare_state(st2, ref2.state)


def test_local_line_solver_batch_matches_solo_runs():
    """The local line solver in a batch (per-scenario block tables) gives
    each scenario's solo run bit for bit."""
    print("[gpu] local line solver batch", flush=True)
    grids = _batch_cases()[:2]
    DeviceGrid = _dev()
    pts = [start_point(g, pi_scale=3000.0, seed=20 + k) for k, g in enumerate(grids)]
    nsw = 30
    dg = DeviceGrid(grids)
    cat = lambda name: np.concatenate([getattr(p[0], name) for p in pts])
    pi = np.concatenate([p[1] for p in pts])
    xb = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), pi)
    dg.qp_build(xb, 0.05, 2)
    dg.admm_init(*dg.rho_scalar(30.0))
    dg.admm_solve(nsw, 0.0, 0.0, sweep_mode=1, block_size=64)
    res = dg.admm_results()
    st = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    for k, g in enumerate(grids):
        x, pik = pts[k]
        solo = DeviceGrid(g)
        xs = solo.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pik)
        solo.qp_build(xs, 0.05, 2)
        solo.admm_init(*solo.rho_scalar(30.0))
        rs = solo.admm_solve(nsw, 0.0, 0.0, sweep_mode=1, block_size=64)
        ss = {k2: v.cpu().numpy() for k2, v in solo.admm_state().items()}
        part = _slice_state(st, dg, k, dg.n_gen, dg.n_line, dg.n_bus)
        for name, a in part.items():
            b = ss[name].reshape(a.shape) if a.ndim == 2 else ss[name]
            assert np.array_equal(a, b), (k, name)
        assert res[k]["sweeps"] == rs["sweeps"] and res[k]["r"] == rs["r"] and res[k]["s"] == rs["s"]


def test_sqp_with_local_line_solver_matches_oracle():
    """Algorithm 1 with the unmodified Hessians and the local line solver on
    the device against the oracle's SQP with the same settings, iteration by
    iteration (fixed sweep budget, no early stop)."""
    from paper_2310_13143_amd import _abi
    print("[gpu] sqp ring14 local line solver", flush=True)
    g = grid_14()
    x0, _ = start_point(g)
    params = sqp.SqpParams(max_iter=4, max_sweeps=150, eps_pri=0.0, eps_dual=0.0, delta0=0.05, tol_step=0.0,
                           tol_primal=0.0, tol_dual=0.0, hessian_mode="raw", line_solver="alm")
    ref = sqp.solve(g, params, x0=x0)
    dg = _dev()(g)
    x = dg.iterate(x0.pg, x0.qg, x0.w, x0.th, x0.wR, x0.wI, None)
    rho_g, rho_l = dg.rho_scalar(params.rho)
    delta = params.delta0
    for k, rec in enumerate(ref.records):
        out = dg.sqp_step(x, delta, rho_g, rho_l, mu=params.mu_merit, delta_max=params.delta_max,
                          hessian_mode=_abi.HESSIAN_RAW_LOCAL, warm_start=k > 0, max_sweeps=params.max_sweeps,
                          eps=0.0, sweep_mode=_abi.SWEEP_LAUNCHES)
        assert bool(out["accepted"]) == rec.accepted, k
        assert abs(out["ared"] - rec.ared) <= 1e-6 * (1.0 + abs(rec.ared)), (k, out["ared"], rec.ared)
        assert abs(out["pred"] - rec.pred) <= 1e-6 * (1.0 + abs(rec.pred)), (k, out["pred"], rec.pred)
        assert abs(out["delta"] - rec.delta) <= 1e-12 * rec.delta, k
        delta = out["delta"]
    xf = {k: v.cpu().numpy() for k, v in x.items()}
    for name in ("pg", "qg", "w", "th", "wR", "wI"):
        assert rel_err(xf[name], getattr(ref.x, name)) <= 1e-7, name


@pytest.mark.parametrize("mode", [1, 2], ids=["launches", "graph"])
@pytest.mark.parametrize("case", ["ring14", "tiny_shunt"])
def test_linfeas_matches_oracle(case, mode):
    """Linear feasibility projection (Section II-A, eq. linfeas) on the
    device: a fixed sweep count against the oracle's decomposed projection
    (1e-8), and a converged run against the oracle's interior-point
    projection (1e-6), with the linear constraints met and the multipliers
    pi untouched."""
    from oracle import linfeas
    print(f"[gpu] linfeas {case} mode={mode}", flush=True)
    g = CASES[case]()
    x0 = acopf.flat_start(g)
    nsw = 150
    ref = linfeas.admm_project(g, x0, 1.0, nsw)
    dg = _dev()(g)
    pi0 = np.random.default_rng(3).standard_normal((g.n_line, 4))
    x = dg.iterate(x0.pg, x0.qg, x0.w, x0.th, x0.wR, x0.wI, pi0)
    res = dg.linfeas(x, rho=1.0, max_sweeps=nsw, eps=0.0, sweep_mode=mode)
    assert res["sweeps"] == nsw and res["infeasible_lines"] == 0
    assert abs(res["r"] - ref.r) <= 1e-7 * ref.r and abs(res["s"] - ref.s) <= 1e-7 * ref.s
    xf = {k: v.cpu().numpy() for k, v in x.items()}
    for name in ("pg", "qg", "w", "th", "wR", "wI"):
        assert rel_err(xf[name], getattr(ref.x, name)) <= TOL, name
    assert np.array_equal(xf["pi"].reshape(4, -1).T, pi0)
    # converged
    x = dg.iterate(x0.pg, x0.qg, x0.w, x0.th, x0.wR, x0.wI, pi0)
    res = dg.linfeas(x, rho=1.0, max_sweeps=20000, eps=1e-10, sweep_mode=mode)
    assert res["converged"]
    xf = {k: v.cpu().numpy() for k, v in x.items()}
    xp = acopf.Iterate(*(xf[n] for n in ("pg", "qg", "w", "th", "wR", "wI")))
    p = linfeas.project(g, x0)
    assert linfeas.violation(g, xp) < 1e-8
    np.testing.assert_allclose(linfeas._vec(xp), linfeas._vec(p.x), atol=1e-6)
    # the workspace serves a QP subproblem again after a build
    dg.qp_build(x, 0.05)
    dg.admm_init(*dg.rho_scalar(2e4))
    assert dg.admm_solve(10, sweep_mode=mode)["sweeps"] == 10


def test_linfeas_batch_matches_solo_runs_and_rejects_the_persistent_mode():
    """Two scenarios projected in one batch give their solo runs bit for
    bit; the persistent sweep mode is refused."""
    from paper_2310_13143_amd import AcopfError
    print("[gpu] linfeas batch", flush=True)
    grids = _batch_cases()[:2]
    DeviceGrid = _dev()
    x0s = [acopf.flat_start(g) for g in grids]
    dg = DeviceGrid(grids)
    cat = lambda name: np.concatenate([getattr(x, name) for x in x0s])
    xb = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)
    dg.linfeas(xb, rho=1.0, max_sweeps=100, eps=0.0, sweep_mode=1)
    xbf = {k: v.cpu().numpy() for k, v in xb.items()}
    offs = {"pg": dg.offsets["gen"], "qg": dg.offsets["gen"], "w": dg.offsets["bus"], "th": dg.offsets["bus"],
            "wR": dg.offsets["line"], "wI": dg.offsets["line"]}
    for k, g in enumerate(grids):
        solo = DeviceGrid(g)
        xs = solo.iterate(x0s[k].pg, x0s[k].qg, x0s[k].w, x0s[k].th, x0s[k].wR, x0s[k].wI, None)
        solo.linfeas(xs, rho=1.0, max_sweeps=100, eps=0.0, sweep_mode=1)
        for name, o in offs.items():
            assert np.array_equal(xbf[name][o[k]:o[k + 1]], xs[name].cpu().numpy()), (k, name)
    with pytest.raises(AcopfError) as e:
        dg.linfeas(xb, sweep_mode=0)
    assert e.value.code == -5


def test_sqp_with_restoration_matches_oracle():
    """Feasibility restoration (hessian mode kModeRestore through
    acopf_sqp_step's restore flag) on the 14-bus grid with its line limits
    halved, where the radius collapses: the device iterations, restoration
    steps included, follow the oracle's SQP with restoration (fixed sweep
    budget): acceptance, the reduction of h of a restoration step, radii and
    the final iterate."""
    import dataclasses
    print("[gpu] sqp ring14 restoration", flush=True)
    g = grid_14()
    g = dataclasses.replace(g, smax_ij=0.5 * g.smax_ij, smax_ji=0.5 * g.smax_ji)
    x0, _ = start_point(g)
    params = sqp.SqpParams(max_iter=8, max_sweeps=60, eps_pri=0.0, eps_dual=0.0, delta0=0.05, tol_step=0.0,
                           tol_primal=0.0, tol_dual=0.0, delta_min=0.02, restore=True)
    ref = sqp.solve(g, params, x0=x0)
    assert any(r.restore and r.accepted for r in ref.records)
    dg = _dev()(g)
    x = dg.iterate(x0.pg, x0.qg, x0.w, x0.th, x0.wR, x0.wI, None)
    rho_g, rho_l = dg.rho_scalar(params.rho)
    delta = params.delta0
    warm = False
    for k, rec in enumerate(ref.records):
        if rec.restore:
            out = dg.sqp_step(x, params.delta0, rho_g, rho_l, mu=params.mu_merit, warm_start=False,
                              max_sweeps=params.max_sweeps, eps=0.0, sweep_mode=1, restore=True)
            assert bool(out["accepted"]) == rec.accepted, k
            assert abs(out["ared"] - rec.ared) <= 1e-6 * (1.0 + abs(rec.ared)), (k, out["ared"], rec.ared)
            assert out["delta"] == params.delta0
            delta, warm = params.delta0, False
            continue
        out = dg.sqp_step(x, delta, rho_g, rho_l, mu=params.mu_merit, delta_max=params.delta_max,
                          warm_start=warm, max_sweeps=params.max_sweeps, eps=0.0, sweep_mode=1)
        assert bool(out["accepted"]) == rec.accepted, k
        assert abs(out["ared"] - rec.ared) <= 1e-6 * (1.0 + abs(rec.ared)), (k, out["ared"], rec.ared)
        # a rejection sets the radius from the step's norm, which the ADMM
        # iterates give to about 1e-8
        assert abs(out["delta"] - rec.delta) <= 1e-8 * rec.delta, k
        delta, warm = out["delta"], True
    xf = {k: v.cpu().numpy() for k, v in x.items()}
    for name in ("pg", "qg", "w", "th", "wR", "wI"):
        assert rel_err(xf[name], getattr(ref.x, name)) <= 1e-7, name


def test_rgg70000_local_line_solver_sampled():
    """The local line solver (RAW_LOCAL) at 70,000 buses in the bench's graph
    sweep mode, with line multipliers of scale 3000 and penalties 30 (many
    indefinite line matrices): one sweep of 400 sampled lines from the GPU's
    own previous state against the oracle's ALM + TRON, started from the same
    previous solution and row multipliers."""
    from paper_2310_13143_amd import _abi
    from oracle import alm
    print("[gpu] rgg70000 local solver sampled", flush=True)
    g = grid_70000()
    x, pi = start_point(g, pi_scale=3000.0, seed=4)
    rho = admm.Rho.scalar(g, 30.0)
    Q = qpm.build_qp(g, x, pi, 0.05, "raw")
    Qm = admm.line_matrices(Q, rho)
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(g.n_line, 400, replace=False))
    assert (np.linalg.eigvalsh(Qm[sample]).min(axis=1) < 0).mean() > 0.2
    dg = _dev()(g)
    xi = dg.iterate(x.pg, x.qg, x.w, x.th, x.wR, x.wI, pi)
    dg.qp_build(xi, 0.05, 2)
    dg.admm_init(*dg.rho_scalar(30.0))
    dg.admm_solve(5, 0.0, 0.0, sweep_mode=_abi.SWEEP_GRAPH)
    s0 = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    dg.admm_solve(1, 0.0, 0.0, sweep_mode=_abi.SWEEP_GRAPH)
    s1 = {k: v.cpu().numpy() for k, v in dg.admm_state().items()}
    L = g.n_line
    xl0, lam0 = s0["xl"].reshape(8, L).T, s0["lam_l"].reshape(8, L).T
    xbf0, mu0 = s0["xbar_f"].reshape(4, L).T, s0["mu"].reshape(2, L).T
    xl1, mu1 = s1["xl"].reshape(8, L).T, s1["mu"].reshape(2, L).T
    Ln = Q.line
    f, t = g.f, g.t
    xbar_v = np.stack([s0["dw"][f], s0["dth"][f], s0["dw"][t], s0["dth"][t]], 1)
    rf, rv = rho.l[:, :4], rho.l[:, 4:]
    c = Ln.q + np.einsum("lf,lfi->li", lam0[:, :4] + rf * (Ln.f0 - xbf0), Ln.F) + lam0[:, 4:] - rv * xbar_v
    bad = 0
    for l in sample:
        r = alm.solve_line(Qm[l], c[l], Ln.lo[l], Ln.hi[l], Ln.G[l], Ln.h[l], z0=xl0[l, 4:8], u0=mu0[l])
        scale = 1.0 + np.abs(r.z).max()
        ok = np.abs(xl1[l, 4:8] - r.z).max() <= 1e-7 * scale and \
            np.abs(mu1[l] - r.u).max() <= 1e-6 * (1.0 + np.abs(r.u).max())
        bad += 0 if ok else 1
    # an iteration whose branches (ratio test, active set) sit on a rounding
    # boundary may part ways on a line now and then; all but 1% must match
    assert bad <= len(sample) // 100, bad


@pytest.mark.parametrize("mode", [0, 2], ids=["persistent", "graph"])
def test_infinity_norm_stop_test_matches_oracle(mode):
    """The stop test on infinity norms (acopf_admm_params.norm_inf): the
    reported norms after a fixed sweep count, and the stop sweep of a
    stopped solve, against the oracle's ADMM with infinity norms."""
    print(f"[gpu] infinity norm mode={mode}", flush=True)
    g = grid_14()
    x, pi = start_point(g, pi_scale=20.0, seed=3)
    rho = _rho(g, 4)
    Q = qpm.build_qp(g, x, pi, 0.05, "psd")
    ref = admm.solve(g, Q, rho, 60, 0.0, 0.0, norm="inf")
    dg, xi, res, st = _run_gpu(g, x, pi, 0.05, rho, None, None, 60, mode=mode, norm_inf=True)
    assert res["sweeps"] == 60
    assert abs(res["r"] - ref.r) <= 1e-7 * ref.r and abs(res["s"] - ref.s) <= 1e-7 * ref.s
    _compare_state(st, ref.state)
    # stop at ||r||_inf <= 3e-3 and ||s||_inf <= 20 (the dual residuals carry
    # the penalties of about 2e4)
    ref2 = admm.solve(g, Q, rho, 400, 3e-3, 20.0, norm="inf")
    assert ref2.converged and ref2.sweeps < 400
    dg.qp_build(xi, 0.05, 0)
    dg.admm_init(rho.g.T.reshape(-1), rho.l.T.reshape(-1))
    res2 = dg.admm_solve(400, 3e-3, 20.0, sweep_mode=mode, norm_inf=True)
    assert res2["converged"] and abs(res2["sweeps"] - ref2.sweeps) <= 1
    assert res2["r"] <= 3e-3 and res2["s"] <= 20.0
