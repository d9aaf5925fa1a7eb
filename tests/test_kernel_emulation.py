"""The library's per-component arithmetic (device code compiled for the host
with g++) against the oracle, on the CPU: line QP solver vs enumeration,
PSD projection, QP build, full ADMM sweeps and the SQP step/multipliers.
This checks the kernels' arithmetic and indexing before a GPU runs them."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from synth.grids import grid_14, grid_2000, tiny_grid, power_flow_start
from oracle import acopf, admm, lineqp, qp as qpm, sqp
from paper_2310_13143_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("emu") / "libemu.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "native", "emulate.cpp"), "-o", out], check=True)
    lib = ctypes.CDLL(out)
    lib.emu_workspace_bytes.restype = ctypes.c_size_t
    lib.emu_workspace_bytes.argtypes = [ctypes.c_int] * 3
    lib.emu_run.restype = ctypes.c_int
    return lib


def ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def test_line_qp_solver_matches_enumeration(emu):
    rng = np.random.default_rng(11)
    n = 400
    A = rng.standard_normal((n, 4, 4))
    Q = A @ np.swapaxes(A, 1, 2) + 0.3 * np.eye(4)
    # badly scaled instances like the ADMM's (rho ~ 1e4 times admittance^2)
    Q[: n // 2] *= rng.uniform(1e2, 1e6, (n // 2, 1, 1))
    c = rng.standard_normal((n, 4)) * np.abs(Q).max(axis=(1, 2))[:, None] * rng.uniform(0.01, 2, (n, 1))
    lo = -rng.uniform(0.01, 0.3, (n, 4))
    hi = rng.uniform(0.01, 0.3, (n, 4))
    G = rng.standard_normal((n, 2, 4))
    h = rng.uniform(0.01, 0.2, (n, 2))
    fx = rng.random(n) < 0.25
    lo[fx, 3] = 0.0
    hi[fx, 3] = 0.0
    P = np.linalg.inv(Q)
    iu = np.triu_indices(4)
    Pp = np.ascontiguousarray(P[:, iu[0], iu[1]])
    z = np.zeros((n, 4)); mu = np.zeros((n, 2)); st = np.zeros(n, dtype=np.int32)
    args = (ptr(Pp), ptr(np.ascontiguousarray(c)), ptr(lo), ptr(hi), ptr(np.ascontiguousarray(G)), ptr(h))
    masks = np.zeros(n, dtype=np.int32)
    emu.emu_line_qp(n, *args, ptr(z), ptr(mu), ptr(st), None, ptr(masks))
    zr, mur, _, feas = lineqp.solve_line_qps(Q, c, lo, hi, G, h)
    assert feas.all() and (st == 0).all()
    scale = 1.0 + np.abs(zr).max(1)
    assert (np.abs(z - zr).max(1) / scale).max() < 1e-8
    mscale = 1.0 + np.abs(mur).max(1)
    assert (np.abs(mu - mur).max(1) / mscale).max() < 1e-6
    assert (masks != 0).sum() > n // 2  # most instances have active constraints
    # warm starts: the optimal working set (accepted by the KKT check), a
    # wrong one (one bit flipped: rejected, then solved from scratch), none
    rng2 = np.random.default_rng(5)
    flip = (1 << rng2.integers(0, 10, n)).astype(np.int32)
    # one active constraint removed: a dual feasible working set whose
    # minimiser violates the removed constraint (the method continues from it)
    drop = np.array([m & ~(1 << int(rng2.choice(np.nonzero([(m >> b) & 1 for b in range(10)])[0])))
                     if m else 0 for m in masks], dtype=np.int32)
    for warm in (masks, masks ^ flip, drop, np.zeros(n, dtype=np.int32)):
        z2 = np.zeros((n, 4)); mu2 = np.zeros((n, 2)); st2 = np.zeros(n, dtype=np.int32)
        m2 = np.zeros(n, dtype=np.int32)
        emu.emu_line_qp(n, *args, ptr(z2), ptr(mu2), ptr(st2), ptr(np.ascontiguousarray(warm, dtype=np.int32)),
                        ptr(m2))
        assert (st2 == 0).all()
        assert (np.abs(z2 - zr).max(1) / scale).max() < 1e-8
        assert (np.abs(mu2 - mur).max(1) / mscale).max() < 1e-6
        # the working set is unique up to degenerate constraints (active with
        # a zero multiplier): a different one must itself certify the
        # minimiser, i.e. be accepted as it stands when given as the warm start
        diff = np.nonzero(m2 != masks)[0]
        assert diff.size <= n // 20
        if diff.size:
            part = [np.ascontiguousarray(a[diff]) for a in (Pp, c, lo, hi, G, h, m2)]  # kept alive for the call
            z3 = np.zeros((diff.size, 4)); mu3 = np.zeros((diff.size, 2)); st3 = np.zeros(diff.size, dtype=np.int32)
            m3 = np.zeros(diff.size, dtype=np.int32)
            emu.emu_line_qp(diff.size, *[ptr(a) for a in part[:6]], ptr(z3), ptr(mu3), ptr(st3), ptr(part[6]), ptr(m3))
            assert np.array_equal(m3, m2[diff]) and (st3 == 0).all()
            assert (np.abs(z3 - zr[diff]).max(1) / scale[diff]).max() < 1e-8


def test_limit_relaxation_matches_oracle(emu):
    """The build's limit-row shift (least-squares violation from the dual:
    the largest support gap over unit normals of the positive quadrant)
    against the oracle's (minimum over the segments of the polygon
    G [lo, hi]), on random boxes and rows (fixed variables, zero rows,
    equal row entries, both rows or one row violated at the least-violation
    point) and on the lines of the 2,000-bus grid at a small trust radius."""
    rng = np.random.default_rng(1)
    n = 5000
    lo = -rng.uniform(0, 0.1, (n, 4)); hi = rng.uniform(0, 0.1, (n, 4))
    lo[::7, 1] = 0.0; hi[::7, 1] = 0.0
    G = rng.standard_normal((n, 2, 4)); h = rng.uniform(-0.3, 0.1, (n, 2))
    G[::11, 1] = 0.0
    G[::13, 0, 2] = G[::13, 1, 2]
    G[::17, :, 3] = 0.0
    cases = [(lo, hi, G, h)]
    g = grid_2000()
    x, pi = _setup(g, 0.00625, 20.0, 2)
    Q = qpm.build_qp(g, x, pi, 0.00625, "psd")
    L = Q.line
    assert (L.relax > 0).any(1).sum() > 10
    cases.append((L.lo, L.hi, L.G, L.h - L.relax))
    for lo_, hi_, G_, h_ in cases:
        lo_, hi_, G_, h_ = (np.ascontiguousarray(a) for a in (lo_, hi_, G_, h_))
        out = np.zeros((lo_.shape[0], 2))
        emu.emu_limit_relaxation(lo_.shape[0], ptr(lo_), ptr(hi_), ptr(G_), ptr(h_), ptr(out))
        ref = lineqp.limit_relaxation(lo_, hi_, G_, h_)
        v = lineqp.min_violation(lo_, hi_, G_, h_)
        assert np.array_equal(out > 0, ref > 0)
        assert (v > 0).all(1).sum() > 5 and ((v > 0).sum(1) == 1).sum() > 5
        scale = 1.0 + np.abs(h_).sum(1) + np.abs(G_).sum((1, 2)) * np.maximum(np.abs(lo_), np.abs(hi_)).max(1)
        assert (np.abs(out - ref).max(1) / scale).max() < 1e-12


def test_neighbour_masks_of_the_wave_search(emu):
    """The 55 neighbours a wave checks for a line: each is a valid working set
    (at most four constraints, never both bounds of a variable), and together
    they cover every valid set one constraint toggle away from the base."""
    def valid(m):
        return bin(m).count("1") <= 4 and (m & (m >> 4) & 0xF) == 0
    rng = np.random.default_rng(3)
    bases = [0] + [int(m) for m in rng.integers(0, 1 << 10, 400) if valid(int(m))]
    for base in bases:
        got = {emu.emu_neighbour_mask(base, i) for i in range(55)} - {-1}
        assert all(valid(m) for m in got)
        assert emu.emu_neighbour_mask(base, 55) == -1 and emu.emu_neighbour_mask(base, -1) == -1
        for k in range(10):
            m = base ^ (1 << k)
            if not (base >> k) & 1 and k < 8:   # an added bound replaces the opposite one
                m &= ~(1 << (k + 4 if k < 4 else k - 4))
            if valid(m):
                assert m in got, (base, k)


def test_psd_projection_matches_oracle(emu):
    rng = np.random.default_rng(12)
    A = rng.standard_normal((50, 4, 4))
    M = np.ascontiguousarray(A + np.swapaxes(A, 1, 2))
    out = M.copy()
    emu.emu_psd_project(50, ptr(out))
    np.testing.assert_allclose(out, qpm.psd_project(M), atol=1e-12)


class HostGrid:
    """acopf_grid / acopf_iterate structs over host numpy arrays."""

    def __init__(self, g):
        self.keep = []
        vals = []
        for n in _abi.GRID_BUS_FIELDS:
            vals.append(self.arr(getattr(g, n)))
        vals += [self.arr(g.f, np.int32), self.arr(g.t, np.int32)]
        for n in _abi.GRID_LINE_FIELDS:
            vals.append(self.arr(getattr(g, n)))
        vals.append(self.arr(g.gbus, np.int32))
        for n in _abi.GRID_GEN_FIELDS:
            vals.append(self.arr(getattr(g, n)))
        self.c = _abi.Grid(g.n_bus, g.n_line, g.n_gen, g.ref, 1, 0, *vals)

    def arr(self, a, dt=np.float64):
        a = np.ascontiguousarray(a, dtype=dt)
        self.keep.append(a)
        return a.ctypes.data

    def iterate(self, x, pi):
        arrays = [np.ascontiguousarray(v, dtype=np.float64) for v in (x.pg, x.qg, x.w, x.th, x.wR, x.wI)]
        arrays.append(np.ascontiguousarray(pi.T.reshape(-1)))
        self.keep += arrays
        return _abi.Iterate(*[a.ctypes.data for a in arrays]), arrays


def _setup(g, delta, pi_scale, seed):
    s = power_flow_start(g)
    x = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    rng = np.random.default_rng(seed)
    pi = rng.standard_normal((g.n_line, 4)) * pi_scale
    pi[:, 2:] = -np.abs(pi[:, 2:])
    return x, pi


@pytest.mark.parametrize("case", ["ring14", "tiny_shunt"])
def test_bus_items_match_per_bus_update(emu, case):
    """The bus phase split by coupling item (launch-mode kernel: per-item
    terms, summed in item order by the bus's first item, then per-item
    multiplier updates), and its one-thread walk over a bus wider than an
    item block, give the bits of the per-bus update over whole sweeps;
    residual norms agree to rounding."""
    g = grid_14() if case == "ring14" else tiny_grid(seed=21, n_bus=7, n_line=10, n_gen=3, shunt_scale=0.04)
    delta = 0.05
    x, pi = _setup(g, delta, 50.0, 3)
    rng = np.random.default_rng(4)
    rho_g = rng.uniform(5e3, 3e4, 2 * g.n_gen)
    rho_l = rng.uniform(5e3, 3e4, 8 * g.n_line)
    lg = rng.standard_normal(2 * g.n_gen) * 100
    ll = rng.standard_normal(8 * g.n_line) * 100
    hg = HostGrid(g)
    cx, _ = hg.iterate(x, pi)
    nsw = 60
    out = []
    for items in (0, 1, 2):
        emu.emu_set_bus_items(items)
        ws = np.zeros(emu.emu_workspace_bytes(g.n_bus, g.n_line, g.n_gen) // 8 + 64)
        base = (ws.ctypes.data + 255) // 256 * 256
        rs = np.zeros(2 * nsw)
        rc = emu.emu_run(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.c_double(delta), 0, ptr(rho_g), ptr(rho_l),
                         ptr(lg), ptr(ll), nsw, ctypes.c_void_p(base), None, ptr(rs))
        assert rc == 0
        lay = _layout(emu, g, base)
        out.append(({k: lay(k, n).copy() for k, n in (("xl", 8 * g.n_line), ("lam_l", 8 * g.n_line),
                                                    ("xbar_f", 4 * g.n_line), ("xg", 2 * g.n_gen),
                                                    ("lam_g", 2 * g.n_gen), ("dw", g.n_bus), ("dth", g.n_bus),
                                                    ("nu", 2 * g.n_bus))}, rs.copy(), ws))
    emu.emu_set_bus_items(0)
    a, ra, _ = out[0]
    for b, rb, _ in out[1:]:
        for k in a:
            assert np.array_equal(a[k], b[k]), k
        np.testing.assert_allclose(rb, ra, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("case", ["ring14", "tiny_shunt"])
def test_sweeps_and_step_match_oracle(emu, case):
    g = grid_14() if case == "ring14" else tiny_grid(seed=21, n_bus=7, n_line=10, n_gen=3, shunt_scale=0.04)
    delta = 0.05
    x, pi = _setup(g, delta, 50.0, 3)
    Q = qpm.build_qp(g, x, pi, delta, "psd")
    rng = np.random.default_rng(4)
    rho = admm.Rho(rng.uniform(5e3, 3e4, (g.n_gen, 2)), rng.uniform(5e3, 3e4, (g.n_line, 8)))
    lam0_g = rng.standard_normal((g.n_gen, 2)) * 100
    lam0_l = rng.standard_normal((g.n_line, 8)) * 100
    nsw = 40
    ref = admm.solve(g, Q, rho, nsw, 0.0, 0.0, state=admm.warm_state(g, lam0_g, lam0_l), record=True)

    hg = HostGrid(g)
    cx, _ = hg.iterate(x, pi)
    ws = np.zeros(emu.emu_workspace_bytes(g.n_bus, g.n_line, g.n_gen) // 8 + 64)
    rho_g = np.ascontiguousarray(rho.g.T.reshape(-1)); rho_l = np.ascontiguousarray(rho.l.T.reshape(-1))
    lg = np.ascontiguousarray(lam0_g.T.reshape(-1)); ll = np.ascontiguousarray(lam0_l.T.reshape(-1))
    d_arrays = [np.zeros(n) for n in (g.n_gen, g.n_gen, g.n_bus, g.n_bus, g.n_line, g.n_line, 4 * g.n_line)]
    cd = _abi.Iterate(*[a.ctypes.data for a in d_arrays])
    rs = np.zeros(2 * nsw)
    base = (ws.ctypes.data + 255) // 256 * 256
    rc = emu.emu_run(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.c_double(delta), 0, ptr(rho_g), ptr(rho_l),
                     ptr(lg), ptr(ll), nsw, ctypes.c_void_p(base), ctypes.byref(cd), ptr(rs))
    assert rc == 0
    # read the state back out of the host workspace through the same layout
    lay = _layout(emu, g, base)
    st = ref.state

    def close(a, b, tol=1e-8):
        scale = max(np.abs(b).max(), 1e-300)
        assert np.abs(a - b).max() <= tol * scale, (np.abs(a - b).max(), scale)

    # line by line in the workspace, 8 slots per line ordered by line end
    slots = [emu.emu_slot8(k) for k in range(8)]
    assert sorted(slots) == list(range(8)) and slots[:4] == [0, 1, 4, 5]
    close(lay("xl", 8 * g.n_line).reshape(-1, 8)[:, slots], st.xl)
    close(lay("lam_l", 8 * g.n_line).reshape(-1, 8)[:, slots], st.lam_l)
    close(lay("xbar_f", 4 * g.n_line).reshape(-1, 4), st.xbar_f)
    close(lay("xg", 2 * g.n_gen).reshape(2, -1).T, st.xg)
    close(lay("lam_g", 2 * g.n_gen).reshape(2, -1).T, st.lam_g)
    close(lay("dw", g.n_bus), st.dw)
    close(lay("dth", g.n_bus), st.dth)
    close(lay("nu", 2 * g.n_bus).reshape(2, -1).T, st.nu)
    hist = np.array(ref.history)
    np.testing.assert_allclose(np.sqrt(rs.reshape(-1, 2)), hist, rtol=1e-7, atol=1e-12)
    # step and multipliers
    dref = sqp.assemble_step(g, Q, st)
    pref = sqp.recover_pi(g, x, Q, st)
    close(d_arrays[4], dref.wR)
    close(d_arrays[5], dref.wI)
    close(d_arrays[0], dref.pg)
    close(d_arrays[6].reshape(4, -1).T, pref, tol=1e-7)
    # merit and model of the SQP acceptance test (Section II-C)
    mer = np.zeros(8)
    emu.emu_merit(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.byref(cd), ctypes.c_void_p(base), ptr(mer))
    mu = 1e5
    ared = (mer[0] + mu * mer[3]) - (mer[1] + mu * mer[4])
    pred = -(mer[2] + mer[6]) + mu * (mer[3] - mer[5])
    xt = x.plus(dref)
    ared_ref = acopf.merit(g, x, mu) - acopf.merit(g, xt, mu)
    pred_ref = sqp.predicted_reduction(g, x, Q, dref, mu)
    scale = acopf.merit(g, x, mu)
    assert abs(ared - ared_ref) <= 1e-9 * abs(scale) and abs(pred - pred_ref) <= 1e-9 * abs(scale)
    assert abs(mer[7] - sqp.step_norm(dref)) <= 1e-12
    # residual report at x with the ADMM's balance multipliers and pi
    res = np.zeros(7)
    emu.emu_residuals(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.c_void_p(base), ptr(res))
    pr = acopf.primal_infeasibility(g, x)
    for k, name in enumerate(("balance", "c11", "c12", "limit", "bounds")):
        assert abs(res[k] - pr[name]) <= 1e-12 * (1 + pr[name]), name
    du = acopf.dual_infeasibility(g, x, st.nu[:, 0], st.nu[:, 1], pi)
    assert abs(res[5] / max(1.0, res[6]) - du) <= 1e-9 * (1 + du)


def _layout(emu, g, base):
    """Reader of the ADMM state arrays inside the host workspace."""
    ptrs = (ctypes.POINTER(ctypes.c_double) * 8)()
    emu.emu_state_ptrs(ctypes.c_void_p(base), g.n_bus, g.n_line, g.n_gen, ptrs)
    names = ("xl", "lam_l", "xbar_f", "xg", "lam_g", "dw", "dth", "nu")
    where = dict(zip(names, ptrs))

    def get(name, n):
        return np.ctypeslib.as_array(where[name], (n,)).copy()
    return get


@pytest.mark.parametrize("feasible", [True, False])
def test_line_qp_vertex_with_a_fifth_violated_constraint(emu, feasible):
    """The unconstrained minimiser lies beyond a vertex of the box (all four
    variables past one of their bounds) and satisfies the first limit row,
    which the vertex violates: the dual method reaches a full working set of
    four bounds with a fifth constraint still violated.  Where the row meets
    the box the result is the enumeration's minimiser; where it cannot, the
    solver reports no feasible point (status 1)."""
    rng = np.random.default_rng(21 if feasible else 22)
    cases = []
    while len(cases) < 300:
        lo = -rng.uniform(0.01, 0.3, 4)
        hi = rng.uniform(0.01, 0.3, 4)
        sgn = rng.choice([-1.0, 1.0], 4)
        v = np.where(sgn > 0, hi, lo)
        zu = v + sgn * rng.uniform(0.5, 3.0, 4) * (hi - lo)
        A = rng.standard_normal((4, 4))
        Q = A @ A.T + 0.3 * np.eye(4)
        Q *= rng.uniform(1.0, 1e5)
        g = rng.standard_normal(4)
        if g @ (zu - v) > 0:
            g = -g
        gmin = np.minimum(g * lo, g * hi).sum()
        top, bot = g @ v, g @ zu
        # h kept away from the interval ends: a row through a vertex of the
        # box makes the minimiser's multipliers non-unique
        lo_h, hi_h = (max(gmin, bot), top) if feasible else (bot, gmin)
        if hi_h - lo_h < 1e-3 * (1.0 + abs(top)):
            continue
        h = rng.uniform(lo_h + 0.05 * (hi_h - lo_h), hi_h - 0.05 * (hi_h - lo_h))
        G = np.stack([g, g])
        hh = np.array([h, h + 100.0])
        cases.append((Q, -Q @ zu, lo, hi, G, hh))
    Q, c, lo, hi, G, h = (np.ascontiguousarray(np.stack(a)) for a in zip(*cases))
    n = Q.shape[0]
    P = np.linalg.inv(Q)
    iu = np.triu_indices(4)
    Pp = np.ascontiguousarray(P[:, iu[0], iu[1]])
    z = np.zeros((n, 4)); mu = np.zeros((n, 2)); st = np.zeros(n, dtype=np.int32); m = np.zeros(n, dtype=np.int32)
    emu.emu_line_qp(n, ptr(Pp), ptr(c), ptr(lo), ptr(hi), ptr(G), ptr(h), ptr(z), ptr(mu), ptr(st), None, ptr(m))
    zr, mur, _, feas = lineqp.solve_line_qps(Q, c, lo, hi, G, h)
    if feasible:
        assert feas.all() and (st == 0).all()
        scale = 1.0 + np.abs(zr).max(1)
        assert (np.abs(z - zr).max(1) / scale).max() < 1e-8
        assert (np.abs(mu - mur).max(1) / (1.0 + np.abs(mur).max(1))).max() < 1e-6
    else:
        assert not feas.any()
        assert (st == 1).all()


@pytest.mark.parametrize("pi_scale,rho", [(300.0, 2e4), (3000.0, 30.0)])
def test_local_line_solver_sweeps_match_oracle(emu, pi_scale, rho):
    """Sweeps with the unmodified line Hessians solved by the paper's local
    method (ALM + TRON, hessian mode RAW_LOCAL) against the oracle's ADMM
    with the same line solver.  At rho = 30 and with line multipliers pi of
    scale 3000, most line subproblems are nonconvex (the exact solver would
    fail on them)."""
    g = grid_14()
    delta = 0.05
    x, pi = _setup(g, delta, pi_scale, 5)
    Q = qpm.build_qp(g, x, pi, delta, "raw")
    R = admm.Rho.scalar(g, rho)
    lam_min = np.linalg.eigvalsh(admm.line_matrices(Q, R)).min(axis=1)
    if rho < 1e3:
        assert (lam_min < 0).sum() >= 5
    nsw = 20
    ref = admm.solve(g, Q, R, nsw, 0.0, 0.0, record=True, line_solver="alm")
    hg = HostGrid(g)
    cx, _ = hg.iterate(x, pi)
    ws = np.zeros(emu.emu_workspace_bytes(g.n_bus, g.n_line, g.n_gen) // 8 + 64)
    rho_g = np.full(2 * g.n_gen, rho); rho_l = np.full(8 * g.n_line, rho)
    rs = np.zeros(2 * nsw)
    base = (ws.ctypes.data + 255) // 256 * 256
    rc = emu.emu_run(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.c_double(delta), 2, ptr(rho_g), ptr(rho_l),
                     None, None, nsw, ctypes.c_void_p(base), None, ptr(rs))
    assert rc % 10000 == ref.infeasible_lines  # lines whose local solve did not converge in the last sweep
    lay = _layout(emu, g, base)
    slots = [emu.emu_slot8(k) for k in range(8)]
    st = ref.state

    def close(a, b, tol):
        scale = max(np.abs(b).max(), 1e-300)
        assert np.abs(a - b).max() <= tol * scale, (np.abs(a - b).max(), scale)

    close(lay("xl", 8 * g.n_line).reshape(-1, 8)[:, slots], st.xl, 1e-7)
    close(lay("lam_l", 8 * g.n_line).reshape(-1, 8)[:, slots], st.lam_l, 1e-7)
    close(lay("dw", g.n_bus), st.dw, 1e-7)
    close(lay("nu", 2 * g.n_bus).reshape(2, -1).T, st.nu, 1e-7)


def test_sweeps_on_relaxed_lines_match_oracle(emu):
    """Sweeps on the 2,000-bus grid at a trust radius where dozens of lines
    have no feasible point: the exact solver of the device code on the
    relaxed rows (least-violation sets, widened by the rounding guard)
    against the oracle, and no line reported infeasible."""
    g = grid_2000()
    delta = 0.00625
    x, pi = _setup(g, delta, 20.0, 2)
    Q = qpm.build_qp(g, x, pi, delta, "psd")
    assert (Q.line.relax > 0).any(1).sum() > 50
    R = admm.Rho.scalar(g, 2e4)
    nsw = 8
    ref = admm.solve(g, Q, R, nsw, 0.0, 0.0)
    assert ref.infeasible_lines == 0
    hg = HostGrid(g)
    cx, _ = hg.iterate(x, pi)
    ws = np.zeros(emu.emu_workspace_bytes(g.n_bus, g.n_line, g.n_gen) // 8 + 64)
    rho_g = np.full(2 * g.n_gen, 2e4); rho_l = np.full(8 * g.n_line, 2e4)
    rs = np.zeros(2 * nsw)
    base = (ws.ctypes.data + 255) // 256 * 256
    rc = emu.emu_run(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.c_double(delta), 0, ptr(rho_g), ptr(rho_l),
                     None, None, nsw, ctypes.c_void_p(base), None, ptr(rs))
    assert rc == 0
    lay = _layout(emu, g, base)
    slots = [emu.emu_slot8(k) for k in range(8)]
    st = ref.state
    # ill-conditioned relaxed lines (rows binding along directions in which
    # their coefficients are tiny): points up to 1e-4 of the box width
    # apart, objectives equal to a few parts in 1e8
    from tests._util import rel_err_cols
    assert rel_err_cols(lay("xl", 8 * g.n_line).reshape(-1, 8)[:, slots], st.xl) <= 1e-4
    assert rel_err_cols(lay("lam_l", 8 * g.n_line).reshape(-1, 8)[:, slots], st.lam_l) <= 1e-4
    assert rel_err_cols(lay("dw", g.n_bus), st.dw) <= 1e-6
    assert rel_err_cols(lay("nu", 2 * g.n_bus).reshape(2, -1).T, st.nu) <= 1e-6


def test_relaxed_line_objectives_match_oracle(emu):
    """Line subproblems of the relaxed lines (2,000-bus grid, trust radius
    0.00625, a first sweep): their optimal objective value is unique and the
    device code's solver matches the oracle's there to 1e-6 relative, with
    the relaxed rows met; the points themselves are ill-determined (see the
    sweep test above)."""
    g = grid_2000()
    x, pi = _setup(g, 0.00625, 20.0, 2)
    Q = qpm.build_qp(g, x, pi, 0.00625, "psd")
    L = Q.line
    idx = np.nonzero((L.relax > 0).any(1))[0]
    R = admm.Rho.scalar(g, 2e4)
    QL = admm.line_matrices(Q, R)[idx]
    c = np.ascontiguousarray((L.q + np.einsum("lf,lfi->li", R.l[:, :4] * L.f0, L.F))[idx])
    lo, hi, G, h = (np.ascontiguousarray(a[idx]) for a in (L.lo, L.hi, L.G, L.h))
    iu = np.triu_indices(4)
    Pp = np.ascontiguousarray(np.linalg.inv(QL)[:, iu[0], iu[1]])
    n = idx.size
    z = np.zeros((n, 4)); mu = np.zeros((n, 2)); st = np.zeros(n, dtype=np.int32)
    emu.emu_line_qp(n, ptr(Pp), ptr(c), ptr(lo), ptr(hi), ptr(G), ptr(h), ptr(z), ptr(mu), ptr(st), None, None)
    zr, _, _, feas = lineqp.solve_line_qps(QL, c, lo, hi, G, h)
    assert feas.all() and (st == 0).all()
    phi = lambda zz: 0.5 * np.einsum("ni,nij,nj->n", zz, QL, zz) + (c * zz).sum(1)
    scale = np.abs(phi(zr)) + np.einsum("ni,ni->n", np.abs(c), np.abs(hi - lo)) + 1e-300
    assert (np.abs(phi(z) - phi(zr)) / scale).max() < 1e-6
    rs = 1 + np.abs(h) + np.einsum("nrj,nj->nr", np.abs(G), np.abs(z))
    assert (np.einsum("nrj,nj->nr", G, z) - h <= 1e-11 * rs).all()   # far inside the 1e-9 guard
    assert (z >= lo).all() and (z <= hi).all()


@pytest.mark.parametrize("case", ["ring14", "tiny_shunt"])
def test_linfeas_sweeps_match_oracle(emu, case):
    """The linear feasibility projection's sweeps (line kernel with free wR,
    wI, generators with a reactive term, the unchanged bus closed form) on
    the host against the oracle's decomposed projection, sweep by sweep in
    the residual norms and in the projected iterate after a fixed count."""
    from oracle import linfeas
    g = grid_14() if case == "ring14" else tiny_grid(seed=21, n_bus=7, n_line=10, n_gen=3, shunt_scale=0.04)
    x0 = acopf.flat_start(g)
    nsw = 60
    ref = linfeas.admm_project(g, x0, 1.0, nsw)
    hg = HostGrid(g)
    cx, arrays = hg.iterate(x0, np.zeros((g.n_line, 4)))
    ws = np.zeros(emu.emu_workspace_bytes(g.n_bus, g.n_line, g.n_gen) // 8 + 64)
    base = (ws.ctypes.data + 255) // 256 * 256
    rs = np.zeros(2 * nsw)
    bad = emu.emu_linfeas_run(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.c_double(1.0), nsw,
                              ctypes.c_void_p(base), ptr(rs))
    assert bad == 0
    assert abs(np.sqrt(rs[-2]) - ref.r) <= 1e-8 * ref.r and abs(np.sqrt(rs[-1]) - ref.s) <= 1e-8 * ref.s
    for name, a in zip(("pg", "qg", "w", "th", "wR", "wI"), arrays[:6]):
        b = getattr(ref.x, name)
        assert np.abs(a - b).max() <= 1e-10 * (1 + np.abs(b).max()), name


def test_restoration_qp_sweeps_and_merit_match_oracle(emu):
    """A feasibility restoration step's QP (objective 0.5 ||d||^2, the same
    constraints; line Hessian mode kModeRestore = 4, generators with unit
    curvature on p and q) built and swept by the device code on the host
    against the oracle's restore-mode QP and ADMM, and the constraint
    violation h at x and x + d against the oracle."""
    g = grid_14()
    delta = 0.05
    x, pi = _setup(g, delta, 50.0, 9)
    Q = qpm.build_qp(g, x, pi, delta, "restore")
    R = admm.Rho.scalar(g, 2e4)
    nsw = 40
    ref = admm.solve(g, Q, R, nsw, 0.0, 0.0)
    hg = HostGrid(g)
    cx, _ = hg.iterate(x, pi)
    ws = np.zeros(emu.emu_workspace_bytes(g.n_bus, g.n_line, g.n_gen) // 8 + 64)
    rho_g = np.full(2 * g.n_gen, 2e4); rho_l = np.full(8 * g.n_line, 2e4)
    d_arrays = [np.zeros(n) for n in (g.n_gen, g.n_gen, g.n_bus, g.n_bus, g.n_line, g.n_line, 4 * g.n_line)]
    cd = _abi.Iterate(*[a.ctypes.data for a in d_arrays])
    rs = np.zeros(2 * nsw)
    base = (ws.ctypes.data + 255) // 256 * 256
    rc = emu.emu_run(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.c_double(delta), 4, ptr(rho_g), ptr(rho_l),
                     None, None, nsw, ctypes.c_void_p(base), ctypes.byref(cd), ptr(rs))
    assert rc == 0
    lay = _layout(emu, g, base)
    slots = [emu.emu_slot8(k) for k in range(8)]
    st = ref.state
    from tests._util import rel_err_cols
    assert rel_err_cols(lay("xl", 8 * g.n_line).reshape(-1, 8)[:, slots], st.xl) <= 1e-8
    assert rel_err_cols(lay("xg", 2 * g.n_gen).reshape(2, -1).T, st.xg) <= 1e-8
    assert rel_err_cols(lay("dw", g.n_bus), st.dw) <= 1e-8
    dref = sqp.assemble_step(g, Q, st)
    for a, name in zip(d_arrays[:6], ("pg", "qg", "w", "th", "wR", "wI")):
        b = getattr(dref, name)
        assert np.abs(a - b).max() <= 1e-8 * (1 + np.abs(b).max()), name
    mer = np.zeros(8)
    emu.emu_merit(ctypes.byref(hg.c), ctypes.byref(cx), ctypes.byref(cd), ctypes.c_void_p(base), ptr(mer))
    assert mer[3] == pytest.approx(acopf.infeas_h(g, x), rel=1e-10)
    assert mer[4] == pytest.approx(acopf.infeas_h(g, x.plus(dref)), rel=1e-7)


@pytest.mark.parametrize("n,bound", [(1, 1), (7, 7), (8, 8), (9, 9), (730, 1457), (688, 688), (1375, 1375),
                                     (5, 40), (61, 64), (64, 61 + 8)])
def test_xcd_block_order_covers_every_block_once(emu, n, bound):
    """The sweep launches' workgroup -> block map: every used block is taken
    by exactly one workgroup of the rounded-up launch, each XCD (workgroups
    b, b + 8, ...) runs one contiguous run of blocks, and the runs follow
    XCD order."""
    out = np.full(bound + 8, -2, dtype=np.int32)
    g = emu.emu_xcd_blocks(n, bound, ptr(out))
    assert g % 8 == 0 and bound <= g < bound + 8
    got = out[:g]
    used = got[got >= 0]
    assert np.array_equal(np.sort(used), np.arange(n))
    assert (got[got < 0] == -1).all()
    starts = []
    for x in range(8):
        run = got[x::8]
        run = run[run >= 0]
        if run.size:
            assert np.array_equal(run, np.arange(run[0], run[0] + run.size))
            starts.append(run[0])
    assert starts == sorted(starts)
