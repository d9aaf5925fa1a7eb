"""Linear feasibility projection (Section II-A, eq. linfeas; Algorithm 1,
the step before the loop).

The start x0 is projected onto the set the ACOPF's linear constraints
define: minimise ||x - x0||^2 over x = (pg, qg, w, th, wR, wI) subject to the
power balance (opfc5, opfc6), which is linear in (pg, qg, w, wR, wI), the
variable bounds (opfc1-4) and the reference angle theta_ref = 0.  The
nonlinear constraints (opfc11-14) are not part of it.  Later QP steps keep
these constraints satisfied (they are linear), so the first QP starts from
a point that meets them.

The balance matrix is read off the model itself: the balance residuals are
affine in x, so column j of their Jacobian is balance(e_j) - balance(0).
The QP is solved by the interior-point method of ``direct.ipm``.

``admm_project`` runs the same projection through the ADMM decomposition of
the QP subproblems (see its section below).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp

from . import acopf
from .acopf import Iterate
from .direct import ipm


@dataclass
class Projection:
    x: Iterate
    objective: float       # ||x - x0||^2
    nu: np.ndarray         # (2B,) multipliers of the balance rows (P then Q)
    iterations: int


def _vec(x: Iterate) -> np.ndarray:
    return np.concatenate([x.pg, x.qg, x.w, x.th, x.wR, x.wI])


def _unvec(grid, v) -> Iterate:
    out, o = [], 0
    for n in (grid.n_gen, grid.n_gen, grid.n_bus, grid.n_bus, grid.n_line, grid.n_line):
        out.append(np.array(v[o:o + n]))
        o += n
    return Iterate(*out)


def balance_matrix(grid):
    """(A, b) with balance residuals (opfc5, opfc6) = A x - b, P rows then Q rows."""
    n = 2 * grid.n_gen + 2 * grid.n_bus + 2 * grid.n_line
    zero = np.zeros(n)

    def bal(v):
        rp, rq = acopf.balance(grid, _unvec(grid, v))
        return np.concatenate([rp, rq])

    r0 = bal(zero)
    cols = []
    for j in range(n):
        e = zero.copy()
        e[j] = 1.0
        cols.append(bal(e) - r0)
    A = np.stack(cols, 1)
    A[np.abs(A) < 1e-300] = 0.0
    return sp.csr_matrix(A), -r0


def bounds(grid):
    """Variable bounds (opfc1-4) with theta_ref = 0; wR, wI are free."""
    thlo = np.full(grid.n_bus, -2 * np.pi)
    thhi = np.full(grid.n_bus, 2 * np.pi)
    thlo[grid.ref] = thhi[grid.ref] = 0.0
    inf = np.full(2 * grid.n_line, np.inf)
    lo = np.concatenate([grid.pmin, grid.qmin, grid.vmin ** 2, thlo, -inf])
    hi = np.concatenate([grid.pmax, grid.qmax, grid.vmax ** 2, thhi, inf])
    return lo, hi


def violation(grid, x: Iterate) -> float:
    """Largest violation of the linear constraints at x."""
    A, b = balance_matrix(grid)
    lo, hi = bounds(grid)
    v = _vec(x)
    return float(max(np.abs(A @ v - b).max(initial=0), np.maximum(lo - v, 0).max(initial=0),
                     np.maximum(v - hi, 0).max(initial=0)))


def project(grid, x0: Iterate, tol: float = 1e-12) -> Projection:
    """Solve eq. linfeas from x0: min 0.5 ||x - x0||^2 under the linear
    constraints (the factor 0.5 does not move the minimiser)."""
    A, b = balance_matrix(grid)
    lo, hi = bounds(grid)
    v0 = _vec(x0)
    n = v0.size
    fixed = lo >= hi
    free = np.nonzero(~fixed)[0]
    vfix = np.where(fixed, hi, 0.0)
    nf = free.size
    I = sp.identity(nf, format="csr")
    flo, fhi = lo[free], hi[free]
    has_hi, has_lo = np.isfinite(fhi), np.isfinite(flo)
    Gin = sp.vstack([I[has_hi], -I[has_lo]]).tocsr()
    hin = np.concatenate([fhi[has_hi], -flo[has_lo]])
    Af = A[:, free]
    bf = b - A @ vfix
    y, nu, _, it = ipm(sp.identity(nf, format="csc"), -v0[free], Af, bf, Gin, hin, tol)
    v = vfix.copy()
    v[free] = y
    return Projection(_unvec(grid, v), float(np.sum((v - v0) ** 2)), nu, it)


# ---------------------------------------------------------------------------
# The same projection through the ADMM decomposition of the QP subproblems
# (Algorithm 2 over eq. cpl), as the device runs it.  Variables are changes
# d = x - x0.  Generators: 0.5 (d_p^2 + d_q^2) on their boxes less x0.  Lines:
# z = (d_w_i, d_wR, d_w_j, d_wI), flows F z exactly (the balance's
# coefficients), objective 0.5 (d_wR^2 + d_wI^2) plus each end's share
# 1/degree of its bus's 0.5 d_w^2, box of d_w from the voltage bounds and
# [-FREE_BOX, FREE_BOX] for d_wR, d_wI, no limit rows; the angle copies are
# held at zero (d_theta enters neither objective nor constraint).  Buses:
# the closed form of the QP subproblems (admm.bus_update) with the start's
# balance constants.

FREE_BOX = 10.0


@dataclass
class AdmmProjection:
    x: Iterate
    sweeps: int
    r: float
    s: float
    converged: bool
    state: object
    d_wR: np.ndarray
    d_wI: np.ndarray


def decomposed_data(grid, x0: Iterate):
    """Per-line (M, F, lo, hi), per-generator boxes and the bus constants of
    the decomposed projection at x0."""
    nb, L = grid.n_bus, grid.n_line
    f, t = grid.f, grid.t
    deg = np.bincount(f, minlength=nb) + np.bincount(t, minlength=nb)
    M = np.zeros((L, 4, 4))
    M[:, 0, 0] = 1.0 / deg[f]
    M[:, 1, 1] = 1.0
    M[:, 2, 2] = 1.0 / deg[t]
    M[:, 3, 3] = 1.0
    z0 = np.zeros(L)
    F = np.stack([np.stack([grid.gii, grid.gij, z0, grid.bij], 1),
                  np.stack([-grid.bii, -grid.bij, z0, grid.gij], 1),
                  np.stack([z0, grid.gji, grid.gjj, -grid.bji], 1),
                  np.stack([z0, -grid.bji, -grid.bjj, -grid.gji], 1)], 1)     # (L, 4 flows, 4 vars)
    whi = grid.vmax ** 2 - x0.w
    wlo = np.minimum(grid.vmin ** 2 - x0.w, whi)
    lo = np.stack([wlo[f], np.full(L, -FREE_BOX), wlo[t], np.full(L, -FREE_BOX)], 1)
    hi = np.stack([whi[f], np.full(L, FREE_BOX), whi[t], np.full(L, FREE_BOX)], 1)
    phi, qhi = grid.pmax - x0.pg, grid.qmax - x0.qg
    glo = np.stack([np.minimum(grid.pmin - x0.pg, phi), np.minimum(grid.qmin - x0.qg, qhi)], 1)
    ghi = np.stack([phi, qhi], 1)
    pij, qij, pji, qji = acopf.flows(grid, x0.w, x0.wR, x0.wI)
    pdk = (grid.pd - np.bincount(grid.gbus, x0.pg, nb) + np.bincount(f, pij, nb) + np.bincount(t, pji, nb)
           + grid.gsh * x0.w)
    qdk = (grid.qd - np.bincount(grid.gbus, x0.qg, nb) + np.bincount(f, qij, nb) + np.bincount(t, qji, nb)
           - grid.bsh * x0.w)
    return M, F, lo, hi, glo, ghi, pdk, qdk


def admm_project(grid, x0: Iterate, rho: float, max_sweeps: int, eps_pri: float = 0.0,
                 eps_dual: float = 0.0) -> AdmmProjection:
    """Eq. linfeas by the sweeps of Algorithm 2 (cold start, every penalty
    rho) until ||r|| <= eps_pri and ||s|| <= eps_dual or max_sweeps."""
    from . import admm
    from .lineqp import solve_line_qps
    from types import SimpleNamespace
    M, F, lo, hi, glo, ghi, pdk, qdk = decomposed_data(grid, x0)
    G, L = grid.n_gen, grid.n_line
    R = admm.Rho.scalar(grid, rho)
    bus_qp = SimpleNamespace(bus=SimpleNamespace(pdk=pdk, qdk=qdk))
    # line matrix: the angle copies are not variables of the line problem
    rv = R.l[:, 4:].copy()
    rv[:, 1] = rv[:, 3] = 0.0
    Qm = M + np.einsum("lf,lfi,lfj->lij", R.l[:, :4], F, F) + np.einsum("li,ij->lij", rv, np.eye(4))
    st = admm.cold_state(grid)
    wri = np.zeros((L, 2))
    r = s = np.inf
    k = 0
    f, t = grid.f, grid.t
    for k in range(1, max_sweeps + 1):
        # generators: 0.5 d^2 + lam (d - xbar) + rho/2 (d - xbar)^2 on the box
        xg = (R.g * st.xbar_g - st.lam_g) / (1.0 + R.g)
        xg = np.minimum(np.maximum(xg, glo), ghi)
        # lines
        xbar_v = np.stack([st.dw[f], st.dth[f], st.dw[t], st.dth[t]], 1)
        c = np.einsum("lf,lfi->li", st.lam_l[:, :4] - R.l[:, :4] * st.xbar_f, F)
        c = c + np.stack([st.lam_l[:, 4] - R.l[:, 4] * xbar_v[:, 0], np.zeros(L),
                          st.lam_l[:, 6] - R.l[:, 6] * xbar_v[:, 2], np.zeros(L)], 1)
        Gz, hz = np.zeros((L, 2, 4)), np.ones((L, 2))
        z, _, _, feas = solve_line_qps(Qm, c, lo, hi, Gz, hz)
        assert feas.all()
        flows = np.einsum("lfi,li->lf", F, z)
        xl = np.concatenate([flows, np.stack([z[:, 0], np.zeros(L), z[:, 2], np.zeros(L)], 1)], 1)
        wri = z[:, [1, 3]]
        # buses, multipliers, residuals (as in admm.sweep)
        xbar_g, xbar_f, dw, dth, nu = admm.bus_update(grid, bus_qp, xg, xl, st, R)
        xbar_l = np.concatenate([xbar_f, np.stack([dw[f], dth[f], dw[t], dth[t]], 1)], 1)
        xbar_l_old = np.concatenate([st.xbar_f, xbar_v], 1)
        lam_g = st.lam_g + R.g * (xg - xbar_g)
        lam_l = st.lam_l + R.l * (xl - xbar_l)
        r = float(np.sqrt(np.sum((xg - xbar_g) ** 2) + np.sum((xl - xbar_l) ** 2)))
        s = float(np.sqrt(np.sum((R.g * (xbar_g - st.xbar_g)) ** 2) + np.sum((R.l * (xbar_l - xbar_l_old)) ** 2)))
        st = admm.AdmmState(xg, xbar_g, lam_g, xl, xbar_f, lam_l, dw, dth, np.zeros((L, 2)), nu)
        if r <= eps_pri and s <= eps_dual:
            break
    x = Iterate(x0.pg + st.xg[:, 0], x0.qg + st.xg[:, 1], x0.w + st.dw, x0.th + st.dth,
                x0.wR + wri[:, 0], x0.wI + wri[:, 1])
    return AdmmProjection(x, k, r, s, bool(r <= eps_pri and s <= eps_dual), st, wri[:, 0], wri[:, 1])
