"""Direct solve of the eliminated QP subproblem (eq. QPsub with eq. elim).

After elimination the QP has one variable per generator output (d_pg, d_qg)
and per bus (d_w, d_th); line flows and the linearised line limits are
affine in the four bus variables of each line.  This module assembles that
sparse QP and solves it with a primal-dual interior-point method
(Mehrotra predictor-corrector, sparse KKT factorised by SuperLU), the
"direct sparse-KKT solve" that the ADMM limit is compared against.

    min 0.5 y^T P y + q^T y   s.t.  A y = b  (power balance),
                                   G y <= h  (line limits, boxes).

Variables with equal bounds (the reference angle) are substituted out.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class QPMatrices:
    P: sp.csr_matrix
    q: np.ndarray
    A: sp.csr_matrix
    b: np.ndarray
    Gl: sp.csr_matrix    # line-limit rows
    hl: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    const: float
    n_gen: int
    n_bus: int


@dataclass
class DirectSolution:
    y: np.ndarray        # (2G + 2B,)
    nu: np.ndarray       # (2B,) balance multipliers (P rows then Q rows)
    mu: np.ndarray       # (2L,) line-limit multipliers (>= 0), rows ordered (line, end)
    objective: float
    iterations: int
    kkt: dict


def var_index(grid):
    G, B = grid.n_gen, grid.n_bus
    return {"pg": np.arange(G), "qg": G + np.arange(G), "w": 2 * G + np.arange(B),
            "th": 2 * G + B + np.arange(B)}


def assemble(grid, qp) -> QPMatrices:
    G, B, L = grid.n_gen, grid.n_bus, grid.n_line
    ix = var_index(grid)
    n = 2 * G + 2 * B
    f, t = grid.f, grid.t
    zi = np.stack([ix["w"][f], ix["th"][f], ix["w"][t], ix["th"][t]], 1)  # (L, 4)
    Lq = qp.line
    # objective
    rows = [ix["pg"], ix["qg"]]
    cols = [ix["pg"], ix["qg"]]
    vals = [qp.gen.fpp, np.zeros(G) if qp.gen.fqq is None else qp.gen.fqq]
    for a in range(4):
        for b_ in range(4):
            rows.append(zi[:, a]); cols.append(zi[:, b_]); vals.append(Lq.M[:, a, b_])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    q = np.zeros(n)
    q[ix["pg"]] += qp.gen.fp
    if qp.gen.fq is not None:
        q[ix["qg"]] += qp.gen.fq
    np.add.at(q, zi.ravel(), Lq.q.ravel())
    const = float(Lq.c0.sum())
    # balance rows: P rows 0..B-1, Q rows B..2B-1
    r, c, v = [], [], []
    r += [grid.gbus, B + grid.gbus]; c += [ix["pg"], ix["qg"]]; v += [np.ones(G), np.ones(G)]
    for k, bus, off in ((0, f, 0), (1, f, B), (2, t, 0), (3, t, B)):
        for a in range(4):
            r.append(off + bus); c.append(zi[:, a]); v.append(-Lq.F[:, k, a])
    r += [np.arange(B), B + np.arange(B)]; c += [ix["w"], ix["w"]]; v += [-grid.gsh, grid.bsh]
    A = sp.coo_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))), shape=(2 * B, n)).tocsr()
    b = np.concatenate([qp.bus.pdk, qp.bus.qdk])
    b = b + np.concatenate([np.bincount(f, Lq.f0[:, 0], B) + np.bincount(t, Lq.f0[:, 2], B),
                            np.bincount(f, Lq.f0[:, 1], B) + np.bincount(t, Lq.f0[:, 3], B)])
    # line-limit rows
    r, c, v = [], [], []
    for e in range(2):
        for a in range(4):
            r.append(2 * np.arange(L) + e); c.append(zi[:, a]); v.append(Lq.G[:, e, a])
    Gl = sp.coo_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))), shape=(2 * L, n)).tocsr()
    hl = Lq.h.ravel()
    lo = np.concatenate([qp.gen.lo[:, 0], qp.gen.lo[:, 1], qp.bus.lo[:, 0], qp.bus.lo[:, 1]])
    hi = np.concatenate([qp.gen.hi[:, 0], qp.gen.hi[:, 1], qp.bus.hi[:, 0], qp.bus.hi[:, 1]])
    return QPMatrices(P, q, A, b, Gl, hl, lo, hi, const, G, B)


def objective_value(m: QPMatrices, y) -> float:
    return float(0.5 * y @ (m.P @ y) + m.q @ y + m.const)


def kkt_report(m: QPMatrices, y, nu, mu, zlo, zhi) -> dict:
    """Stationarity, primal, dual-sign and complementarity residuals."""
    gr = m.P @ y + m.q + m.A.T @ nu + m.Gl.T @ mu - zlo + zhi
    prim = max(np.abs(m.A @ y - m.b).max(initial=0),
               np.maximum(m.Gl @ y - m.hl, 0).max(initial=0),
               np.maximum(m.lo - y, 0).max(initial=0), np.maximum(y - m.hi, 0).max(initial=0))
    dual = max(np.maximum(-mu, 0).max(initial=0), np.maximum(-zlo, 0).max(initial=0),
               np.maximum(-zhi, 0).max(initial=0))
    comp = max(np.abs(mu * (m.Gl @ y - m.hl)).max(initial=0), np.abs(zlo * (y - m.lo)).max(initial=0),
               np.abs(zhi * (m.hi - y)).max(initial=0))
    return {"stationarity": float(np.abs(gr).max()), "primal": float(prim), "dual": float(dual),
            "complementarity": float(comp)}


def ipm(P, q, A, b, Gin, hin, tol: float = 1e-11, max_iter: int = 200):
    """Primal-dual interior point (Mehrotra predictor-corrector) for
    min 0.5 y^T P y + q^T y  s.t.  A y = b,  Gin y <= hin, with the KKT
    system factorised by SuperLU.  Returns (y, nu, z, iterations) with z >= 0
    the multipliers of the inequalities."""
    P, A, Gin = sp.csc_matrix(P), sp.csc_matrix(A), sp.csr_matrix(Gin)
    nf = P.shape[0]
    mi, me = Gin.shape[0], A.shape[0]
    y = np.zeros(nf)
    s = np.maximum(hin - Gin @ y, 1.0)
    z = np.ones(mi)
    nu = np.zeros(me)
    GT, AT = Gin.T.tocsr(), A.T.tocsr()
    scale = 1.0 + max(np.abs(q).max(initial=0), np.abs(b).max(initial=0), np.abs(hin).max(initial=0))
    it = 0
    for it in range(1, max_iter + 1):
        rd = P @ y + q + AT @ nu + GT @ z
        rp = A @ y - b
        ri = Gin @ y + s - hin
        mu_c = s @ z / mi
        if (np.abs(rd).max() <= tol * scale and np.abs(rp).max(initial=0) <= tol * scale
                and np.abs(ri).max() <= tol * scale and mu_c <= 1e-3 * tol * scale):
            break
        D = z / s
        H = (P + GT @ sp.diags(D) @ Gin + 1e-13 * sp.identity(nf)).tocsc()
        K = sp.bmat([[H, AT], [A, -1e-13 * sp.identity(me)]], format="csc")
        lu = spla.splu(K)

        def newton(rc):
            rhs1 = -rd - GT @ (D * ri) - GT @ (rc / s)
            sol = lu.solve(np.concatenate([rhs1, -rp]))
            dy, dnu = sol[:nf], sol[nf:]
            dz = D * (Gin @ dy + ri) + rc / s
            ds = (rc - s * dz) / z
            return dy, dnu, ds, dz

        def step_len(v, dv):
            neg = dv < 0
            return min(1.0, float(np.min(-v[neg] / dv[neg]))) if neg.any() else 1.0

        dy, dnu, ds, dz = newton(-s * z)
        a_aff = min(step_len(s, ds), step_len(z, dz))
        mu_aff = (s + a_aff * ds) @ (z + a_aff * dz) / mi
        sigma = (mu_aff / mu_c) ** 3
        rc = -s * z - ds * dz + sigma * mu_c
        dy, dnu, ds, dz = newton(rc)
        a = 0.99 * min(step_len(s, ds), step_len(z, dz))
        a = min(a, 1.0)
        y += a * dy
        nu += a * dnu
        s += a * ds
        z += a * dz
    return y, nu, z, it


def solve(grid, qp, tol: float = 1e-11, max_iter: int = 200) -> DirectSolution:
    m = assemble(grid, qp)
    n = m.P.shape[0]
    fixed = m.lo >= m.hi
    free = np.nonzero(~fixed)[0]
    yfix = np.where(fixed, m.hi, 0.0)
    # reduced problem in the free variables
    Pf = m.P[free][:, free].tocsc()
    qf = m.q[free] + (m.P @ yfix)[free]
    Af = m.A[:, free].tocsc()
    bf = m.b - m.A @ yfix
    nf = free.size
    I = sp.identity(nf, format="csr")
    Gin = sp.vstack([m.Gl[:, free], I, -I]).tocsr()
    hin = np.concatenate([m.hl - m.Gl @ yfix, m.hi[free], -m.lo[free]])
    y, nu, z, it = ipm(Pf, qf, Af, bf, Gin, hin, tol, max_iter)
    yfull = yfix.copy()
    yfull[free] = y
    nl = m.Gl.shape[0]
    mu = z[:nl]
    zhi = np.zeros(n)
    zlo = np.zeros(n)
    zhi[free] = z[nl:nl + nf]
    zlo[free] = z[nl + nf:]
    # multipliers of fixed variables absorb their stationarity residual
    grf = m.P @ yfull + m.q + m.A.T @ nu + m.Gl.T @ mu
    zlo[fixed] = np.maximum(grf[fixed], 0)
    zhi[fixed] = np.maximum(-grf[fixed], 0)
    rep = kkt_report(m, yfull, nu, mu, zlo, zhi)
    return DirectSolution(yfull, nu, mu, objective_value(m, yfull), it, rep)


def max_violation(grid, qp, y) -> float:
    """Largest violation of the constraints of the eliminated QP at y."""
    m = assemble(grid, qp)
    return float(max(np.abs(m.A @ y - m.b).max(initial=0),
                     np.maximum(m.Gl @ y - m.hl, 0).max(initial=0),
                     np.maximum(m.lo - y, 0).max(initial=0), np.maximum(y - m.hi, 0).max(initial=0)))
