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
