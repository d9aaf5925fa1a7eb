"""Exact minimiser of the line subproblem (Section IV-B2, eq. line_kernel).

Once the flows are substituted, each line subproblem is a QP in the four
voltage copies z:

    minimise 0.5 z^T Q z + c^T z   s.t.  lo <= z <= hi,  G z <= h  (2 rows).

The paper solves it with an augmented Lagrangian and TRON (eq.
line_kernel_alm), an iterative local method whose limit is the minimiser.
With Q positive definite the minimiser is unique, and this module computes
it by brute force: for every face of the feasible polyhedron (each variable
free, at its lower bound or at its upper bound; each limit row inactive or
active) solve the equality-constrained QP on that face, and keep the
primal-feasible face solution of smallest objective.  The minimiser of a
convex QP is the minimiser over the affine hull of the smallest face that
contains it, so it is among the candidates.  Variables with lo == hi are
fixed.  Before enumerating, a line whose unconstrained minimiser is feasible
is answered directly (that point is then the minimiser).

Returns z, the multipliers mu >= 0 of the two limit rows and the face
multipliers of the bounds; lines without a feasible point are flagged.

``limit_relaxation`` gives the shift of the limit rows that the QP build
applies to a line whose box and rows have no common point (the paper's
ADMM keeps progressing on such QPs, Section V, because its augmented
Lagrangian line solver does not fail on them: it ends at the point of
least squared violation, ``min_violation``, and the shift reproduces that
limit for the exact solver).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import itertools
import numpy as np

FEAS_TOL = 1e-11
CHUNK = 128


def _face_masks():
    """All faces as masks over the 10 constraints (4 lower bounds, 4 upper
    bounds, 2 limit rows); a variable is free, at its lower or at its upper
    bound, each row inactive or active."""
    out = []
    for vs in itertools.product((0, 1, 2), repeat=4):      # 0 free, 1 lower, 2 upper
        for rs in itertools.product((0, 1), repeat=2):
            m = np.zeros(10, dtype=bool)
            for k in range(4):
                if vs[k] == 1:
                    m[k] = True
                elif vs[k] == 2:
                    m[4 + k] = True
            m[8], m[9] = rs
            out.append(m)
    return np.array(out)


FACES = _face_masks()   # (324, 10)


def _feasible(z, lo, hi, G, h, tol):
    sl = np.abs(lo) + np.abs(hi) + 1.0
    ok = np.all(z >= lo - tol * sl, axis=-1) & np.all(z <= hi + tol * sl, axis=-1)
    g = np.einsum("...rj,...j->...r", G, z)
    rs = np.abs(h) + np.einsum("...rj,...j->...r", np.abs(G), np.abs(z)) + 1.0
    return ok & np.all(g <= h + tol * rs, axis=-1)


RELAX_ABS = 1e-9   # rounding guard of the relaxation, per unit of the rows' scale


def min_max_violation(lo, hi, G, h):
    """t* = min over lo <= z <= hi of max_r (G_r z - h_r), per line.

    An LP in (z, t): minimise t subject to G_r z - h_r <= t and the box.
    Its feasible set has no line, so an optimal vertex exists, with five
    independent active constraints: either four bounds (z a vertex of the
    box) and a row, or three bounds and both rows (z on an edge of the box,
    where the two rows are equal).  Both kinds are enumerated (16 vertices,
    32 edges) and the smallest objective kept."""
    n = lo.shape[0]
    best = np.full(n, np.inf)
    corners = np.array(list(itertools.product((0, 1), repeat=4)), dtype=bool)   # (16, 4)
    for cb in corners:
        z = np.where(cb[None], hi, lo)
        best = np.minimum(best, np.max(np.einsum("nrj,nj->nr", G, z) - h, axis=1))
    dG = G[:, 0] - G[:, 1]
    dh = h[:, 0] - h[:, 1]
    for d in range(4):
        others = [e for e in range(4) if e != d]
        for cb in itertools.product((0, 1), repeat=3):
            z = lo.copy()
            for e, b in zip(others, cb):
                z[:, e] = hi[:, e] if b else lo[:, e]
            # rows equal: dG . z = dh, solved for z_d
            rest = sum(dG[:, e] * z[:, e] for e in others)
            ok = dG[:, d] != 0.0
            zd = np.where(ok, (dh - rest) / np.where(ok, dG[:, d], 1.0), 0.0)
            ok &= (zd >= lo[:, d]) & (zd <= hi[:, d])
            z[:, d] = zd
            t = np.max(np.einsum("nrj,nj->nr", G, z) - h, axis=1)
            best = np.where(ok, np.minimum(best, t), best)
    return best


def _segment_min(a, e, h):
    """min over t in [0, 1] of f(t) = 0.5 sum_r max(0, a_r + t e_r - h_r)^2
    (a, e, h of shape (..., 2)); returns (f_min, t_min).  f is convex and
    piecewise quadratic: its minimiser is an end point, a breakpoint
    a_r + t e_r = h_r, or the stationary point of one of its pieces (rows
    {0}, {1} or {0, 1} positive)."""
    b = a - h
    with np.errstate(divide="ignore", invalid="ignore"):
        cand = [np.zeros(b.shape[:-1]), np.ones(b.shape[:-1])]
        for r in range(2):
            cand.append(np.where(e[..., r] != 0.0, -b[..., r] / e[..., r], 0.0))      # breakpoint / piece {r}
        ee = (e * e).sum(-1)
        cand.append(np.where(ee > 0.0, -(b * e).sum(-1) / ee, 0.0))               # piece {0, 1}
    best_f = np.full(b.shape[:-1], np.inf)
    best_t = np.zeros(b.shape[:-1])
    for t in cand:
        t = np.clip(t, 0.0, 1.0)
        f = 0.5 * (np.maximum(b + t[..., None] * e, 0.0) ** 2).sum(-1)
        better = f < best_f
        best_f = np.where(better, f, best_f)
        best_t = np.where(better, t, best_t)
    return best_f, best_t


def min_violation(lo, hi, G, h):
    """v* = (G z* - h)^+ for z* minimising 0.5 ||(G z - h)^+||^2 over the box,
    per line (the violation the paper's augmented Lagrangian line solver
    drives its iterates to when the box and the rows have no common point:
    its subproblems' penalty terms weigh this sum of squares with a penalty
    parameter that goes to zero).  v* is unique, z* need not be.

    The objective depends on z only through y = G z, which ranges over the
    polygon Z = G [lo, hi] (the convex hull of the 16 images of the box
    vertices).  When the minimum is positive it lies on the boundary of Z
    (in the interior a move against the gradient (y - h)^+ would still
    decrease it); every edge of Z is a segment between two of the 16
    images, all of which lie in Z, so the minimum over the 120 segments is
    the minimum over Z.  Lines whose box and rows intersect (min_max_violation
    <= 0) get v* = 0."""
    n = lo.shape[0]
    corners = np.array(list(itertools.product((0, 1), repeat=4)), dtype=bool)   # (16, 4)
    pts = np.stack([np.einsum("nrj,nj->nr", G, np.where(cb[None], hi, lo)) for cb in corners], 1)  # (n, 16, 2)
    best_f = np.full(n, np.inf)
    best_y = np.zeros((n, 2))
    for i, j in itertools.combinations(range(16), 2):
        a, e = pts[:, i], pts[:, j] - pts[:, i]
        f, t = _segment_min(a, e, h)
        better = f < best_f
        best_f = np.where(better, f, best_f)
        best_y = np.where(better[:, None], a + t[:, None] * e, best_y)
    v = np.maximum(best_y - h, 0.0)
    return np.where((min_max_violation(lo, hi, G, h) > 0.0)[:, None], v, 0.0)


def relax_guard(lo, hi, G, h):
    """RELAX_ABS times the scale of the rows' terms, 1 + |h_0| + |h_1| +
    sum_j (|G_0j| + |G_1j|) max(|lo_j|, |hi_j|): a bound on the rounding
    error of v* many times over."""
    zmax = np.maximum(np.abs(lo), np.abs(hi))
    return RELAX_ABS * (1.0 + np.abs(h).sum(1) + np.einsum("nrj,nj->n", np.abs(G), zmax))


def limit_relaxation(lo, hi, G, h):
    """Shift (n, 2) added to the limit rows of each line: 0 when the box and
    the rows G z <= h have a common point, else v* (``min_violation``) plus
    the rounding guard on both rows.  The QP on the relaxed rows then has as
    its minimiser the limit of the paper's augmented Lagrangian line solver
    (the minimiser over the points of least violation), up to the guard."""
    v = min_violation(lo, hi, G, h)
    infeasible = (v > 0.0).any(1)
    return np.where(infeasible[:, None], v + relax_guard(lo, hi, G, h)[:, None], 0.0)


def solve_line_qps(Q, c, lo, hi, G, h, tol: float = FEAS_TOL):
    """Vectorised over lines: Q (n,4,4) PD, c (n,4), lo/hi (n,4), G (n,2,4), h (n,2).

    Returns (z, mu, bound_mult, feasible) with mu (n,2) >= 0 the multipliers
    of G z <= h and bound_mult (n,4) the signed multipliers of the active
    bounds (Q z + c + mu^T G + bound_mult = 0)."""
    n = Q.shape[0]
    fixed = lo >= hi
    z_best = np.zeros((n, 4))
    mu_best = np.zeros((n, 2))
    bm_best = np.zeros((n, 4))
    feasible = np.ones(n, dtype=bool)

    # unconstrained minimiser (only when no variable is fixed)
    zu = -np.linalg.solve(Q, c[:, :, None])[:, :, 0]
    ok = _feasible(zu, lo, hi, G, h, tol) & ~fixed.any(1)
    z_best[ok] = zu[ok]
    todo = np.nonzero(~ok)[0]
    if todo.size == 0:
        return z_best, mu_best, bm_best, feasible

    for i0 in range(0, todo.size, CHUNK):
        sel = todo[i0:i0 + CHUNK]
        z_best[sel], mu_best[sel], bm_best[sel], feasible[sel] = _enumerate(
            Q[sel], c[sel], lo[sel], hi[sel], G[sel], h[sel], fixed[sel], tol)
    return z_best, mu_best, bm_best, feasible


def _enumerate(Q, c, lo, hi, G, h, fx, tol):
    m = Q.shape[0]
    nf = FACES.shape[0]
    # a fixed variable is only enumerated with its lower bound active
    valid = np.ones((m, nf), dtype=bool)
    for k in range(4):
        valid &= ~(fx[:, k][:, None] & ~FACES[None, :, k])
        valid &= ~(fx[:, k][:, None] & FACES[None, :, 4 + k])
    act = np.broadcast_to(FACES, (m, nf, 10)) & valid[:, :, None]
    # constraint normals N (10 x 4) as equalities N z = r: z_k = lo_k, z_k = hi_k, G_r z = h_r
    N = np.zeros((m, 10, 4))
    N[:, :4, :] = np.eye(4)
    N[:, 4:8, :] = np.eye(4)
    N[:, 8:, :] = G
    r = np.concatenate([lo, hi, h], 1)
    # KKT of each face in one padded 14x14 system; inactive constraints get an
    # identity row so their multiplier is 0
    K = np.zeros((m, nf, 14, 14))
    K[:, :, :4, :4] = Q[:, None]
    a = act[..., None]                                        # (m, nf, 10, 1)
    Nb = np.broadcast_to(N[:, None], (m, nf, 10, 4))
    K[:, :, 4:, :4] = np.where(a, Nb, 0.0)
    K[:, :, :4, 4:] = np.swapaxes(K[:, :, 4:, :4], 2, 3)
    eye10 = np.eye(10)[None, None]
    K[:, :, 4:, 4:] = np.where(act[:, :, :, None], 0.0, eye10)
    rhs = np.zeros((m, nf, 14))
    rhs[:, :, :4] = -c[:, None]
    rhs[:, :, 4:] = np.where(act, r[:, None], 0.0)
    # a face whose active constraint normals are linearly dependent has a
    # singular KKT matrix: test the Gram determinant of the unit normals
    Nn = N / np.linalg.norm(N, axis=2, keepdims=True)
    gram = np.einsum("mik,mjk->mij", Nn, Nn)
    both = act[:, :, :, None] & act[:, :, None, :]
    gm = np.where(both, gram[:, None], np.eye(10)[None, None])
    good = valid & (act.sum(2) <= 4) & (np.linalg.det(gm) > 1e-12)
    K = np.where(good[..., None, None], K, np.eye(14)[None, None])
    sol = np.linalg.solve(K, rhs[..., None])[..., 0]
    z = sol[..., :4]
    feas = good & _feasible(z, lo[:, None], hi[:, None], G[:, None], h[:, None], tol)
    obj = 0.5 * np.einsum("lfi,lij,lfj->lf", z, Q, z) + np.einsum("li,lfi->lf", c, z)
    obj = np.where(feas, obj, np.inf)
    best = np.argmin(obj, axis=1)
    rows = np.arange(m)
    has = np.isfinite(obj[rows, best])
    nu = sol[rows, best, 4:]
    # lower-bound multipliers enter as -mult, upper as +mult in Q z + c + ... = 0
    return z[rows, best], nu[:, 8:], nu[:, 4:8] + nu[:, :4], has
