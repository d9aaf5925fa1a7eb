"""Local line solver of the paper (Section IV-B2): augmented Lagrangian
method over the slack form (eqs. line_kernel_simp, line_kernel_simp1,
line_kernel_alm) with a projected trust-region Newton method for the
box-constrained subproblems (TRON, Lin and More 1999).

The line subproblem after the flow substitution is

    minimise phi(z) = 0.5 z^T Q z + c^T z   s.t.  lo <= z <= hi,  g(z) = G z - h <= 0,

where Q need not be positive definite (the unmodified Lagrangian Hessian).
With slacks s >= 0 for g(z) + s = 0 (eq. line_kernel_simp1) and the
penalised Lagrangian of eq. line_kernel_alm (multipliers u, penalty
parameter mu; the paper's formula is garbled, read here as
phi + u^T (g + s) + ||g + s||^2 / (2 mu)), minimising over s >= 0 in closed
form (s = max(0, -g - mu u)) leaves the box-constrained, continuously
differentiable, piecewise quadratic

    psi(z) = phi(z) + sum_r [max(0, g_r(z) + mu u_r)^2 - (mu u_r)^2] / (2 mu).

The paper defers the ALM's parameter updates to its reference [ALM3]; the
schedule here is the textbook bound-constrained Lagrangian method
(Nocedal and Wright, Algorithm 17.4, in the spirit of LANCELOT):
  * solve psi to a projected-gradient tolerance omega;
  * if the constraint violation ||max(g, -mu u)||_inf <= eta: update the
    multipliers u <- max(0, u + g / mu), tighten eta <- eta mu^0.9 and
    omega <- omega mu; otherwise decrease mu <- 0.1 mu and reset
    eta <- 0.1 mu^0.1, omega <- mu;
  * stop when the violation is <= tol_feas and the projected gradient of
    the last subproblem is <= tol_opt.
All tolerances are scaled by the size of the data (scale below).

TRON for psi on the box (one trust-region step per iteration):
  1. Cauchy step: projected search s(t) = P[z - t g] - z from t = Delta /
     ||g||, halving t until the model q(s) = g^T s + 0.5 s^T B s satisfies
     q(s) <= 0.01 g^T s (B the Hessian of psi at z: Q plus G_r^T G_r / mu
     for the rows with g_r + mu u_r > 0);
  2. subspace step: on the variables that the Cauchy point leaves strictly
     inside the box, conjugate gradients on the model (stopping at the trust
     region boundary or at negative curvature), followed by a projected
     search along the resulting direction with the same decrease rule;
  3. ratio test rho = (psi(z + s) - psi(z)) / q(s), the change of psi
     formed from s without subtracting the two values (which cancel near a
     minimiser whose psi is large): the step is taken if
     rho > 1e-4; Delta <- 0.25 ||s|| if rho < 0.25, Delta <- max(Delta,
     2 ||s||) if rho > 0.75; stop at a projected gradient <= omega.

This is an iteration, not a closed form: on convex lines it approaches the
unique minimiser (the exact solver's result), on nonconvex ones a local
minimiser.  Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np


@dataclass
class AlmParams:
    mu0: float = 0.1           # initial penalty parameter m (dimensionless, see solve_line)
    tol_feas: float = 1e-9     # constraint violation, relative
    tol_opt: float = 1e-9      # projected gradient, relative
    max_outer: int = 30
    max_inner: int = 50
    delta0: float = 1.0        # initial trust radius, relative to the box size


@dataclass
class AlmResult:
    z: np.ndarray
    u: np.ndarray      # multipliers (>= 0) of g(z) <= 0
    mu: float
    outer: int
    inner: int
    converged: bool


def _proj(z, lo, hi):
    return np.minimum(np.maximum(z, lo), hi)


def psi(z, Q, c, G, h, u, mu):
    g = G @ z - h
    t = np.maximum(0.0, g + mu * u)
    return 0.5 * z @ Q @ z + c @ z + float(np.sum(t * t - (mu * u) ** 2)) / (2.0 * mu)


def psi_change(z, s, Q, c, G, h, u, mu):
    """psi(z + s) - psi(z), in the algebraically equal form s^T (Q z + c) +
    0.5 s^T Q s + sum_r (a1_r - a0_r)(a1_r + a0_r) / (2 mu) with a =
    max(0, g + mu u): the difference of the two values themselves loses all
    its digits near a minimiser whose psi is large."""
    d_obj = float(s @ (Q @ z + c) + 0.5 * s @ Q @ s)
    a0 = np.maximum(0.0, G @ z - h + mu * u)
    a1 = np.maximum(0.0, G @ (z + s) - h + mu * u)
    return d_obj + float(np.sum((a1 - a0) * (a1 + a0))) / (2.0 * mu)


def psi_grad_hess(z, Q, c, G, h, u, mu):
    g = G @ z - h
    t = np.maximum(0.0, g + mu * u)
    grad = Q @ z + c + G.T @ t / mu
    act = (g + mu * u) > 0.0
    B = Q + (G[act].T @ G[act]) / mu
    return grad, B


def proj_grad_norm(z, grad, lo, hi):
    """Infinity norm of the projected gradient in gradient units: a
    component counts in full inside the box and only its descent-blocking
    sign at a bound (a bound's multiplier absorbs the other sign)."""
    pg = np.where(z <= lo, np.minimum(grad, 0.0), np.where(z >= hi, np.maximum(grad, 0.0), grad))
    pg = np.where(lo >= hi, 0.0, pg)
    return float(np.abs(pg).max())


def _model(s, grad, B):
    return float(grad @ s + 0.5 * s @ B @ s)


def _cg_box(s, z, grad, B, lo, hi, delta):
    """Conjugate gradients for the model on the variables that z + s leaves
    strictly inside the box (others fixed), from s; stops at the trust
    region boundary, at negative curvature or after as many steps as free
    variables.  Returns the direction d (zero on fixed variables)."""
    n = z.size
    zc = z + s
    free = (zc > lo) & (zc < hi)
    d = np.zeros(n)
    if not free.any():
        return d
    r = -(grad + B @ s)[free]
    BF = B[np.ix_(free, free)]
    w = np.zeros(int(free.sum()))
    p = r.copy()
    rr = float(r @ r)
    for _ in range(int(free.sum())):
        if rr <= 0.0:
            break
        Bp = BF @ p
        curv = float(p @ Bp)
        # largest alpha with ||s + w + alpha p|| <= delta
        base = s.copy()
        base[free] += w
        a2 = float(p @ p)
        b2 = 2.0 * float(base[free] @ p)
        c2 = float(base @ base) - delta * delta
        a_tr = (-b2 + np.sqrt(max(b2 * b2 - 4.0 * a2 * c2, 0.0))) / (2.0 * a2)
        if curv <= 0.0:
            w = w + a_tr * p       # negative curvature: to the boundary
            break
        alpha = rr / curv
        if alpha >= a_tr:
            w = w + a_tr * p
            break
        w = w + alpha * p
        r = r - alpha * Bp
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    d[free] = w
    return d


def tron_step(z, grad, B, lo, hi, delta):
    """One TRON trial step from z: the Cauchy step, then minor iterations
    (conjugate gradients on the free variables and a projected search along
    their direction) while they keep adding bounds, at most n of them."""
    n = z.size
    gn = float(np.linalg.norm(grad))
    if gn == 0.0:
        return np.zeros(n)
    # 1. Cauchy step by projected search
    t = delta / gn
    s = _proj(z - t * grad, lo, hi) - z
    for _ in range(60):
        if np.linalg.norm(s) <= delta * (1 + 1e-12) and _model(s, grad, B) <= 0.01 * float(grad @ s):
            break
        t *= 0.5
        s = _proj(z - t * grad, lo, hi) - z
    # 2. minor iterations on the free subspace
    for _ in range(n):
        d = _cg_box(s, z, grad, B, lo, hi, delta)
        if not d.any():
            break
        qc = _model(s, grad, B)
        gq = grad + B @ s
        zc = z + s
        beta, took = 1.0, False
        for _ in range(30):
            sn = _proj(zc + beta * d, lo, hi) - z
            if np.linalg.norm(sn) <= delta * (1 + 1e-12) and \
                    _model(sn, grad, B) <= qc + 0.01 * min(0.0, float(gq @ (sn - s))):
                took = True
                break
            beta *= 0.5
        if not took:
            break
        hit = np.any((zc + beta * d < lo) | (zc + beta * d > hi))
        s = sn
        if not hit:
            break
    return s


def tron(z0, Q, c, G, h, u, mu, lo, hi, omega, delta, max_iter):
    """Box-constrained minimisation of psi from z0 to projected gradient <= omega."""
    z = _proj(z0, lo, hi)
    dmin = 1e-15 * (1.0 + float(np.abs(lo).max() + np.abs(hi).max()))
    it = 0
    for it in range(1, max_iter + 1):
        grad, B = psi_grad_hess(z, Q, c, G, h, u, mu)
        if proj_grad_norm(z, grad, lo, hi) <= omega or delta < dmin:
            return z, it - 1, max(delta, dmin)
        s = tron_step(z, grad, B, lo, hi, delta)
        q = _model(s, grad, B)
        rho = psi_change(z, s, Q, c, G, h, u, mu) / q if q < 0 else -1.0
        if rho > 1e-4:
            z = _proj(z + s, lo, hi)
        sn = float(np.linalg.norm(s))
        if rho < 0.25:
            delta = 0.25 * sn if sn > 0 else 0.25 * delta
        elif rho > 0.75:
            delta = max(delta, 2.0 * sn)
    return z, it, delta


def solve_line(Q, c, lo, hi, G, h, z0=None, u0=None, mu0=None, p: AlmParams = AlmParams()) -> AlmResult:
    """ALM + TRON for one line subproblem (see the module docstring).  The
    penalty parameter is mu = m mu_ref with mu_ref = gscale^2 / scale (so a
    penalty of m = 1 weighs the rows like the objective) and the schedule
    runs on the dimensionless m."""
    zs = max(float(np.abs(lo).max()), float(np.abs(hi).max()), 1e-12)
    scale = 1.0 + float(np.abs(Q).max()) * zs + float(np.abs(c).max())
    gscale = 1.0 + float(np.abs(G).sum(1).max()) * zs + float(np.abs(h).max())
    mu_ref = gscale * gscale / scale
    z = _proj(np.zeros(4) if z0 is None else np.asarray(z0, float), lo, hi)
    u = np.zeros(2) if u0 is None else np.asarray(u0, float).copy()
    m = p.mu0 if mu0 is None else float(mu0) / mu_ref
    omega, eta = m, 0.1 * m ** 0.1
    delta = p.delta0 * float(np.max(hi - lo)) + 1e-12
    inner_total = 0
    for outer in range(1, p.max_outer + 1):
        mu = m * mu_ref
        # each subproblem starts with a fresh trust radius
        z, inner, _ = tron(z, Q, c, G, h, u, mu, lo, hi, max(omega, p.tol_opt) * scale, delta, p.max_inner)
        inner_total += inner
        g = G @ z - h
        viol = float(np.abs(np.maximum(g, -mu * u)).max()) / gscale
        grad, _ = psi_grad_hess(z, Q, c, G, h, u, mu)
        pg = proj_grad_norm(z, grad, lo, hi) / scale
        if viol <= p.tol_feas and pg <= p.tol_opt:
            u = np.maximum(0.0, u + g / mu)
            return AlmResult(z, u, mu, outer, inner_total, True)
        if viol <= eta:
            u = np.maximum(0.0, u + g / mu)
            eta, omega = eta * m ** 0.9, omega * m
        else:
            m *= 0.1
            eta, omega = 0.1 * m ** 0.1, m
        omega = max(omega, p.tol_opt)
        eta = max(eta, p.tol_feas)
    return AlmResult(z, u, m * mu_ref, p.max_outer, inner_total, False)
