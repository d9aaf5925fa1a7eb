// Local solver of one line subproblem (Section IV-B2): the augmented
// Lagrangian method over the slack form (eqs. line_kernel_simp,
// line_kernel_simp1, line_kernel_alm) with a projected trust-region Newton
// method (TRON, Lin and More 1999) for its box-constrained subproblems:
//
//   minimise phi(z) = 0.5 z^T Q z + c^T z   s.t.  lo <= z <= hi,  g(z) = G z - h <= 0,
//
// for Q that need not be positive definite (the unmodified Hessian).  The
// slacks of g(z) + s = 0, s >= 0, are minimised out in closed form, which
// leaves the box-constrained piecewise quadratic
//
//   psi(z) = phi(z) + sum_r [max(0, g_r(z) + mu u_r)^2 - (mu u_r)^2] / (2 mu)
//
// with multipliers u >= 0 and penalty parameter mu.  Outer iterations
// (textbook bound-constrained Lagrangian schedule, on the dimensionless
// m = mu / mu_ref with mu_ref = gscale^2 / scale): solve psi to a
// projected-gradient tolerance omega; if the violation ||max(g, -mu u)||
// <= eta update u <- max(0, u + g / mu), eta <- eta m^0.9, omega <- omega m;
// otherwise m <- m / 10, eta <- 0.1 m^0.1, omega <- m; stop at violation
// and projected gradient <= 1e-9 (relative).  TRON step: Cauchy point by a
// projected search along -grad (halving from t = Delta / ||grad|| to the
// decrease q(s) <= 0.01 grad^T s), then up to four minor iterations of
// conjugate gradients on the variables strictly inside the box, each
// followed by a projected search; ratio test 1e-4, radius 0.25 ||s|| below
// a ratio of 0.25 and max(Delta, 2 ||s||) above 0.75.  On convex lines the
// result is the exact minimiser within the tolerances; on nonconvex ones a
// local minimiser.  All loops have fixed trip-count bounds and the arrays
// stay in registers.
#pragma once

#include "small_linalg.h"

namespace acopf {

struct LineAlmResult {
  double z[4];
  double u[2];    // multipliers (>= 0) of G z <= h
  int converged;
  int iterations;  // TRON iterations over all outer iterations
};

namespace alm {

constexpr double kTolFeas = 1e-9;
constexpr double kTolOpt = 1e-9;
constexpr double kM0 = 0.1;
constexpr int kMaxOuter = 30;
constexpr int kMaxInner = 50;

ACOPF_HD double proj1(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

ACOPF_HD double dot(const double a[4], const double b[4]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

ACOPF_HD double norm(const double a[4]) { return sqrt(dot(a, a)); }

ACOPF_HD void matvec(const double A[4][4], const double v[4], double out[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = A[i][0] * v[0] + A[i][1] * v[1] + A[i][2] * v[2] + A[i][3] * v[3];
}

struct Problem {
  double Q[4][4], c[4], lo[4], hi[4], G[2][4], h[2];
};

// psi(z + s) - psi(z) without subtracting the two values: s^T (Q z + c) +
// 0.5 s^T Q s + sum_r (a1 - a0)(a1 + a0) / (2 mu), a = max(0, g + mu u).
ACOPF_HD double psi_change(const Problem& P, const double z[4], const double s[4], const double u[2], double mu) {
  double Qz[4], Qs[4];
  matvec(P.Q, z, Qz);
  matvec(P.Q, s, Qs);
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) v += s[i] * (Qz[i] + P.c[i]);
  v += 0.5 * dot(s, Qs);
  double pen = 0.0;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const double g0 = dot(P.G[r], z) - P.h[r];
    const double gs = dot(P.G[r], s);
    const double a0 = fmax(0.0, g0 + mu * u[r]);
    const double a1 = fmax(0.0, g0 + gs + mu * u[r]);
    pen += (a1 - a0) * (a1 + a0);
  }
  return v + pen / (2.0 * mu);
}

ACOPF_HD void grad_hess(const Problem& P, const double z[4], const double u[2], double mu, double grad[4],
                        double B[4][4]) {
  matvec(P.Q, z, grad);
  double t[2], a[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const double g = dot(P.G[r], z) - P.h[r];
    t[r] = fmax(0.0, g + mu * u[r]);
    a[r] = (g + mu * u[r]) > 0.0 ? 1.0 : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    grad[i] += P.c[i] + (P.G[0][i] * t[0] + P.G[1][i] * t[1]) / mu;
#pragma unroll
    for (int j = 0; j < 4; ++j) B[i][j] = P.Q[i][j] + (a[0] * P.G[0][i] * P.G[0][j] + a[1] * P.G[1][i] * P.G[1][j]) / mu;
  }
}

ACOPF_HD double proj_grad_norm(const Problem& P, const double z[4], const double grad[4]) {
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double g = grad[i];
    g = (z[i] <= P.lo[i]) ? fmin(g, 0.0) : ((z[i] >= P.hi[i]) ? fmax(g, 0.0) : g);
    g = (P.lo[i] >= P.hi[i]) ? 0.0 : g;
    m = fmax(m, fabs(g));
  }
  return m;
}

ACOPF_HD double model(const double s[4], const double grad[4], const double B[4][4]) {
  double Bs[4];
  matvec(B, s, Bs);
  return dot(grad, s) + 0.5 * dot(s, Bs);
}

// Conjugate gradients for the model on the variables z + s leaves strictly
// inside the box, from s (see the file comment).
ACOPF_HD void cg_box(const Problem& P, const double s[4], const double z[4], const double grad[4],
                     const double B[4][4], double delta, double d[4]) {
  double fr[4], Bs[4];
  int nfree = 0;
  matvec(B, s, Bs);
  double r[4], p[4], w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double zc = z[i] + s[i];
    fr[i] = (zc > P.lo[i] && zc < P.hi[i]) ? 1.0 : 0.0;
    nfree += fr[i] != 0.0 ? 1 : 0;
    r[i] = -fr[i] * (grad[i] + Bs[i]);
    p[i] = r[i];
    w[i] = 0.0;
    d[i] = 0.0;
  }
  if (nfree == 0) return;
  double rr = dot(r, r);
  for (int it = 0; it < nfree; ++it) {
    if (rr <= 0.0) break;
    double Bp[4];
    matvec(B, p, Bp);
#pragma unroll
    for (int i = 0; i < 4; ++i) Bp[i] *= fr[i];
    const double curv = dot(p, Bp);
    double base[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) base[i] = s[i] + w[i];
    const double a2 = dot(p, p);
    const double b2 = 2.0 * dot(base, p);
    const double c2 = dot(base, base) - delta * delta;
    const double a_tr = (-b2 + sqrt(fmax(b2 * b2 - 4.0 * a2 * c2, 0.0))) / (2.0 * a2);
    if (curv <= 0.0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] += a_tr * p[i];
      break;
    }
    const double alpha = rr / curv;
    if (alpha >= a_tr) {
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] += a_tr * p[i];
      break;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      w[i] += alpha * p[i];
      r[i] -= alpha * Bp[i];
    }
    const double rr_new = dot(r, r);
#pragma unroll
    for (int i = 0; i < 4; ++i) p[i] = r[i] + (rr_new / rr) * p[i];
    rr = rr_new;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) d[i] = w[i];
}

// One TRON trial step from z.
ACOPF_HD void tron_step(const Problem& P, const double z[4], const double grad[4], const double B[4][4],
                        double delta, double s[4]) {
  const double gn = norm(grad);
#pragma unroll
  for (int i = 0; i < 4; ++i) s[i] = 0.0;
  if (gn == 0.0) return;
  double t = delta / gn;
#pragma unroll
  for (int i = 0; i < 4; ++i) s[i] = proj1(z[i] - t * grad[i], P.lo[i], P.hi[i]) - z[i];
  for (int k = 0; k < 60; ++k) {
    if (norm(s) <= delta * (1.0 + 1e-12) && model(s, grad, B) <= 0.01 * dot(grad, s)) break;
    t *= 0.5;
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = proj1(z[i] - t * grad[i], P.lo[i], P.hi[i]) - z[i];
  }
  for (int minor = 0; minor < 4; ++minor) {
    double d[4];
    cg_box(P, s, z, grad, B, delta, d);
    if (d[0] == 0.0 && d[1] == 0.0 && d[2] == 0.0 && d[3] == 0.0) break;
    const double qc = model(s, grad, B);
    double Bs[4], gq[4], zc[4];
    matvec(B, s, Bs);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      gq[i] = grad[i] + Bs[i];
      zc[i] = z[i] + s[i];
    }
    double beta = 1.0, sn[4];
    bool took = false;
    for (int k = 0; k < 30; ++k) {
      double ds[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        sn[i] = proj1(zc[i] + beta * d[i], P.lo[i], P.hi[i]) - z[i];
        ds[i] = sn[i] - s[i];
      }
      if (norm(sn) <= delta * (1.0 + 1e-12) && model(sn, grad, B) <= qc + 0.01 * fmin(0.0, dot(gq, ds))) {
        took = true;
        break;
      }
      beta *= 0.5;
    }
    if (!took) break;
    bool hit = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double v = zc[i] + beta * d[i];
      hit = hit || v < P.lo[i] || v > P.hi[i];
      s[i] = sn[i];
    }
    if (!hit) break;
  }
}

// Box-constrained minimisation of psi from z to projected gradient <= omega;
// returns the TRON iterations taken.
ACOPF_HD int tron(const Problem& P, double z[4], const double u[2], double mu, double omega, double delta,
                  int max_iter) {
#pragma unroll
  for (int i = 0; i < 4; ++i) z[i] = proj1(z[i], P.lo[i], P.hi[i]);
  double amax = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) amax = fmax(amax, fabs(P.lo[i]));
  double bmax = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) bmax = fmax(bmax, fabs(P.hi[i]));
  const double dmin = 1e-15 * (1.0 + (amax + bmax));
  for (int it = 1; it <= max_iter; ++it) {
    double grad[4], B[4][4];
    grad_hess(P, z, u, mu, grad, B);
    if (proj_grad_norm(P, z, grad) <= omega || delta < dmin) return it - 1;
    double s[4];
    tron_step(P, z, grad, B, delta, s);
    const double q = model(s, grad, B);
    const double rho = (q < 0.0) ? psi_change(P, z, s, u, mu) / q : -1.0;
    if (rho > 1e-4) {
#pragma unroll
      for (int i = 0; i < 4; ++i) z[i] = proj1(z[i] + s[i], P.lo[i], P.hi[i]);
    }
    const double sn = norm(s);
    if (rho < 0.25)
      delta = (sn > 0.0) ? 0.25 * sn : 0.25 * delta;
    else if (rho > 0.75)
      delta = fmax(delta, 2.0 * sn);
  }
  return max_iter;
}

}  // namespace alm

// ALM + TRON for one line subproblem from z0 and multipliers u0 (the
// previous sweep's solution), penalty m starting at 0.1.
ACOPF_HD LineAlmResult solve_line_alm(const double Qp[10], const double c[4], const double lo[4], const double hi[4],
                                      const double G[2][4], const double h[2], const double z0[4],
                                      const double u0[2]) {
  alm::Problem P;
  sym_unpack(Qp, P.Q);
  double qmax = 0.0, cmax = 0.0, zs = 1e-12, hmax = 0.0, gsum = 0.0, width = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    P.c[i] = c[i];
    P.lo[i] = lo[i];
    P.hi[i] = hi[i];
    P.G[0][i] = G[0][i];
    P.G[1][i] = G[1][i];
    cmax = fmax(cmax, fabs(c[i]));
    zs = fmax(zs, fmax(fabs(lo[i]), fabs(hi[i])));
    width = fmax(width, hi[i] - lo[i]);
#pragma unroll
    for (int j = 0; j < 4; ++j) qmax = fmax(qmax, fabs(P.Q[i][j]));
  }
  P.h[0] = h[0];
  P.h[1] = h[1];
  hmax = fmax(fabs(h[0]), fabs(h[1]));
  gsum = fmax(fabs(G[0][0]) + fabs(G[0][1]) + fabs(G[0][2]) + fabs(G[0][3]),
              fabs(G[1][0]) + fabs(G[1][1]) + fabs(G[1][2]) + fabs(G[1][3]));
  const double scale = 1.0 + qmax * zs + cmax;
  const double gscale = 1.0 + gsum * zs + hmax;
  const double mu_ref = gscale * gscale / scale;
  LineAlmResult res;
  double z[4] = {z0[0], z0[1], z0[2], z0[3]};
  double u[2] = {u0[0], u0[1]};
  double m = alm::kM0;
  double omega = m, eta = 0.1 * pow(m, 0.1);
  const double delta = width + 1e-12;
  int inner_total = 0;
  res.converged = 0;
  for (int outer = 1; outer <= alm::kMaxOuter; ++outer) {
    const double mu = m * mu_ref;
    inner_total += alm::tron(P, z, u, mu, fmax(omega, alm::kTolOpt) * scale, delta, alm::kMaxInner);
    double g[2], viol = 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      g[r] = alm::dot(P.G[r], z) - P.h[r];
      viol = fmax(viol, fabs(fmax(g[r], -mu * u[r])));
    }
    viol /= gscale;
    double grad[4], B[4][4];
    alm::grad_hess(P, z, u, mu, grad, B);
    const double pg = alm::proj_grad_norm(P, z, grad) / scale;
    if (viol <= alm::kTolFeas && pg <= alm::kTolOpt) {
      u[0] = fmax(0.0, u[0] + g[0] / mu);
      u[1] = fmax(0.0, u[1] + g[1] / mu);
      res.converged = 1;
      break;
    }
    if (viol <= eta) {
      u[0] = fmax(0.0, u[0] + g[0] / mu);
      u[1] = fmax(0.0, u[1] + g[1] / mu);
      eta *= pow(m, 0.9);
      omega *= m;
    } else {
      m *= 0.1;
      eta = 0.1 * pow(m, 0.1);
      omega = m;
    }
    omega = fmax(omega, alm::kTolOpt);
    eta = fmax(eta, alm::kTolFeas);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) res.z[i] = z[i];
  res.u[0] = u[0];
  res.u[1] = u[1];
  res.iterations = inner_total;
  return res;
}

}  // namespace acopf
