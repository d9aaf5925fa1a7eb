// Exact solver for one line subproblem (Section IV-B2, eq. line_kernel):
//
//   minimise 0.5 z^T Q z + c^T z   s.t.  lo <= z <= hi,   G z <= h (2 rows),
//
// with Q symmetric positive definite, given its inverse P = Q^{-1}.  The
// paper solves this problem with an augmented Lagrangian and TRON; its limit
// is the unique minimiser, which this routine computes exactly:
//
//  1. warm start: the working set that was optimal in the previous ADMM
//     sweep is tried first; its equality-constrained minimiser is accepted
//     when it satisfies every constraint and its multipliers are
//     non-negative (the KKT conditions, which certify the minimiser of a
//     strictly convex QP).  Between sweeps the working set rarely changes.
//     Otherwise a primal-dual guess (that set without its constraints of
//     negative multiplier, plus the constraints its minimiser violates) is
//     checked the same way; it settles most working-set changes.
//  2. otherwise the dual active-set method of Goldfarb and Idnani (Math.
//     Programming 27, 1983) runs: add the most violated constraint, take the
//     primal/dual step that keeps the active multipliers non-negative
//     (dropping a constraint whose multiplier reaches zero), until no
//     constraint is violated.  It starts from the previous working set when
//     that set's multipliers are non-negative (a valid state of the method),
//     else from the unconstrained minimiser with an empty working set.
//
// Constraints are numbered 0-3 (lower bounds of z_0..z_3), 4-7 (upper
// bounds) and 8-9 (the two rows), written as n_k . z >= b_k.  The working
// set never holds more than four linearly independent constraints.  All
// loops have fixed trip counts so the arrays stay in registers.
#pragma once

#include "small_linalg.h"

namespace acopf {

struct LineQPResult {
  double z[4];
  double mu[2];   // multipliers (>= 0) of the rows G z <= h
  int status;     // 0 solved, 1 infeasible, 2 iteration cap
  int mask;       // bit k set: constraint k in the optimal working set
};

ACOPF_HD double dot4(const double a[4], const double b[4]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

ACOPF_HD void matvec4(const double P[4][4], const double v[4], double out[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = P[i][0] * v[0] + P[i][1] * v[1] + P[i][2] * v[2] + P[i][3] * v[3];
}

// Normal and right-hand side of constraint k (n_k . z >= b_k).
ACOPF_HD void gi_constraint(int k, const double G[2][4], const double lo[4], const double hi[4],
                            const double h[2], double n[4], double& b) {
  const bool row = k >= 8;
  const int r = k - 8;
  const int v = k & 3;
  const double sgn = (k < 4) ? 1.0 : -1.0;
#pragma unroll
  for (int d = 0; d < 4; ++d) n[d] = row ? -(r == 0 ? G[0][d] : G[1][d]) : ((d == v) ? sgn : 0.0);
  b = row ? -(r == 0 ? h[0] : h[1]) : ((k < 4) ? lo[v] : -hi[v]);
}

// Solve S y = rhs for the q x q leading block of S (symmetric positive
// definite, lower triangle read), padded to 4x4 with the identity: LDL^T
// without square roots (E = L D is kept beside L).
ACOPF_HD void spd_solve_padded(const double S[4][4], int q, const double rhs[4], double y[4]) {
  double L[4][4], E[4][4], dinv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double d = (j < q) ? S[j][j] : 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < j) d -= L[j][k] * E[j][k];
    dinv[j] = 1.0 / fmax(d, 1e-300);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i > j) {
        double e = (i < q && j < q) ? S[i][j] : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < j) e -= L[i][k] * E[j][k];
        E[i][j] = e;
        L[i][j] = e * dinv[j];
      }
    }
  }
  double t[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s = (i < q) ? rhs[i] : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < i) s -= L[i][k] * t[k];
    t[i] = s;
  }
#pragma unroll
  for (int ii = 0; ii < 4; ++ii) {
    const int i = 3 - ii;
    double s = t[i] * dinv[i];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k > i) s -= L[k][i] * y[k];
    y[i] = s;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) y[a] = (a < q) ? y[a] : 0.0;
}

// Working-set products: W[:, j] = P N_j and the lower triangle of
// S = N^T P N (padded).
ACOPF_HD void gi_products(const double P[4][4], const double N[4][4], int q, double W[4][4], double S[4][4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double t[4];
    matvec4(P, N[j], t);
#pragma unroll
    for (int i = 0; i < 4; ++i) W[i][j] = (j < q) ? t[i] : 0.0;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (b <= a) S[a][b] = N[a][0] * W[0][b] + N[a][1] * W[1][b] + N[a][2] * W[2][b] + N[a][3] * W[3][b];
}

// Most violated constraint outside the working set at z (scaled by the
// constraint's 1-norm gn, ign = 1 / gn or 0); -1 if none is violated beyond
// the tolerance.
ACOPF_HD int gi_most_violated(const double z[4], int mask, const double lo[4], const double hi[4],
                              const double G[2][4], const double h[2], const double gn[2], const double ign[2]) {
  const double zs = fabs(z[0]) + fabs(z[1]) + fabs(z[2]) + fabs(z[3]);
  int p = -1;
  double worst = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double sl = z[k] - lo[k];
    const bool vl = !((mask >> k) & 1) && sl < -1e-12 * (1.0 + fabs(lo[k]) + zs) && sl < worst;
    worst = vl ? sl : worst;
    p = vl ? k : p;
    const double su = hi[k] - z[k];
    const bool vu = !((mask >> (k + 4)) & 1) && su < -1e-12 * (1.0 + fabs(hi[k]) + zs) && su < worst;
    worst = vu ? su : worst;
    p = vu ? k + 4 : p;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const double gz = G[r][0] * z[0] + G[r][1] * z[1] + G[r][2] * z[2] + G[r][3] * z[3];
    const double s = h[r] - gz;
    const double sc = s * ign[r];
    const bool v = gn[r] > 0.0 && !((mask >> (8 + r)) & 1) && s < -1e-12 * (1.0 + fabs(h[r]) + gn[r] * zs) &&
                   sc < worst;
    worst = v ? sc : worst;
    p = v ? 8 + r : p;
  }
  return p;
}

// KKT check of a working set (warm start), in the variables' own
// coordinates: an active bound fixes its variable (t_v = +1 lower, -1
// upper, 0 free), an active row enters through v_r = P G_r^T.  The
// multipliers y solve the 6x6 Schur system (N P N^T) y = b - N zu with the
// inactive entries replaced by identity rows, so no branch or register
// placement depends on which constraints are active; LDL^T without
// pivoting (the system is positive definite).  Returns true, with the
// minimiser z and the rows' multipliers, if the working set is optimal.
//
// dual_ok reports whether the working set is at least dual feasible (its
// minimiser exists, its multipliers y, by variable then row, are all
// non-negative and its constraints hold): the dual active-set method may
// then continue from it instead of starting over.
ACOPF_HD bool warm_check(const double P[4][4], const double zu[4], const double lo[4], const double hi[4],
                         const double G[2][4], const double h[2], const double gn[2], const double ign[2],
                         int warm_mask, double cs, double z[4], double mu[2], double y[6], bool& dual_ok) {
  double t[4], a[4], beta[4], ar[2];
  bool ok = (warm_mask & (warm_mask >> 4) & 0xF) == 0;  // a lower and an upper bound of one variable
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const bool lower = (warm_mask >> v) & 1, upper = (warm_mask >> (v + 4)) & 1;
    a[v] = (lower || upper) ? 1.0 : 0.0;
    t[v] = lower ? 1.0 : (upper ? -1.0 : 0.0);
    beta[v] = lower ? lo[v] : hi[v];
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) ar[r] = ((warm_mask >> (8 + r)) & 1) ? 1.0 : 0.0;
  double vr[2][4];
  matvec4(P, G[0], vr[0]);
  matvec4(P, G[1], vr[1]);
  // lower triangle of the Schur system and its right-hand side
  double S[6][6], rhs[6];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j <= i) S[i][j] = t[i] * t[j] * P[i][j] + ((i == j) ? 1.0 - a[i] : 0.0);
    rhs[i] = t[i] * (beta[i] - zu[i]);
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
#pragma unroll
    for (int j = 0; j < 4; ++j) S[4 + r][j] = -ar[r] * t[j] * vr[r][j];
#pragma unroll
    for (int r2 = 0; r2 < 2; ++r2)
      if (r2 <= r) S[4 + r][4 + r2] = ar[r] * ar[r2] * dot4(G[r], vr[r2]) + ((r == r2) ? 1.0 - ar[r] : 0.0);
    rhs[4 + r] = ar[r] * (dot4(G[r], zu) - h[r]);
  }
  // LDL^T: S = L D L^T with unit lower triangular L
  double L[6][6], D[6], dinv[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double d = S[j][j];
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k < j) d -= L[j][k] * L[j][k] * D[k];
    D[j] = d;
    ok = ok && d > 0.0;
    dinv[j] = 1.0 / d;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (i > j) {
        double s = S[i][j];
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (k < j) s -= L[i][k] * L[j][k] * D[k];
        L[i][j] = s * dinv[j];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = rhs[i];
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k < i) s -= L[i][k] * y[k];
    y[i] = s;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) y[i] *= dinv[i];
#pragma unroll
  for (int ii = 0; ii < 6; ++ii) {
    const int i = 5 - ii;
    double s = y[i];
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k > i) s -= L[k][i] * y[k];
    y[i] = s;
  }
  // minimiser of the working set: z = zu + P N^T y
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double zi = zu[i] - ar[0] * y[4] * vr[0][i] - ar[1] * y[5] * vr[1][i];
#pragma unroll
    for (int v = 0; v < 4; ++v) zi += t[v] * y[v] * P[i][v];
    z[i] = zi;
  }
  // KKT: non-negative multipliers (free sign for a bound of a fixed
  // variable), active constraints met, every other constraint satisfied
  bool strict = ok;  // every multiplier non-negative, no exception
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const bool fixed_var = lo[v] >= hi[v];
    const bool met = a[v] == 0.0 || fabs(z[v] - beta[v]) <= 1e-9 * (1.0 + fabs(beta[v]));
    ok = ok && (a[v] == 0.0 || fixed_var || y[v] >= -1e-10 * cs) && met;
    strict = strict && (a[v] == 0.0 || y[v] >= 0.0) && met;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const bool met = ar[r] == 0.0 || fabs(dot4(G[r], z) - h[r]) <= 1e-9 * (1.0 + fabs(h[r]));
    ok = ok && (ar[r] == 0.0 || y[4 + r] >= -1e-10 * cs) && met;
    strict = strict && (ar[r] == 0.0 || y[4 + r] >= 0.0) && met;
    mu[r] = ar[r] * y[4 + r];
  }
  dual_ok = strict;
  ok = ok && gi_most_violated(z, warm_mask, lo, hi, G, h, gn, ign) < 0;
  return ok;
}

// Primal-dual guess of the optimal working set from a working set `mask`,
// its minimiser z and its multipliers y (by variable, then row, as
// warm_check returns them): the active constraints with a negative
// multiplier are dropped (a fixed variable keeps its bound) and the
// constraints z violates are added (a violated bound replaces the opposite
// bound of its variable).
ACOPF_HD int pd_guess(int mask, const double z[4], const double y[6], const double lo[4], const double hi[4],
                      const double G[2][4], const double h[2], const double gn[2]) {
  int m = mask;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const bool drop = y[v] < 0.0 && !(lo[v] >= hi[v]);
    m = drop ? (m & ~((1 << v) | (1 << (v + 4)))) : m;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) m = (y[4 + r] < 0.0) ? (m & ~(1 << (8 + r))) : m;
  const double zs = fabs(z[0]) + fabs(z[1]) + fabs(z[2]) + fabs(z[3]);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const bool below = z[v] - lo[v] < -1e-12 * (1.0 + fabs(lo[v]) + zs);
    const bool above = hi[v] - z[v] < -1e-12 * (1.0 + fabs(hi[v]) + zs);
    m = below ? ((m | (1 << v)) & ~(1 << (v + 4))) : m;
    m = above ? ((m | (1 << (v + 4))) & ~(1 << v)) : m;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const double gz = G[r][0] * z[0] + G[r][1] * z[1] + G[r][2] * z[2] + G[r][3] * z[3];
    const bool viol = gn[r] > 0.0 && h[r] - gz < -1e-12 * (1.0 + fabs(h[r]) + gn[r] * zs);
    m = viol ? (m | (1 << (8 + r))) : m;
  }
  return m;
}

// Quantities every check starts from (as at the start of solve_line_qp): P
// unpacked, the rows' 1-norms, the unconstrained minimiser zu = -P c and the
// scale of c.
ACOPF_HD void line_qp_start(const double Pp[10], const double c[4], const double G[2][4], double P[4][4],
                            double gn[2], double zu[4], double& cs) {
  sym_unpack(Pp, P);
  gn[0] = fabs(G[0][0]) + fabs(G[0][1]) + fabs(G[0][2]) + fabs(G[0][3]);
  gn[1] = fabs(G[1][0]) + fabs(G[1][1]) + fabs(G[1][2]) + fabs(G[1][3]);
  matvec4(P, c, zu);
#pragma unroll
  for (int i = 0; i < 4; ++i) zu[i] = -zu[i];
  cs = 1.0 + fabs(c[0]) + fabs(c[1]) + fabs(c[2]) + fabs(c[3]);
}

// Steps 1 and 1b alone (no dual active-set method): true, with the result,
// when the warm set or the primal-dual guess is optimal (or, with no warm
// set, the unconstrained minimiser is feasible); otherwise false, with
// `base` the last working set checked.  solve_line_qp repeats these checks
// before its dual method (same result bits).
ACOPF_HD bool solve_line_qp_fast(const double Pp[10], const double c[4], const double lo[4], const double hi[4],
                                 const double G[2][4], const double h[2], int warm_mask, LineQPResult& res,
                                 int& base) {
  double P[4][4], gn[2], zu[4], cs;
  line_qp_start(Pp, c, G, P, gn, zu, cs);
  const double ign[2] = {gn[0] > 0.0 ? 1.0 / gn[0] : 0.0, gn[1] > 0.0 ? 1.0 / gn[1] : 0.0};
  base = warm_mask;
  double zg[4] = {zu[0], zu[1], zu[2], zu[3]}, yg[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (warm_mask != 0 && __builtin_popcount(warm_mask) <= 4) {
    double zw[4], muw[2];
    bool dual_ok = false;
    if (warm_check(P, zu, lo, hi, G, h, gn, ign, warm_mask, cs, zw, muw, yg, dual_ok)) {
#pragma unroll
      for (int i = 0; i < 4; ++i) res.z[i] = fmin(fmax(zw[i], lo[i]), hi[i]);
      res.mu[0] = muw[0];
      res.mu[1] = muw[1];
      res.status = 0;
      res.mask = warm_mask;
      return true;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) zg[i] = zw[i];
  } else if (warm_mask == 0) {
    if (gi_most_violated(zu, 0, lo, hi, G, h, gn, ign) < 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) res.z[i] = fmin(fmax(zu[i], lo[i]), hi[i]);
      res.mu[0] = 0.0;
      res.mu[1] = 0.0;
      res.status = 0;
      res.mask = 0;
      return true;
    }
  } else {
    return false;
  }
  const int m1 = pd_guess(warm_mask, zg, yg, lo, hi, G, h, gn);
  if (m1 == warm_mask || __builtin_popcount(m1) > 4) return false;
  base = m1;
  double z1[4], mu1[2], y1[6];
  bool d1 = false;
  if (!warm_check(P, zu, lo, hi, G, h, gn, ign, m1, cs, z1, mu1, y1, d1)) return false;
#pragma unroll
  for (int i = 0; i < 4; ++i) res.z[i] = fmin(fmax(z1[i], lo[i]), hi[i]);
  res.mu[0] = mu1[0];
  res.mu[1] = mu1[1];
  res.status = 0;
  res.mask = m1;
  return true;
}

// Neighbour `idx` of working set `base` for a search by many threads at
// once: idx 0-9 toggle one constraint, idx 10-54 toggle a pair (a bound
// that is added replaces the opposite bound of its variable); -1 when idx
// is out of range or the set would hold more than four constraints.
ACOPF_HD int neighbour_mask(int base, int idx) {
  if (idx < 0 || idx >= 55) return -1;
  int a = idx, b = -1;
  if (idx >= 10) {
    int p = idx - 10, i = 0;
    while (p >= 9 - i) {
      p -= 9 - i;
      ++i;
    }
    a = i;
    b = i + 1 + p;
  }
  int m = base;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int k = (t == 0) ? a : b;
    if (k < 0) continue;
    if ((m >> k) & 1) {
      m &= ~(1 << k);
    } else {
      m |= 1 << k;
      if (k < 8) m &= ~(1 << (k < 4 ? k + 4 : k - 4));
    }
  }
  return __builtin_popcount(m) <= 4 ? m : -1;
}

// KKT check of working set `mask` for the subproblem (Pp, c, lo, hi, G, h):
// true, with the result, if the set is optimal.
ACOPF_HD bool check_working_set(const double Pp[10], const double c[4], const double lo[4], const double hi[4],
                                const double G[2][4], const double h[2], int mask, LineQPResult& res) {
  double P[4][4], gn[2], zu[4], cs;
  line_qp_start(Pp, c, G, P, gn, zu, cs);
  const double ign[2] = {gn[0] > 0.0 ? 1.0 / gn[0] : 0.0, gn[1] > 0.0 ? 1.0 / gn[1] : 0.0};
  double z[4], mu[2], y[6];
  bool d = false;
  if (!warm_check(P, zu, lo, hi, G, h, gn, ign, mask, cs, z, mu, y, d)) return false;
#pragma unroll
  for (int i = 0; i < 4; ++i) res.z[i] = fmin(fmax(z[i], lo[i]), hi[i]);
  res.mu[0] = mu[0];
  res.mu[1] = mu[1];
  res.status = 0;
  res.mask = mask;
  return true;
}

ACOPF_HD LineQPResult solve_line_qp(const double Pp[10], const double c[4], const double lo[4],
                                    const double hi[4], const double G[2][4], const double h[2],
                                    int warm_mask) {
  const double INF = 1e300;
  const int MAX_STEPS = 48;
  double P[4][4];
  sym_unpack(Pp, P);
  const double gn[2] = {fabs(G[0][0]) + fabs(G[0][1]) + fabs(G[0][2]) + fabs(G[0][3]),
                        fabs(G[1][0]) + fabs(G[1][1]) + fabs(G[1][2]) + fabs(G[1][3])};
  const double ign[2] = {gn[0] > 0.0 ? 1.0 / gn[0] : 0.0, gn[1] > 0.0 ? 1.0 / gn[1] : 0.0};
  double zu[4];
  matvec4(P, c, zu);
#pragma unroll
  for (int i = 0; i < 4; ++i) zu[i] = -zu[i];
  const double cs = 1.0 + fabs(c[0]) + fabs(c[1]) + fabs(c[2]) + fabs(c[3]);

  LineQPResult res;
  double z[4] = {zu[0], zu[1], zu[2], zu[3]};
  int act[4] = {-1, -1, -1, -1};
  double N[4][4], u[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int d = 0; d < 4; ++d) N[j][d] = 0.0;
  int q = 0, mask = 0, status = 0;
  bool done = false;

  // 1. warm start from the previous working set
  double zg[4] = {zu[0], zu[1], zu[2], zu[3]}, yg[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  bool try_guess = false;
  if (warm_mask != 0 && __builtin_popcount(warm_mask) <= 4) {
    double zw[4], muw[2], yw[6];
    bool dual_ok = false;
    if (warm_check(P, zu, lo, hi, G, h, gn, ign, warm_mask, cs, zw, muw, yw, dual_ok)) {
#pragma unroll
      for (int i = 0; i < 4; ++i) res.z[i] = fmin(fmax(zw[i], lo[i]), hi[i]);
      res.mu[0] = muw[0];
      res.mu[1] = muw[1];
      res.status = 0;
      res.mask = warm_mask;
      return res;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) zg[i] = zw[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) yg[i] = yw[i];
    try_guess = true;
    if (dual_ok) {
      // The working set's minimiser with non-negative multipliers is a valid
      // state of the dual active-set method: continue from it (it then only
      // adds the constraints it violates) instead of starting over.
      int qq = 0;
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        if ((warm_mask >> k) & 1) {
          double n[4], bk;
          gi_constraint(k, G, lo, hi, h, n, bk);
          const double uk = (k < 8) ? yw[k & 3] : yw[4 + (k - 8)];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const bool here = (j == qq);
            act[j] = here ? k : act[j];
            u[j] = here ? uk : u[j];
#pragma unroll
            for (int d = 0; d < 4; ++d) N[j][d] = here ? n[d] : N[j][d];
          }
          qq += 1;
        }
      }
      q = qq;
      mask = warm_mask;
#pragma unroll
      for (int i = 0; i < 4; ++i) z[i] = zw[i];
    }
  } else if (warm_mask == 0) {
    try_guess = gi_most_violated(zu, 0, lo, hi, G, h, gn, ign) >= 0;  // the unconstrained minimiser is infeasible
  }
  // 1b. primal-dual guess, checked like the warm start
  if (try_guess) {
    const int m1 = pd_guess(warm_mask, zg, yg, lo, hi, G, h, gn);
    if (m1 != warm_mask && __builtin_popcount(m1) <= 4) {
      double z1[4], mu1[2], y1[6];
      bool d1 = false;
      if (warm_check(P, zu, lo, hi, G, h, gn, ign, m1, cs, z1, mu1, y1, d1)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) res.z[i] = fmin(fmax(z1[i], lo[i]), hi[i]);
        res.mu[0] = mu1[0];
        res.mu[1] = mu1[1];
        res.status = 0;
        res.mask = m1;
        return res;
      }
    }
  }

  // 2. dual active-set method
  int steps = 0;
  while (!done) {
    const int p = gi_most_violated(z, mask, lo, hi, G, h, gn, ign);
    if (p < 0) break;
    double np_[4], bp;
    gi_constraint(p, G, lo, hi, h, np_, bp);
    double v[4];
    matvec4(P, np_, v);
    const double npn = dot4(np_, v);
    double up = 0.0;
    bool added = false;
    while (!added) {
      if (++steps > MAX_STEPS) { status = 2; break; }
      double W[4][4], S[4][4], rhs[4], r[4];
      gi_products(P, N, q, W, S);
#pragma unroll
      for (int j = 0; j < 4; ++j) rhs[j] = (j < q) ? dot4(N[j], v) : 0.0;
      spd_solve_padded(S, q, rhs, r);
      double dz[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) dz[i] = v[i] - (W[i][0] * r[0] + W[i][1] * r[1] + W[i][2] * r[2] + W[i][3] * r[3]);
      // dual step length: first active multiplier that would become negative
      // (smallest u_j / r_j over r_j > 0, compared as u_j r_k < u_k r_j)
      int kdrop = -1;
      double un = 0.0, rd = 1.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool cand = (j < q) && (r[j] > 0.0);
        const bool better = cand && (kdrop < 0 || u[j] * rd < un * r[j]);
        un = better ? u[j] : un;
        rd = better ? r[j] : rd;
        kdrop = better ? j : kdrop;
      }
      const double t1 = (kdrop >= 0) ? un / rd : INF;
      // primal step length: reach constraint p
      const double nz = dot4(np_, dz);
      // (a full working set of four independent constraints leaves no primal
      // direction: dz vanishes up to rounding)
      const double t2 = (q < 4 && nz > 1e-14 * npn) ? -(dot4(np_, z) - bp) / nz : INF;
      const double t = fmin(t1, t2);
      if (t >= INF) { status = 1; break; }
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = (j < q) ? u[j] - t * r[j] : u[j];
      up += t;
      if (t2 < INF) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] += t * dz[i];
      }
      if (t2 <= t1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool here = (j == q);
          act[j] = here ? p : act[j];
          u[j] = here ? up : u[j];
#pragma unroll
          for (int d = 0; d < 4; ++d) N[j][d] = here ? np_[d] : N[j][d];
        }
        q += 1;
        mask |= 1 << p;
        added = true;
      } else {
        const int kd = act[kdrop];
        mask &= ~(1 << kd);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const bool shift = (j >= kdrop);
          act[j] = shift ? act[j + 1] : act[j];
          u[j] = shift ? u[j + 1] : u[j];
#pragma unroll
          for (int d = 0; d < 4; ++d) N[j][d] = shift ? N[j + 1][d] : N[j][d];
        }
        act[3] = -1;
        u[3] = 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) N[3][d] = 0.0;
        q -= 1;
      }
    }
    if (status != 0) break;
  }

#pragma unroll
  for (int i = 0; i < 4; ++i) res.z[i] = fmin(fmax(z[i], lo[i]), hi[i]);
  res.mu[0] = 0.0;
  res.mu[1] = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    res.mu[0] = (act[j] == 8) ? u[j] : res.mu[0];
    res.mu[1] = (act[j] == 9) ? u[j] : res.mu[1];
  }
  res.status = status;
  res.mask = (status == 0) ? mask : 0;
  return res;
}

}  // namespace acopf
