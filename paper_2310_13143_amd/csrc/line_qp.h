// Exact solver for one line subproblem (Section IV-B2, eq. line_kernel):
//
//   minimise 0.5 z^T Q z + c^T z   s.t.  lo <= z <= hi,   G z <= h (2 rows),
//
// with Q symmetric positive definite, given its inverse P = Q^{-1}.  The
// paper solves this problem with an augmented Lagrangian and TRON; its limit
// is the unique minimiser, which this routine computes in finitely many steps
// with the dual active-set method of Goldfarb and Idnani (Math. Programming
// 27, 1983): start at the unconstrained minimiser, add the most violated
// constraint, take the primal/dual step that keeps the active multipliers
// non-negative (dropping a constraint whose multiplier reaches zero), until
// no constraint is violated.  The working set never holds more than four
// linearly independent constraints.  Everything is unrolled over the 10
// constraints (4 lower bounds, 4 upper bounds, 2 rows) so it stays in
// registers.
#pragma once

#include "small_linalg.h"

namespace acopf {

struct LineQPResult {
  double z[4];
  double mu[2];   // multipliers (>= 0) of the rows G z <= h
  int status;     // 0 solved, 1 infeasible, 2 iteration cap
};

// Constraint k in "n_k . z >= b_k" form: k < 4 lower bound of z_k, 4 <= k < 8
// upper bound of z_{k-4}, k = 8, 9 row k-8 of G z <= h.
ACOPF_HD void gi_normal(int k, const double G[2][4], double n[4]) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    double v = 0.0;
    v = (k == d) ? 1.0 : v;
    v = (k == d + 4) ? -1.0 : v;
    v = (k == 8) ? -G[0][d] : v;
    v = (k == 9) ? -G[1][d] : v;
    n[d] = v;
  }
}

ACOPF_HD double gi_rhs(int k, const double lo[4], const double hi[4], const double h[2]) {
  double b = 0.0;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    b = (k == d) ? lo[d] : b;
    b = (k == d + 4) ? -hi[d] : b;
  }
  b = (k == 8) ? -h[0] : b;
  b = (k == 9) ? -h[1] : b;
  return b;
}

ACOPF_HD double dot4(const double a[4], const double b[4]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

ACOPF_HD void matvec4(const double P[4][4], const double v[4], double out[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = P[i][0] * v[0] + P[i][1] * v[1] + P[i][2] * v[2] + P[i][3] * v[3];
}

// Direction of adding constraint with normal np to the working set with
// normals N[0..q-1]: dual direction r = (N^T P N)^{-1} N^T P np and primal
// direction dz = P np - P N r.
ACOPF_HD void gi_directions(const double P[4][4], const double N[4][4], int q, const double np[4],
                            double r[4], double dz[4]) {
  double v[4];
  matvec4(P, np, v);
  double W[4][4];  // W[:, j] = P N[j]
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double t[4];
    matvec4(P, N[j], t);
#pragma unroll
    for (int i = 0; i < 4; ++i) W[i][j] = (j < q) ? t[i] : 0.0;
  }
  // S = N^T P N (q x q, padded with identity), rhs = N^T v
  double S[4][4], rhs[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double s = N[a][0] * W[0][b] + N[a][1] * W[1][b] + N[a][2] * W[2][b] + N[a][3] * W[3][b];
      S[a][b] = (a < q && b < q) ? s : ((a == b) ? 1.0 : 0.0);
    }
    rhs[a] = (a < q) ? dot4(N[a], v) : 0.0;
  }
  double L[4][4];
  chol4(S, L);
  // solve L L^T r = rhs
  double y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s = rhs[i];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < i) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
#pragma unroll
  for (int ii = 0; ii < 4; ++ii) {
    int i = 3 - ii;
    double s = y[i];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k > i) s -= L[k][i] * r[k];
    r[i] = s / L[i][i];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) r[a] = (a < q) ? r[a] : 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    dz[i] = v[i] - (W[i][0] * r[0] + W[i][1] * r[1] + W[i][2] * r[2] + W[i][3] * r[3]);
}

ACOPF_HD LineQPResult solve_line_qp(const double Pp[10], const double c[4], const double lo[4],
                                    const double hi[4], const double G[2][4], const double h[2]) {
  const double INF = 1e300;
  const int MAX_STEPS = 48;
  double P[4][4];
  sym_unpack(Pp, P);
  LineQPResult res;
  double z[4];
  matvec4(P, c, z);
#pragma unroll
  for (int i = 0; i < 4; ++i) z[i] = -z[i];

  int act[4] = {-1, -1, -1, -1};
  double N[4][4];
  double u[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int d = 0; d < 4; ++d) N[j][d] = 0.0;
  int q = 0;
  int status = 0;
  int steps = 0;
  // feasibility tolerance, relative to the size of each constraint
  double zs = fabs(z[0]) + fabs(z[1]) + fabs(z[2]) + fabs(z[3]);

  while (true) {
    // most violated constraint outside the working set (scaled violation)
    int p = -1;
    double worst = 0.0;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      bool inw = (act[0] == k) || (act[1] == k) || (act[2] == k) || (act[3] == k);
      double n[4];
      gi_normal(k, G, n);
      double b = gi_rhs(k, lo, hi, h);
      double nn = fabs(n[0]) + fabs(n[1]) + fabs(n[2]) + fabs(n[3]);
      double s = dot4(n, z) - b;
      double tol = 1e-12 * (1.0 + fabs(b) + nn * zs);
      double sc = s / fmax(nn, 1e-300);
      bool viol = !inw && nn > 0.0 && s < -tol && sc < worst;
      worst = viol ? sc : worst;
      p = viol ? k : p;
    }
    if (p < 0) break;
    double np_[4];
    gi_normal(p, G, np_);
    double bp = gi_rhs(p, lo, hi, h);
    double up = 0.0;
    bool added = false;
    while (!added) {
      if (++steps > MAX_STEPS) { status = 2; break; }
      double r[4], dz[4];
      gi_directions(P, N, q, np_, r, dz);
      // dual step length: first active multiplier that would become negative
      double t1 = INF;
      int kdrop = -1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bool cand = (j < q) && (r[j] > 0.0);
        double ratio = cand ? u[j] / r[j] : INF;
        bool better = cand && ratio < t1;
        t1 = better ? ratio : t1;
        kdrop = better ? j : kdrop;
      }
      // primal step length: reach the constraint
      double v[4];
      matvec4(P, np_, v);
      double npn = dot4(np_, v);
      double nz = dot4(np_, dz);
      double t2 = (nz > 1e-14 * npn) ? -(dot4(np_, z) - bp) / nz : INF;
      double t = fmin(t1, t2);
      if (t >= INF) { status = 1; break; }
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = (j < q) ? u[j] - t * r[j] : u[j];
      up += t;
      if (t2 < INF) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] += t * dz[i];
      }
      if (t2 <= t1) {
        // add p to the working set
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bool here = (j == q);
          act[j] = here ? p : act[j];
          u[j] = here ? up : u[j];
#pragma unroll
          for (int d = 0; d < 4; ++d) N[j][d] = here ? np_[d] : N[j][d];
        }
        q += 1;
        added = true;
      } else {
        // drop constraint kdrop (shift the later ones down)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          bool shift = (j >= kdrop);
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
    zs = fabs(z[0]) + fabs(z[1]) + fabs(z[2]) + fabs(z[3]);
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
  return res;
}

}  // namespace acopf
