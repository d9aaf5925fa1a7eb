// Linear feasibility projection (Section II-A, eq. linfeas; Algorithm 1,
// the step before its loop) through the ADMM sweeps of the QP subproblems.
//
// The projection of a start x0 onto the ACOPF's linear constraints,
//   minimise 0.5 ||x - x0||^2  s.t.  power balance (opfc5, opfc6), bounds
//   (opfc1-4), theta_ref = 0,
// is a QP in d = x - x0 with the identity as Hessian, whose constraints are
// those of the QP subproblem without the linearised (opfc11-14).  It runs
// through the same decomposition (eq. cpl) with these line subproblems:
//   * the variables are z = (d_w_i, d_wR, d_w_j, d_wI): with (opfc11,
//     opfc12) gone, wR and wI are free variables of their line and the
//     flows are linear in z exactly (the same coefficients as the balance);
//   * the objective is 0.5 (d_wR^2 + d_wI^2) plus each end's share of its
//     bus's 0.5 d_w^2 (1 / degree per incident line, so the shares add up
//     at the consensus);
//   * the w copies are coupled to the bus values as before; the angle copies
//     are held at zero: d_theta enters neither objective nor constraint and
//     its projection is 0 (theta_ref stays 0);
//   * the box of d_w is the voltage bounds less w0; wR, wI are free, given
//     the box [-10, 10] (per unit squared, far beyond any voltage product)
//     so that the exact line solver applies; there are no limit rows.
// Generators take 0.5 (d_pg^2 + d_qg^2) with their bounds less (pg0, qg0);
// buses keep their balance rows (eq. bus_kernel_simp) with the constants of
// the start.  After the solve x <- x0 + d with d_wR, d_wI the lines' own
// values.
#pragma once

#include "components.h"

namespace acopf {

constexpr double kLinfeasFreeBox = 10.0;

// Line data of the projection for line l at the start x.
ACOPF_HD void build_line_linfeas(const acopf_grid& g, const acopf_iterate& x, const Workspace& w, int l) {
  const int L = g.n_line;
  const int i = g.line_from[l], j = g.line_to[l];
  double* d = w.line;
#pragma unroll
  for (int k = 0; k < LF_COUNT; ++k) d[k * L + l] = 0.0;
  const double deg_i = (double)(w.bus_end_ptr[i + 1] - w.bus_end_ptr[i]);
  const double deg_j = (double)(w.bus_end_ptr[j + 1] - w.bus_end_ptr[j]);
  // packed upper triangle: diagonal entries at 0, 4, 7, 9
  d[(LF_M + 0) * L + l] = 1.0 / deg_i;
  d[(LF_M + 4) * L + l] = 1.0;
  d[(LF_M + 7) * L + l] = 1.0 / deg_j;
  d[(LF_M + 9) * L + l] = 1.0;
  // flows (p_ij, q_ij, p_ji, q_ji) over z = (w_i, wR, w_j, wI)
  const double F[4][4] = {{g.gii[l], g.gij[l], 0.0, g.bij[l]},
                          {-g.bii[l], -g.bij[l], 0.0, g.gij[l]},
                          {0.0, g.gji[l], g.gjj[l], -g.bji[l]},
                          {0.0, -g.bji[l], -g.bjj[l], -g.gji[l]}};
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) d[(LF_F + 4 * r + k) * L + l] = F[r][k];
  const double wi_hi = g.vmax[i] * g.vmax[i] - x.w[i], wj_hi = g.vmax[j] * g.vmax[j] - x.w[j];
  d[(LF_LO + 0) * L + l] = fmin(g.vmin[i] * g.vmin[i] - x.w[i], wi_hi);
  d[(LF_HI + 0) * L + l] = wi_hi;
  d[(LF_LO + 2) * L + l] = fmin(g.vmin[j] * g.vmin[j] - x.w[j], wj_hi);
  d[(LF_HI + 2) * L + l] = wj_hi;
  d[(LF_LO + 1) * L + l] = -kLinfeasFreeBox;
  d[(LF_HI + 1) * L + l] = kLinfeasFreeBox;
  d[(LF_LO + 3) * L + l] = -kLinfeasFreeBox;
  d[(LF_HI + 3) * L + l] = kLinfeasFreeBox;
  // no limit rows: 0 <= 1
  d[(LF_H + 0) * L + l] = 1.0;
  d[(LF_H + 1) * L + l] = 1.0;
}

// Generator data of the projection: 0.5 d^2 for p and q, bounds less x0.
ACOPF_HD void build_gen_linfeas(const acopf_grid& g, const acopf_iterate& x, const Workspace& w, int k) {
  const int G = g.n_gen;
  double* d = w.gen;
  const double phi = g.pmax[k] - x.pg[k], qhi = g.qmax[k] - x.qg[k];
  d[GF_FP * G + k] = 0.0;
  d[GF_FPP * G + k] = 1.0;
  d[GF_PLO * G + k] = fmin(g.pmin[k] - x.pg[k], phi);
  d[GF_PHI * G + k] = phi;
  d[GF_QLO * G + k] = fmin(g.qmin[k] - x.qg[k], qhi);
  d[GF_QHI * G + k] = qhi;
  d[GF_FQ * G + k] = 0.0;
  d[GF_FQQ * G + k] = 1.0;
}

// Line update of a projection sweep: the exact minimiser of the line's
// subproblem (its angle-coupling terms vanish: those multipliers and bus
// values stay zero), stored as flows, w copies, zero angle copies, and
// (d_wR, d_wI) in the limit-multiplier slots.  Returns the solver status.
ACOPF_HD int update_line_linfeas(const Workspace& w, int l) {
  double Pp[10], c[4], lo[4], hi[4], G[2][4], h[2];
  line_sweep_data(w, l, Pp, c, lo, hi, G, h);
  const LineQPResult res = solve_line_qp(Pp, c, lo, hi, G, h, w.line_mask[l]);
  const int L = w.n_line;
  const double* d = w.line;
  w.line_mask[l] = res.mask;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    w.xl[lc8(l, r)] = d[(LF_F + 4 * r) * L + l] * res.z[0] + d[(LF_F + 4 * r + 1) * L + l] * res.z[1] +
                      d[(LF_F + 4 * r + 2) * L + l] * res.z[2] + d[(LF_F + 4 * r + 3) * L + l] * res.z[3];
  w.xl[lc8(l, 4)] = res.z[0];
  w.xl[lc8(l, 5)] = 0.0;
  w.xl[lc8(l, 6)] = res.z[2];
  w.xl[lc8(l, 7)] = 0.0;
  w.mu[l] = res.z[1];
  w.mu[L + l] = res.z[3];
  return res.status;
}

}  // namespace acopf
