// Per-component arithmetic of the ADMM QP solver: one call handles one line,
// one generator or one bus.  The GPU kernels call these from one thread per
// component; every memory access is an explicit structure-of-arrays index so
// that the same source can be compiled for the host to test its arithmetic.
#pragma once

#include "line_alm.h"
#include "line_qp.h"
#include "small_linalg.h"
#include "workspace.h"
#include "../../include/acopf_admm.h"

namespace acopf {

// The coupling state of the lines (x, lambda, rho and the starting
// multipliers: 8 couplings per line) is stored line by line, each line's 8
// slots ordered by line end: the from end's (p_ij, q_ij, w_i, th_i), then
// the to end's (p_ji, q_ji, w_j, th_j), so the bus update of one line end
// reads and writes one aligned 32-byte half of each record.  Couplings are
// numbered 0-3 for the flows (p_ij, q_ij, p_ji, q_ji) and 4-7 for the
// voltage copies (w_i, th_i, w_j, th_j); slot8 maps that number to its
// slot.  The bus-side copies are two arrays of 4 per line (flows; the end
// buses' d_w, d_th), in coupling order.
ACOPF_HD constexpr int slot8(int k) { return (k & 1) | ((k & 2) << 1) | ((k & 4) >> 1); }
ACOPF_HD size_t lc8(int l, int k) { return 8 * (size_t)l + slot8(k); }
ACOPF_HD size_t lc4(int l, int k) { return 4 * (size_t)l + k; }

static constexpr double kTwoPi = 6.283185307179586476925286766559;

// phi(n) = sum_d min(g_d lo_d, g_d hi_d) - n . h with g = n_0 G_0 + n_1 G_1:
// the smallest value of n . (G z - h) over the box.
ACOPF_HD double box_support(const double lo[4], const double hi[4], const double G[2][4], const double h[2],
                            double n0, double n1) {
  double phi = -n0 * h[0] - n1 * h[1];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const double gd = n0 * G[0][d] + n1 * G[1][d];
    phi += fmin(gd * lo[d], gd * hi[d]);
  }
  return phi;
}

// Relaxation of the limit rows of a line whose box lo <= z <= hi and rows
// G z <= h have no common point (the paper's ADMM keeps progressing on QPs
// without a feasible point, Section V: its augmented Lagrangian line solver
// ends at the point of least squared violation).  Writes shift[r] = v_r +
// guard to both rows, 0 for lines with a common point; returns true if
// relaxed.
//  * Common point: t* = min over the box of max_r (G_r z - h_r) <= 0.  By LP
//    duality t* is the maximum of phi over n = (a, 1 - a), a in [0, 1]; phi
//    is concave and piecewise linear, so the maximum lies at a = 0, a = 1
//    or a breakpoint where some g_d vanishes.
//  * v = (G z* - h)^+ for z* minimising ||(G z - h)^+||^2 over the box is
//    the vector from the quadrant {y <= h} to its nearest point of the
//    polygon G [lo, hi]; its length is the largest phi(n) over unit n >= 0
//    and its direction the maximising n (distance between convex sets).
//    On the quarter circle n = (cos th, sin th) phi is linear, n . c, within
//    each sector between breakpoint angles (sign pattern of g fixed), so its
//    maximum lies at th = 0, th = pi/2, a breakpoint, or a sector's
//    stationary direction c / |c|.  Each breakpoint and end angle gives the
//    sign patterns on both of its sides; phi itself is evaluated at every
//    candidate.
//  * guard = 1e-9 (1 + |h_0| + |h_1| + sum_d (|G_0d| + |G_1d|) max(|lo_d|,
//    |hi_d|)) on both rows, many times the rounding error of v.
ACOPF_HD bool limit_relaxation(const double lo[4], const double hi[4], const double G[2][4], const double h[2],
                               double shift[2]) {
  shift[0] = shift[1] = 0.0;
  double alpha[6] = {0.0, 1.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const double den = G[1][d] - G[0][d];
    const double a = (den != 0.0) ? G[1][d] / den : 0.0;
    alpha[2 + d] = fmin(fmax(a, 0.0), 1.0);
  }
  double t = -1e300;
#pragma unroll
  for (int k = 0; k < 6; ++k) t = fmax(t, box_support(lo, hi, G, h, alpha[k], 1.0 - alpha[k]));
  if (!(t > 0.0)) return false;
  // candidate angles: the ends of the quarter circle and the breakpoints in it
  constexpr double kHalfPi = 1.5707963267948966192313216916398;
  constexpr double kPi = 3.1415926535897932384626433832795;
  double th[6] = {0.0, kHalfPi, -1.0, -1.0, -1.0, -1.0};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (G[0][d] == 0.0 && G[1][d] == 0.0) continue;
    double a = atan2(-G[0][d], G[1][d]);
    if (a < 0.0) a += kPi;
    if (a <= kHalfPi) th[2 + d] = a;
  }
  double best = -1e300, bn0 = 1.0, bn1 = 0.0;
  auto consider = [&](double n0, double n1) {
    const double phi = box_support(lo, hi, G, h, n0, n1);
    if (phi > best) {
      best = phi;
      bn0 = n0;
      bn1 = n1;
    }
  };
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (th[k] < 0.0) continue;
    const double n0 = cos(th[k]), n1 = sin(th[k]);
    consider(n0, n1);
    // the sectors on both sides: the sign of g_d there, from g_d at th or,
    // where g_d vanishes at th, from its derivative along the circle
#pragma unroll
    for (int side = -1; side <= 1; side += 2) {
      double c0 = -h[0], c1 = -h[1];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        double gd = n0 * G[0][d] + n1 * G[1][d];
        if (th[2 + d] == th[k]) gd = side * (-n1 * G[0][d] + n0 * G[1][d]);
        const double sel = (gd >= 0.0) ? lo[d] : hi[d];
        c0 += G[0][d] * sel;
        c1 += G[1][d] * sel;
      }
      const double nc = sqrt(c0 * c0 + c1 * c1);
      if (c0 >= 0.0 && c1 >= 0.0 && nc > 0.0) consider(c0 / nc, c1 / nc);
    }
  }
  double scale = 1.0 + fabs(h[0]) + fabs(h[1]);
#pragma unroll
  for (int d = 0; d < 4; ++d) scale += (fabs(G[0][d]) + fabs(G[1][d])) * fmax(fabs(lo[d]), fabs(hi[d]));
  const double guard = 1e-9 * scale;
  const double dist = fmax(best, 0.0);
  shift[0] = dist * bn0 + guard;
  shift[1] = dist * bn1 + guard;
  return true;
}

// QP data of line l at the iterate (Sections III-B, III-C and IV-B2).
// Returns false if the elimination pivot wR cos + wI sin vanishes or the
// data are not finite.  *relaxed (optional): the limit rows were relaxed.
// cshift (optional, 4 values): added to c11..c14 of (opfc11-14) at x in
// their linearisations (the QP of a second-order correction).
ACOPF_HD bool build_line(const acopf_grid& g, const acopf_iterate& x, double delta, int mode,
                         const Workspace& w, int l, bool* relaxed = nullptr, const double* cshift = nullptr) {
  const int L = g.n_line;
  const int f = g.line_from[l], t = g.line_to[l];
  const double wi = x.w[f], wj = x.w[t], thi = x.th[f], thj = x.th[t];
  const double wR = x.wR[l], wI = x.wI[l];
  const double p11 = x.pi[l], p12 = x.pi[L + l], p13 = x.pi[2 * L + l], p14 = x.pi[3 * L + l];
  const double gii = g.gii[l], bii = g.bii[l], gij = g.gij[l], bij = g.bij[l];
  const double gji = g.gji[l], bji = g.bji[l], gjj = g.gjj[l], bjj = g.bjj[l];
  const double ph = thi - thj;
  const double s = sin(ph), c = cos(ph);
  // elimination (eq. elim): linearised opfc11, opfc12 solved for d_wR, d_wI
  const double K = wR * c + wI * s;
  double r1 = wi * wj - wR * wR - wI * wI;  // -c11
  double r2 = -wR * s + wI * c;             // -c12
  if (cshift) {
    r1 -= cshift[0];
    r2 -= cshift[1];
  }
  bool ok = fabs(K) >= 1e-8;
  const double K2 = 2.0 * (ok ? K : 1.0);
  const double aR[4] = {c * wj / K2, -wI, c * wi / K2, wI};
  const double aI[4] = {s * wj / K2, wR, s * wi / K2, -wR};
  const double bR = (c * r1 + 2.0 * wI * r2) / K2;
  const double bI = (s * r1 - 2.0 * wR * r2) / K2;

  // Hessian of L_ij (eq. lag) in u = (w_i, th_i, wR, wI, w_j, th_j); for a
  // restoration step (kModeRestore) the Hessian of 0.5 ||d||^2 instead,
  // each bus variable's term shared among its lines by 1 / degree
  double H[6][6];
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = 0; b < 6; ++b) H[a][b] = 0.0;
  if (mode == kModeRestore) {
    const double sf = 1.0 / (double)(w.bus_end_ptr[f + 1] - w.bus_end_ptr[f]);
    const double st = 1.0 / (double)(w.bus_end_ptr[t + 1] - w.bus_end_ptr[t]);
    H[0][0] = sf;
    H[1][1] = sf;
    H[2][2] = 1.0;
    H[3][3] = 1.0;
    H[4][4] = st;
    H[5][5] = st;
  } else {
    H[2][2] += 2.0 * p11;
    H[3][3] += 2.0 * p11;
    H[0][4] -= p11;
    H[4][0] -= p11;
    const double T = -wR * s + wI * c;
    H[1][1] += p12 * T;
    H[5][5] += p12 * T;
    H[1][5] -= p12 * T;
    H[5][1] -= p12 * T;
    H[2][1] += p12 * c; H[1][2] += p12 * c;
    H[2][5] -= p12 * c; H[5][2] -= p12 * c;
    H[3][1] += p12 * s; H[1][3] += p12 * s;
    H[3][5] -= p12 * s; H[5][3] -= p12 * s;
    {
      const double gp_ij[6] = {gii, 0.0, gij, bij, 0.0, 0.0};
      const double gq_ij[6] = {-bii, 0.0, -bij, gij, 0.0, 0.0};
      const double gp_ji[6] = {0.0, 0.0, gji, -bji, gjj, 0.0};
      const double gq_ji[6] = {0.0, 0.0, -bji, -gji, -bjj, 0.0};
#pragma unroll
      for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b < 6; ++b)
          H[a][b] -= 2.0 * p13 * (gp_ij[a] * gp_ij[b] + gq_ij[a] * gq_ij[b]) +
                     2.0 * p14 * (gp_ji[a] * gp_ji[b] + gq_ji[a] * gq_ji[b]);
    }
  }
  // A (6x4): rows e0, e1, aR, aI, e2, e3; M = A^T H A, q = A^T H b
  double A[6][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    A[0][k] = (k == 0) ? 1.0 : 0.0;
    A[1][k] = (k == 1) ? 1.0 : 0.0;
    A[2][k] = aR[k];
    A[3][k] = aI[k];
    A[4][k] = (k == 2) ? 1.0 : 0.0;
    A[5][k] = (k == 3) ? 1.0 : 0.0;
  }
  double HA[6][4];
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < 6; ++b) v += H[a][b] * A[b][k];
      HA[a][k] = v;
    }
  double M[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < 6; ++a) v += A[a][i] * HA[a][j];
      M[i][j] = v;
    }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i + 1; j < 4; ++j) {
      double v = 0.5 * (M[i][j] + M[j][i]);
      M[i][j] = v;
      M[j][i] = v;
    }
  if (mode == ACOPF_HESSIAN_PSD) psd_project4(M);
  double q[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = HA[2][i] * bR + HA[3][i] * bI;  // (A^T H b)_i = (HA)^T b
  const double c0 = 0.5 * (bR * bR * H[2][2] + 2.0 * bR * bI * H[2][3] + bI * bI * H[3][3]);

  // flow map (substitution after eq. line_kernel)
  double F[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double e0 = (k == 0) ? 1.0 : 0.0, e2 = (k == 2) ? 1.0 : 0.0;
    F[0][k] = gii * e0 + gij * aR[k] + bij * aI[k];
    F[1][k] = -bii * e0 - bij * aR[k] + gij * aI[k];
    F[2][k] = gjj * e2 + gji * aR[k] - bji * aI[k];
    F[3][k] = -bjj * e2 - bji * aR[k] - gji * aI[k];
  }
  const double f0[4] = {gij * bR + bij * bI, -bij * bR + gij * bI, gji * bR - bji * bI,
                        -bji * bR - gji * bI};
  // boxes of the voltage copies: bounds shifted to the iterate and the TR
  double lo[4], hi[4];
  {
    const int bus[2] = {f, t};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = bus[e];
      const double vl = g.vmin[i], vh = g.vmax[i];
      double wl = fmax(-delta, vl * vl - x.w[i]);
      double wh = fmin(delta, vh * vh - x.w[i]);
      double tl = fmax(-delta, -kTwoPi - x.th[i]);
      double th = fmin(delta, kTwoPi - x.th[i]);
      if (w.bus_flags[i] & BUS_REF) { tl = 0.0; th = 0.0; }
      lo[2 * e] = fmin(wl, wh);
      hi[2 * e] = wh;
      lo[2 * e + 1] = fmin(tl, th);
      hi[2 * e + 1] = th;
    }
  }
  // flows at the iterate and linearised limits (opfqpc13, opfqpc14)
  const double pij = gii * wi + gij * wR + bij * wI;
  const double qij = -bii * wi - bij * wR + gij * wI;
  const double pji = gjj * wj + gji * wR - bji * wI;
  const double qji = -bjj * wj - bji * wR - gji * wI;
  double Gr[2][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Gr[0][k] = 2.0 * pij * F[0][k] + 2.0 * qij * F[1][k];
    Gr[1][k] = 2.0 * pji * F[2][k] + 2.0 * qji * F[3][k];
  }
  const double sij = g.smax_ij[l], sji = g.smax_ji[l];
  double hr[2] = {sij * sij - pij * pij - qij * qij - 2.0 * pij * f0[0] - 2.0 * qij * f0[1],
                  sji * sji - pji * pji - qji * qji - 2.0 * pji * f0[2] - 2.0 * qji * f0[3]};
  if (cshift) {  // c13 + e13 - 2 p_ij dp_ij - 2 q_ij dq_ij >= 0  <=>  G z <= h + e13
    hr[0] += cshift[2];
    hr[1] += cshift[3];
  }
  double shift[2];
  const bool rel = limit_relaxation(lo, hi, Gr, hr, shift);
  const double hr0 = hr[0] + shift[0], hr1 = hr[1] + shift[1];
  if (relaxed) *relaxed = rel;
  ok = ok && isfinite(hr0) && isfinite(hr1) && isfinite(c0);

  double* d = w.line;
  double Mp[10];
  sym_pack(M, Mp);
#pragma unroll
  for (int k = 0; k < 10; ++k) d[(LF_M + k) * L + l] = Mp[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    d[(LF_Q + k) * L + l] = q[k];
    d[(LF_F0 + k) * L + l] = f0[k];
    d[(LF_LO + k) * L + l] = lo[k];
    d[(LF_HI + k) * L + l] = hi[k];
    d[(LF_AR + k) * L + l] = aR[k];
    d[(LF_AI + k) * L + l] = aI[k];
    d[(LF_G + k) * L + l] = Gr[0][k];
    d[(LF_G + 4 + k) * L + l] = Gr[1][k];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) d[(LF_F + 4 * r + k) * L + l] = F[r][k];
  d[(LF_H + 0) * L + l] = hr0;
  d[(LF_H + 1) * L + l] = hr1;
  d[LF_BR * L + l] = bR;
  d[LF_BI * L + l] = bI;
  d[(LF_PK + 0) * L + l] = pij;
  d[(LF_PK + 1) * L + l] = qij;
  d[(LF_PK + 2) * L + l] = pji;
  d[(LF_PK + 3) * L + l] = qji;
  d[LF_C0 * L + l] = c0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    d[(LF_HR + k) * L + l] = H[2][k];
    d[(LF_HI_ROW + k) * L + l] = H[3][k];
  }
  return ok;
}

// restore: the objective 0.5 (d_p^2 + d_q^2) of a restoration step.
ACOPF_HD void build_gen(const acopf_grid& g, const acopf_iterate& x, double delta, const Workspace& w,
                        int k, bool restore = false) {
  const int G = g.n_gen;
  const double p = x.pg[k], qv = x.qg[k];
  double* d = w.gen;
  d[GF_FP * G + k] = restore ? 0.0 : 2.0 * g.cost2[k] * p + g.cost1[k];
  d[GF_FPP * G + k] = restore ? 1.0 : 2.0 * g.cost2[k];
  const double phi = fmin(delta, g.pmax[k] - p), qhi = fmin(delta, g.qmax[k] - qv);
  d[GF_PLO * G + k] = fmin(fmax(-delta, g.pmin[k] - p), phi);
  d[GF_PHI * G + k] = phi;
  d[GF_QLO * G + k] = fmin(fmax(-delta, g.qmin[k] - qv), qhi);
  d[GF_QHI * G + k] = qhi;
  d[GF_FQ * G + k] = 0.0;
  d[GF_FQQ * G + k] = restore ? 1.0 : 0.0;
}

// p^{d,(k)}, q^{d,(k)} of bus i (constants after eq. acopf_qppf).
ACOPF_HD void build_bus(const acopf_grid& g, const acopf_iterate& x, const Workspace& w, int i) {
  double pd = g.pd[i] + g.gsh[i] * x.w[i];
  double qd = g.qd[i] - g.bsh[i] * x.w[i];
  for (int e = w.bus_gen_ptr[i]; e < w.bus_gen_ptr[i + 1]; ++e) {
    const int k = w.bus_gen[e];
    pd -= x.pg[k];
    qd -= x.qg[k];
  }
  for (int e = w.bus_end_ptr[i]; e < w.bus_end_ptr[i + 1]; ++e) {
    const int code = w.bus_end[e];
    const int l = code >> 1;
    const double wR = x.wR[l], wI = x.wI[l];
    if ((code & 1) == 0) {
      pd += g.gii[l] * x.w[i] + g.gij[l] * wR + g.bij[l] * wI;
      qd += -g.bii[l] * x.w[i] - g.bij[l] * wR + g.gij[l] * wI;
    } else {
      pd += g.gjj[l] * x.w[i] + g.gji[l] * wR - g.bji[l] * wI;
      qd += -g.bjj[l] * x.w[i] - g.bji[l] * wR - g.gji[l] * wI;
    }
  }
  w.bus_pdk[i] = pd;
  w.bus_qdk[i] = qd;
}

// Factorisation of line l's subproblem matrix for the current penalties:
// P = Q^{-1}, Q = M + sum_f rho_f F_f^T F_f + diag(rho_v), and the constant
// part of its linear term, q + sum_f rho_f f0_f F_f.  False if Q is not
// positive definite.  With the local line solver (RAW_LOCAL) Q itself is
// kept in P's place and need not be definite.
ACOPF_HD bool prep_line(const Workspace& w, int l) {
  const int L = w.n_line;
  const double* d = w.line;
  double Mp[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) Mp[k] = d[(LF_M + k) * L + l];
  double Q[4][4];
  sym_unpack(Mp, Q);
  double cc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) cc[i] = d[(LF_Q + i) * L + l];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double rho = w.rho_l[lc8(l, r)];
    const double f0 = d[(LF_F0 + r) * L + l];
    double Fr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) Fr[k] = d[(LF_F + 4 * r + k) * L + l];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cc[i] += rho * f0 * Fr[i];
#pragma unroll
      for (int j = 0; j < 4; ++j) Q[i][j] += rho * Fr[i] * Fr[j];
    }
  }
  // in the linear feasibility projection z = (w_i, wR, w_j, wI): only the
  // w copies are coupled to bus values (the angle copies are held at zero)
  const bool lf = w.sync->hessian_mode == kModeLinfeas;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (!lf || (i & 1) == 0) Q[i][i] += w.rho_l[lc8(l, 4 + i)];
  double Pp[10];
  bool ok = true;
  if (w.sync->hessian_mode == ACOPF_HESSIAN_RAW_LOCAL) {
    sym_pack(Q, Pp);
  } else {
    double Lc[4][4], Pinv[4][4];
    ok = chol4(Q, Lc);
    chol4_inverse(Lc, Pinv);
    sym_pack(Pinv, Pp);
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) w.line_P[k * L + l] = Pp[k];
#pragma unroll
  for (int i = 0; i < 4; ++i) w.line_cc[i * L + l] = cc[i];
  return ok;
}

// Data of line l's subproblem in this sweep (eq. line_kernel): the factor
// P (packed), the linear term c from the multipliers and the bus-side
// values of the previous sweep, the box and the limit rows.
ACOPF_HD void line_sweep_data(const Workspace& w, int l, double Pp[10], double c[4], double lo[4], double hi[4],
                              double G[2][4], double h[2]) {
  const int L = w.n_line;
  const double* d = w.line;
#pragma unroll
  for (int k = 0; k < 10; ++k) Pp[k] = w.line_P[k * L + l];
  double F[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) F[r][k] = d[(LF_F + 4 * r + k) * L + l];
  // bus-side values of the voltage copies, stored in the line's record by
  // the last bus update (the end buses' d_w, d_th)
  const double xbv[4] = {w.xbar_v[lc4(l, 0)], w.xbar_v[lc4(l, 1)], w.xbar_v[lc4(l, 2)], w.xbar_v[lc4(l, 3)]};
#pragma unroll
  for (int i = 0; i < 4; ++i)
    c[i] = w.line_cc[i * L + l] + w.lam_l[lc8(l, 4 + i)] - w.rho_l[lc8(l, 4 + i)] * xbv[i];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double a = w.lam_l[lc8(l, r)] - w.rho_l[lc8(l, r)] * w.xbar_f[lc4(l, r)];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] += F[r][i] * a;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    lo[k] = d[(LF_LO + k) * L + l];
    hi[k] = d[(LF_HI + k) * L + l];
    G[0][k] = d[(LF_G + k) * L + l];
    G[1][k] = d[(LF_G + 4 + k) * L + l];
  }
  h[0] = d[(LF_H + 0) * L + l];
  h[1] = d[(LF_H + 1) * L + l];
}

// Line-side values of the 8 couplings (flows F z + f0, then z), the limit-
// row multipliers and the working set of a solved line subproblem.  The
// flow map is read again (from cache) rather than kept in registers across
// the solver, which spilled it; an opaque copy of the index keeps the
// compiler from reusing the first load.
ACOPF_HD void line_sweep_store(const Workspace& w, int l, const LineQPResult& res) {
  const int L = w.n_line;
  const double* d = w.line;
  w.line_mask[l] = res.mask;
  int lf = l;
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(lf));
#endif
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double fl = d[(LF_F + 4 * r) * L + lf] * res.z[0] + d[(LF_F + 4 * r + 1) * L + lf] * res.z[1] +
                      d[(LF_F + 4 * r + 2) * L + lf] * res.z[2] + d[(LF_F + 4 * r + 3) * L + lf] * res.z[3] +
                      d[(LF_F0 + r) * L + l];
    w.xl[lc8(l, r)] = fl;
    w.xl[lc8(l, 4 + r)] = res.z[r];
  }
  w.mu[l] = res.mu[0];
  w.mu[L + l] = res.mu[1];
}

// Line update with the local solver (hessian mode RAW_LOCAL; line_P holds Q
// itself): ALM + TRON from the previous sweep's solution and limit-row
// multipliers.  Not converged counts like an infeasible line (status 2).
// The sweep kernels that call it are separate instantiations, so that its
// registers do not weigh on the exact solver's kernels.
ACOPF_HD int update_line_local(const Workspace& w, int l) {
  double Qp[10], c[4], lo[4], hi[4], G[2][4], h[2];
  line_sweep_data(w, l, Qp, c, lo, hi, G, h);
  const double z0[4] = {w.xl[lc8(l, 4)], w.xl[lc8(l, 5)], w.xl[lc8(l, 6)], w.xl[lc8(l, 7)]};
  const double u0[2] = {w.mu[l], w.mu[w.n_line + l]};
  const LineAlmResult a = solve_line_alm(Qp, c, lo, hi, G, h, z0, u0);
  LineQPResult res;
#pragma unroll
  for (int i = 0; i < 4; ++i) res.z[i] = a.z[i];
  res.mu[0] = a.u[0];
  res.mu[1] = a.u[1];
  res.status = a.converged ? 0 : 2;
  res.mask = 0;
  line_sweep_store(w, l, res);
  return res.status;
}

// Line update of one ADMM sweep (eq. line_kernel): exact minimiser of the
// line subproblem given the multipliers and the bus-side values of the
// previous sweep.  Writes the line-side values of the 8 couplings and the
// limit-row multipliers; returns the solver status (0 solved).
ACOPF_HD int update_line(const acopf_grid& g, const Workspace& w, int l) {
  (void)g;
  double Pp[10], c[4], lo[4], hi[4], G[2][4], h[2];
  line_sweep_data(w, l, Pp, c, lo, hi, G, h);
  const LineQPResult res = solve_line_qp(Pp, c, lo, hi, G, h, w.line_mask[l]);
  line_sweep_store(w, l, res);
  return res.status;
}

// The line update when the previous working set or the primal-dual guess
// settles it (the common case between sweeps): returns false, writing
// nothing, with `base` the last working set checked, when a search or
// update_line must run instead.
ACOPF_HD bool update_line_fast(const Workspace& w, int l, int& base) {
  double Pp[10], c[4], lo[4], hi[4], G[2][4], h[2];
  line_sweep_data(w, l, Pp, c, lo, hi, G, h);
  LineQPResult res;
  if (!solve_line_qp_fast(Pp, c, lo, hi, G, h, w.line_mask[l], res, base)) return false;
  line_sweep_store(w, l, res);
  return true;
}

// Neighbour `idx` of working set `base` checked for line l (one thread of a
// search over a line's neighbouring working sets): true, with the result
// in res, if it is optimal.
ACOPF_HD bool line_neighbour_check(const Workspace& w, int l, int base, int idx, LineQPResult& res) {
  const int m = neighbour_mask(base, idx);
  if (m < 0) return false;
  double Pp[10], c[4], lo[4], hi[4], G[2][4], h[2];
  line_sweep_data(w, l, Pp, c, lo, hi, G, h);
  return check_working_set(Pp, c, lo, hi, G, h, m, res);
}

// A residual term added to a running norm of the stop test: the sum of
// squares (Euclidean norms) or the largest square (infinity norms; the
// square root of either is the norm).
ACOPF_HD void acc_norm(double& acc, double v2, bool inf) { acc = inf ? fmax(acc, v2) : acc + v2; }

// Generator update (eq. gen_kernel, closed form clamp) of generator k.
ACOPF_HD void update_gen(const Workspace& w, int k) {
  const int G = w.n_gen;
  const double* d = w.gen;
  const double rp = w.rho_g[k], rq = w.rho_g[G + k];
  double xp = (rp * w.xbar_g[k] - w.lam_g[k] - d[GF_FP * G + k]) / (d[GF_FPP * G + k] + rp);
  double xq = (rq * w.xbar_g[G + k] - w.lam_g[G + k] - d[GF_FQ * G + k]) / (d[GF_FQQ * G + k] + rq);
  xp = fmin(fmax(xp, d[GF_PLO * G + k]), d[GF_PHI * G + k]);
  xq = fmin(fmax(xq, d[GF_QLO * G + k]), d[GF_QHI * G + k]);
  w.xg[k] = xp;
  w.xg[G + k] = xq;
}

// Bus update (eq. bus_kernel, closed form of eq. bus_kernel_simp with
// diagonal Q), multiplier update (eq. multiplier) of every coupling that
// ends at bus i, and that bus's contribution to ||r||^2 and ||s||^2.
// Generators of the bus are updated first (they only read values of the
// previous bus update), which keeps the two-block order of Algorithm 2.
//
// With Q_c = rho_c and c_c = rho_c x_c + lam_c the closed form gives, for a
// generator or flow copy with balance coefficient a_c = +-1,
//   xbar_c = x_c + (lam_c - a_c nu) / rho_c,   lam_c + rho_c (x_c - xbar_c) = a_c nu,
// so the multiplier update of these couplings is written as a_c nu.
// kTrace: also add |r_c| and |s_c| of every coupling at the bus to the
// workspace's trace sums.
template <bool kTrace = false>
ACOPF_HD void update_bus(const acopf_grid& g, const Workspace& w, int i, double& r2, double& s2,
                         bool inf = false) {
  // Line ends are visited in chunks of kChunk: the chunk's CSR entries are
  // loaded together, then all of its coupling values, so a bus of degree d
  // waits on 2 ceil(d / kChunk) memory round trips per pass instead of 2 d.
  constexpr int kChunk = 4;
  const int G = w.n_gen, L = w.n_line;
  const int g0 = w.bus_gen_ptr[i], g1 = w.bus_gen_ptr[i + 1];
  const int e0 = w.bus_end_ptr[i], e1 = w.bus_end_ptr[i + 1];
  double spp = 0.0, sqq = 0.0, rp = 0.0, rq = 0.0, qw = 0.0, cw = 0.0, qt = 0.0, ct = 0.0;
  for (int e = g0; e < g1; ++e) {
    const int k = w.bus_gen[e];
    update_gen(w, k);
    const double ip = 1.0 / w.rho_g[k], iq = 1.0 / w.rho_g[G + k];
    spp += ip;
    sqq += iq;
    rp += w.xg[k] + w.lam_g[k] * ip;
    rq += w.xg[G + k] + w.lam_g[G + k] * iq;
  }
  for (int e = e0; e < e1; e += kChunk) {
    int l[kChunk], sd[kChunk];
    bool on[kChunk];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      on[j] = e + j < e1;
      const int code = on[j] ? w.bus_end[e + j] : 0;
      l[j] = code >> 1;
      sd[j] = code & 1;
    }
    double v[kChunk][12];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      const int kp = 2 * sd[j], kw = 4 + 2 * sd[j];
#pragma unroll
      for (int m = 0; m < 12; ++m) v[j][m] = 0.0;
      if (on[j]) {
        v[j][0] = w.rho_l[lc8(l[j], kp)];
        v[j][1] = w.rho_l[lc8(l[j], kp + 1)];
        v[j][2] = w.rho_l[lc8(l[j], kw)];
        v[j][3] = w.rho_l[lc8(l[j], kw + 1)];
        v[j][4] = w.xl[lc8(l[j], kp)];
        v[j][5] = w.xl[lc8(l[j], kp + 1)];
        v[j][6] = w.xl[lc8(l[j], kw)];
        v[j][7] = w.xl[lc8(l[j], kw + 1)];
        v[j][8] = w.lam_l[lc8(l[j], kp)];
        v[j][9] = w.lam_l[lc8(l[j], kp + 1)];
        v[j][10] = w.lam_l[lc8(l[j], kw)];
        v[j][11] = w.lam_l[lc8(l[j], kw + 1)];
      }
    }
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      if (!on[j]) continue;
      const double ip = 1.0 / v[j][0], iq = 1.0 / v[j][1];
      spp += ip;
      sqq += iq;
      rp -= v[j][4] + v[j][8] * ip;
      rq -= v[j][5] + v[j][9] * iq;
      qw += v[j][2];
      cw += v[j][2] * v[j][6] + v[j][10];
      qt += v[j][3];
      ct += v[j][3] * v[j][7] + v[j][11];
    }
  }
  const double gsh = g.gsh[i], bsh = g.bsh[i];
  const double iqw = 1.0 / qw;
  spp += gsh * gsh * iqw;
  sqq += bsh * bsh * iqw;
  const double spq = -gsh * bsh * iqw;
  rp += -gsh * cw * iqw - w.bus_pdk[i];
  rq += bsh * cw * iqw - w.bus_qdk[i];
  const double idet = 1.0 / (spp * sqq - spq * spq);
  const double nup = (sqq * rp - spq * rq) * idet;
  const double nuq = (spp * rq - spq * rp) * idet;
  const double dw_new = (cw + gsh * nup - bsh * nuq) * iqw;
  const double dth_new = (w.bus_flags[i] & BUS_REF) ? 0.0 : ct / qt;
  const double dw_old = w.dw[i], dth_old = w.dth[i];
  double rr = 0.0, ss = 0.0;
  for (int e = g0; e < g1; ++e) {
    const int k = w.bus_gen[e];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int idx = j * G + k;
      const double rho = w.rho_g[idx], xv = w.xg[idx], lam = w.lam_g[idx];
      const double lam_new = (j == 0) ? nup : nuq;
      const double xb = xv + (lam - lam_new) / rho;
      const double ds = rho * (xb - w.xbar_g[idx]);
      w.lam_g[idx] = lam_new;
      w.xbar_g[idx] = xb;
      acc_norm(rr, (xv - xb) * (xv - xb), inf);
      acc_norm(ss, ds * ds, inf);
      if (kTrace) {
        w.tr_r_g[idx] += fabs(xv - xb);
        w.tr_s_g[idx] += fabs(ds);
      }
    }
  }
  for (int e = e0; e < e1; e += kChunk) {
    int l[kChunk], sd[kChunk];
    bool on[kChunk];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      on[j] = e + j < e1;
      const int code = on[j] ? w.bus_end[e + j] : 0;
      l[j] = code >> 1;
      sd[j] = code & 1;
    }
    double v[kChunk][14];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      const int kp = 2 * sd[j], kw = 4 + 2 * sd[j];
#pragma unroll
      for (int m = 0; m < 14; ++m) v[j][m] = 1.0;
      if (on[j]) {
        v[j][0] = w.rho_l[lc8(l[j], kp)];
        v[j][1] = w.rho_l[lc8(l[j], kp + 1)];
        v[j][2] = w.rho_l[lc8(l[j], kw)];
        v[j][3] = w.rho_l[lc8(l[j], kw + 1)];
        v[j][4] = w.xl[lc8(l[j], kp)];
        v[j][5] = w.xl[lc8(l[j], kp + 1)];
        v[j][6] = w.xl[lc8(l[j], kw)];
        v[j][7] = w.xl[lc8(l[j], kw + 1)];
        v[j][8] = w.lam_l[lc8(l[j], kp)];
        v[j][9] = w.lam_l[lc8(l[j], kp + 1)];
        v[j][10] = w.lam_l[lc8(l[j], kw)];
        v[j][11] = w.lam_l[lc8(l[j], kw + 1)];
        v[j][12] = w.xbar_f[lc4(l[j], kp)];
        v[j][13] = w.xbar_f[lc4(l[j], kp + 1)];
      }
    }
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      if (!on[j]) continue;
      const int kp = 2 * sd[j], kw = 4 + 2 * sd[j];
      // flow copies p, q (balance coefficient -1): new multiplier -nu
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const double rho = v[j][m], xv = v[j][4 + m], lam = v[j][8 + m];
        const double lam_new = -((m == 0) ? nup : nuq);
        const double xb = xv + (lam - lam_new) / rho;
        const double ds = rho * (xb - v[j][12 + m]);
        w.lam_l[lc8(l[j], kp + m)] = lam_new;
        w.xbar_f[lc4(l[j], kp + m)] = xb;
        acc_norm(rr, (xv - xb) * (xv - xb), inf);
        acc_norm(ss, ds * ds, inf);
        if (kTrace) {
          w.tr_r_l[(kp + m) * L + l[j]] += fabs(xv - xb);
          w.tr_s_l[(kp + m) * L + l[j]] += fabs(ds);
        }
      }
      // voltage copies w, th
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const double rho = v[j][2 + m], xv = v[j][6 + m], lam = v[j][10 + m];
        const double xb = (m == 0) ? dw_new : dth_new;
        const double ds = rho * (xb - ((m == 0) ? dw_old : dth_old));
        w.lam_l[lc8(l[j], kw + m)] = lam + rho * (xv - xb);
        w.xbar_v[lc4(l[j], 2 * sd[j] + m)] = xb;
        acc_norm(rr, (xv - xb) * (xv - xb), inf);
        acc_norm(ss, ds * ds, inf);
        if (kTrace) {
          w.tr_r_l[(kw + m) * L + l[j]] += fabs(xv - xb);
          w.tr_s_l[(kw + m) * L + l[j]] += fabs(ds);
        }
      }
    }
  }
  w.dw[i] = dw_new;
  w.dth[i] = dth_new;
  w.nu[i] = nup;
  w.nu[w.n_bus + i] = nuq;
  acc_norm(r2, rr, inf);
  acc_norm(s2, ss, inf);
}

// The bus update of update_bus split by coupling item (one line end or one
// generator of the bus), for a bus phase that gives each item its own
// thread.  Same formulas; the bus sums are added in the same order
// (generators, then line ends in CSR order).
//
// First half: the item's terms of the bus sums (spp, sqq, rp, rq, qw, cw,
// qt, ct); a generator is updated first (eq. gen_kernel).  v keeps the
// item's values for the second half: a line end rho, x, lam of its p, q, w,
// th couplings and the bus-side flow copies; a generator rho, x, lam and the
// bus-side copies of p and q.
ACOPF_HD void bus_item_terms(const Workspace& w, int code, double v[14], double a[8]) {
#pragma unroll
  for (int m = 0; m < 8; ++m) a[m] = 0.0;
#pragma unroll
  for (int m = 0; m < 14; ++m) v[m] = 1.0;
  if (code >= 0) {
    const int l = code >> 1, sd = code & 1;
    const int kp = 2 * sd, kw = 4 + 2 * sd;
    v[0] = w.rho_l[lc8(l, kp)];
    v[1] = w.rho_l[lc8(l, kp + 1)];
    v[2] = w.rho_l[lc8(l, kw)];
    v[3] = w.rho_l[lc8(l, kw + 1)];
    v[4] = w.xl[lc8(l, kp)];
    v[5] = w.xl[lc8(l, kp + 1)];
    v[6] = w.xl[lc8(l, kw)];
    v[7] = w.xl[lc8(l, kw + 1)];
    v[8] = w.lam_l[lc8(l, kp)];
    v[9] = w.lam_l[lc8(l, kp + 1)];
    v[10] = w.lam_l[lc8(l, kw)];
    v[11] = w.lam_l[lc8(l, kw + 1)];
    v[12] = w.xbar_f[lc4(l, kp)];
    v[13] = w.xbar_f[lc4(l, kp + 1)];
    const double ip = 1.0 / v[0], iq = 1.0 / v[1];
    a[0] = ip;
    a[1] = iq;
    a[2] = -(v[4] + v[8] * ip);
    a[3] = -(v[5] + v[9] * iq);
    a[4] = v[2];
    a[5] = v[2] * v[6] + v[10];
    a[6] = v[3];
    a[7] = v[3] * v[7] + v[11];
  } else if (code != kItemPad && code != kItemBus) {
    const int G = w.n_gen, k = -code - 1;
    update_gen(w, k);
    v[0] = w.rho_g[k];
    v[1] = w.rho_g[G + k];
    v[2] = w.xg[k];
    v[3] = w.xg[G + k];
    v[4] = w.lam_g[k];
    v[5] = w.lam_g[G + k];
    v[6] = w.xbar_g[k];
    v[7] = w.xbar_g[G + k];
    const double ip = 1.0 / v[0], iq = 1.0 / v[1];
    a[0] = ip;
    a[1] = iq;
    a[2] = v[2] + v[4] * ip;
    a[3] = v[3] + v[5] * iq;
  }
}

// Constants of bus i for its closed form: shunt g, b, p^{d,(k)}, q^{d,(k)},
// reference flag, and the bus values of the previous sweep.
ACOPF_HD void bus_item_consts(const acopf_grid& g, const Workspace& w, int i, double bc[7]) {
  bc[0] = g.gsh[i];
  bc[1] = g.bsh[i];
  bc[2] = w.bus_pdk[i];
  bc[3] = w.bus_qdk[i];
  bc[4] = (w.bus_flags[i] & BUS_REF) ? 1.0 : 0.0;
  bc[5] = w.dw[i];
  bc[6] = w.dth[i];
}

// Closed form of bus i from its summed terms (as in update_bus):
// out = (nu_p, nu_q, d_w, d_th, previous d_w, previous d_th).
ACOPF_HD void bus_item_solve(const double sum[8], const double bc[7], double out[6]) {
  double spp = sum[0], sqq = sum[1], rp = sum[2], rq = sum[3];
  const double qw = sum[4], cw = sum[5], qt = sum[6], ct = sum[7];
  const double gsh = bc[0], bsh = bc[1];
  const double iqw = 1.0 / qw;
  spp += gsh * gsh * iqw;
  sqq += bsh * bsh * iqw;
  const double spq = -gsh * bsh * iqw;
  rp += -gsh * cw * iqw - bc[2];
  rq += bsh * cw * iqw - bc[3];
  const double idet = 1.0 / (spp * sqq - spq * spq);
  const double nup = (sqq * rp - spq * rq) * idet;
  const double nuq = (spp * rq - spq * rp) * idet;
  out[0] = nup;
  out[1] = nuq;
  out[2] = (cw + gsh * nup - bsh * nuq) * iqw;
  out[3] = (bc[4] != 0.0) ? 0.0 : ct / qt;
  out[4] = bc[5];
  out[5] = bc[6];
}

// Second half: the item's multiplier and bus-side copy updates (eq.
// multiplier) given its bus's closed form, and its terms of ||r||^2 and
// ||s||^2 (kTrace: also the trace sums).
template <bool kTrace = false>
ACOPF_HD void bus_item_update(const Workspace& w, int code, const double v[14], const double res[6], double& rr,
                              double& ss, bool inf = false) {
  if (code >= 0) {
    const int L = w.n_line;
    const int l = code >> 1, sd = code & 1;
    const int kp = 2 * sd, kw = 4 + 2 * sd;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const double rho = v[m], xv = v[4 + m], lam = v[8 + m];
      const double lam_new = -res[m];
      const double xb = xv + (lam - lam_new) / rho;
      const double ds = rho * (xb - v[12 + m]);
      w.lam_l[lc8(l, kp + m)] = lam_new;
      w.xbar_f[lc4(l, kp + m)] = xb;
      acc_norm(rr, (xv - xb) * (xv - xb), inf);
      acc_norm(ss, ds * ds, inf);
      if (kTrace) {
        w.tr_r_l[(kp + m) * L + l] += fabs(xv - xb);
        w.tr_s_l[(kp + m) * L + l] += fabs(ds);
      }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const double rho = v[2 + m], xv = v[6 + m], lam = v[10 + m];
      const double xb = res[2 + m];
      const double ds = rho * (xb - res[4 + m]);
      w.lam_l[lc8(l, kw + m)] = lam + rho * (xv - xb);
      w.xbar_v[lc4(l, 2 * sd + m)] = xb;
      acc_norm(rr, (xv - xb) * (xv - xb), inf);
      acc_norm(ss, ds * ds, inf);
      if (kTrace) {
        w.tr_r_l[(kw + m) * L + l] += fabs(xv - xb);
        w.tr_s_l[(kw + m) * L + l] += fabs(ds);
      }
    }
  } else if (code != kItemPad && code != kItemBus) {
    const int G = w.n_gen, k = -code - 1;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int idx = j * G + k;
      const double rho = v[j], xv = v[2 + j], lam = v[4 + j];
      const double lam_new = res[j];
      const double xb = xv + (lam - lam_new) / rho;
      const double ds = rho * (xb - v[6 + j]);
      w.lam_g[idx] = lam_new;
      w.xbar_g[idx] = xb;
      acc_norm(rr, (xv - xb) * (xv - xb), inf);
      acc_norm(ss, ds * ds, inf);
      if (kTrace) {
        w.tr_r_g[idx] += fabs(xv - xb);
        w.tr_s_g[idx] += fabs(ds);
      }
    }
  }
}

// A whole bus by the item functions, one item at a time (a bus with more
// items than an item block): the same sums, closed form and updates in the
// same order as update_bus, with the register footprint of one item.  Each
// item's values are loaded again for its update; nothing has changed them
// in between (a generator's own update is recomputed with the same result).
template <bool kTrace = false>
ACOPF_HD void bus_whole_update(const acopf_grid& g, const Workspace& w, int i, double& rr, double& ss,
                               bool inf = false) {
  const int g0 = w.bus_gen_ptr[i], g1 = w.bus_gen_ptr[i + 1];
  const int e0 = w.bus_end_ptr[i], e1 = w.bus_end_ptr[i + 1];
  const int n = (g1 - g0) + (e1 - e0);
  double sum[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < n; ++j) {
    const int code = (j < g1 - g0) ? -(w.bus_gen[g0 + j] + 1) : w.bus_end[e0 + j - (g1 - g0)];
    double v[14], a[8];
    bus_item_terms(w, code, v, a);
#pragma unroll
    for (int m = 0; m < 8; ++m) sum[m] += a[m];
  }
  double bc[7], out[6];
  bus_item_consts(g, w, i, bc);
  bus_item_solve(sum, bc, out);
  w.dw[i] = out[2];
  w.dth[i] = out[3];
  w.nu[i] = out[0];
  w.nu[w.n_bus + i] = out[1];
  for (int j = 0; j < n; ++j) {
    const int code = (j < g1 - g0) ? -(w.bus_gen[g0 + j] + 1) : w.bus_end[e0 + j - (g1 - g0)];
    double v[14], a[8];
    bus_item_terms(w, code, v, a);
    bus_item_update<kTrace>(w, code, v, out, rr, ss, inf);
  }
}

// Step and multiplier estimates of line l (Section IV-B5).
ACOPF_HD void step_line(const acopf_grid& g, const acopf_iterate& x, const Workspace& w,
                        const acopf_iterate& d, int l) {
  const int L = w.n_line;
  const double* q = w.line;
  const int f = g.line_from[l], t = g.line_to[l];
  double aR[4], aI[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    aR[k] = q[(LF_AR + k) * L + l];
    aI[k] = q[(LF_AI + k) * L + l];
  }
  const double bR = q[LF_BR * L + l], bI = q[LF_BI * L + l];
  // step: elimination applied to the bus-side values
  const double zb[4] = {w.dw[f], w.dth[f], w.dw[t], w.dth[t]};
  d.wR[l] = aR[0] * zb[0] + aR[1] * zb[1] + aR[2] * zb[2] + aR[3] * zb[3] + bR;
  d.wI[l] = aI[0] * zb[0] + aI[1] * zb[1] + aI[2] * zb[2] + aI[3] * zb[3] + bI;
  // multipliers from the line subproblem's KKT conditions at its own solution
  double z[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) z[k] = w.xl[lc8(l, 4 + k)];
  const double u[6] = {z[0], z[1], aR[0] * z[0] + aR[1] * z[1] + aR[2] * z[2] + aR[3] * z[3] + bR,
                       aI[0] * z[0] + aI[1] * z[1] + aI[2] * z[2] + aI[3] * z[3] + bI, z[2], z[3]};
  double huR = 0.0, huI = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    huR += q[(LF_HR + k) * L + l] * u[k];
    huI += q[(LF_HI_ROW + k) * L + l] * u[k];
  }
  const double gij = g.gij[l], bij = g.bij[l], gji = g.gji[l], bji = g.bji[l];
  const double pij = q[(LF_PK + 0) * L + l], qij = q[(LF_PK + 1) * L + l];
  const double pji = q[(LF_PK + 2) * L + l], qji = q[(LF_PK + 3) * L + l];
  const double lam[4] = {w.lam_l[lc8(l, 0)], w.lam_l[lc8(l, 1)], w.lam_l[lc8(l, 2)], w.lam_l[lc8(l, 3)]};
  const double mu0 = w.mu[l], mu1 = w.mu[L + l];
  const double gR = huR + lam[0] * gij - lam[1] * bij + lam[2] * gji - lam[3] * bji +
                    mu0 * (2.0 * pij * gij - 2.0 * qij * bij) + mu1 * (2.0 * pji * gji - 2.0 * qji * bji);
  const double gI = huI + lam[0] * bij + lam[1] * gij - lam[2] * bji - lam[3] * gji +
                    mu0 * (2.0 * pij * bij + 2.0 * qij * gij) + mu1 * (-2.0 * pji * bji - 2.0 * qji * gji);
  const double ph = x.th[f] - x.th[t];
  const double s = sin(ph), c = cos(ph);
  const double wR = x.wR[l], wI = x.wI[l];
  // [2wR  s] [pi11]     [gR]
  // [2wI -c] [pi12] = - [gI]
  const double det = -2.0 * wR * c - 2.0 * wI * s;
  d.pi[l] = (gR * c + s * gI) / det;
  d.pi[L + l] = (-2.0 * wR * gI + 2.0 * wI * gR) / det;
  d.pi[2 * L + l] = -mu0;
  d.pi[3 * L + l] = -mu1;
}

}  // namespace acopf

namespace acopf {

// Merit pieces of line l (Section II-C) at x and at the trial point x + d:
// out[0] = h contribution at x, out[1] = at x + d, out[2] = m(d)
// contribution (linearised constraints), out[3] = the line's model
// quadratic 0.5 z^T M z + q^T z + 0.5 b^T H b at the bus-side step z.
ACOPF_HD void merit_line(const acopf_grid& g, const acopf_iterate& x, const Workspace& w,
                         const acopf_iterate& d, int l, double out[4]) {
  const int L = w.n_line;
  const int f = g.line_from[l], t = g.line_to[l];
  const double gii = g.gii[l], bii = g.bii[l], gij = g.gij[l], bij = g.bij[l];
  const double gji = g.gji[l], bji = g.bji[l], gjj = g.gjj[l], bjj = g.bjj[l];
  const double s2ij = g.smax_ij[l] * g.smax_ij[l], s2ji = g.smax_ji[l] * g.smax_ji[l];
  double hv[2];
#pragma unroll
  for (int trial = 0; trial < 2; ++trial) {
    const double a = trial ? 1.0 : 0.0;
    const double wi = x.w[f] + a * d.w[f], wj = x.w[t] + a * d.w[t];
    const double wR = x.wR[l] + a * d.wR[l], wI = x.wI[l] + a * d.wI[l];
    const double ph = (x.th[f] + a * d.th[f]) - (x.th[t] + a * d.th[t]);
    const double c11 = wR * wR + wI * wI - wi * wj;
    const double c12 = wR * sin(ph) - wI * cos(ph);
    const double pij = gii * wi + gij * wR + bij * wI, qij = -bii * wi - bij * wR + gij * wI;
    const double pji = gjj * wj + gji * wR - bji * wI, qji = -bjj * wj - bji * wR - gji * wI;
    const double c13 = s2ij - pij * pij - qij * qij, c14 = s2ji - pji * pji - qji * qji;
    hv[trial] = fabs(c11) + fabs(c12) + fmax(0.0, -c13) + fmax(0.0, -c14);
  }
  // linearised constraints at x along d
  const double wi = x.w[f], wj = x.w[t], wR = x.wR[l], wI = x.wI[l];
  const double ph = x.th[f] - x.th[t];
  const double s = sin(ph), c = cos(ph);
  const double K = wR * c + wI * s;
  const double c11 = wR * wR + wI * wI - wi * wj, c12 = wR * s - wI * c;
  const double pij = gii * wi + gij * wR + bij * wI, qij = -bii * wi - bij * wR + gij * wI;
  const double pji = gjj * wj + gji * wR - bji * wI, qji = -bjj * wj - bji * wR - gji * wI;
  const double c13 = s2ij - pij * pij - qij * qij, c14 = s2ji - pji * pji - qji * qji;
  const double dwi = d.w[f], dwj = d.w[t], dR = d.wR[l], dI = d.wI[l];
  const double l11 = c11 + 2.0 * wR * dR + 2.0 * wI * dI - wj * dwi - wi * dwj;
  const double l12 = c12 + s * dR - c * dI + K * (d.th[f] - d.th[t]);
  const double dpij = gii * dwi + gij * dR + bij * dI, dqij = -bii * dwi - bij * dR + gij * dI;
  const double dpji = gjj * dwj + gji * dR - bji * dI, dqji = -bjj * dwj - bji * dR - gji * dI;
  const double l13 = c13 - 2.0 * pij * dpij - 2.0 * qij * dqij;
  const double l14 = c14 - 2.0 * pji * dpji - 2.0 * qji * dqji;
  // model quadratic 0.5 u^T H u over the full step u = A z + b (eq. elim,
  // Section II-C): 0.5 z^T M z + q^T z + 0.5 b^T H b with the QP's reduced
  // (possibly projected) M
  const double z[4] = {d.w[f], d.th[f], d.w[t], d.th[t]};
  double Mp[10], M[4][4];
#pragma unroll
  for (int k = 0; k < 10; ++k) Mp[k] = w.line[(LF_M + k) * L + l];
  sym_unpack(Mp, M);
  double quad = w.line[LF_C0 * L + l];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double mz = M[i][0] * z[0] + M[i][1] * z[1] + M[i][2] * z[2] + M[i][3] * z[3];
    quad += 0.5 * z[i] * mz + w.line[(LF_Q + i) * L + l] * z[i];
  }
  out[0] = hv[0];
  out[1] = hv[1];
  out[2] = fabs(l11) + fabs(l12) + fmax(0.0, -l13) + fmax(0.0, -l14);
  out[3] = quad;
}

// Second-order error of the trial step d at line l: e = c(x + d) - c(x) -
// grad c(x)^T d for (opfc11-14), the shift of the correction QP.
ACOPF_HD void soc_error_line(const acopf_grid& g, const acopf_iterate& x, const acopf_iterate& d, int l,
                             double e[4]) {
  const int f = g.line_from[l], t = g.line_to[l];
  const double gii = g.gii[l], bii = g.bii[l], gij = g.gij[l], bij = g.bij[l];
  const double gji = g.gji[l], bji = g.bji[l], gjj = g.gjj[l], bjj = g.bjj[l];
  const double s2ij = g.smax_ij[l] * g.smax_ij[l], s2ji = g.smax_ji[l] * g.smax_ji[l];
  double cn[4];
  {
    const double wi = x.w[f] + d.w[f], wj = x.w[t] + d.w[t];
    const double wR = x.wR[l] + d.wR[l], wI = x.wI[l] + d.wI[l];
    const double ph = (x.th[f] + d.th[f]) - (x.th[t] + d.th[t]);
    const double pij = gii * wi + gij * wR + bij * wI, qij = -bii * wi - bij * wR + gij * wI;
    const double pji = gjj * wj + gji * wR - bji * wI, qji = -bjj * wj - bji * wR - gji * wI;
    cn[0] = wR * wR + wI * wI - wi * wj;
    cn[1] = wR * sin(ph) - wI * cos(ph);
    cn[2] = s2ij - pij * pij - qij * qij;
    cn[3] = s2ji - pji * pji - qji * qji;
  }
  const double wi = x.w[f], wj = x.w[t], wR = x.wR[l], wI = x.wI[l];
  const double ph = x.th[f] - x.th[t];
  const double s = sin(ph), c = cos(ph);
  const double K = wR * c + wI * s;
  const double pij = gii * wi + gij * wR + bij * wI, qij = -bii * wi - bij * wR + gij * wI;
  const double pji = gjj * wj + gji * wR - bji * wI, qji = -bjj * wj - bji * wR - gji * wI;
  const double dwi = d.w[f], dwj = d.w[t], dR = d.wR[l], dI = d.wI[l];
  const double l11 = wR * wR + wI * wI - wi * wj + 2.0 * wR * dR + 2.0 * wI * dI - wj * dwi - wi * dwj;
  const double l12 = wR * s - wI * c + s * dR - c * dI + K * (d.th[f] - d.th[t]);
  const double dpij = gii * dwi + gij * dR + bij * dI, dqij = -bii * dwi - bij * dR + gij * dI;
  const double dpji = gjj * dwj + gji * dR - bji * dI, dqji = -bjj * dwj - bji * dR - gji * dI;
  const double l13 = s2ij - pij * pij - qij * qij - 2.0 * pij * dpij - 2.0 * qij * dqij;
  const double l14 = s2ji - pji * pji - qji * qji - 2.0 * pji * dpji - 2.0 * qji * dqji;
  e[0] = cn[0] - l11;
  e[1] = cn[1] - l12;
  e[2] = cn[2] - l13;
  e[3] = cn[3] - l14;
}

// Objective pieces of generator k: f(p), f(p + d), model f'(p) d + 0.5 f'' d^2.
ACOPF_HD void merit_gen(const acopf_grid& g, const acopf_iterate& x, const acopf_iterate& d, int k,
                        double out[3]) {
  const double p = x.pg[k], dp = d.pg[k], pt = p + dp;
  out[0] = g.cost2[k] * p * p + g.cost1[k] * p;
  out[1] = g.cost2[k] * pt * pt + g.cost1[k] * pt;
  out[2] = (2.0 * g.cost2[k] * p + g.cost1[k]) * dp + g.cost2[k] * dp * dp;
}

// Residual report pieces.  Each routine returns maxima so the reduction is
// order independent.  primal[0..4] = balance, c11, c12, limit, bounds;
// dual = projected Lagrangian-gradient magnitude; gradf = |f'(p)|.
ACOPF_HD double proj_grad(double gr, double v, double lo, double hi) {
  const double tol = 1e-6;
  const bool atlo = v <= lo + tol, athi = v >= hi - tol;
  double r = fabs(gr);
  r = atlo ? fmax(-gr, 0.0) : r;
  r = athi ? fmax(gr, 0.0) : r;
  return (atlo && athi) ? 0.0 : r;
}

ACOPF_HD void residual_line(const acopf_grid& g, const acopf_iterate& x, const Workspace& w, int l,
                            double primal[5], double& dual) {
  const int L = w.n_line, B = w.n_bus;
  const int f = g.line_from[l], t = g.line_to[l];
  const double gii = g.gii[l], bii = g.bii[l], gij = g.gij[l], bij = g.bij[l];
  const double gji = g.gji[l], bji = g.bji[l], gjj = g.gjj[l], bjj = g.bjj[l];
  const double wi = x.w[f], wj = x.w[t], wR = x.wR[l], wI = x.wI[l];
  const double ph = x.th[f] - x.th[t];
  const double s = sin(ph), c = cos(ph);
  const double pij = gii * wi + gij * wR + bij * wI, qij = -bii * wi - bij * wR + gij * wI;
  const double pji = gjj * wj + gji * wR - bji * wI, qji = -bjj * wj - bji * wR - gji * wI;
  const double c11 = wR * wR + wI * wI - wi * wj, c12 = wR * s - wI * c;
  const double c13 = g.smax_ij[l] * g.smax_ij[l] - pij * pij - qij * qij;
  const double c14 = g.smax_ji[l] * g.smax_ji[l] - pji * pji - qji * qji;
  primal[1] = fabs(c11);
  primal[2] = fabs(c12);
  primal[3] = fmax(fmax(0.0, -c13), fmax(0.0, -c14));
  const double p11 = x.pi[l], p12 = x.pi[L + l], p13 = x.pi[2 * L + l], p14 = x.pi[3 * L + l];
  const double ypf = w.nu[f], yqf = w.nu[B + f], ypt = w.nu[t], yqt = w.nu[B + t];
  const double gR = -ypf * gij + yqf * bij - ypt * gji + yqt * bji + 2.0 * p11 * wR + p12 * s +
                    p13 * (-2.0 * pij * gij + 2.0 * qij * bij) + p14 * (-2.0 * pji * gji + 2.0 * qji * bji);
  const double gI = -ypf * bij - yqf * gij + ypt * bji + yqt * gji + 2.0 * p11 * wI - p12 * c +
                    p13 * (-2.0 * pij * bij - 2.0 * qij * gij) + p14 * (2.0 * pji * bji + 2.0 * qji * gji);
  dual = fmax(fabs(gR), fabs(gI));
}

ACOPF_HD void residual_bus(const acopf_grid& g, const acopf_iterate& x, const Workspace& w, int i,
                           double primal[5], double& dual) {
  const int L = w.n_line, B = w.n_bus;
  const double wi = x.w[i];
  const double yp = w.nu[i], yq = w.nu[B + i];
  double rp = -g.pd[i] - g.gsh[i] * wi, rq = -g.qd[i] + g.bsh[i] * wi;
  double gw = -g.gsh[i] * yp + g.bsh[i] * yq, gth = 0.0;
  for (int e = w.bus_gen_ptr[i]; e < w.bus_gen_ptr[i + 1]; ++e) {
    const int k = w.bus_gen[e];
    rp += x.pg[k];
    rq += x.qg[k];
  }
  for (int e = w.bus_end_ptr[i]; e < w.bus_end_ptr[i + 1]; ++e) {
    const int code = w.bus_end[e];
    const int l = code >> 1, side = code & 1;
    const int o = side ? g.line_from[l] : g.line_to[l];
    const double wo = x.w[o], wR = x.wR[l], wI = x.wI[l];
    const double p11 = x.pi[l], p12 = x.pi[L + l], p13 = x.pi[2 * L + l], p14 = x.pi[3 * L + l];
    const double ph = side ? (x.th[o] - x.th[i]) : (x.th[i] - x.th[o]);
    const double K = wR * cos(ph) + wI * sin(ph);
    if (side == 0) {
      const double gii = g.gii[l], bii = g.bii[l];
      const double p = gii * wi + g.gij[l] * wR + g.bij[l] * wI, q = -bii * wi - g.bij[l] * wR + g.gij[l] * wI;
      rp -= p;
      rq -= q;
      gw += -yp * gii + yq * bii - p11 * wo + p13 * (-2.0 * p * gii + 2.0 * q * bii);
      gth += p12 * K;
    } else {
      const double gjj = g.gjj[l], bjj = g.bjj[l];
      const double p = gjj * wi + g.gji[l] * wR - g.bji[l] * wI, q = -bjj * wi - g.bji[l] * wR - g.gji[l] * wI;
      rp -= p;
      rq -= q;
      gw += -yp * gjj + yq * bjj - p11 * wo + p14 * (-2.0 * p * gjj + 2.0 * q * bjj);
      gth -= p12 * K;
    }
  }
  const double v2lo = g.vmin[i] * g.vmin[i], v2hi = g.vmax[i] * g.vmax[i];
  primal[0] = fmax(fabs(rp), fabs(rq));
  const double thv = fmax(fmax(0.0, -(x.th[i] + kTwoPi)), fmax(0.0, x.th[i] - kTwoPi));
  primal[4] = fmax(fmax(fmax(0.0, v2lo - wi), fmax(0.0, wi - v2hi)), thv);
  dual = fmax(proj_grad(gw, wi, v2lo, v2hi), (w.bus_flags[i] & BUS_REF) ? 0.0 : fabs(gth));
}

ACOPF_HD void residual_gen(const acopf_grid& g, const acopf_iterate& x, const Workspace& w, int k,
                           double& bound, double& dual, double& gradf) {
  const int B = w.n_bus;
  const int i = g.gen_bus[k];
  const double p = x.pg[k], q = x.qg[k];
  const double fp = 2.0 * g.cost2[k] * p + g.cost1[k];
  bound = fmax(fmax(fmax(0.0, g.pmin[k] - p), fmax(0.0, p - g.pmax[k])),
               fmax(fmax(0.0, g.qmin[k] - q), fmax(0.0, q - g.qmax[k])));
  dual = fmax(proj_grad(fp + w.nu[i], p, g.pmin[k], g.pmax[k]), proj_grad(w.nu[B + i], q, g.qmin[k], g.qmax[k]));
  gradf = fabs(fp);
}

}  // namespace acopf
