// Device workspace of one grid: topology tables, QP data, ADMM state and
// reduction scratch, carved out of one caller-allocated buffer.  All arrays
// are structure-of-arrays with one entry per component so that consecutive
// threads touch consecutive addresses; field k of an array with n entries
// per field lives at [k * n + index].
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace acopf {

// Number of per-line FP64 fields written by the QP build.
enum LineField {
  LF_M = 0,        // 10: reduced Hessian (packed upper triangle)
  LF_Q = 10,       // 4: linear term A^T H b
  LF_F = 14,       // 16: flow map rows (p_ij, q_ij, p_ji, q_ji) x z
  LF_F0 = 30,      // 4: flow offsets
  LF_LO = 34,      // 4
  LF_HI = 38,      // 4
  LF_G = 42,       // 8: two limit rows
  LF_H = 50,       // 2
  LF_AR = 52,      // 4
  LF_BR = 56,      // 1
  LF_AI = 57,      // 4
  LF_BI = 61,      // 1
  LF_PK = 62,      // 4: flows at the iterate
  LF_C0 = 66,      // 1: 0.5 b^T H b
  LF_HR = 67,      // 6: row wR of the raw Hessian
  LF_HI_ROW = 73,  // 6: row wI of the raw Hessian
  LF_COUNT = 79
};

enum GenField { GF_FP = 0, GF_FPP, GF_PLO, GF_PHI, GF_QLO, GF_QHI, GF_COUNT };

struct SyncState {
  unsigned int count;      // grid-barrier arrivals
  unsigned int gen;        // grid-barrier generation
  int done;                // stop flag of the current solve
  int sweeps;              // sweeps completed
  int barrier_error;       // a barrier wait timed out
  int numeric_error;       // non-finite data / vanishing pivot in the QP build
  int nonconvex;           // raw mode: a line matrix failed its Cholesky
  int infeasible[2];       // infeasible line subproblems, by sweep parity
  int converged;           // the stop test held at the last sweep
  int blocks;              // grid size of the last solve
  unsigned int go;         // grid-barrier release epoch (persistent kernel)
  int pad;
  double r_norm, s_norm;
};

// Outcome of one trust-region SQP step (Algorithm 1), decided on the device.
struct SqpDecision {
  double f_x, f_xd, h_x, h_xd, m_d, quad;   // objective, merit h, model pieces
  double ared, pred, step_inf;
  double delta_in, delta_out;
  int accepted;
  int pad;
};

// Residual report (maxima; order independent).
struct ResidualReport {
  double balance, c11, c12, limit, bounds, dual, gradf;
};

constexpr int kMeritFields = 8;     // f_x, f_xd, quad_gen, h_x, h_xd, m_d, quad_line, step max
constexpr int kResidFields = 7;     // balance, c11, c12, limit, bounds, dual, gradf

struct Workspace {
  int32_t n_bus, n_line, n_gen, max_partials;
  // topology
  int32_t* bus_end_ptr;    // [n_bus + 1]
  int32_t* bus_end;        // [2 n_line] entry 2 l + side (0 from end, 1 to end)
  int32_t* bus_gen_ptr;    // [n_bus + 1]
  int32_t* bus_gen;        // [n_gen]
  // QP data
  double* line;            // [LF_COUNT][n_line]
  double* gen;             // [GF_COUNT][n_gen]
  double* bus_pdk;         // [n_bus]
  double* bus_qdk;         // [n_bus]
  // per-solve factorisation
  double* line_P;          // [10][n_line]  Q^{-1} packed
  double* line_cc;         // [4][n_line]   q + sum_f rho_f f0_f F_f
  // ADMM state
  double *xg, *xbar_g, *lam_g, *rho_g;   // [2][n_gen]
  double *xl, *lam_l, *rho_l;            // [8][n_line]
  double *xbar_f;                        // [4][n_line]
  double *dw, *dth, *nu;                 // [n_bus], [n_bus], [2][n_bus]
  double *mu;                            // [2][n_line]
  int32_t* line_mask;                    // [n_line] optimal working set of the last line solve
  // reductions
  double* partials;        // [2][max_partials]
  unsigned int* arrive;    // [max_partials * kArriveStride] grid-barrier arrival epochs
  double* merit_partials;  // [kMeritFields][max_partials]
  double* resid_partials;  // [kResidFields][max_partials]
  SyncState* sync;
  SqpDecision* decision;
  ResidualReport* report;
};

// Arrival flags of different blocks sit on different 128-byte lines.
constexpr int kArriveStride = 32;

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Lays the workspace out from base (or, with base == nullptr, only counts
// its size).  Returns the number of bytes used.
inline size_t layout_workspace(void* base, int32_t nb, int32_t nl, int32_t ng, Workspace* w) {
  size_t off = 0;
  char* b = static_cast<char*>(base);
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? (void*)(b + off) : nullptr;
    off += align_up(bytes);
    return p;
  };
  const size_t D = sizeof(double), I = sizeof(int32_t);
  int32_t maxp = 4096;
  int32_t need = (nb > nl ? nb : nl) / 64 + 64;
  if (need > maxp) maxp = need;
  Workspace t;
  t.n_bus = nb; t.n_line = nl; t.n_gen = ng; t.max_partials = maxp;
  t.bus_end_ptr = (int32_t*)take((size_t)(nb + 1) * I);
  t.bus_end = (int32_t*)take((size_t)2 * nl * I);
  t.bus_gen_ptr = (int32_t*)take((size_t)(nb + 1) * I);
  t.bus_gen = (int32_t*)take((size_t)(ng > 0 ? ng : 1) * I);
  t.line = (double*)take((size_t)LF_COUNT * nl * D);
  t.gen = (double*)take((size_t)GF_COUNT * ng * D);
  t.bus_pdk = (double*)take((size_t)nb * D);
  t.bus_qdk = (double*)take((size_t)nb * D);
  t.line_P = (double*)take((size_t)10 * nl * D);
  t.line_cc = (double*)take((size_t)4 * nl * D);
  t.xg = (double*)take((size_t)2 * ng * D);
  t.xbar_g = (double*)take((size_t)2 * ng * D);
  t.lam_g = (double*)take((size_t)2 * ng * D);
  t.rho_g = (double*)take((size_t)2 * ng * D);
  t.xl = (double*)take((size_t)8 * nl * D);
  t.lam_l = (double*)take((size_t)8 * nl * D);
  t.rho_l = (double*)take((size_t)8 * nl * D);
  t.xbar_f = (double*)take((size_t)4 * nl * D);
  t.dw = (double*)take((size_t)nb * D);
  t.dth = (double*)take((size_t)nb * D);
  t.nu = (double*)take((size_t)2 * nb * D);
  t.mu = (double*)take((size_t)2 * nl * D);
  t.line_mask = (int32_t*)take((size_t)nl * I);
  t.partials = (double*)take((size_t)2 * maxp * D);
  t.arrive = (unsigned int*)take((size_t)maxp * kArriveStride * sizeof(unsigned int));
  t.merit_partials = (double*)take((size_t)kMeritFields * maxp * D);
  t.resid_partials = (double*)take((size_t)kResidFields * maxp * D);
  t.sync = (SyncState*)take(sizeof(SyncState));
  t.decision = (SqpDecision*)take(sizeof(SqpDecision));
  t.report = (ResidualReport*)take(sizeof(ResidualReport));
  if (w) *w = t;
  return off;
}

}  // namespace acopf
