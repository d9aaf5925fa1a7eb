// Device workspace of one batch of grids (a single grid is a batch of one):
// topology tables, QP data, ADMM state and reduction scratch, carved out of
// one caller-allocated buffer.  The scenarios of a batch are packed one after
// another (buses, lines and generators of scenario s occupy contiguous index
// ranges) and never reference each other's components.  Arrays are
// structure-of-arrays with one entry per component, so that consecutive
// threads touch consecutive addresses (field k of an array with n entries per
// field at [k * n + index]), except the lines' coupling state, which the bus
// update gathers per line end and which is therefore stored line by line
// (8 slots per line, ordered by line end; see lc8).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace acopf {

// Per-line FP64 fields written by the QP build.
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

// f', f'' of the active power's objective, its box, the reactive power's
// box, and the reactive power's f', f'' (zero in the SQP's QP, whose cost
// has no reactive term; one in the linear feasibility projection).
enum GenField { GF_FP = 0, GF_FPP, GF_PLO, GF_PHI, GF_QLO, GF_QHI, GF_FQ, GF_FQQ, GF_COUNT };

// hessian_mode value of a workspace holding the linear feasibility
// projection's QP (Section II-A, eq. linfeas) instead of an SQP subproblem.
constexpr int kModeLinfeas = 3;

// Line Hessian mode of a feasibility restoration step's QP: the objective
// 0.5 ||d||^2 in place of the Lagrangian's Hessian (build_line).
constexpr int kModeRestore = 4;

enum BusFlag { BUS_REF = 1 };

// Whole-batch synchronisation and error state.
struct SyncState {
  unsigned int go;         // grid-barrier release epoch (persistent kernel)
  int done;                // every scenario has stopped
  int n_done;              // scenarios stopped so far
  int barrier_error;       // a barrier wait timed out
  int numeric_error;       // non-finite data / vanishing pivot in the QP build
  int nonconvex;           // raw mode: a line matrix failed its Cholesky
  int blocks;              // grid size of the last solve
  int hessian_mode;        // acopf_hessian_mode of the last QP build, or kModeLinfeas
  int norm_inf;            // the running solve's stop test uses infinity norms
};

// Per-scenario ADMM and SQP state.
struct ScenState {
  int done;                // stopped (converged or at the sweep cap)
  int sweeps;              // sweeps completed
  int converged;           // the stop test held at the last sweep
  int infeasible[2];       // infeasible line subproblems, by sweep parity
  int status;              // 0, or the acopf_status of a failed QP build / factorisation
  int relaxed;             // lines whose limit rows the last QP build relaxed
  int skip;                // left out of the next solve (a second-order correction pass of other scenarios)
  double r_norm, s_norm;   // residual norms of the last sweep
  double delta;            // trust radius of the current SQP iteration
  double rho_factor;       // residual balancing: factor on the penalties decided after the last sweep
  int sqp_done;            // the SQP run of this scenario has stopped (its iterate is frozen)
  int sqp_reason;          // why: 1 primal and dual infeasibility met, 2 small accepted step, 3 radius collapse
  int sqp_iters;           // SQP iterations taken since the radius was set
  int pad2;
  long long t_start;       // device wall clock when the radius was set (start of the run)
  long long t_done;        // device wall clock when the run stopped
};

// Outcome of one trust-region SQP step (Algorithm 1), decided on the device.
struct SqpDecision {
  double f_x, f_xd, h_x, h_xd, m_d, quad;   // objective, merit h, model pieces
  double ared, pred, step_inf;
  double delta_in, delta_out;
  int accepted;
  int update_pi;           // accepted and the multiplier rule allows the new estimates
  int soc;                 // second-order correction: 0 none, 1 tried (step rejected), 2 taken
  int soc_sweeps;          // sweeps of the correction's ADMM solve
};

// Residual report (maxima; order independent).
struct ResidualReport {
  double balance, c11, c12, limit, bounds, dual, gradf;
};

// Arrival flags of different blocks sit on different 128-byte lines.
constexpr int kArriveStride = 32;
// Most blocks per scenario of the per-scenario reductions (merit sums,
// residual maxima): each writes its block's partial to Workspace::red.
constexpr int kRedBlocks = 256;

struct Workspace {
  int32_t n_bus, n_line, n_gen, n_scen, max_partials;
  // topology
  int32_t* bus_end_ptr;    // [n_bus + 1]
  int32_t* bus_end;        // [2 n_line] entry 2 l + side (0 from end, 1 to end)
  int32_t* bus_gen_ptr;    // [n_bus + 1]
  int32_t* bus_gen;        // [n_gen]
  int32_t* bus_scen;       // [n_bus] scenario of each bus
  int32_t* bus_flags;      // [n_bus] BusFlag bits
  int32_t* scen_bus_off;   // [n_scen + 1]
  int32_t* scen_line_off;  // [n_scen + 1]
  int32_t* scen_gen_off;   // [n_scen + 1]
  int32_t* line_blk_off;   // [n_scen + 1] first block of each scenario in the line phase
  int32_t* bus_blk_off;    // [n_scen + 1] same for the bus phase
  // bus phase by coupling items (launch modes): the generators, then the
  // line ends of each bus in consecutive slots of one block (kItemBlock slots)
  int32_t* item_code;      // [slots] 2 l + side for a line end, -(k + 1) for generator k, kItemBus, kItemPad
  int32_t* item_bus;       // [slots] bus of the item (-1 for padding)
  int32_t* item_head;      // [slots] slot (within the block) of the bus's first item
  int32_t* item_len;       // [slots] number of items of the bus
  int32_t* item_blk_off;   // [n_scen + 1] first item block of each scenario
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
  double *xl, *lam_l, *rho_l;            // [n_line][8] line by line
  double *xbar_f;                        // [n_line][4] line by line: bus-side flow copies
  double *xbar_v;                        // [n_line][4] line by line: the end buses' d_w, d_th (w_i, th_i, w_j, th_j)
  double *dw, *dth, *nu;                 // [n_bus], [n_bus], [2][n_bus]
  double *mu;                            // [2][n_line]
  int32_t* line_mask;                    // [n_line] optimal working set of the last line solve
  double *lam0_g, *lam0_l;               // [2][n_gen], [n_line][8] multipliers the last solve started from
  double* soc_e;                         // [4][n_line] second-order error of the trial step (correction QP)
  // per-coupling sums of |r_c| and |s_c| over the sweeps of a traced solve
  double *tr_r_g, *tr_s_g;               // [2][n_gen]
  double *tr_r_l, *tr_s_l;               // [8][n_line]
  // reductions
  double* partials;        // [2][max_partials]
  unsigned int* arrive;    // [max_partials * kArriveStride] grid-barrier arrival epochs
  double* line_comp;       // [4][n_line] per-component merit / residual pieces
  double* gen_comp;        // [4][n_gen]
  double* bus_comp;        // [3][n_bus]
  SyncState* sync;
  ScenState* scen;         // [n_scen]
  SqpDecision* decision;   // [n_scen]
  ResidualReport* report;  // [n_scen]
  double* red;             // [n_scen][kRedBlocks][8] block partials of the per-scenario reductions
};

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Item blocks of the bus phase, one thread per slot.  A bus's items never
// straddle two blocks, so two consecutive blocks of a scenario hold more
// slots than one block together; this bounds the block count by the sizes
// alone (blocks past a scenario's last one exit at once).  A bus with more
// items than a block takes one slot (kItemBus) whose thread runs the whole
// per-bus update.  Blocks have 64 slots, one wave each: a wave solves its
// buses with no workgroup barrier (with blocks in XCD order, faster than
// 128- and 256-slot blocks).  A bus-phase workgroup runs item_waves_for
// item blocks, one per wave, and adds their residual terms into one partial:
// on large grids four (the stop test then reads a quarter as many
// partials), on small, latency-bound ones one (the most workgroups, spread
// over the most CUs).  A scenario's item blocks start at a multiple of that
// count, so that a workgroup serves one scenario.
constexpr int32_t kItemPad = -0x7fffffff;
constexpr int32_t kItemBus = -0x7ffffffe;
constexpr int32_t kItemBlock = 64;
// Grids below this many lines run the line phase's wave search and
// one-wave bus-phase workgroups.
constexpr int32_t kSearchMaxLines = 16384;

inline int32_t item_waves_for(int32_t nl) { return nl < kSearchMaxLines ? 1 : 4; }

// Item blocks (a multiple of item_waves_for) for the sizes.
inline int32_t item_blocks_bound(int32_t nl, int32_t ng, int32_t ns) {
  const int64_t items = 2 * (int64_t)nl + ng, b = kItemBlock, wv = item_waves_for(nl);
  const int64_t n = 2 * ((items + b - 1) / b) + 2 * (int64_t)ns + 1 + (wv - 1) * ((int64_t)ns + 1);
  return (int32_t)((n + wv - 1) / wv * wv);
}

inline int32_t max_partials_for(int32_t nb, int32_t nl, int32_t ng, int32_t ns) {
  // bus-phase blocks of 64 threads (plus one partial block per scenario),
  // item blocks and the largest persistent grid
  int32_t need = (nb > nl ? nb : nl) / 64 + 2 * ns + 64;
  const int32_t items = item_blocks_bound(nl, ng, ns);
  need = need > items ? need : items;
  return need > 4096 ? need : 4096;
}

// Lays the workspace out from base (or, with base == nullptr, only counts
// its size).  Returns the number of bytes used.
inline size_t layout_workspace(void* base, int32_t nb, int32_t nl, int32_t ng, int32_t ns, Workspace* w) {
  size_t off = 0;
  char* b = static_cast<char*>(base);
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? (void*)(b + off) : nullptr;
    off += align_up(bytes > 0 ? bytes : 1);
    return p;
  };
  const size_t D = sizeof(double), I = sizeof(int32_t);
  const int32_t maxp = max_partials_for(nb, nl, ng, ns);
  Workspace t;
  t.n_bus = nb; t.n_line = nl; t.n_gen = ng; t.n_scen = ns; t.max_partials = maxp;
  t.bus_end_ptr = (int32_t*)take((size_t)(nb + 1) * I);
  t.bus_end = (int32_t*)take((size_t)2 * nl * I);
  t.bus_gen_ptr = (int32_t*)take((size_t)(nb + 1) * I);
  t.bus_gen = (int32_t*)take((size_t)ng * I);
  t.bus_scen = (int32_t*)take((size_t)nb * I);
  t.bus_flags = (int32_t*)take((size_t)nb * I);
  t.scen_bus_off = (int32_t*)take((size_t)(ns + 1) * I);
  t.scen_line_off = (int32_t*)take((size_t)(ns + 1) * I);
  t.scen_gen_off = (int32_t*)take((size_t)(ns + 1) * I);
  t.line_blk_off = (int32_t*)take((size_t)(ns + 1) * I);
  t.bus_blk_off = (int32_t*)take((size_t)(ns + 1) * I);
  const size_t slots = (size_t)item_blocks_bound(nl, ng, ns) * kItemBlock;
  t.item_code = (int32_t*)take(slots * I);
  t.item_bus = (int32_t*)take(slots * I);
  t.item_head = (int32_t*)take(slots * I);
  t.item_len = (int32_t*)take(slots * I);
  t.item_blk_off = (int32_t*)take((size_t)(ns + 1) * I);
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
  t.xbar_v = (double*)take((size_t)4 * nl * D);
  t.dw = (double*)take((size_t)nb * D);
  t.dth = (double*)take((size_t)nb * D);
  t.nu = (double*)take((size_t)2 * nb * D);
  t.mu = (double*)take((size_t)2 * nl * D);
  t.line_mask = (int32_t*)take((size_t)nl * I);
  t.lam0_g = (double*)take((size_t)2 * ng * D);
  t.lam0_l = (double*)take((size_t)8 * nl * D);
  t.soc_e = (double*)take((size_t)4 * nl * D);
  t.tr_r_g = (double*)take((size_t)2 * ng * D);
  t.tr_s_g = (double*)take((size_t)2 * ng * D);
  t.tr_r_l = (double*)take((size_t)8 * nl * D);
  t.tr_s_l = (double*)take((size_t)8 * nl * D);
  t.partials = (double*)take((size_t)2 * maxp * D);
  t.arrive = (unsigned int*)take((size_t)maxp * kArriveStride * sizeof(unsigned int));
  t.line_comp = (double*)take((size_t)4 * nl * D);
  t.gen_comp = (double*)take((size_t)4 * ng * D);
  t.bus_comp = (double*)take((size_t)3 * nb * D);
  t.sync = (SyncState*)take(sizeof(SyncState));
  t.scen = (ScenState*)take((size_t)ns * sizeof(ScenState));
  t.decision = (SqpDecision*)take((size_t)ns * sizeof(SqpDecision));
  t.report = (ResidualReport*)take((size_t)ns * sizeof(ResidualReport));
  t.red = (double*)take((size_t)ns * kRedBlocks * 8 * D);
  if (w) *w = t;
  return off;
}

}  // namespace acopf
