/*
 * acopf_admm.h -- C ABI of the MI355X (gfx950) ADMM QP solver for the SQP
 * method of "GPU-Accelerated Sequential Quadratic Programming Algorithm for
 * Solving ACOPF" (Li, Schanen, Kim; arXiv 2310.13143).
 *
 * Every array argument is a DEVICE pointer unless its comment says "host".
 * The caller owns all memory: it allocates the grid arrays, the iterate and
 * one workspace of acopf_workspace_bytes() bytes per grid; the library
 * never allocates or frees device memory.  Calls enqueue work on the given
 * HIP stream and return; results are valid once the stream has completed
 * (calls taking a host result pointer synchronise the stream themselves).
 * All arithmetic is FP64.  Indices are int32, zero based.  A workspace must
 * not be used by two calls at the same time.
 *
 * Errors: every entry point returns ACOPF_OK (0) or a negative
 * acopf_status; acopf_last_error() then describes the failure (per host
 * thread).  Convergence outcomes are not errors: they are reported in the
 * result structs.
 */
#ifndef ACOPF_ADMM_H
#define ACOPF_ADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ACOPF_OK = 0,
  ACOPF_ERR_INVALID_ARG = -1,     /* bad size, null pointer, index out of range */
  ACOPF_ERR_HIP = -2,             /* a HIP runtime call failed */
  ACOPF_ERR_NONCONVEX_LINE = -3,  /* raw Hessian mode: a line subproblem matrix is not positive definite */
  ACOPF_ERR_NUMERIC = -4,         /* non-finite data or a vanishing elimination pivot */
  ACOPF_ERR_UNSUPPORTED = -5,     /* request outside what the build supports */
  ACOPF_ERR_BARRIER = -6          /* the persistent sweep kernel's grid barrier timed out */
} acopf_status;

typedef enum {
  ACOPF_ADMM_CONVERGED = 0,       /* ||r|| <= eps_pri and ||s|| <= eps_dual (norm_inf) */
  ACOPF_ADMM_MAX_SWEEPS = 1,      /* stopped at max_sweeps */
  ACOPF_ADMM_FAILED = 2           /* not solved: the scenario's QP build or factorisation failed (status) */
} acopf_admm_outcome;

/* Line Hessians and line solver.  PSD: the reduced line Hessians are
 * projected onto the positive semidefinite cone and each line subproblem is
 * solved exactly.  RAW: the unmodified Hessians, solved exactly; a line
 * whose subproblem matrix is not positive definite fails the solve with
 * ACOPF_ERR_NONCONVEX_LINE.  RAW_LOCAL: the unmodified Hessians, every line
 * subproblem solved by the paper's local method, the augmented Lagrangian
 * over the slack form with a projected trust-region Newton inner solver
 * (Section IV-B2, eqs. line_kernel_simp1, line_kernel_alm), started from
 * the previous sweep's solution: on nonconvex lines it finds a local
 * minimiser. */
typedef enum { ACOPF_HESSIAN_PSD = 0, ACOPF_HESSIAN_RAW = 1, ACOPF_HESSIAN_RAW_LOCAL = 2 } acopf_hessian_mode;
/* How the sweeps of a solve are issued: one cooperative kernel for all
 * sweeps (single scenario); kernel launches per phase; or the same launches
 * replayed from an instantiated HIP graph of one chunk of sweeps (64; the
 * stop flag is read between chunks), built on first use and cached for the
 * process per workspace, grid arrays and launch parameters (at most 256
 * graphs; past that, and on a stream being captured, plain launches). */
typedef enum { ACOPF_SWEEP_PERSISTENT = 0, ACOPF_SWEEP_LAUNCHES = 1, ACOPF_SWEEP_GRAPH = 2 } acopf_sweep_mode;

/*
 * Network data of the ACOPF model (Section III-A, eqs. acopf and acopf_pf),
 * per unit.  Branch (i, j) = (line_from, line_to); g_ii + j b_ii, g_ij + j
 * b_ij, g_ji + j b_ji, g_jj + j b_jj are the entries of the branch's own
 * 2x2 admittance matrix used by the flow definitions; smax_* are the limits
 * s_bar (not squared).  Generator cost f(p) = cost2 p^2 + cost1 p.  Shunt
 * g_sh + j b_sh enters the balance as in (opfc5, opfc6).  Every bus must be
 * the end of at least one branch.
 *
 * A batch of independent scenarios (n_scen > 1) packs the scenarios' arrays
 * one after another; acopf_setup_batch gives their index ranges and
 * reference buses (ref_bus is then unused).  n_scen 0 or 1 = one grid.
 */
typedef struct {
  int32_t n_bus, n_line, n_gen, ref_bus;
  int32_t n_scen, reserved;
  const double *vmin, *vmax, *pd, *qd, *gsh, *bsh;                   /* [n_bus]  */
  const int32_t *line_from, *line_to;                                /* [n_line] */
  const double *gii, *bii, *gij, *bij, *gji, *bji, *gjj, *bjj;       /* [n_line] */
  const double *smax_ij, *smax_ji;                                   /* [n_line] */
  const int32_t *gen_bus;                                            /* [n_gen]  */
  const double *pmin, *pmax, *qmin, *qmax, *cost2, *cost1;           /* [n_gen]  */
} acopf_grid;

/* SQP iterate x^(k) (Section III-B) and line multipliers pi of (eq. lag):
 * pi[k * n_line + l] multiplies constraint (opfc11 + k) of line l, with the
 * paper's plus-sign Lagrangian (limits' multipliers are <= 0). */
typedef struct {
  double *pg, *qg;      /* [n_gen]      */
  double *w, *th;       /* [n_bus]      w = v^2, angle */
  double *wR, *wI;      /* [n_line]     */
  double *pi;           /* [4 * n_line] */
} acopf_iterate;

typedef struct {
  int32_t max_sweeps;   /* cap on ADMM iterations (Algorithm 2)                    */
  double eps_pri;       /* stop when ||r|| <= eps_pri ...                         */
  double eps_dual;      /* ... and ||s|| <= eps_dual (Section IV-B5; Euclidean
                           norms unless norm_inf); 0 = never                      */
  int32_t sweep_mode;   /* acopf_sweep_mode                                       */
  int32_t block_size;   /* threads per block, multiple of 64, <= 256; 0 = 256     */
  int32_t max_blocks;   /* persistent grid size cap; 0 = as many as fit resident  */
  int32_t trace;        /* 1 = also sum |r_c| and |s_c| of every coupling over the
                           sweeps (reset at the start of the solve; exported by
                           acopf_admm_state_get; launch-per-phase mode only)   */
  int32_t balance_every;/* residual balancing of the penalties after every
                           balance_every-th sweep (a multiple of 64; 0 = off;
                           launch-per-phase modes): all penalties of a scenario
                           times balance_tau when ||r|| > balance_mu ||s||,
                           divided by it when ||s|| > balance_mu ||r||; the
                           multipliers are not scaled.  The heuristic the paper
                           names beside its stop rule (Section IV-B5); the
                           final penalties are exported by acopf_admm_state_get */
  double balance_mu;    /* e.g. 10 */
  double balance_tau;   /* e.g. 2, > 1 */
  int32_t norm_inf;     /* 1: the stop test, r_norm and s_norm use infinity norms
                           (largest |r_c|, |s_c| over the couplings) instead of
                           Euclidean ones; 0 (default): Euclidean */
} acopf_admm_params;

typedef struct {
  int32_t sweeps;            /* sweeps run                                           */
  int32_t outcome;           /* acopf_admm_outcome                                   */
  double r_norm, s_norm;     /* ||r||, ||s|| of the last sweep (the solve's norm)    */
  int32_t infeasible_lines;  /* line subproblems without a feasible point, last sweep */
  int32_t blocks;            /* grid size the sweeps ran with                        */
  int32_t status;            /* 0, or ACOPF_ERR_NUMERIC / ACOPF_ERR_NONCONVEX_LINE when the
                                scenario's QP could not be built or factored (not solved) */
  int32_t relaxed_lines;     /* lines whose limit rows the QP build relaxed because the
                                line's box and linearised limits had no common point */
} acopf_admm_result;

/* Layout of an ADMM state held by the caller (export / warm start), line-
 * major like the coupling order of (eq. cpl):
 *   per generator 2 couplings (p, q): xg, xbar_g, lam_g, rho_g  [2 * n_gen], index c * n_gen + g
 *   per line 8 couplings (p_ij, q_ij, p_ji, q_ji, w_i, th_i, w_j, th_j):
 *       xl, lam_l, rho_l [8 * n_line], index c * n_line + l; xbar_f [4 * n_line] (flow copies)
 *   per bus: dw, dth [n_bus], nu [2 * n_bus] (balance multipliers, P rows then Q rows)
 *   per line: mu [2 * n_line] (multipliers of the two limit rows in the last line solve)
 * x is the generator/line side, xbar the bus side of a coupling.  A traced
 * solve (acopf_admm_params.trace) also sums, per coupling, |r_c| = |x_c -
 * xbar_c| and |s_c| = |rho_c (xbar_c - xbar_c of the sweep before)| over
 * its sweeps (Section IV-B5 residuals, per coupling). */
typedef struct {
  double *xg, *xbar_g, *lam_g, *rho_g;
  double *xl, *xbar_f, *lam_l, *rho_l;
  double *dw, *dth, *nu, *mu;
  double *sum_r_g, *sum_s_g;   /* [2 * n_gen]  sums of |r_c|, |s_c| of the last traced solve */
  double *sum_r_l, *sum_s_l;   /* [8 * n_line] */
} acopf_admm_state;

/* Bytes of device workspace for one grid or batch (QP data, ADMM state,
 * topology, reduction scratch); 0 for invalid sizes. */
size_t acopf_workspace_bytes(int32_t n_bus, int32_t n_line, int32_t n_gen, int32_t n_scen);

/* Validate the grid and build the bus incidence tables in the workspace.
 * Copies the three index arrays to the host once (synchronous).  Must be
 * called once per workspace, with the same grid, before any other call on
 * it; the library keeps no state outside the workspace. */
acopf_status acopf_setup(const acopf_grid* grid, void* workspace, size_t workspace_bytes,
                         void* stream);

/* Batched setup: scenario s owns buses [bus_offset[s], bus_offset[s+1]),
 * lines [line_offset[s], ...) and generators [gen_offset[s], ...) of the
 * packed arrays (host arrays of n_scen + 1 entries starting at 0 and ending
 * at the totals), and ref_bus[s] (host, global index) is its reference bus.
 * Lines and generators may only reference buses of their own scenario.
 * Every later call then works on all scenarios at once, each with its own
 * trust radius, stop test and SQP decision (a single grid is a batch of one). */
acopf_status acopf_setup_batch(const acopf_grid* grid, const int32_t* bus_offset, const int32_t* line_offset,
                               const int32_t* gen_offset, const int32_t* ref_bus, void* workspace,
                               size_t workspace_bytes, void* stream);

/* Set the per-scenario trust radii (device array of n_scen entries, > 0). */
acopf_status acopf_set_delta(const acopf_grid* grid, const double* delta, void* workspace, void* stream);

/* Build the QP subproblem (QPsub) at iterate x with trust radius delta
 * (delta > 0: every scenario; delta == 0: each scenario's radius held in the
 * workspace, see acopf_set_delta and acopf_sqp_step_batch):
 * elimination of d_wR, d_wI (eq. elim), line Hessian of (eq. lag) reduced
 * by A_ij (Section IV-B2; PSD-projected in ACOPF_HESSIAN_PSD mode), flow
 * map, linearised limits (opfqpc13, opfqpc14), boxes (opfqpc1-4 with the
 * trust region; the reference angle fixed), generator gradients and the
 * bus constants p^{d,(k)}, q^{d,(k)}.  A line whose box and linearised
 * limits have no common point gets its limit rows relaxed by the least-
 * squares violation over the box, plus a rounding guard of 1e-9 of the
 * rows' scale (the point the paper's augmented Lagrangian line solver runs
 * to on such a line, Section V; counted in relaxed_lines).  The Hessian
 * mode also picks the line solver of the solves that follow on this
 * workspace (exact, or the local ALM + TRON for ACOPF_HESSIAN_RAW_LOCAL).
 * Returns ACOPF_ERR_NUMERIC if a line has |wR cos + wI sin| < 1e-8 at x
 * (after the stream syncs this is reported by the next solve). */
acopf_status acopf_qp_build(const acopf_grid* grid, const acopf_iterate* x, double delta,
                            int32_t hessian_mode, void* workspace, void* stream);

/* Start an ADMM solve: copy the penalties rho (host-layout arrays of
 * acopf_admm_state, each entry > 0) and the warm-start multipliers
 * (lam_g, lam_l; NULL = cold start, all zero) into the workspace, zero the
 * primal values x, xbar and the bus values (Algorithm 2, line 1), and
 * factor each line subproblem matrix Q = M + sum rho_f F_f^T F_f +
 * diag(rho_v).  Requires a built QP. */
acopf_status acopf_admm_init(const acopf_grid* grid, const double* rho_g, const double* rho_l,
                             const double* lam_g, const double* lam_l, void* workspace, void* stream);

/* Run ADMM sweeps (Algorithm 2) from the workspace state until the stop
 * test of Section IV-B5 holds or max_sweeps: generator closed form (eq.
 * gen_kernel), line subproblem (eq. line_kernel: the dual active-set
 * method on the 4-variable strictly convex QP, or ALM + TRON in the
 * RAW_LOCAL mode), bus closed form (eq.
 * bus_kernel_simp), multiplier update (eq. multiplier), residuals.  If
 * result is non-NULL (host) the stream is synchronised and the result
 * copied; otherwise the result is kept in the workspace
 * (acopf_admm_result_get). */
acopf_status acopf_admm_solve(const acopf_grid* grid, const acopf_admm_params* params,
                              void* workspace, void* stream, acopf_admm_result* result);

/* Per-scenario results of the last solve (host array of n_scen entries;
 * synchronises the stream).  A scenario whose QP build met non-finite data
 * or a vanishing pivot, or whose line matrix could not be factored, is not
 * solved (outcome ACOPF_ADMM_FAILED, its status set); the other scenarios
 * are unaffected.  For a single grid (n_scen <= 1) such a failure is also
 * returned (ACOPF_ERR_NUMERIC, ACOPF_ERR_NONCONVEX_LINE); a batch returns
 * ACOPF_OK and reports failures per scenario.  ACOPF_ERR_BARRIER is always
 * returned. */
acopf_status acopf_admm_result_batch(const acopf_grid* grid, void* workspace, void* stream,
                                     acopf_admm_result* results);

/* Copy the last solve's result (scenario 0) to host memory (synchronises the stream). */
acopf_status acopf_admm_result_get(const acopf_grid* grid, void* workspace, void* stream,
                                   acopf_admm_result* result);

/* Export the ADMM state to caller arrays in the line-major layout above
 * (any member may be NULL to skip it). */
acopf_status acopf_admm_state_get(const acopf_grid* grid, void* workspace,
                                  const acopf_admm_state* out, void* stream);

/* Step returned to SQP and multiplier estimates (Section IV-B5): d_pg,
 * d_qg from the generator side, d_w, d_th from the bus side, d_wR, d_wI by
 * the elimination applied to the bus-side values; pi13, pi14 = -mu of the
 * last line solve, pi11, pi12 from the stationarity of the line subproblem
 * in (d_wR, d_wI) (a 2x2 solve).  Outputs: d (an iterate layout whose pi
 * member receives the new multipliers). */
acopf_status acopf_step(const acopf_grid* grid, const acopf_iterate* x, void* workspace,
                        const acopf_iterate* d, void* stream);

/* When an accepted step also replaces x.pi by the new estimates.  The
 * paper's Algorithm 1 always does (ACOPF_PI_ALWAYS).  ACOPF_PI_IF_CONVERGED
 * keeps the previous pi unless the solve met its stop test: on a QP without
 * a feasible point ADMM's multipliers grow with every sweep, and their
 * estimates would scale the next line Hessians without bound. */
typedef enum { ACOPF_PI_ALWAYS = 0, ACOPF_PI_IF_CONVERGED = 1 } acopf_pi_update;

/* Multipliers an SQP iteration's ADMM solve starts from (the primal
 * values always start at zero). */
typedef enum {
  ACOPF_START_ZERO = 0,      /* all zero                                              */
  ACOPF_START_PREVIOUS = 1,  /* the previous solve's in this workspace (zero after setup) */
  ACOPF_START_GIVEN = 2      /* acopf_sqp_params.lam_g0 / lam_l0 (e.g. acopf_warm_decode) */
} acopf_start;

/* One iteration of the basic trust-region SQP (Section II, Algorithm 1):
 * build the QP at x with radius state->delta, solve it by ADMM (params
 * admm, starting multipliers per warm_start, penalties rho_g, rho_l in the
 * layout of acopf_admm_state), form the step d (caller scratch in the
 * iterate layout) and multiplier estimates, evaluate the l1 merit
 * phi_1 = f + mu h and its model q (Section II-C), accept the step iff
 * ared > 0 and pred > 0, and update the radius: doubled (up to delta_max)
 * after an accepted step that reached it with ared >= grow_ratio * pred,
 * unchanged after another accepted step, 0.5 min(delta, ||d||_inf) after a
 * rejection.  On acceptance x <- x + d and x.pi <- the new estimates, on
 * the device.  Synchronises the stream and fills *state (host).
 *
 * With soc = 1 a rejected step with a positive predicted reduction gets a
 * second-order correction (the remedy the paper names as future work at the
 * end of Section II-D): e = c(x + d) - c(x) - grad c(x)^T d of (opfc11-14) is
 * added to c(x) in the linearised constraints, that QP is solved by ADMM
 * from the rejected solve's multipliers, and its step replaces d when its
 * actual reduction is positive (judged against the first step's pred; the
 * radius then grows as after any accepted step that reached it). */
typedef struct {
  double mu;             /* l1 merit penalty (the paper uses 1e5)         */
  double delta_max;      /* trust-radius cap                              */
  double grow_ratio;     /* radius growth threshold on ared / pred        */
  int32_t hessian_mode;  /* acopf_hessian_mode                            */
  int32_t warm_start;    /* acopf_start                                   */
  acopf_admm_params admm;
  const double* lam_g0;  /* ACOPF_START_GIVEN: starting multipliers,      */
  const double* lam_l0;  /* layout of acopf_admm_state (device)           */
  int32_t pi_update;     /* acopf_pi_update                               */
  int32_t soc;           /* 1: second-order correction of rejected steps  */
  /* Termination of a scenario's run on the device (Algorithm 1, the stop
   * rule after the algorithm): with stop = 1, after each iteration the
   * residual report is formed on the device and a scenario stops when its
   * step was accepted with primal <= tol_primal and dual <= tol_dual, or
   * accepted with ||d||_inf < tol_step, or its radius fell below
   * delta_min.  A stopped scenario's iterate, radius and multipliers are
   * frozen: later calls leave it out until acopf_set_delta starts a new
   * run.  See acopf_sqp_outcome_batch. */
  int32_t stop;
  /* restore = 1: this call takes a feasibility restoration step instead (a
   * remedy the paper names as missing, Section V): the QP with the same
   * linearised constraints (opfqpc5, opfqpc6, opfqpc11-14; lines without a
   * feasible point relaxed as in acopf_qp_build) and the objective
   * 0.5 ||d||^2 over (pg, qg, w, theta, wR, wI) (each bus variable's term
   * shared among its lines by 1/degree; pi and the costs unused; exact line
   * solver), within the radius held for the scenario.  The step is accepted
   * iff it lowers the constraint violation h of the merit function
   * (state->ared = h(x) - h(x + d), pred = 0); the radius and x.pi are left
   * as they are, and soc is ignored.  The caller calls it when a run's
   * radius has collapsed and restarts the radius after an accepted step. */
  int32_t restore;
  double tol_primal, tol_dual, tol_step, delta_min;
} acopf_sqp_params;

typedef struct {
  double delta;          /* in: radius of this iteration; out: the next  */
  int32_t accepted;      /* the step was accepted                         */
  int32_t admm_sweeps;   /* sweeps of this iteration's ADMM solve         */
  double ared, pred;     /* actual and predicted merit reduction          */
  double step_inf;       /* ||d||_inf over (pg, qg, w, th)                */
  double objective;      /* f at the returned iterate                     */
  double merit;          /* phi_1 at the returned iterate                 */
  double admm_r, admm_s; /* final ADMM residual norms                     */
  double admm_ms;        /* duration of the ADMM sweeps (HIP events on the stream) */
  int32_t status;        /* the scenario's acopf_admm_result.status; a failed QP
                            counts as a rejected step (radius halved)      */
  int32_t soc_sweeps;    /* sweeps of the second-order correction's solve (0: not tried);
                            accepted with soc_sweeps > 0: the corrected step was taken */
} acopf_sqp_state;

acopf_status acopf_sqp_step(const acopf_grid* grid, const acopf_iterate* x, const acopf_iterate* d,
                            const double* rho_g, const double* rho_l, const acopf_sqp_params* params,
                            void* workspace, void* stream, acopf_sqp_state* state);

/* The same step for every scenario of a batch, each with its own radius
 * (held in the workspace; set it with acopf_set_delta) and its own
 * decision.  states (host, n_scen entries) may be NULL: then nothing is
 * copied back and the call does not synchronise the stream.  With states =
 * NULL and eps_pri = eps_dual = 0 the call enqueues device work only, so a
 * caller may record it under stream capture and replay the graph as SQP
 * iterations (the iterate, radii and multipliers stay on the device).  Under
 * capture the ADMM stop test (eps > 0) runs on the device: every chunk of
 * sweeps up to max_sweeps is recorded, and launches of a stopped scenario
 * return at once; with stop = 1 stopped scenarios leave the later
 * iterations of the recorded loop. */
acopf_status acopf_sqp_step_batch(const acopf_grid* grid, const acopf_iterate* x, const acopf_iterate* d,
                                  const double* rho_g, const double* rho_l, const acopf_sqp_params* params,
                                  void* workspace, void* stream, acopf_sqp_state* states);

/* Per-scenario state of device-stopped SQP runs (acopf_sqp_params.stop). */
typedef struct {
  int32_t done;          /* the run has stopped                                     */
  int32_t reason;        /* 0 running; 1 primal and dual infeasibility met after an
                            accepted step; 2 accepted step below tol_step; 3 radius
                            below delta_min                                         */
  int32_t iterations;    /* SQP iterations taken (up to and including the stopping one) */
  int32_t reserved;
  double seconds;        /* device wall-clock time from acopf_set_delta to the stop
                            (0 while running)                                       */
} acopf_sqp_outcome;

/* Reads the per-scenario outcomes (host array of n_scen entries;
 * synchronises the stream). */
acopf_status acopf_sqp_outcome_batch(const acopf_grid* grid, void* workspace, void* stream, acopf_sqp_outcome* out);

/* Linear feasibility projection (Section II-A, eq. linfeas; Algorithm 1,
 * the step before its loop): replaces the start x (device arrays, updated
 * in place; x.pi is not touched) by the nearest point, in the Euclidean
 * norm over (pg, qg, w, theta, wR, wI), that meets the ACOPF's linear
 * constraints: power balance (opfc5, opfc6), bounds (opfc1-4), theta_ref
 * unchanged; wR, wI free (boxed at +-10 around x for the line solver).  A
 * positive distance certifies that x violated them.  Runs the identity-
 * Hessian QP through the ADMM sweeps of acopf_admm_solve (params:
 * max_sweeps, eps_pri, eps_dual, the launch or graph sweep mode, block
 * size; no trace or balancing): every penalty is rho (> 0), and each line
 * solves a 4-variable QP in (d_w_i, d_wR, d_w_j, d_wI) exactly.  The
 * workspace then holds the projection, not a QP subproblem: call
 * acopf_qp_build before the next acopf_admm_solve.  result (host, optional)
 * as acopf_admm_solve's, read after the iterate is updated.  Errors:
 * ACOPF_ERR_INVALID_ARG (null argument, rho <= 0), ACOPF_ERR_UNSUPPORTED
 * (persistent sweep mode, trace, balancing). */
acopf_status acopf_linfeas(const acopf_grid* grid, const acopf_iterate* x, double rho,
                           const acopf_admm_params* params, void* workspace, void* stream,
                           acopf_admm_result* result);

/* Infeasibility report of the ACOPF (eq. acopf) at x (synchronises; host
 * result): infinity norms of the power-balance residuals, of (opfc11),
 * (opfc12), of the line-limit violations and of the bound violations;
 * primal = their maximum; dual = infinity norm of the Lagrangian gradient
 * projected at active bounds, with the balance multipliers of the last bus
 * update and the line multipliers x.pi, divided by max(1, |f'|_inf). */
typedef struct {
  double primal, balance, c11, c12, limit, bounds, dual;
} acopf_residuals_report;

acopf_status acopf_residuals(const acopf_grid* grid, const acopf_iterate* x, void* workspace, void* stream,
                             acopf_residuals_report* out);

/* The report per scenario of a batch (host array of n_scen entries). */
acopf_status acopf_residuals_batch(const acopf_grid* grid, const acopf_iterate* x, void* workspace, void* stream,
                                   acopf_residuals_report* out);

/*
 * Learned warm start (an extension: the paper starts ADMM from zero or the
 * previous point).  A per-component network (acopf_mlp.h) maps local
 * features of each line and generator to a correction of the plain start of
 * its couplings' multipliers (the multipliers held in the workspace: the
 * previous solve's; zero at the first QP of an SQP run, `first`) and to a
 * factor on each coupling's penalty.
 *
 * Line features (ACOPF_LINE_FEATURES, in order): p_d, q_d of the from bus,
 * p_d, q_d of the to bus; g_ij, b_ij, g_ii, b_ii, g_jj, b_jj divided by 100;
 * w_i, w_j, wR, wI; sin(th_i - th_j); smax_ij; the 8 plain-start
 * multipliers divided by ACOPF_WARM_LAM_SCALE; 1 if `first`, else 0.  Generator features (ACOPF_GEN_FEATURES): p_d, q_d of its
 * bus; cost2 / 1e4; cost1 / 1e3; pg, qg; pmax, qmax; its 2 plain-start
 * multipliers / ACOPF_WARM_LAM_SCALE; the flag.  Outputs and training
 * targets (ACOPF_LINE_OUTPUTS per line: the change of the 8 multipliers over
 * a solve divided by ACOPF_WARM_LAM_SCALE, then 8 log penalty factors;
 * ACOPF_GEN_OUTPUTS per generator: the same for its 2 couplings).  The
 * target penalty factor of a coupling is the residual balance of a traced
 * solve, clip(sqrt((rho sum|r_c| + ACOPF_WARM_RHO_REG) / (sum|s_c| +
 * ACOPF_WARM_RHO_REG)), 1/ACOPF_WARM_RHO_CLIP, ACOPF_WARM_RHO_CLIP): the
 * regulariser gives factor 1 to couplings that never move (the reference
 * angle), whatever rounding noise their sums hold.  All feature, target and
 * output arrays are FP32, feature-major: feature f of component c at
 * a[f * ld + c].
 */
#define ACOPF_LINE_FEATURES 25
#define ACOPF_GEN_FEATURES 11
#define ACOPF_LINE_OUTPUTS 16
#define ACOPF_GEN_OUTPUTS 4
#define ACOPF_WARM_LAM_SCALE 1e3
#define ACOPF_WARM_RHO_CLIP 10.0
#define ACOPF_WARM_RHO_REG 1e-6

/* Features of every line and generator at iterate x (the workspace's
 * multipliers as the plain start, or zero if first = 1). */
acopf_status acopf_features(const acopf_grid* grid, const acopf_iterate* x, void* workspace, int32_t first,
                            float* line_x, int64_t ld_line, float* gen_x, int64_t ld_gen, void* stream);

/* Training targets from the last solve in the workspace: the change of its
 * multipliers from their start to their end and, from its trace sums (a
 * solve with trace = 1), the target log penalty factors. */
acopf_status acopf_warm_targets(const acopf_grid* grid, void* workspace, float* line_t, int64_t ld_line,
                                float* gen_t, int64_t ld_gen, void* stream);

/* Starting point from network outputs y: multipliers lam + y *
 * ACOPF_WARM_LAM_SCALE if use_lam, else lam (lam = the plain start: the
 * workspace's multipliers, or zero if first = 1); penalties rho0 exp(y) with y clipped to
 * +-log(ACOPF_WARM_RHO_CLIP) if use_rho, else rho0 (rho_l0 for lines, rho_g0
 * for generators, > 0).  A non-finite output keeps the plain start of its
 * coupling.  Outputs (device, layout of acopf_admm_state) feed
 * acopf_admm_init or acopf_sqp_step with ACOPF_START_GIVEN. */
acopf_status acopf_warm_decode(const acopf_grid* grid, void* workspace, const float* line_y, int64_t ld_line,
                               const float* gen_y, int64_t ld_gen, double rho_l0, double rho_g0, int32_t first,
                               int32_t use_lam, int32_t use_rho, double* lam_l, double* lam_g, double* rho_l,
                               double* rho_g, void* stream);

#ifdef __cplusplus
}
#endif

/* Last error message of the calling host thread (never NULL). */
#ifdef __cplusplus
extern "C"
#endif
const char* acopf_last_error(void);

#endif /* ACOPF_ADMM_H */
