// MI355X (gfx950) kernels and C ABI of the ADMM QP solver for the SQP
// method for ACOPF (arXiv 2310.13143, Sections III-IV).
//
// One thread per component: the line update (the only non-closed-form
// subproblem) runs one 4-variable QP per lane; buses gather the couplings of
// their incident line ends and generators through CSR tables.  A sweep is
// phase A (lines) -> phase B (generators, buses, multipliers, residual
// partials) -> sweep end (fixed-order sums of the partials, stop test).
//
// A batch packs independent scenarios one after another.  In the
// launch-per-phase mode every block of a phase belongs to one scenario (a
// block table built on the device), so block partials are per scenario and
// each scenario stops on its own residuals; blocks of stopped scenarios exit
// at once.  The persistent mode (one cooperative launch for all sweeps, grid
// barriers between phases) serves a single scenario.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "components.h"
#include "errors.h"
#include "launch_order.h"
#include "linfeas.h"

using namespace acopf;

std::string& acopf::last_error() {
  thread_local std::string msg = "no error";
  return msg;
}

namespace {

constexpr int kDefaultBlock = 256;
// Most blocks of a sweep launch: its work items (blocks x up to 256
// threads, rounded up for the XCD order) must count below 2^32.
constexpr long long kMaxSweepBlocks = 1LL << 22;
constexpr long long kSpinLimit = 1LL << 25;
// Most lines per wave that the line phase's neighbour search serves.
constexpr int kSearchLines = 2;
// Sweeps enqueued between two looks at the stop flag (launch mode).
constexpr int kSweepChunk = 64;
// Learned warm start: multiplier scale and penalty-factor clip of the
// network's outputs.
constexpr double kLamScale = ACOPF_WARM_LAM_SCALE;
constexpr double kRhoClip = ACOPF_WARM_RHO_CLIP;
constexpr double kRhoReg = ACOPF_WARM_RHO_REG;

__device__ __forceinline__ int gtid() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int gstride() { return gridDim.x * blockDim.x; }

// Sum of v over the block in a fixed order (wave shuffles, then waves in order).
__device__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += lds[k];
  __syncthreads();
  return t;
}

// block_sum of two values at once (inf: their maxima), the result valid in
// thread 0 only (the same order and arithmetic as block_sum; two barriers
// instead of six).
__device__ void block_sum2_to_first(double& a, double& b, double* lds, bool inf = false) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ta = __shfl_xor(a, off, 64), tb = __shfl_xor(b, off, 64);
    a = inf ? fmax(a, ta) : a + ta;
    b = inf ? fmax(b, tb) : b + tb;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    lds[wave] = a;
    lds[8 + wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int k = 0; k < nw; ++k) ta = inf ? fmax(ta, lds[k]) : ta + lds[k];
    for (int k = 0; k < nw; ++k) tb = inf ? fmax(tb, lds[8 + k]) : tb + lds[8 + k];
    a = ta;
    b = tb;
  }
}

__device__ double block_max(double v, double* lds) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double m = 0.0;
  for (int k = 0; k < nw; ++k) m = fmax(m, lds[k]);
  __syncthreads();
  return m;
}

// Orders a wave's LDS stores before the loads of its other lanes (the
// fences of a workgroup barrier without the barrier: the exchange stays
// within one wave).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Scenario owning block b of a phase whose per-scenario first blocks are
// blk_off[0..ns]; -1 past the last block.
__device__ __forceinline__ int scen_of_block(const int32_t* blk_off, int ns, int b) {
  if (b >= blk_off[ns]) return -1;
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk_off[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Scenario owning component i of a kind whose per-scenario first indices are
// off[0..ns] (binary search).
__device__ __forceinline__ int scen_of_index(const int32_t* off, int ns, int i) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// A failed QP build or factorisation of a line marks its scenario (the
// most negative status wins) and the batch-wide flag.
__device__ void fail_line(const Workspace& w, int l, int status, int* flag) {
  atomicAdd(flag, 1);
  atomicMin(&w.scen[scen_of_index(w.scen_line_off, w.n_scen, l)].status, status);
}

// ---------------------------------------------------------------- QP build
// Setting the radii starts a new SQP run: the device stop state is cleared
// and the run's start time recorded.
__device__ void start_run(ScenState* sc, double delta) {
  sc->delta = delta;
  sc->sqp_done = 0;
  sc->sqp_reason = 0;
  sc->sqp_iters = 0;
  sc->t_start = wall_clock64();
  sc->t_done = 0;
}

__global__ void k_set_delta(Workspace w, double delta) {
  for (int s = gtid(); s < w.n_scen; s += gstride()) start_run(&w.scen[s], delta);
}

__global__ void k_copy_delta(Workspace w, const double* delta) {
  for (int s = gtid(); s < w.n_scen; s += gstride()) start_run(&w.scen[s], delta[s]);
}

// soc = 1: only the lines of scenarios taking a second-order correction,
// with the constraint shift of their trial step (soc_e).
__global__ void k_build_lines(acopf_grid g, acopf_iterate x, int mode, Workspace w, int soc) {
  const int L = g.n_line;
  for (int l = gtid(); l < L; l += gstride()) {
    const int s = w.bus_scen[g.line_from[l]];
    if (soc && w.decision[s].soc != 1) continue;
    ScenState* sc = &w.scen[s];
    double e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = soc ? w.soc_e[k * L + l] : 0.0;
    bool relaxed = false;
    // the correction QP has the rejected step's radius (k_decide has already
    // stored the next one)
    const double delta = soc ? w.decision[s].delta_in : sc->delta;
    if (!build_line(g, x, delta, mode, w, l, &relaxed, soc ? e : nullptr))
      fail_line(w, l, ACOPF_ERR_NUMERIC, &w.sync->numeric_error);
    if (relaxed) atomicAdd(&sc->relaxed, 1);
  }
}

__global__ void k_build_gens(acopf_grid g, acopf_iterate x, Workspace w, int restore) {
  for (int k = gtid(); k < g.n_gen; k += gstride())
    build_gen(g, x, w.scen[w.bus_scen[g.gen_bus[k]]].delta, w, k, restore != 0);
}

__global__ void k_build_buses(acopf_grid g, acopf_iterate x, Workspace w) {
  for (int i = gtid(); i < g.n_bus; i += gstride()) build_bus(g, x, w, i);
}

// QP of the linear feasibility projection at the start x (lines, generators;
// the buses take k_build_buses).
__global__ void k_build_lines_linfeas(acopf_grid g, acopf_iterate x, Workspace w) {
  for (int l = gtid(); l < g.n_line; l += gstride()) build_line_linfeas(g, x, w, l);
}

__global__ void k_build_gens_linfeas(acopf_grid g, acopf_iterate x, Workspace w) {
  for (int k = gtid(); k < g.n_gen; k += gstride()) build_gen_linfeas(g, x, w, k);
}

// x <- x + d of the projection: generators and buses from their ADMM values,
// wR, wI from the lines' own values.
__global__ void k_apply_linfeas(acopf_grid g, acopf_iterate x, Workspace w) {
  const int G = g.n_gen, L = g.n_line, B = g.n_bus;
  for (int t = gtid(); t < G + B + L; t += gstride()) {
    if (t < G) {
      x.pg[t] += w.xg[t];
      x.qg[t] += w.xg[G + t];
    } else if (t < G + B) {
      const int i = t - G;
      x.w[i] += w.dw[i];
      x.th[i] += w.dth[i];
    } else {
      const int l = t - G - B;
      x.wR[l] += w.mu[l];
      x.wI[l] += w.mu[L + l];
    }
  }
}

// ---------------------------------------------------------------- ADMM init
__global__ void k_fill(double* p, long long n, double v) {
  for (long long i = gtid(); i < n; i += gstride()) p[i] = v;
}

__global__ void k_fill_int(int32_t* p, long long n, int32_t v) {
  for (long long i = gtid(); i < n; i += gstride()) p[i] = v;
}

__global__ void k_copy(double* dst, const double* src, long long n) {
  for (long long i = gtid(); i < n; i += gstride()) dst[i] = src[i];
}

// Line-by-line coupling state (8 slots per line, lc8) from / to the
// field-by-field layout [8][n] of the C ABI.
__global__ void k_fields_to_lines(double* dst, const double* src, int n) {
  const long long total = 8LL * n;
  for (long long e = gtid(); e < total; e += gstride()) {
    const int i = (int)(e / 8), f = (int)(e - 8LL * i);
    dst[lc8(i, f)] = src[(long long)f * n + i];
  }
}

__global__ void k_lines_to_fields(double* dst, const double* src, int n) {
  const long long total = 8LL * n;
  for (long long e = gtid(); e < total; e += gstride()) {
    const int f = (int)(e / n), i = (int)(e - (long long)f * n);
    dst[e] = src[lc8(i, f)];
  }
}

// Line-by-line [n][4] arrays (bus-side copies) to the layout [4][n].
__global__ void k_lines4_to_fields(double* dst, const double* src, int n) {
  const long long total = 4LL * n;
  for (long long e = gtid(); e < total; e += gstride()) {
    const int f = (int)(e / n), i = (int)(e - (long long)f * n);
    dst[e] = src[lc4(i, f)];
  }
}

__global__ void k_prep_lines(Workspace w) {
  for (int l = gtid(); l < w.n_line; l += gstride())
    if (!prep_line(w, l)) fail_line(w, l, ACOPF_ERR_NONCONVEX_LINE, &w.sync->nonconvex);
}

__global__ void k_clear_flags(Workspace w, int mode) {
  if (gtid() == 0) {
    w.sync->numeric_error = 0;
    w.sync->nonconvex = 0;
    w.sync->hessian_mode = mode;
  }
  for (int s = gtid(); s < w.n_scen; s += gstride()) {
    w.scen[s].status = 0;
    w.scen[s].relaxed = 0;
    w.scen[s].skip = 0;
  }
}

// Start of a solve: per-scenario stop state, barrier flags, block tables of
// both phases for block size bs.  items: the bus phase runs by workgroups
// of that many item blocks (0: by buses).
__global__ void k_reset_solve(Workspace w, int blocks, int bs, int items, int norm_inf) {
  for (int b = gtid(); b < w.max_partials; b += gstride()) w.arrive[b * kArriveStride] = 0u;
  for (int s = gtid(); s < w.n_scen; s += gstride()) {
    ScenState* sc = &w.scen[s];
    if (sc->skip) {  // left out: its results of the last solve stay
      sc->done = 1;
      continue;
    }
    sc->done = sc->status != 0 ? 1 : 0;  // a failed QP is not solved
    sc->sweeps = 0;
    sc->converged = 0;
    sc->infeasible[0] = 0;
    sc->infeasible[1] = 0;
    sc->r_norm = 0.0;
    sc->s_norm = 0.0;
  }
  if (gtid() == 0) {
    SyncState* sy = w.sync;
    int failed = 0;
    for (int s = 0; s < w.n_scen; ++s) failed += (w.scen[s].status != 0 || w.scen[s].skip) ? 1 : 0;
    sy->go = 0u;
    sy->done = failed == w.n_scen ? 1 : 0;
    sy->n_done = failed;
    sy->barrier_error = 0;
    sy->blocks = blocks;
    sy->norm_inf = norm_inf;
    int lb = 0, bb = 0;
    for (int s = 0; s < w.n_scen; ++s) {
      w.line_blk_off[s] = lb;
      w.bus_blk_off[s] = bb;
      lb += (w.scen_line_off[s + 1] - w.scen_line_off[s] + bs - 1) / bs;
      bb += (w.scen_bus_off[s + 1] - w.scen_bus_off[s] + bs - 1) / bs;
    }
    w.line_blk_off[w.n_scen] = lb;
    w.bus_blk_off[w.n_scen] = bb;
    if (items)  // the bus phase runs by item blocks: its partials follow them
      for (int s = 0; s <= w.n_scen; ++s) w.bus_blk_off[s] = w.item_blk_off[s] / items;
  }
}

// ---------------------------------------------------------------- sweeps
// Sum of scenario s's partials [p0, p1) (fixed order), stop decision.
__device__ void finish_scenario(const Workspace& w, int s, int p0, int p1, int max_sweeps, double eps_pri,
                                double eps_dual, double* lds) {
  const bool inf = w.sync->norm_inf != 0;
  double r2 = 0.0, s2 = 0.0;
  for (int b = p0 + (int)threadIdx.x; b < p1; b += blockDim.x) {
    acc_norm(r2, w.partials[b], inf);
    acc_norm(s2, w.partials[w.max_partials + b], inf);
  }
  r2 = inf ? block_max(r2, lds) : block_sum(r2, lds);
  s2 = inf ? block_max(s2, lds) : block_sum(s2, lds);
  if (threadIdx.x == 0) {
    ScenState* sc = &w.scen[s];
    const int k = sc->sweeps + 1;
    sc->sweeps = k;
    const double r = sqrt(r2), sn = sqrt(s2);
    sc->r_norm = r;
    sc->s_norm = sn;
    const bool conv = (eps_pri > 0.0 || eps_dual > 0.0) && r <= eps_pri && sn <= eps_dual;
    sc->converged = conv ? 1 : 0;
    sc->infeasible[k & 1] = 0;  // counter of the next sweep
    if (conv || k >= max_sweeps || w.sync->barrier_error) {
      sc->done = 1;
      if (atomicAdd(&w.sync->n_done, 1) + 1 == w.n_scen) w.sync->done = 1;
    }
  }
}

// Launch modes end a sweep without a kernel of their own: the next line
// phase evaluates the stop test of the sweep before it, every block from
// the same partials, and one kernel per chunk of sweeps (k_finish_phase)
// records the norms of the chunk's last sweep.  The bus phase counts the
// sweeps, so the count a line block reads is never written during its
// kernel.
//
// Residual sums of a scenario's last sweep from its bus-phase partials
// [p0, p1): the first wave adds them lane-strided, then by a butterfly of
// shuffles (every lane ends with the same bits), so each kernel that
// evaluates the stop test gets the same value.  Valid in the first wave.
// kInf: the partials are maxima of squares (infinity norms); a template
// parameter, so that the Euclidean sum is a plain chain of adds.
template <bool kInf>
__device__ void sweep_sums(const Workspace& w, int p0, int p1, double& r2, double& s2) {
  constexpr bool inf = kInf;
  double a = 0.0, b = 0.0;
  if (threadIdx.x < 64) {
    // up to 16 partials per lane are loaded before any is added (one round
    // of memory latency for up to 1,024 bus blocks), then added in order
    for (int k0 = p0 + (int)threadIdx.x; k0 < p1; k0 += 16 * 64) {
      double ra[16], rb[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int k = k0 + 64 * j;
        ra[j] = k < p1 ? w.partials[k] : 0.0;
        rb[j] = k < p1 ? w.partials[w.max_partials + k] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc_norm(a, ra[j], inf);
        acc_norm(b, rb[j], inf);
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    acc_norm(a, __shfl_xor(a, off, 64), inf);
    acc_norm(b, __shfl_xor(b, off, 64), inf);
  }
  r2 = a;
  s2 = b;
}

__device__ __forceinline__ bool stop_met(double r2, double s2, double eps_pri, double eps_dual) {
  return (eps_pri > 0.0 || eps_dual > 0.0) && sqrt(r2) <= eps_pri && sqrt(s2) <= eps_dual;
}

// Norms and stop state of scenario s after its last sweep (one thread).
__device__ void record_sweep(const Workspace& w, int s, double r2, double s2, bool stop, double eps_pri,
                             double eps_dual) {
  ScenState* sc = &w.scen[s];
  sc->r_norm = sqrt(r2);
  sc->s_norm = sqrt(s2);
  sc->converged = stop_met(r2, s2, eps_pri, eps_dual) ? 1 : 0;
  if (stop) {
    sc->done = 1;
    if (atomicAdd(&w.sync->n_done, 1) + 1 == w.n_scen) w.sync->done = 1;
  }
}

__device__ __forceinline__ bool batch_done(const Workspace& w) {
  return __hip_atomic_load(&w.sync->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// `single`: one scenario, ceil(n / block) blocks used (the launch rounded up
// to the XCD order's multiple of 8), so a block needs no table lookup (one
// flag read before the line work).  Blocks b are logical: in XCD order
// (xcd_block) with kXcdOrder, else in workgroup order.  At
// most 256 registers per lane: two waves per SIMD (measured faster than one
// wave with more registers; a cap of three waves spills hundreds of bytes).
// Start of a line-phase block: its scenario s and, with `test`, the stop
// test of the previous sweep (launch modes; 1 on Euclidean norms, 2 on
// infinity norms, an argument so that no flag load precedes the test).
// False when the block has nothing to do (scenario done or stopped now).
template <bool kXcdOrder>
__device__ __forceinline__ int line_block(int n) {
  if (kXcdOrder) return xcd_block(blockIdx.x, n);
  return (int)blockIdx.x < n ? (int)blockIdx.x : -1;
}

template <bool kXcdOrder>
__device__ __forceinline__ bool line_phase_begin(const Workspace& w, int single, int test, double eps_pri,
                                                 double eps_dual, int& s, int& b, int* s_stop) {
  s = 0;
  if (single) {
    if (w.scen[0].done) return false;
    b = line_block<kXcdOrder>((w.n_line + (int)blockDim.x - 1) / (int)blockDim.x);
    if (b < 0) return false;
  } else {
    if (batch_done(w)) return false;
    b = line_block<kXcdOrder>(w.line_blk_off[w.n_scen]);
    s = b < 0 ? -1 : scen_of_block(w.line_blk_off, w.n_scen, b);
    if (s < 0 || w.scen[s].done) return false;
  }
  if (test) {
    double r2, s2;
    if (test == 2) sweep_sums<true>(w, w.bus_blk_off[s], w.bus_blk_off[s + 1], r2, s2);
    else sweep_sums<false>(w, w.bus_blk_off[s], w.bus_blk_off[s + 1], r2, s2);
    if (threadIdx.x == 0) {
      const bool stop = stop_met(r2, s2, eps_pri, eps_dual);
      // the scenario's first block records the stop; every block obeys it
      if (stop && b == (single ? 0 : w.line_blk_off[s])) record_sweep(w, s, r2, s2, true, eps_pri, eps_dual);
      *s_stop = stop ? 1 : 0;
    }
    __syncthreads();
    if (*s_stop) return false;
  }
  return true;
}

// Line of this thread in scenario s, -1 past the scenario's lines.
__device__ __forceinline__ int line_of_thread(const Workspace& w, int single, int s, int b) {
  const int l = single ? (int)(b * blockDim.x + threadIdx.x)
                       : w.scen_line_off[s] + (int)((b - w.line_blk_off[s]) * blockDim.x + threadIdx.x);
  return l < (single ? w.n_line : w.scen_line_off[s + 1]) ? l : -1;
}

// `test`: first evaluate the stop test of the previous sweep (launch modes;
// 1 Euclidean, 2 infinity norms).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_line_phase(acopf_grid g, Workspace w, int single, int test, int search, double eps_pri, double eps_dual) {
  __shared__ int s_stop;
  int s, b;
  if (!line_phase_begin<true>(w, single, test, eps_pri, eps_dual, s, b, &s_stop)) return;
  const int l = line_of_thread(w, single, s, b);
  if (l < 0) return;
  // one full solve per thread (the exact solver's own warm start and guess)
  if (!search) {
    if (update_line(g, w, l) != 0) atomicAdd(&w.scen[s].infeasible[w.scen[s].sweeps & 1], 1);
    return;
  }
  // 1. the warm working set or the primal-dual guess settles most lines
  int base = 0;
  bool left = !update_line_fast(w, l, base);
  // 2. for each line they leave, the wave's threads check the neighbours of
  // its last working set at once (one per thread; the line's data are
  // loaded by every thread from the same addresses); the first thread
  // whose set passes the KKT check stores the result.  The searches run one
  // line after another while the dual method runs the wave's lines
  // together, so only a wave with at most kSearchLines such lines searches.
  // Used for small, latency-bound grids (`search`): there it shortens the
  // wave's tail; on large grids and batches it measured slower.
  const int lane = (int)__lane_id();
  unsigned long long todo = __ballot(left);
  if (__popcll(todo) > kSearchLines) todo = 0ull;
  while (todo != 0ull) {
    const int f = __ffsll((long long)todo) - 1;
    todo &= todo - 1ull;
    const int lf = __shfl(l, f), bf = __shfl(base, f);
    LineQPResult r;
    const bool ok = line_neighbour_check(w, lf, bf, lane, r);
    const unsigned long long hit = __ballot(ok);
    if (hit != 0ull) {
      if (lane == __ffsll((long long)hit) - 1) line_sweep_store(w, lf, r);
      if (lane == f) left = false;
    }
  }
  // 3. the dual active-set method for the rest; an opaque copy of the index
  // keeps the compiler from carrying step 1's values across steps 2 and 3
  if (left) {
    int lr = l;
    asm volatile("" : "+v"(lr));
    if (update_line(g, w, lr) != 0) atomicAdd(&w.scen[s].infeasible[w.scen[s].sweeps & 1], 1);
  }
}

// Line phase with the local line solver (hessian mode RAW_LOCAL): one
// ALM + TRON solve per thread.  A kernel of its own, so that the exact
// solver's kernel keeps its register budget.  Its blocks run in workgroup
// order: the solve is compute-bound and its cost varies from line to line,
// and contiguous runs of blocks per XCD measured slower (spatial clusters
// of expensive lines land on one XCD).
__global__ void __launch_bounds__(256)
k_line_phase_local(Workspace w, int single, int test, double eps_pri, double eps_dual) {
  __shared__ int s_stop;
  int s, b;
  if (!line_phase_begin<false>(w, single, test, eps_pri, eps_dual, s, b, &s_stop)) return;
  const int l = line_of_thread(w, single, s, b);
  if (l < 0) return;
  if (update_line_local(w, l) != 0) atomicAdd(&w.scen[s].infeasible[w.scen[s].sweeps & 1], 1);
}

// Line phase of the linear feasibility projection: one exact solve per
// thread from the line's previous working set.
__global__ void __launch_bounds__(256)
k_line_phase_linfeas(Workspace w, int single, int test, double eps_pri, double eps_dual) {
  __shared__ int s_stop;
  int s, b;
  if (!line_phase_begin<true>(w, single, test, eps_pri, eps_dual, s, b, &s_stop)) return;
  const int l = line_of_thread(w, single, s, b);
  if (l < 0) return;
  if (update_line_linfeas(w, l) != 0) atomicAdd(&w.scen[s].infeasible[w.scen[s].sweeps & 1], 1);
}

// Bus phase by coupling items (launch modes): one thread per line end or
// generator, the items of a bus in consecutive threads of one block.  Each
// thread loads its item's couplings and writes its terms of the bus sums to
// LDS; the bus's first thread adds them (fixed order) and solves the bus's
// closed form; then every thread updates its couplings.  A bus of degree d
// costs one round of independent loads on d threads instead of a
// dependent walk over its CSR on one.  Each wave runs one item block on its
// own (the item block is the wave: its lanes exchange terms through LDS
// without a workgroup barrier); workgroup b runs item blocks
// [kWaves b, kWaves (b + 1)), taken in XCD order (xcd_block), and writes
// one partial.  Workgroups past a scenario's last item block exit at
// once; the scenario's first workgroup counts the sweep.  kInf: the
// residual partials are maxima of squares (infinity norms), a template
// parameter so that the Euclidean kernel carries no selects.
template <bool kTrace, bool kInf, int kWaves>
__global__ void __launch_bounds__(kItemBlock * kWaves) k_bus_items(acopf_grid g, Workspace w, int single) {
  constexpr int kThreads = kItemBlock * kWaves;
  __shared__ double terms[8][kThreads];
  __shared__ double bres[6][kThreads];
  __shared__ double lds[16];
  int s = 0, b;
  if (single) {
    if (w.scen[0].done) return;
    b = xcd_block(blockIdx.x, w.item_blk_off[1] / kWaves);
    if (b < 0) return;
  } else {
    if (batch_done(w)) return;
    b = xcd_block(blockIdx.x, w.item_blk_off[w.n_scen] / kWaves);
    s = b < 0 ? -1 : scen_of_block(w.item_blk_off, w.n_scen, b * kWaves);
    if (s < 0 || w.scen[s].done) return;
  }
  const int t = threadIdx.x, seg = t & ~(kItemBlock - 1);  // seg: the wave's item block in LDS
  const size_t slot = (size_t)b * kThreads + t;
  const int code = w.item_code[slot], bus = w.item_bus[slot], head = w.item_head[slot], len = w.item_len[slot];
  constexpr bool inf = kInf;
  const bool whole = code == kItemBus;  // a bus wider than a block: its thread walks all its items
  const bool lead = bus >= 0 && t - seg == head && !whole;
  double bc[7];
  if (lead) bus_item_consts(g, w, bus, bc);
  double v[14], a[8];
  bus_item_terms(w, code, v, a);
#pragma unroll
  for (int m = 0; m < 8; ++m) terms[m][t] = a[m];
  wave_lds_sync();
  if (lead) {
    double sum[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < len; ++j)
#pragma unroll
      for (int m = 0; m < 8; ++m) sum[m] += terms[m][t + j];
    double out[6];
    bus_item_solve(sum, bc, out);
    w.dw[bus] = out[2];
    w.dth[bus] = out[3];
    w.nu[bus] = out[0];
    w.nu[w.n_bus + bus] = out[1];
#pragma unroll
    for (int m = 0; m < 6; ++m) bres[m][t] = out[m];
  }
  wave_lds_sync();
  double rr = 0.0, ss = 0.0;
  if (whole) {
    bus_whole_update<kTrace>(g, w, bus, rr, ss, inf);
  } else if (bus >= 0) {
    double res[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) res[m] = bres[m][seg + head];
    bus_item_update<kTrace>(w, code, v, res, rr, ss, inf);
  }
  block_sum2_to_first(rr, ss, lds, inf);
  if (t == 0) {
    w.partials[b] = rr;
    w.partials[w.max_partials + b] = ss;
    if (b * kWaves == w.item_blk_off[s]) {
      ScenState* sc = &w.scen[s];
      const int k = sc->sweeps + 1;
      sc->sweeps = k;
      sc->infeasible[k & 1] = 0;  // counter of the next sweep
    }
  }
}

// End of a chunk of launch-mode sweeps: records the norms of each running
// scenario's last sweep and applies its stop test and the sweep cap.  One
// 64-thread block per scenario.
__global__ void k_finish_phase(Workspace w, int max_sweeps, double eps_pri, double eps_dual) {
  const int s = blockIdx.x;
  if (w.sync->done || w.scen[s].done) return;
  double r2, s2;
  if (w.sync->norm_inf) sweep_sums<true>(w, w.bus_blk_off[s], w.bus_blk_off[s + 1], r2, s2);
  else sweep_sums<false>(w, w.bus_blk_off[s], w.bus_blk_off[s + 1], r2, s2);
  if (threadIdx.x == 0) {
    const bool stop = stop_met(r2, s2, eps_pri, eps_dual) || w.scen[s].sweeps >= max_sweeps;
    record_sweep(w, s, r2, s2, stop, eps_pri, eps_dual);
  }
}

// Residual balancing after a sweep (one thread per scenario): the factor on
// the penalties of each running scenario from the norms of its last sweep
// (recorded by k_finish_phase).
__global__ void k_rho_balance(Workspace w, double mu, double tau) {
  for (int s = gtid(); s < w.n_scen; s += gstride()) {
    ScenState* sc = &w.scen[s];
    double f = 1.0;
    if (!sc->done) {
      if (sc->r_norm > mu * sc->s_norm) f = tau;
      else if (sc->s_norm > mu * sc->r_norm) f = 1.0 / tau;
    }
    sc->rho_factor = f;
  }
}

// The factors applied: penalties scaled, lines of those scenarios factored
// again (P = Q^{-1} and the constant part of the linear term depend on rho).
__global__ void k_rho_apply(acopf_grid g, Workspace w) {
  const int L = g.n_line, G = g.n_gen;
  for (int l = gtid(); l < L; l += gstride()) {
    const double f = w.scen[w.bus_scen[g.line_from[l]]].rho_factor;
    if (f == 1.0) continue;
#pragma unroll
    for (int k = 0; k < 8; ++k) w.rho_l[lc8(l, k)] *= f;
    if (!prep_line(w, l)) fail_line(w, l, ACOPF_ERR_NONCONVEX_LINE, &w.sync->nonconvex);
  }
  for (int k = gtid(); k < G; k += gstride()) {
    const double f = w.scen[w.bus_scen[g.gen_bus[k]]].rho_factor;
    if (f == 1.0) continue;
    w.rho_g[k] *= f;
    w.rho_g[G + k] *= f;
  }
}

// Grid barrier for a cooperative launch (all blocks resident).  Each block
// publishes its arrival by storing the barrier's epoch to its own flag (no
// contended read-modify-write); block 0 waits for every flag, runs `last`
// with the other blocks' writes visible, and releases the grid by storing
// the epoch to `go`.  Only one wave per block executes the device-scope
// fences; the workgroup barrier orders the block's other waves around them.
// Waits are bounded: on timeout the barrier error flag is raised and the
// block continues, so every block reaches the end of the kernel.
template <typename F>
__device__ void grid_barrier(const Workspace& w, unsigned int epoch, F&& last) {
  SyncState* sy = w.sync;
  __syncthreads();
  if (blockIdx.x != 0) {
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&w.arrive[blockIdx.x * kArriveStride], epoch, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      long long spins = 0;
      while (__hip_atomic_load(&sy->go, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          __hip_atomic_store(&sy->barrier_error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return;
  }
  for (unsigned int b = 1 + threadIdx.x; b < gridDim.x; b += blockDim.x) {
    long long spins = 0;
    while (__hip_atomic_load(&w.arrive[b * kArriveStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        __hip_atomic_store(&sy->barrier_error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  last();
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&sy->go, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// Persistent sweep loop of a single scenario (LOCAL: the local line solver).
template <bool LOCAL>
__global__ void __launch_bounds__(256) k_sweep_persistent(acopf_grid g, Workspace w, int max_sweeps,
                                                          double eps_pri, double eps_dual) {
  __shared__ double lds[16];
  __shared__ int s_stop;
  SyncState* sy = w.sync;
  ScenState* sc = &w.scen[0];
  if (__hip_atomic_load(&sy->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;  // failed QP: same for all blocks
  for (int k = 0; k < max_sweeps; ++k) {
    for (int l = gtid(); l < g.n_line; l += gstride())
      if ((LOCAL ? update_line_local(w, l) : update_line(g, w, l)) != 0) atomicAdd(&sc->infeasible[k & 1], 1);
    grid_barrier(w, 2u * k + 1u, [] {});
    double r2 = 0.0, s2 = 0.0;
    const bool inf = sy->norm_inf != 0;
    for (int i = gtid(); i < g.n_bus; i += gstride()) update_bus(g, w, i, r2, s2, inf);
    r2 = inf ? block_max(r2, lds) : block_sum(r2, lds);
    s2 = inf ? block_max(s2, lds) : block_sum(s2, lds);
    if (threadIdx.x == 0) {
      w.partials[blockIdx.x] = r2;
      w.partials[w.max_partials + blockIdx.x] = s2;
    }
    grid_barrier(w, 2u * k + 2u, [&] { finish_scenario(w, 0, 0, gridDim.x, max_sweeps, eps_pri, eps_dual, lds); });
    if (threadIdx.x == 0) {
      const int done = __hip_atomic_load(&sy->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int berr = __hip_atomic_load(&sy->barrier_error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_stop = (done || berr) ? 1 : 0;
    }
    __syncthreads();
    if (s_stop) break;
  }
}

// ---------------------------------------------------------------- step
// soc_only = 1: only the components of scenarios taking a second-order
// correction (the others keep the step already written).
__global__ void k_step_lines(acopf_grid g, acopf_iterate x, Workspace w, acopf_iterate d, int soc_only) {
  for (int l = gtid(); l < g.n_line; l += gstride()) {
    if (soc_only && w.decision[w.bus_scen[g.line_from[l]]].soc != 1) continue;
    step_line(g, x, w, d, l);
  }
}

__global__ void k_step_nodes(acopf_grid g, Workspace w, acopf_iterate d, int soc_only) {
  for (int i = gtid(); i < g.n_bus; i += gstride()) {
    if (soc_only && w.decision[w.bus_scen[i]].soc != 1) continue;
    d.w[i] = w.dw[i];
    d.th[i] = w.dth[i];
  }
  for (int k = gtid(); k < g.n_gen; k += gstride()) {
    if (soc_only && w.decision[w.bus_scen[g.gen_bus[k]]].soc != 1) continue;
    d.pg[k] = w.xg[k];
    d.qg[k] = w.xg[g.n_gen + k];
  }
}

// ---------------------------------------------------------------- SQP step
// Per-component merit pieces: lines (h at x, h at x + d, m(d), model
// quadratic), generators (f at x, f at x + d, model terms, |step|), buses
// (|step|).
__global__ void k_merit_parts(acopf_grid g, acopf_iterate x, Workspace w, acopf_iterate d) {
  const int L = g.n_line, G = g.n_gen;
  for (int l = gtid(); l < L; l += gstride()) {
    double o[4];
    merit_line(g, x, w, d, l, o);
#pragma unroll
    for (int k = 0; k < 4; ++k) w.line_comp[k * L + l] = o[k];
  }
  for (int k = gtid(); k < G; k += gstride()) {
    double o[3];
    merit_gen(g, x, d, k, o);
    w.gen_comp[k] = o[0];
    w.gen_comp[G + k] = o[1];
    w.gen_comp[2 * G + k] = o[2];
    w.gen_comp[3 * G + k] = fmax(fabs(d.pg[k]), fabs(d.qg[k]));
  }
  for (int i = gtid(); i < g.n_bus; i += gstride()) w.bus_comp[i] = fmax(fabs(d.w[i]), fabs(d.th[i]));
}

// Fixed-order sums of scenario s's merit pieces (one block): a = (f at x,
// f at x + d, generator model terms, h at x, h at x + d, m(d), line model
// terms); smax = ||d||_inf over (pg, qg, w, th).
// Chunk k of K of the components [c0, c1) of a scenario.
__device__ __forceinline__ void red_chunk(int c0, int c1, int k, int K, int& a, int& b) {
  const long long n = c1 - c0;
  a = c0 + (int)(n * k / K);
  b = c0 + (int)(n * (k + 1) / K);
}

__device__ __forceinline__ double* red_slot(const Workspace& w, int s, int k) {
  return w.red + ((size_t)s * kRedBlocks + k) * 8;
}

// Block partials of the merit sums: block s K + k adds chunk k of scenario
// s's line, generator and bus pieces (block sums in fixed order) and writes
// them with the chunk's largest step component to Workspace::red.
__global__ void k_merit_partial(Workspace w, int K) {
  __shared__ double lds[16];
  const int s = blockIdx.x / K, k = blockIdx.x % K;
  const int L = w.n_line, G = w.n_gen;
  int l0, l1, g0, g1, b0, b1;
  red_chunk(w.scen_line_off[s], w.scen_line_off[s + 1], k, K, l0, l1);
  red_chunk(w.scen_gen_off[s], w.scen_gen_off[s + 1], k, K, g0, g1);
  red_chunk(w.scen_bus_off[s], w.scen_bus_off[s + 1], k, K, b0, b1);
  double a[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, smax = 0.0;
  for (int l = l0 + (int)threadIdx.x; l < l1; l += blockDim.x) {
    a[3] += w.line_comp[l];
    a[4] += w.line_comp[L + l];
    a[5] += w.line_comp[2 * L + l];
    a[6] += w.line_comp[3 * L + l];
  }
  for (int q = g0 + (int)threadIdx.x; q < g1; q += blockDim.x) {
    a[0] += w.gen_comp[q];
    a[1] += w.gen_comp[G + q];
    a[2] += w.gen_comp[2 * G + q];
    smax = fmax(smax, w.gen_comp[3 * G + q]);
  }
  for (int i = b0 + (int)threadIdx.x; i < b1; i += blockDim.x) smax = fmax(smax, w.bus_comp[i]);
#pragma unroll
  for (int j = 0; j < 7; ++j) a[j] = block_sum(a[j], lds);
  smax = block_max(smax, lds);
  if (threadIdx.x == 0) {
    double* r = red_slot(w, s, k);
#pragma unroll
    for (int j = 0; j < 7; ++j) r[j] = a[j];
    r[7] = smax;
  }
}

// Merit sums of scenario s from its K block partials, by one wave (the
// block's first 64 threads): lane t adds partials t, t + 64, ... in order,
// then a butterfly of shuffles combines the lanes (both partners of a step
// add the same two values, so every lane ends with the same bits).
__device__ void merit_sums(const Workspace& w, int s, int K, double a[7], double& smax) {
  const int lane = (int)threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 7; ++j) a[j] = 0.0;
  smax = 0.0;
  for (int k = lane; k < K; k += 64) {
    const double* r = red_slot(w, s, k);
#pragma unroll
    for (int j = 0; j < 7; ++j) a[j] += r[j];
    smax = fmax(smax, r[7]);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int j = 0; j < 7; ++j) a[j] += __shfl_xor(a[j], off, 64);
    smax = fmax(smax, __shfl_xor(smax, off, 64));
  }
}

// Acceptance test and trust-radius update of Algorithm 1, one 64-thread
// block per scenario (fixed-order sums of the scenario's block partials).  soc = 1: a
// rejected step with pred > 0 of a scenario whose QP was solved is marked
// for a second-order correction (decided by k_soc_decide).
// restore: a restoration step, accepted iff it lowers h; radius and pi kept.
__global__ void k_decide(Workspace w, int K, double mu, double delta_max, double grow, int pi_rule, int soc,
                         int restore) {
  const int s = blockIdx.x;
  double a[7], smax;
  merit_sums(w, s, K, a, smax);
  if (threadIdx.x == 0) {
    SqpDecision* dc = &w.decision[s];
    const double delta = w.scen[s].delta;
    if (w.scen[s].sqp_done) {  // a stopped run: nothing changes
      dc->ared = 0.0;
      dc->pred = 0.0;
      dc->step_inf = 0.0;
      dc->delta_in = delta;
      dc->delta_out = delta;
      dc->accepted = 0;
      dc->update_pi = 0;
      dc->soc = 0;
      dc->soc_sweeps = 0;
      return;
    }
    dc->f_x = a[0];
    dc->f_xd = a[1];
    dc->h_x = a[3];
    dc->h_xd = a[4];
    dc->m_d = a[5];
    dc->quad = a[2] + a[6];
    const double ared = (a[0] + mu * a[3]) - (a[1] + mu * a[4]);
    const double pred = -(a[2] + a[6]) + mu * (a[3] - a[5]);
    dc->ared = ared;
    dc->pred = pred;
    dc->step_inf = smax;
    dc->delta_in = delta;
    const bool failed = w.scen[s].status != 0;
    if (restore) {
      const bool acc = !failed && a[4] < a[3];
      dc->ared = a[3] - a[4];
      dc->pred = 0.0;
      dc->delta_out = delta;
      dc->accepted = acc ? 1 : 0;
      dc->update_pi = 0;
      dc->soc = 0;
      dc->soc_sweeps = 0;
      return;
    }
    const bool ok = !failed && ared > 0.0 && pred > 0.0;
    double dn = delta;
    if (ok) {
      if (smax >= 0.99 * delta && ared >= grow * pred) dn = fmin(2.0 * delta, delta_max);
    } else if (failed) {
      dn = 0.5 * delta;  // a QP that could not be built or factored counts as a rejected step
    } else {
      dn = 0.5 * fmin(delta, smax);
    }
    dc->delta_out = dn;
    dc->accepted = ok ? 1 : 0;
    dc->update_pi = (ok && (pi_rule == ACOPF_PI_ALWAYS || w.scen[s].converged)) ? 1 : 0;
    dc->soc = (soc && !ok && !failed && pred > 0.0) ? 1 : 0;
    dc->soc_sweeps = 0;
    w.scen[s].delta = dn;
  }
}

// Start of the second-order correction pass: scenarios not taking it are
// left out of the next solve; each line of a scenario taking it gets the
// second-order error of its rejected trial step d.
__global__ void k_soc_begin(acopf_grid g, acopf_iterate x, acopf_iterate d, Workspace w) {
  const int L = g.n_line;
  for (int s = gtid(); s < w.n_scen; s += gstride()) {
    const bool on = w.decision[s].soc == 1;
    w.scen[s].skip = on ? 0 : 1;
    if (on) w.scen[s].relaxed = 0;
  }
  for (int l = gtid(); l < L; l += gstride()) {
    if (w.decision[w.bus_scen[g.line_from[l]]].soc != 1) continue;
    double e[4];
    soc_error_line(g, x, d, l, e);
#pragma unroll
    for (int k = 0; k < 4; ++k) w.soc_e[k * L + l] = e[k];
  }
}

// ADMM start of the correction solve, for the scenarios taking it only: the
// multipliers of the rejected step's solve are kept, primal values and bus
// values start at zero, line matrices and linear terms are factored again.
__global__ void k_soc_init(acopf_grid g, Workspace w) {
  const int L = g.n_line, G = g.n_gen, B = g.n_bus;
  for (int l = gtid(); l < L; l += gstride()) {
    if (w.decision[w.bus_scen[g.line_from[l]]].soc != 1) continue;
#pragma unroll
    for (int k = 0; k < 8; ++k) w.xl[lc8(l, k)] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w.xbar_f[lc4(l, k)] = 0.0;
      w.xbar_v[lc4(l, k)] = 0.0;
    }
    w.mu[l] = 0.0;
    w.mu[L + l] = 0.0;
    w.line_mask[l] = 0;
    if (!prep_line(w, l)) fail_line(w, l, ACOPF_ERR_NONCONVEX_LINE, &w.sync->nonconvex);
  }
  for (int k = gtid(); k < G; k += gstride()) {
    if (w.decision[w.bus_scen[g.gen_bus[k]]].soc != 1) continue;
    w.xg[k] = 0.0;
    w.xg[G + k] = 0.0;
    w.xbar_g[k] = 0.0;
    w.xbar_g[G + k] = 0.0;
  }
  for (int i = gtid(); i < B; i += gstride()) {
    if (w.decision[w.bus_scen[i]].soc != 1) continue;
    w.dw[i] = 0.0;
    w.dth[i] = 0.0;
    w.nu[i] = 0.0;
    w.nu[B + i] = 0.0;
  }
}

// Decision on the corrected step of each scenario that took the correction
// (one block per scenario): accepted iff its actual merit reduction is
// positive, judged against the first step's model (pred of k_decide); the
// radius grows as after an accepted step that reached it.  Clears the
// left-out marks of every scenario.
__global__ void k_soc_decide(Workspace w, int K, double mu, double delta_max, double grow, int pi_rule) {
  const int s = blockIdx.x;
  SqpDecision* dc = &w.decision[s];
  if (dc->soc != 1) {
    if (threadIdx.x == 0) w.scen[s].skip = 0;
    return;
  }
  double a[7], smax;
  merit_sums(w, s, K, a, smax);
  if (threadIdx.x == 0) {
    ScenState* sc = &w.scen[s];
    dc->soc_sweeps = sc->sweeps;
    const double ared = (dc->f_x + mu * dc->h_x) - (a[1] + mu * a[4]);
    if (sc->status == 0 && ared > 0.0) {
      dc->soc = 2;
      dc->accepted = 1;
      dc->ared = ared;
      dc->f_xd = a[1];
      dc->h_xd = a[4];
      double dn = dc->delta_in;
      if (dc->step_inf >= 0.99 * dc->delta_in && ared >= grow * dc->pred) dn = fmin(2.0 * dc->delta_in, delta_max);
      dc->delta_out = dn;
      dc->update_pi = (pi_rule == ACOPF_PI_ALWAYS || sc->converged) ? 1 : 0;
      sc->delta = dn;
    }
    sc->skip = 0;
  }
}

// x <- x + d and pi <- new estimates in every scenario whose step was
// accepted: phase 0 after the first decision, phase 1 the corrected steps.
__device__ __forceinline__ bool apply_now(const SqpDecision& dc, int phase) {
  return phase == 0 ? dc.accepted != 0 : dc.soc == 2;
}

__global__ void k_apply(acopf_grid g, acopf_iterate x, acopf_iterate d, Workspace w, int phase) {
  const int L = g.n_line;
  for (int k = gtid(); k < g.n_gen; k += gstride()) {
    if (!apply_now(w.decision[w.bus_scen[g.gen_bus[k]]], phase)) continue;
    x.pg[k] += d.pg[k];
    x.qg[k] += d.qg[k];
  }
  for (int i = gtid(); i < g.n_bus; i += gstride()) {
    if (!apply_now(w.decision[w.bus_scen[i]], phase)) continue;
    x.w[i] += d.w[i];
    x.th[i] += d.th[i];
  }
  for (int l = gtid(); l < L; l += gstride()) {
    const SqpDecision& dc = w.decision[w.bus_scen[g.line_from[l]]];
    if (!apply_now(dc, phase)) continue;
    x.wR[l] += d.wR[l];
    x.wI[l] += d.wI[l];
    if (!dc.update_pi) continue;
#pragma unroll
    for (int k = 0; k < 4; ++k) x.pi[k * L + l] = d.pi[k * L + l];
  }
}

// Start of an SQP iteration with device stops: stopped runs are left out
// of the iteration's solves.
__global__ void k_sqp_begin(Workspace w) {
  for (int s = gtid(); s < w.n_scen; s += gstride()) w.scen[s].skip = w.scen[s].sqp_done ? 1 : 0;
}

// End of an SQP iteration with device stops (one thread per scenario): the
// stop rule on the residual report of the new iterate (k_residual_reduce)
// and the iteration's decision; clears the left-out marks.
__global__ void k_sqp_stop(Workspace w, double tol_primal, double tol_dual, double tol_step, double delta_min) {
  for (int s = gtid(); s < w.n_scen; s += gstride()) {
    ScenState* sc = &w.scen[s];
    sc->skip = 0;
    if (sc->sqp_done) continue;
    sc->sqp_iters += 1;
    const ResidualReport& r = w.report[s];
    const double primal = fmax(fmax(fmax(r.balance, r.c11), fmax(r.c12, r.limit)), r.bounds);
    const double dual = r.dual / fmax(1.0, r.gradf);
    const SqpDecision& dc = w.decision[s];
    int reason = 0;
    if (dc.accepted && primal <= tol_primal && dual <= tol_dual) reason = 1;
    else if (dc.accepted && dc.step_inf < tol_step) reason = 2;
    else if (sc->delta < delta_min) reason = 3;
    if (reason) {
      sc->sqp_done = 1;
      sc->sqp_reason = reason;
      sc->t_done = wall_clock64();
    }
  }
}

// ---------------------------------------------------------------- residuals
__global__ void k_residual_parts(acopf_grid g, acopf_iterate x, Workspace w) {
  const int L = g.n_line, G = g.n_gen, B = g.n_bus;
  for (int l = gtid(); l < L; l += gstride()) {
    double pr[5] = {0, 0, 0, 0, 0}, du = 0.0;
    residual_line(g, x, w, l, pr, du);
    w.line_comp[l] = pr[1];
    w.line_comp[L + l] = pr[2];
    w.line_comp[2 * L + l] = pr[3];
    w.line_comp[3 * L + l] = du;
  }
  for (int i = gtid(); i < B; i += gstride()) {
    double pr[5] = {0, 0, 0, 0, 0}, du = 0.0;
    residual_bus(g, x, w, i, pr, du);
    w.bus_comp[i] = pr[0];
    w.bus_comp[B + i] = pr[4];
    w.bus_comp[2 * B + i] = du;
  }
  for (int k = gtid(); k < G; k += gstride()) {
    double bnd, du, gf;
    residual_gen(g, x, w, k, bnd, du, gf);
    w.gen_comp[k] = bnd;
    w.gen_comp[G + k] = du;
    w.gen_comp[2 * G + k] = gf;
  }
}

// Block partials of the residual maxima: block s K + k takes chunk k of
// scenario s's components.
__global__ void k_residual_partial(Workspace w, int K) {
  __shared__ double lds[16];
  const int s = blockIdx.x / K, k = blockIdx.x % K, L = w.n_line, G = w.n_gen, B = w.n_bus;
  int l0, l1, g0, g1, b0, b1;
  red_chunk(w.scen_line_off[s], w.scen_line_off[s + 1], k, K, l0, l1);
  red_chunk(w.scen_gen_off[s], w.scen_gen_off[s + 1], k, K, g0, g1);
  red_chunk(w.scen_bus_off[s], w.scen_bus_off[s + 1], k, K, b0, b1);
  double a[7] = {0, 0, 0, 0, 0, 0, 0};  // balance, c11, c12, limit, bounds, dual, gradf
  for (int l = l0 + (int)threadIdx.x; l < l1; l += blockDim.x) {
    a[1] = fmax(a[1], w.line_comp[l]);
    a[2] = fmax(a[2], w.line_comp[L + l]);
    a[3] = fmax(a[3], w.line_comp[2 * L + l]);
    a[5] = fmax(a[5], w.line_comp[3 * L + l]);
  }
  for (int i = b0 + (int)threadIdx.x; i < b1; i += blockDim.x) {
    a[0] = fmax(a[0], w.bus_comp[i]);
    a[4] = fmax(a[4], w.bus_comp[B + i]);
    a[5] = fmax(a[5], w.bus_comp[2 * B + i]);
  }
  for (int q = g0 + (int)threadIdx.x; q < g1; q += blockDim.x) {
    a[4] = fmax(a[4], w.gen_comp[q]);
    a[5] = fmax(a[5], w.gen_comp[G + q]);
    a[6] = fmax(a[6], w.gen_comp[2 * G + q]);
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) a[j] = block_max(a[j], lds);
  if (threadIdx.x == 0) {
    double* r = red_slot(w, s, k);
#pragma unroll
    for (int j = 0; j < 7; ++j) r[j] = a[j];
  }
}

// The residual report of each scenario (one 64-thread block per scenario):
// the largest of its K block partials, lane-strided then by shuffles.
__global__ void k_residual_reduce(Workspace w, int K) {
  const int s = blockIdx.x, lane = (int)threadIdx.x;
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int k = lane; k < K; k += 64) {
    const double* r = red_slot(w, s, k);
#pragma unroll
    for (int j = 0; j < 7; ++j) a[j] = fmax(a[j], r[j]);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int j = 0; j < 7; ++j) a[j] = fmax(a[j], __shfl_xor(a[j], off, 64));
  if (lane == 0) {
    ResidualReport* r = &w.report[s];
    r->balance = a[0];
    r->c11 = a[1];
    r->c12 = a[2];
    r->limit = a[3];
    r->bounds = a[4];
    r->dual = a[5];
    r->gradf = a[6];
  }
}

// ---------------------------------------------------------------- host helpers
// Two HIP events released when the owner goes out of scope.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t create() {
    hipError_t e = hipEventCreate(&a);
    return e == hipSuccess ? hipEventCreate(&b) : e;
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

int blocks_for(long long n, int bs) {
  long long b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (int)b;
}

// Blocks per scenario of the per-scenario reductions: about 1,024 of a
// scenario's components (by the batch's average) per block, at most
// kRedBlocks.  Fixed by the sizes, so the order of the sums is too.
int red_blocks(const acopf_grid* g, int ns) {
  const long long n = std::max(std::max((long long)g->n_line, (long long)g->n_bus), (long long)g->n_gen);
  const long long per = (n + ns - 1) / ns;
  return (int)std::min<long long>(kRedBlocks, std::max<long long>(1, (per + 1023) / 1024));
}

// ---------------------------------------------------------------- learned warm start
static_assert(ACOPF_LINE_FEATURES == 16 + 8 + 1, "line feature layout");
static_assert(ACOPF_GEN_FEATURES == 8 + 2 + 1, "generator feature layout");

// Features of every line and generator (FP32, feature-major with leading
// dimensions ldl, ldg); the previous multipliers are the workspace's, zero
// at the first QP of a run.
__global__ void k_features(acopf_grid g, acopf_iterate x, Workspace w, int first, float* fl, long long ldl,
                           float* fg, long long ldg) {
  const int L = g.n_line, G = g.n_gen;
  const double flag = first ? 1.0 : 0.0;
  for (int l = gtid(); l < L; l += gstride()) {
    const int i = g.line_from[l], j = g.line_to[l];
    const double v[16] = {g.pd[i], g.qd[i], g.pd[j], g.qd[j],
                          g.gij[l] / 100.0, g.bij[l] / 100.0, g.gii[l] / 100.0, g.bii[l] / 100.0,
                          g.gjj[l] / 100.0, g.bjj[l] / 100.0, x.w[i], x.w[j], x.wR[l], x.wI[l],
                          sin(x.th[i] - x.th[j]), g.smax_ij[l]};
#pragma unroll
    for (int f = 0; f < 16; ++f) fl[f * ldl + l] = (float)v[f];
#pragma unroll
    for (int c = 0; c < 8; ++c) fl[(16 + c) * ldl + l] = first ? 0.0f : (float)(w.lam_l[lc8(l, c)] / kLamScale);
    fl[24 * ldl + l] = (float)flag;
  }
  for (int k = gtid(); k < G; k += gstride()) {
    const int b = g.gen_bus[k];
    const double v[ACOPF_GEN_FEATURES] = {g.pd[b], g.qd[b], g.cost2[k] / 1e4, g.cost1[k] / 1e3, x.pg[k], x.qg[k],
                                          g.pmax[k], g.qmax[k], first ? 0.0 : w.lam_g[k] / kLamScale,
                                          first ? 0.0 : w.lam_g[G + k] / kLamScale, flag};
#pragma unroll
    for (int f = 0; f < ACOPF_GEN_FEATURES; ++f) fg[f * ldg + k] = (float)v[f];
  }
}

// log clip(sqrt((rho sum_r + reg) / (sum_s + reg)), 1 / clip, clip).
__device__ double log_rho_factor(double rho, double sum_r, double sum_s) {
  const double fac = sqrt((rho * sum_r + kRhoReg) / (sum_s + kRhoReg));
  return log(fmin(fmax(fac, 1.0 / kRhoClip), kRhoClip));
}

__global__ void k_targets(Workspace w, float* tl, long long ldl, float* tg, long long ldg) {
  const int L = w.n_line, G = w.n_gen;
  for (int l = gtid(); l < L; l += gstride()) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const size_t q = lc8(l, c);  // line-by-line state
      const int t = c * L + l;     // trace sums, field by field
      tl[c * ldl + l] = (float)((w.lam_l[q] - w.lam0_l[q]) / kLamScale);
      tl[(8 + c) * ldl + l] = (float)log_rho_factor(w.rho_l[q], w.tr_r_l[t], w.tr_s_l[t]);
    }
  }
  for (int k = gtid(); k < G; k += gstride()) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int q = c * G + k;
      tg[c * ldg + k] = (float)((w.lam_g[q] - w.lam0_g[q]) / kLamScale);
      tg[(2 + c) * ldg + k] = (float)log_rho_factor(w.rho_g[q], w.tr_r_g[q], w.tr_s_g[q]);
    }
  }
}

// ADMM start from network outputs: the plain start (the workspace's
// multipliers, the base penalty) corrected by the outputs; a non-finite
// output keeps the plain start of its coupling.
__global__ void k_decode(Workspace w, const float* yl, long long ldl, const float* yg, long long ldg, double rho_l0,
                         double rho_g0, int first, int use_lam, int use_rho, double* lam_l, double* lam_g,
                         double* rho_l, double* rho_g) {
  const int L = w.n_line, G = w.n_gen;
  const double lmax = log(kRhoClip);
  for (int l = gtid(); l < L; l += gstride()) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int q = c * L + l;  // caller layout
      const double base = first ? 0.0 : w.lam_l[lc8(l, c)];
      const double a = base + (double)yl[c * ldl + l] * kLamScale;
      lam_l[q] = (use_lam && isfinite(a)) ? a : base;
      const double o = (double)yl[(8 + c) * ldl + l];
      rho_l[q] = (use_rho && isfinite(o)) ? rho_l0 * exp(fmin(fmax(o, -lmax), lmax)) : rho_l0;
    }
  }
  for (int k = gtid(); k < G; k += gstride()) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int q = c * G + k;
      const double base = first ? 0.0 : w.lam_g[q];
      const double a = base + (double)yg[c * ldg + k] * kLamScale;
      lam_g[q] = (use_lam && isfinite(a)) ? a : base;
      const double o = (double)yg[(2 + c) * ldg + k];
      rho_g[q] = (use_rho && isfinite(o)) ? rho_g0 * exp(fmin(fmax(o, -lmax), lmax)) : rho_g0;
    }
  }
}

int n_scen_of(const acopf_grid* g) { return g->n_scen > 1 ? g->n_scen : 1; }

bool grid_ok(const acopf_grid* g) {
  return g && g->n_bus > 0 && g->n_line > 0 && g->n_gen >= 0 && g->n_scen >= 0 && n_scen_of(g) <= g->n_bus &&
         g->vmin && g->vmax && g->pd && g->qd && g->gsh && g->bsh && g->line_from && g->line_to && g->gii &&
         g->bii && g->gij && g->bij && g->gji && g->bji && g->gjj && g->bjj && g->smax_ij && g->smax_ji &&
         (g->n_gen == 0 || (g->gen_bus && g->pmin && g->pmax && g->qmin && g->qmax && g->cost2 && g->cost1));
}

bool iterate_ok(const acopf_iterate* x) {
  return x && x->pg && x->qg && x->w && x->th && x->wR && x->wI && x->pi;
}

Workspace ws_of(const acopf_grid* g, void* base) {
  Workspace w;
  layout_workspace(base, g->n_bus, g->n_line, g->n_gen, n_scen_of(g), &w);
  return w;
}

acopf_status read_sync(const Workspace& w, hipStream_t s, SyncState* out) {
  HIP_TRY(hipMemcpyAsync(out, w.sync, sizeof(SyncState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return ACOPF_OK;
}

// ---------------------------------------------------------------- line solver per workspace
// Hessian mode of the last QP build on each workspace, kept on the host:
// it picks the line kernels of the solves that follow (the local line
// solver's kernels are separate instantiations).  acopf_setup resets it.
struct ModeTable {
  std::mutex mu;
  std::map<const void*, int> mode;
};

ModeTable& mode_table() {
  static ModeTable* t = new ModeTable();
  return *t;
}

void set_hessian_mode(const void* workspace, int mode) {
  ModeTable& t = mode_table();
  std::lock_guard<std::mutex> lock(t.mu);
  if (mode == ACOPF_HESSIAN_PSD)
    t.mode.erase(workspace);
  else
    t.mode[workspace] = mode;
}

// 0 exact line solver, 1 local line solver, 2 the projection's line kernel.
int line_solver_of(const void* workspace) {
  ModeTable& t = mode_table();
  std::lock_guard<std::mutex> lock(t.mu);
  auto it = t.mode.find(workspace);
  if (it == t.mode.end()) return 0;
  return it->second == ACOPF_HESSIAN_RAW_LOCAL ? 1 : (it->second == kModeLinfeas ? 2 : 0);
}

acopf_status setup_impl(const acopf_grid* g, const int32_t* bus_off_h, const int32_t* line_off_h,
                        const int32_t* gen_off_h, const int32_t* ref_h, void* workspace, size_t bytes,
                        void* stream) {
  const int nb = g->n_bus, nl = g->n_line, ng = g->n_gen, ns = n_scen_of(g);
  const size_t need = layout_workspace(nullptr, nb, nl, ng, ns, nullptr);
  if (bytes < need)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: workspace of " + std::to_string(bytes) + " bytes, need " +
                                           std::to_string(need));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // scenario tables
  for (int k = 0; k < ns; ++k) {
    if (bus_off_h[k + 1] <= bus_off_h[k] || line_off_h[k + 1] <= line_off_h[k] || gen_off_h[k + 1] < gen_off_h[k])
      return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: scenario " + std::to_string(k) + " has an empty or reversed range");
    if (ref_h[k] < bus_off_h[k] || ref_h[k] >= bus_off_h[k + 1])
      return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: reference bus of scenario " + std::to_string(k) + " out of range");
  }
  if (bus_off_h[0] != 0 || line_off_h[0] != 0 || gen_off_h[0] != 0 || bus_off_h[ns] != nb ||
      line_off_h[ns] != nl || gen_off_h[ns] != ng)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: scenario ranges do not cover the arrays");
  std::vector<int32_t> from(nl), to(nl), gb(ng);
  HIP_TRY(hipMemcpyAsync(from.data(), g->line_from, nl * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(to.data(), g->line_to, nl * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  if (ng > 0) HIP_TRY(hipMemcpyAsync(gb.data(), g->gen_bus, ng * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int32_t> scen(nb), flags(nb, 0);
  for (int k = 0; k < ns; ++k) {
    for (int i = bus_off_h[k]; i < bus_off_h[k + 1]; ++i) scen[i] = k;
    flags[ref_h[k]] |= BUS_REF;
  }
  std::vector<int32_t> deg(nb, 0), gdeg(nb, 0);
  for (int k = 0; k < ns; ++k) {
    for (int l = line_off_h[k]; l < line_off_h[k + 1]; ++l) {
      const int f = from[l], t = to[l];
      if (f < bus_off_h[k] || f >= bus_off_h[k + 1] || t < bus_off_h[k] || t >= bus_off_h[k + 1] || f == t)
        return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: line " + std::to_string(l) + " has a bad end bus");
      deg[f]++;
      deg[t]++;
    }
    for (int q = gen_off_h[k]; q < gen_off_h[k + 1]; ++q) {
      if (gb[q] < bus_off_h[k] || gb[q] >= bus_off_h[k + 1])
        return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: generator " + std::to_string(q) + " has a bad bus");
      gdeg[gb[q]]++;
    }
  }
  for (int i = 0; i < nb; ++i)
    if (deg[i] == 0) return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: bus " + std::to_string(i) + " has no line");
  // CSR of line ends per bus (ends in line order) and of generators per bus
  std::vector<int32_t> eptr(nb + 1, 0), gptr(nb + 1, 0), ends(2 * (size_t)nl), gens(ng > 0 ? ng : 1);
  for (int i = 0; i < nb; ++i) {
    eptr[i + 1] = eptr[i] + deg[i];
    gptr[i + 1] = gptr[i] + gdeg[i];
  }
  std::vector<int32_t> fill(eptr.begin(), eptr.end() - 1), gfill(gptr.begin(), gptr.end() - 1);
  for (int l = 0; l < nl; ++l) {
    ends[fill[from[l]]++] = 2 * l;
    ends[fill[to[l]]++] = 2 * l + 1;
  }
  for (int q = 0; q < ng; ++q) gens[gfill[gb[q]]++] = q;
  // coupling items of the bus phase: per scenario, bus by bus, its
  // generators then its line ends (CSR order) in consecutive slots of one
  // block; a bus that does not fit the current block starts the next one,
  // and a bus with more items than a block takes one whole-bus slot
  const int32_t ib = kItemBlock, waves = item_waves_for(nl);
  const int32_t nib = item_blocks_bound(nl, ng, ns);
  std::vector<int32_t> icode((size_t)nib * ib, kItemPad), ibus((size_t)nib * ib, -1), ihead((size_t)nib * ib),
      ilen((size_t)nib * ib, 0), iblk(ns + 1);
  for (size_t q = 0; q < ihead.size(); ++q) ihead[q] = (int32_t)(q % ib);
  int32_t blk = 0;
  for (int k = 0; k < ns; ++k) {
    blk = (blk + waves - 1) / waves * waves;  // a workgroup serves one scenario
    iblk[k] = blk;
    int fill = 0;
    bool open = false;
    for (int i = bus_off_h[k]; i < bus_off_h[k + 1]; ++i) {
      const int items = gdeg[i] + deg[i];
      const bool whole = items > ib;
      const int n = whole ? 1 : items;
      if (!open || fill + n > ib) {
        if (open) ++blk;
        open = true;
        fill = 0;
      }
      const size_t base = (size_t)blk * ib;
      int j = fill;
      if (whole) {
        icode[base + j++] = kItemBus;
      } else {
        for (int q = gptr[i]; q < gptr[i + 1]; ++q) icode[base + j++] = -(gens[q] + 1);
        for (int e = eptr[i]; e < eptr[i + 1]; ++e) icode[base + j++] = ends[e];
      }
      for (int m = fill; m < fill + n; ++m) {
        ibus[base + m] = i;
        ihead[base + m] = fill;
        ilen[base + m] = n;
      }
      fill += n;
    }
    if (open) ++blk;
  }
  blk = (blk + waves - 1) / waves * waves;
  iblk[ns] = blk;
  if (blk > nib) return fail(ACOPF_ERR_UNSUPPORTED, "acopf_setup: item blocks exceed their bound");
  Workspace w = ws_of(g, workspace);
  const size_t used = (size_t)blk * ib * sizeof(int32_t);
  HIP_TRY(hipMemcpy(w.item_code, icode.data(), used, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.item_bus, ibus.data(), used, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.item_head, ihead.data(), used, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.item_len, ilen.data(), used, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.item_blk_off, iblk.data(), (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.bus_end_ptr, eptr.data(), (nb + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.bus_end, ends.data(), 2 * (size_t)nl * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.bus_gen_ptr, gptr.data(), (nb + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  if (ng > 0) HIP_TRY(hipMemcpy(w.bus_gen, gens.data(), ng * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.bus_scen, scen.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.bus_flags, flags.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.scen_bus_off, bus_off_h, (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.scen_line_off, line_off_h, (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.scen_gen_off, gen_off_h, (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  SyncState zero;
  std::memset(&zero, 0, sizeof(zero));
  HIP_TRY(hipMemcpy(w.sync, &zero, sizeof(zero), hipMemcpyHostToDevice));
  std::vector<ScenState> sz(ns);
  std::memset(sz.data(), 0, ns * sizeof(ScenState));
  for (auto& e : sz) e.delta = 1.0;
  HIP_TRY(hipMemcpy(w.scen, sz.data(), ns * sizeof(ScenState), hipMemcpyHostToDevice));
  // multipliers start at zero (the previous-iterate start of a first solve)
  // and so do the trace sums
  const size_t D = sizeof(double);
  if (ng > 0) HIP_TRY(hipMemset(w.lam_g, 0, 2 * (size_t)ng * D));
  HIP_TRY(hipMemset(w.lam_l, 0, 8 * (size_t)nl * D));
  if (ng > 0) HIP_TRY(hipMemset(w.tr_r_g, 0, 2 * (size_t)ng * D));
  if (ng > 0) HIP_TRY(hipMemset(w.tr_s_g, 0, 2 * (size_t)ng * D));
  HIP_TRY(hipMemset(w.tr_r_l, 0, 8 * (size_t)nl * D));
  HIP_TRY(hipMemset(w.tr_s_l, 0, 8 * (size_t)nl * D));
  set_hessian_mode(workspace, ACOPF_HESSIAN_PSD);
  return ACOPF_OK;
}

// rho_fill > 0: every penalty is rho_fill (rho_g, rho_l unused).
acopf_status admm_init_impl(const acopf_grid* g, const double* rho_g, const double* rho_l, const double* lam_g,
                            const double* lam_l, bool keep_lam, void* workspace, void* stream,
                            double rho_fill = 0.0) {
  if (!grid_ok(g) || !workspace || (rho_fill <= 0.0 && (!rho_l || (g->n_gen > 0 && !rho_g))))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_init: null argument");
  if ((lam_l == nullptr && lam_g != nullptr) || (lam_l != nullptr && lam_g == nullptr && g->n_gen > 0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_init: give both warm-start multiplier arrays or neither");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int bs = kDefaultBlock;
  const long long G2 = 2LL * g->n_gen, L8 = 8LL * g->n_line;
  auto fill = [&](double* p, long long n, double v) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, bs)), dim3(bs), 0, s, p, n, v);
  };
  auto copy = [&](double* d, const double* src, long long n) {
    if (n > 0) hipLaunchKernelGGL(k_copy, dim3(blocks_for(n, bs)), dim3(bs), 0, s, d, src, n);
  };
  auto to_lines = [&](double* d, const double* src, int n) {
    hipLaunchKernelGGL(k_fields_to_lines, dim3(blocks_for(8LL * n, bs)), dim3(bs), 0, s, d, src, n);
  };
  if (rho_fill > 0.0) {
    fill(w.rho_g, G2, rho_fill);
    fill(w.rho_l, L8, rho_fill);
  } else {
    copy(w.rho_g, rho_g, G2);
    to_lines(w.rho_l, rho_l, g->n_line);
  }
  if (keep_lam) {
    // multipliers of the previous solve stay in place (previous-iterate warm start)
  } else if (lam_l) {
    copy(w.lam_g, lam_g, G2);
    to_lines(w.lam_l, lam_l, g->n_line);
  } else {
    fill(w.lam_g, G2, 0.0);
    fill(w.lam_l, L8, 0.0);
  }
  copy(w.lam0_g, w.lam_g, G2);  // the start of this solve (training targets)
  copy(w.lam0_l, w.lam_l, L8);
  fill(w.xg, G2, 0.0);
  fill(w.xbar_g, G2, 0.0);
  fill(w.xl, L8, 0.0);
  fill(w.xbar_f, 4LL * g->n_line, 0.0);
  fill(w.xbar_v, 4LL * g->n_line, 0.0);
  fill(w.dw, g->n_bus, 0.0);
  fill(w.dth, g->n_bus, 0.0);
  fill(w.nu, 2LL * g->n_bus, 0.0);
  fill(w.mu, 2LL * g->n_line, 0.0);
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, w.line_mask,
                     (long long)g->n_line, 0);
  hipLaunchKernelGGL(k_prep_lines, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, w);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

// ---------------------------------------------------------------- sweep launches
// Arguments of the launch-per-phase sweeps of one solve.
struct SweepLaunch {
  acopf_grid g;
  Workspace w;
  int nbl, nbb, bs, single, ns, trace, max_sweeps;
  int solver;  // line kernel: 0 exact, 1 local (ALM + TRON), 2 linear feasibility projection
  int norm_inf;  // infinity norms (bus partials, stop test)
  double eps_pri, eps_dual;
};

template <bool kTrace, int kWaves>
void launch_bus_items_norm(const SweepLaunch& a, hipStream_t s) {
  const dim3 grid(xcd_grid(a.nbb)), block(kItemBlock * kWaves);
  if (a.norm_inf)
    hipLaunchKernelGGL((k_bus_items<kTrace, true, kWaves>), grid, block, 0, s, a.g, a.w, a.single);
  else
    hipLaunchKernelGGL((k_bus_items<kTrace, false, kWaves>), grid, block, 0, s, a.g, a.w, a.single);
}

void launch_bus_items(const SweepLaunch& a, hipStream_t s) {
  const bool one = item_waves_for(a.g.n_line) == 1;
  if (a.trace && one) launch_bus_items_norm<true, 1>(a, s);
  else if (a.trace) launch_bus_items_norm<true, 4>(a, s);
  else if (one) launch_bus_items_norm<false, 1>(a, s);
  else launch_bus_items_norm<false, 4>(a, s);
}

// n sweeps: each line phase but the first tests the sweep before it; the
// chunk ends with k_finish_phase.
void enqueue_sweeps(const SweepLaunch& a, int n, hipStream_t s) {
  const int search = a.g.n_line < kSearchMaxLines ? 1 : 0;
  const int stop_test = (a.eps_pri > 0.0 || a.eps_dual > 0.0) ? (a.norm_inf ? 2 : 1) : 0;
  for (int k = 0; k < n; ++k) {
    if (a.solver == 1)
      hipLaunchKernelGGL(k_line_phase_local, dim3(xcd_grid(a.nbl)), dim3(a.bs), 0, s, a.w, a.single,
                         (k > 0) ? stop_test : 0, a.eps_pri, a.eps_dual);
    else if (a.solver == 2)
      hipLaunchKernelGGL(k_line_phase_linfeas, dim3(xcd_grid(a.nbl)), dim3(a.bs), 0, s, a.w, a.single,
                         (k > 0) ? stop_test : 0, a.eps_pri, a.eps_dual);
    else
      hipLaunchKernelGGL(k_line_phase, dim3(xcd_grid(a.nbl)), dim3(a.bs), 0, s, a.g, a.w, a.single,
                         (k > 0) ? stop_test : 0, search, a.eps_pri, a.eps_dual);
    launch_bus_items(a, s);
  }
  hipLaunchKernelGGL(k_finish_phase, dim3(a.ns), dim3(64), 0, s, a.w, a.max_sweeps, a.eps_pri, a.eps_dual);
}

// Instantiated graphs of n launch-per-phase sweeps, cached per process and
// keyed by everything their kernels receive (device, workspace, grid
// arrays, sizes, launch shape, stop parameters), so that a hit replays
// exactly the launches the plain mode would enqueue.  Entries live until
// the process ends; past kMaxGraphs distinct keys the solve launches
// without a graph.
constexpr size_t kMaxGraphs = 256;

struct GraphCache {
  std::mutex mu;
  std::map<std::string, hipGraphExec_t> execs;
  std::map<int, hipStream_t> capture_streams;
};

GraphCache& graph_cache() {
  static GraphCache* c = new GraphCache();  // never destroyed: graphs may be in flight at exit
  return *c;
}

std::string graph_key(const SweepLaunch& a, int n, int dev) {
  std::string k;
  auto put = [&](const void* p, size_t b) { k.append(static_cast<const char*>(p), b); };
  put(&dev, sizeof dev);
  put(&n, sizeof n);
  const acopf_grid& g = a.g;
  const int32_t ints[6] = {g.n_bus, g.n_line, g.n_gen, g.ref_bus, g.n_scen, g.reserved};
  put(ints, sizeof ints);
  const void* ptrs[] = {g.vmin, g.vmax, g.pd, g.qd, g.gsh, g.bsh, g.line_from, g.line_to, g.gii, g.bii, g.gij,
                        g.bij, g.gji, g.bji, g.gjj, g.bjj, g.smax_ij, g.smax_ji, g.gen_bus, g.pmin, g.pmax,
                        g.qmin, g.qmax, g.cost2, g.cost1, a.w.bus_end_ptr /* workspace base */};
  put(ptrs, sizeof ptrs);
  const int shape[9] = {a.nbl, a.nbb, a.bs, a.single, a.ns, a.trace, a.max_sweeps, a.solver, a.norm_inf};
  put(shape, sizeof shape);
  put(&a.eps_pri, sizeof a.eps_pri);
  put(&a.eps_dual, sizeof a.eps_dual);
  return k;
}

// Graph of n sweeps for a (built on first use); *exec = nullptr when the
// cache is full.
acopf_status sweep_graph(const SweepLaunch& a, int n, hipGraphExec_t* exec) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  const std::string key = graph_key(a, n, dev);
  GraphCache& c = graph_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  auto it = c.execs.find(key);
  if (it != c.execs.end()) {
    *exec = it->second;
    return ACOPF_OK;
  }
  *exec = nullptr;
  if (c.execs.size() >= kMaxGraphs) return ACOPF_OK;
  auto cs = c.capture_streams.find(dev);
  if (cs == c.capture_streams.end()) {
    hipStream_t st;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    cs = c.capture_streams.emplace(dev, st).first;
  }
  HIP_TRY(hipStreamBeginCapture(cs->second, hipStreamCaptureModeThreadLocal));
  enqueue_sweeps(a, n, cs->second);
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamEndCapture(cs->second, &graph));
  hipGraphExec_t ge = nullptr;
  const hipError_t e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
  HIP_TRY(hipGraphDestroy(graph));
  HIP_TRY(e);
  c.execs.emplace(key, ge);
  *exec = ge;
  return ACOPF_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char* acopf_last_error(void) { return last_error().c_str(); }

size_t acopf_workspace_bytes(int32_t n_bus, int32_t n_line, int32_t n_gen, int32_t n_scen) {
  if (n_bus <= 0 || n_line <= 0 || n_gen < 0 || n_scen < 0 || n_scen > n_bus) return 0;
  return layout_workspace(nullptr, n_bus, n_line, n_gen, n_scen > 1 ? n_scen : 1, nullptr);
}

acopf_status acopf_setup(const acopf_grid* g, void* workspace, size_t bytes, void* stream) {
  if (!grid_ok(g)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: incomplete grid description");
  if (!workspace) return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: null workspace");
  if (n_scen_of(g) != 1) return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: use acopf_setup_batch for n_scen > 1");
  if (g->ref_bus < 0 || g->ref_bus >= g->n_bus) return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: bad reference bus");
  const int32_t bo[2] = {0, g->n_bus}, lo[2] = {0, g->n_line}, go[2] = {0, g->n_gen}, rf[1] = {g->ref_bus};
  return setup_impl(g, bo, lo, go, rf, workspace, bytes, stream);
}

acopf_status acopf_setup_batch(const acopf_grid* g, const int32_t* bus_offset, const int32_t* line_offset,
                               const int32_t* gen_offset, const int32_t* ref_bus, void* workspace, size_t bytes,
                               void* stream) {
  if (!grid_ok(g)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup_batch: incomplete grid description");
  if (!workspace || !bus_offset || !line_offset || !gen_offset || !ref_bus)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup_batch: null argument");
  return setup_impl(g, bus_offset, line_offset, gen_offset, ref_bus, workspace, bytes, stream);
}

acopf_status acopf_set_delta(const acopf_grid* g, const double* delta, void* workspace, void* stream) {
  if (!grid_ok(g) || !workspace || !delta) return fail(ACOPF_ERR_INVALID_ARG, "acopf_set_delta: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  hipLaunchKernelGGL(k_copy_delta, dim3(blocks_for(w.n_scen, 256)), dim3(256), 0, s, w, delta);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

}  // extern "C"

namespace {
// QP build; mode may also be kModeRestore (a restoration step's QP: exact
// line solver, generators with 0.5 (d_p^2 + d_q^2)).
acopf_status qp_build_impl(const acopf_grid* g, const acopf_iterate* x, double delta, int mode, void* workspace,
                           void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int bs = kDefaultBlock;
  const bool restore = mode == kModeRestore;
  if (delta > 0.0) hipLaunchKernelGGL(k_set_delta, dim3(blocks_for(w.n_scen, bs)), dim3(bs), 0, s, w, delta);
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, w, mode);
  set_hessian_mode(workspace, restore ? ACOPF_HESSIAN_PSD : mode);
  hipLaunchKernelGGL(k_build_lines, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, *g, *x, mode, w, 0);
  if (g->n_gen > 0)
    hipLaunchKernelGGL(k_build_gens, dim3(blocks_for(g->n_gen, bs)), dim3(bs), 0, s, *g, *x, w, restore ? 1 : 0);
  hipLaunchKernelGGL(k_build_buses, dim3(blocks_for(g->n_bus, bs)), dim3(bs), 0, s, *g, *x, w);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}
}  // namespace

extern "C" {

acopf_status acopf_qp_build(const acopf_grid* g, const acopf_iterate* x, double delta, int32_t mode,
                            void* workspace, void* stream) {
  if (!grid_ok(g) || !iterate_ok(x) || !workspace)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_qp_build: null argument");
  if (!(delta >= 0.0)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_qp_build: trust radius must be >= 0");
  if (mode != ACOPF_HESSIAN_PSD && mode != ACOPF_HESSIAN_RAW && mode != ACOPF_HESSIAN_RAW_LOCAL)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_qp_build: unknown Hessian mode");
  return qp_build_impl(g, x, delta, mode, workspace, stream);
}

acopf_status acopf_admm_init(const acopf_grid* g, const double* rho_g, const double* rho_l,
                             const double* lam_g, const double* lam_l, void* workspace, void* stream) {
  return admm_init_impl(g, rho_g, rho_l, lam_g, lam_l, false, workspace, stream);
}

acopf_status acopf_admm_solve(const acopf_grid* g, const acopf_admm_params* p, void* workspace, void* stream,
                              acopf_admm_result* result) {
  if (!grid_ok(g) || !p || !workspace) return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: null argument");
  if (p->max_sweeps < 0 || !(p->eps_pri >= 0.0) || !(p->eps_dual >= 0.0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: bad parameters");
  if (p->norm_inf != 0 && p->norm_inf != 1)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: norm_inf must be 0 or 1");
  const int bs = p->block_size > 0 ? p->block_size : kDefaultBlock;
  if (bs % 64 != 0 || bs > 256)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: block_size must be a multiple of 64, <= 256");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int ns = w.n_scen;
  const int reset_blocks = blocks_for(std::max(w.max_partials, ns), 256);
  if (p->max_sweeps == 0) {
    hipLaunchKernelGGL(k_reset_solve, dim3(reset_blocks), dim3(256), 0, s, w, 0, bs, 0, p->norm_inf);
    HIP_TRY(hipGetLastError());
    if (result) return acopf_admm_result_get(g, workspace, stream, result);
    return ACOPF_OK;
  }
  if (p->trace != 0 && p->trace != 1) return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: trace must be 0 or 1");
  if (p->trace && p->sweep_mode == ACOPF_SWEEP_PERSISTENT)
    return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: traced solves run in the launch-per-phase modes");
  const bool balance = p->balance_every > 0;
  if (p->balance_every < 0 || p->balance_every % kSweepChunk != 0)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: balance_every must be 0 or a positive multiple of 64");
  if (balance && !(p->balance_mu >= 1.0 && p->balance_tau > 1.0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: residual balancing needs balance_mu >= 1 and balance_tau > 1");
  if (balance && p->sweep_mode == ACOPF_SWEEP_PERSISTENT)
    return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: residual balancing runs in the launch-per-phase modes");
  const int solver = line_solver_of(workspace);
  const bool local = solver == 1;
  if (p->trace) {
    const int bz = kDefaultBlock;
    const long long G2 = 2LL * g->n_gen, L8 = 8LL * g->n_line;
    if (G2 > 0) {
      hipLaunchKernelGGL(k_fill, dim3(blocks_for(G2, bz)), dim3(bz), 0, s, w.tr_r_g, G2, 0.0);
      hipLaunchKernelGGL(k_fill, dim3(blocks_for(G2, bz)), dim3(bz), 0, s, w.tr_s_g, G2, 0.0);
    }
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(L8, bz)), dim3(bz), 0, s, w.tr_r_l, L8, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(L8, bz)), dim3(bz), 0, s, w.tr_s_l, L8, 0.0);
  }
  if (p->sweep_mode == ACOPF_SWEEP_LAUNCHES || p->sweep_mode == ACOPF_SWEEP_GRAPH) {
    // one scenario: exact block counts; a batch: upper bounds of the
    // per-scenario block counts (excess blocks exit)
    const int single = ns == 1 ? 1 : 0;
    const long long nbl = (g->n_line + bs - 1) / bs + (single ? 0 : ns);
    // bus phase by workgroups of item_waves_for item blocks (bound from
    // the sizes; excess workgroups exit)
    const long long nbb = item_blocks_bound(g->n_line, g->n_gen, ns) / item_waves_for(g->n_line);
    if (nbb > w.max_partials || nbl > kMaxSweepBlocks || nbb > kMaxSweepBlocks)
      return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: grid too large for the block size");
    SweepLaunch a;
    a.g = *g;
    a.w = w;
    a.nbl = (int)nbl;
    a.nbb = (int)nbb;
    a.bs = bs;
    a.single = single;
    a.ns = ns;
    a.trace = p->trace;
    a.max_sweeps = p->max_sweeps;
    a.solver = solver;
    a.norm_inf = p->norm_inf;
    a.eps_pri = p->eps_pri;
    a.eps_dual = p->eps_dual;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    // a stream under capture records plain launches, and every chunk up to
    // the cap (the stop test then acts on the device only)
    const bool use_graph = p->sweep_mode == ACOPF_SWEEP_GRAPH && !capturing;
    hipLaunchKernelGGL(k_reset_solve, dim3(reset_blocks), dim3(256), 0, s, w, (int)nbb, bs,
                       item_waves_for(g->n_line), p->norm_inf);
    for (int k0 = 0; k0 < p->max_sweeps; k0 += kSweepChunk) {
      const int k1 = std::min(p->max_sweeps, k0 + kSweepChunk);
      hipGraphExec_t ge = nullptr;
      if (use_graph) {
        acopf_status rc = sweep_graph(a, k1 - k0, &ge);
        if (rc != ACOPF_OK) return rc;
      }
      if (ge)
        HIP_TRY(hipGraphLaunch(ge, s));
      else
        enqueue_sweeps(a, k1 - k0, s);
      if (balance && k1 % p->balance_every == 0 && k1 < p->max_sweeps) {
        hipLaunchKernelGGL(k_rho_balance, dim3(blocks_for(ns, 64)), dim3(64), 0, s, w, p->balance_mu,
                           p->balance_tau);
        hipLaunchKernelGGL(k_rho_apply, dim3(blocks_for(std::max(g->n_line, g->n_gen), 256)), dim3(256), 0, s, *g,
                           w);
      }
      HIP_TRY(hipGetLastError());
      if (k1 < p->max_sweeps && (p->eps_pri > 0.0 || p->eps_dual > 0.0) && !capturing) {
        // look at the stop flag before enqueueing more sweeps
        SyncState st;
        acopf_status rc = read_sync(w, s, &st);
        if (rc != ACOPF_OK) return rc;
        if (st.done) break;
      }
    }
  } else if (p->sweep_mode == ACOPF_SWEEP_PERSISTENT) {
    if (ns != 1) return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: the persistent mode serves one scenario");
    if (solver == 2)
      return fail(ACOPF_ERR_UNSUPPORTED, "acopf_linfeas: the projection runs in the launch-per-phase modes");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int cus = 0, coop = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: device has no cooperative launch");
    int per_cu = 0;
    const void* kern = local ? (const void*)k_sweep_persistent<true> : (const void*)k_sweep_persistent<false>;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, bs, 0));
    if (per_cu < 1) return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: persistent kernel does not fit a CU");
    long long want = std::max(blocks_for(g->n_line, bs), blocks_for(g->n_bus, bs));
    long long nblk = std::min<long long>(want, (long long)per_cu * cus);
    if (p->max_blocks > 0) nblk = std::min<long long>(nblk, p->max_blocks);
    nblk = std::min<long long>(nblk, w.max_partials);
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_reset_solve, dim3(reset_blocks), dim3(256), 0, s, w, (int)nblk, bs, 0, p->norm_inf);
    acopf_grid gg = *g;
    int ms = p->max_sweeps;
    double ep = p->eps_pri, ed = p->eps_dual;
    void* args[] = {&gg, &w, &ms, &ep, &ed};
    HIP_TRY(hipLaunchCooperativeKernel(kern, dim3((unsigned)nblk), dim3(bs), args, 0, s));
  } else {
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: unknown sweep mode");
  }
  if (result) return acopf_admm_result_get(g, workspace, stream, result);
  return ACOPF_OK;
}

acopf_status acopf_admm_result_batch(const acopf_grid* g, void* workspace, void* stream, acopf_admm_result* out) {
  if (!grid_ok(g) || !workspace || !out) return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_result: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  std::vector<ScenState> sc(w.n_scen);
  SyncState st;
  HIP_TRY(hipMemcpyAsync(sc.data(), w.scen, w.n_scen * sizeof(ScenState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&st, w.sync, sizeof(SyncState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < w.n_scen; ++k) {
    out[k].sweeps = sc[k].sweeps;
    out[k].outcome = sc[k].status != 0 ? ACOPF_ADMM_FAILED
                     : sc[k].converged ? ACOPF_ADMM_CONVERGED : ACOPF_ADMM_MAX_SWEEPS;
    out[k].r_norm = sc[k].r_norm;
    out[k].s_norm = sc[k].s_norm;
    out[k].infeasible_lines = sc[k].sweeps > 0 ? sc[k].infeasible[(sc[k].sweeps - 1) & 1] : 0;
    out[k].blocks = st.blocks;
    out[k].status = sc[k].status;
    out[k].relaxed_lines = sc[k].relaxed;
  }
  if (st.barrier_error) return fail(ACOPF_ERR_BARRIER, "acopf_admm_solve: grid barrier timed out");
  if (w.n_scen > 1) return ACOPF_OK;  // failures of a batch are per-scenario outcomes
  if (st.numeric_error)
    return fail(ACOPF_ERR_NUMERIC, "acopf_admm_solve: the QP build met a vanishing elimination pivot or non-finite data");
  if (st.nonconvex)
    return fail(ACOPF_ERR_NONCONVEX_LINE, "acopf_admm_solve: a line subproblem matrix is not positive definite");
  return ACOPF_OK;
}

acopf_status acopf_admm_result_get(const acopf_grid* g, void* workspace, void* stream, acopf_admm_result* result) {
  if (!grid_ok(g) || !workspace || !result) return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_result_get: null argument");
  Workspace w = ws_of(g, workspace);
  std::vector<acopf_admm_result> all(w.n_scen);
  acopf_status rc = acopf_admm_result_batch(g, workspace, stream, all.data());
  *result = all[0];
  return rc;
}

acopf_status acopf_admm_state_get(const acopf_grid* g, void* workspace, const acopf_admm_state* o, void* stream) {
  if (!grid_ok(g) || !workspace || !o) return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_state_get: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const size_t D = sizeof(double);
  const size_t G2 = 2 * (size_t)g->n_gen, L8 = 8 * (size_t)g->n_line, L4 = 4 * (size_t)g->n_line;
  auto cp = [&](double* dst, const double* src, size_t n) -> hipError_t {
    if (!dst || n == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, n * D, hipMemcpyDeviceToDevice, s);
  };
  auto fields = [&](double* dst, const double* src, int F) -> hipError_t {  // line-by-line -> caller layout
    if (!dst) return hipSuccess;
    const long long n = (long long)g->n_line * F;
    if (F == 8)
      hipLaunchKernelGGL(k_lines_to_fields, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst, src, g->n_line);
    else
      hipLaunchKernelGGL(k_lines4_to_fields, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst, src, g->n_line);
    return hipGetLastError();
  };
  (void)L8;
  (void)L4;
  HIP_TRY(cp(o->xg, w.xg, G2));
  HIP_TRY(cp(o->xbar_g, w.xbar_g, G2));
  HIP_TRY(cp(o->lam_g, w.lam_g, G2));
  HIP_TRY(cp(o->rho_g, w.rho_g, G2));
  HIP_TRY(fields(o->xl, w.xl, 8));
  HIP_TRY(fields(o->xbar_f, w.xbar_f, 4));
  HIP_TRY(fields(o->lam_l, w.lam_l, 8));
  HIP_TRY(fields(o->rho_l, w.rho_l, 8));
  HIP_TRY(cp(o->dw, w.dw, g->n_bus));
  HIP_TRY(cp(o->dth, w.dth, g->n_bus));
  HIP_TRY(cp(o->nu, w.nu, 2 * (size_t)g->n_bus));
  HIP_TRY(cp(o->mu, w.mu, 2 * (size_t)g->n_line));
  HIP_TRY(cp(o->sum_r_g, w.tr_r_g, G2));
  HIP_TRY(cp(o->sum_s_g, w.tr_s_g, G2));
  HIP_TRY(cp(o->sum_r_l, w.tr_r_l, L8));
  HIP_TRY(cp(o->sum_s_l, w.tr_s_l, L8));
  return ACOPF_OK;
}

acopf_status acopf_step(const acopf_grid* g, const acopf_iterate* x, void* workspace, const acopf_iterate* d,
                        void* stream) {
  if (!grid_ok(g) || !iterate_ok(x) || !iterate_ok(d) || !workspace)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_step: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int bs = kDefaultBlock;
  hipLaunchKernelGGL(k_step_lines, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, *g, *x, w, *d, 0);
  hipLaunchKernelGGL(k_step_nodes, dim3(blocks_for(std::max(g->n_bus, g->n_gen), bs)), dim3(bs), 0, s, *g, w, *d, 0);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_sqp_step_batch(const acopf_grid* g, const acopf_iterate* x, const acopf_iterate* d,
                                  const double* rho_g, const double* rho_l, const acopf_sqp_params* p,
                                  void* workspace, void* stream, acopf_sqp_state* states) {
  if (!grid_ok(g) || !iterate_ok(x) || !iterate_ok(d) || !p || !workspace)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: null argument");
  if (!(p->mu > 0.0) || !(p->delta_max > 0.0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: penalty and radius cap must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (capturing && states)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step_batch: host results need a synchronisation; pass states = NULL "
                                       "while the stream is being captured");
  if (p->stop && !(p->tol_primal >= 0.0 && p->tol_dual >= 0.0 && p->tol_step >= 0.0 && p->delta_min >= 0.0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: stop tolerances must be >= 0");
  if (p->restore != 0 && p->restore != 1) return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: restore must be 0 or 1");
  if (p->hessian_mode != ACOPF_HESSIAN_PSD && p->hessian_mode != ACOPF_HESSIAN_RAW &&
      p->hessian_mode != ACOPF_HESSIAN_RAW_LOCAL)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: unknown Hessian mode");
  acopf_status rc = qp_build_impl(g, x, 0.0, p->restore ? kModeRestore : p->hessian_mode, workspace, stream);
  if (rc != ACOPF_OK) return rc;
  const bool soc = p->soc && !p->restore;
  if (p->stop) hipLaunchKernelGGL(k_sqp_begin, dim3(blocks_for(w.n_scen, 64)), dim3(64), 0, s, w);
  if (p->pi_update != ACOPF_PI_ALWAYS && p->pi_update != ACOPF_PI_IF_CONVERGED)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: unknown multiplier update rule");
  if (p->warm_start < ACOPF_START_ZERO || p->warm_start > ACOPF_START_GIVEN)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: unknown warm-start mode");
  if (p->warm_start == ACOPF_START_GIVEN && (!p->lam_l0 || (g->n_gen > 0 && !p->lam_g0)))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: ACOPF_START_GIVEN needs lam_g0 and lam_l0");
  if (p->warm_start == ACOPF_START_GIVEN)
    rc = admm_init_impl(g, rho_g, rho_l, p->lam_g0, p->lam_l0, false, workspace, stream);
  else
    rc = admm_init_impl(g, rho_g, rho_l, nullptr, nullptr, p->warm_start == ACOPF_START_PREVIOUS, workspace,
                        stream);
  if (rc != ACOPF_OK) return rc;
  // under stream capture (a caller recording the SQP loop in a graph) the
  // iteration is recorded without timing events and without results
  EventPair ev;
  if (!capturing) {
    HIP_TRY(ev.create());
    HIP_TRY(hipEventRecord(ev.a, s));
  }
  rc = acopf_admm_solve(g, &p->admm, workspace, stream, nullptr);
  if (rc != ACOPF_OK) return rc;
  if (!capturing) HIP_TRY(hipEventRecord(ev.b, s));
  rc = acopf_step(g, x, workspace, d, stream);
  if (rc != ACOPF_OK) return rc;
  const int bs = 256;
  const int nb = blocks_for(std::max(std::max(g->n_line, g->n_bus), g->n_gen), bs);
  const int K = red_blocks(g, w.n_scen);
  hipLaunchKernelGGL(k_merit_parts, dim3(nb), dim3(bs), 0, s, *g, *x, w, *d);
  hipLaunchKernelGGL(k_merit_partial, dim3(w.n_scen * K), dim3(256), 0, s, w, K);
  hipLaunchKernelGGL(k_decide, dim3(w.n_scen), dim3(64), 0, s, w, K, p->mu, p->delta_max, p->grow_ratio,
                     (int)p->pi_update, soc ? 1 : 0, p->restore);
  hipLaunchKernelGGL(k_apply, dim3(nb), dim3(bs), 0, s, *g, *x, *d, w, 0);
  HIP_TRY(hipGetLastError());
  std::vector<acopf_admm_result> ar(w.n_scen);
  bool have_ar = false;
  if (soc) {
    // second-order correction of the rejected steps (end of Section II-D):
    // under capture the pass is always recorded (scenarios without a
    // rejected step are left out of it); otherwise it runs only when a
    // scenario asks for it
    bool run = true;
    if (!capturing) {
      std::vector<SqpDecision> d0(w.n_scen);
      HIP_TRY(hipMemcpyAsync(d0.data(), w.decision, w.n_scen * sizeof(SqpDecision), hipMemcpyDeviceToHost, s));
      rc = acopf_admm_result_batch(g, workspace, stream, ar.data());  // synchronises
      if (rc != ACOPF_OK) return rc;
      have_ar = true;
      run = false;
      for (int k = 0; k < w.n_scen; ++k) run = run || d0[k].soc == 1;
    }
    if (run) {
      const int nl = blocks_for(g->n_line, bs);
      hipLaunchKernelGGL(k_soc_begin, dim3(nb), dim3(bs), 0, s, *g, *x, *d, w);
      hipLaunchKernelGGL(k_build_lines, dim3(nl), dim3(bs), 0, s, *g, *x, (int)p->hessian_mode, w, 1);
      hipLaunchKernelGGL(k_soc_init, dim3(nb), dim3(bs), 0, s, *g, w);
      HIP_TRY(hipGetLastError());
      acopf_admm_params a2 = p->admm;
      a2.trace = 0;  // traces describe the first solve
      rc = acopf_admm_solve(g, &a2, workspace, stream, nullptr);
      if (rc != ACOPF_OK) return rc;
      hipLaunchKernelGGL(k_step_lines, dim3(nl), dim3(bs), 0, s, *g, *x, w, *d, 1);
      hipLaunchKernelGGL(k_step_nodes, dim3(blocks_for(std::max(g->n_bus, g->n_gen), bs)), dim3(bs), 0, s, *g, w, *d,
                         1);
      hipLaunchKernelGGL(k_merit_parts, dim3(nb), dim3(bs), 0, s, *g, *x, w, *d);
      hipLaunchKernelGGL(k_merit_partial, dim3(w.n_scen * K), dim3(256), 0, s, w, K);
      hipLaunchKernelGGL(k_soc_decide, dim3(w.n_scen), dim3(64), 0, s, w, K, p->mu, p->delta_max, p->grow_ratio,
                         (int)p->pi_update);
      hipLaunchKernelGGL(k_apply, dim3(nb), dim3(bs), 0, s, *g, *x, *d, w, 1);
      HIP_TRY(hipGetLastError());
    }
  }
  if (p->stop) {
    hipLaunchKernelGGL(k_residual_parts, dim3(nb), dim3(bs), 0, s, *g, *x, w);
    hipLaunchKernelGGL(k_residual_partial, dim3(w.n_scen * K), dim3(256), 0, s, w, K);
    hipLaunchKernelGGL(k_residual_reduce, dim3(w.n_scen), dim3(64), 0, s, w, K);
    hipLaunchKernelGGL(k_sqp_stop, dim3(blocks_for(w.n_scen, 64)), dim3(64), 0, s, w, p->tol_primal, p->tol_dual,
                       p->tol_step, p->delta_min);
    HIP_TRY(hipGetLastError());
  }
  if (!states) return ACOPF_OK;
  std::vector<SqpDecision> dc(w.n_scen);
  HIP_TRY(hipMemcpyAsync(dc.data(), w.decision, w.n_scen * sizeof(SqpDecision), hipMemcpyDeviceToHost, s));
  if (!have_ar) {
    rc = acopf_admm_result_batch(g, workspace, stream, ar.data());
    if (rc != ACOPF_OK) return rc;
  } else {
    HIP_TRY(hipStreamSynchronize(s));
  }
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
  for (int k = 0; k < w.n_scen; ++k) {
    acopf_sqp_state* st = &states[k];
    st->delta = dc[k].delta_out;
    st->accepted = dc[k].accepted;
    st->ared = dc[k].ared;
    st->pred = dc[k].pred;
    st->step_inf = dc[k].step_inf;
    st->objective = dc[k].accepted ? dc[k].f_xd : dc[k].f_x;
    st->merit = dc[k].accepted ? dc[k].f_xd + p->mu * dc[k].h_xd : dc[k].f_x + p->mu * dc[k].h_x;
    st->admm_sweeps = ar[k].sweeps;
    st->admm_r = ar[k].r_norm;
    st->admm_s = ar[k].s_norm;
    st->admm_ms = ms;
    st->status = ar[k].status;
    st->soc_sweeps = dc[k].soc_sweeps;
  }
  return ACOPF_OK;
}

acopf_status acopf_sqp_step(const acopf_grid* g, const acopf_iterate* x, const acopf_iterate* d,
                            const double* rho_g, const double* rho_l, const acopf_sqp_params* p, void* workspace,
                            void* stream, acopf_sqp_state* state) {
  if (!grid_ok(g) || !state || !workspace) return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: null argument");
  if (n_scen_of(g) != 1) return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: use acopf_sqp_step_batch for batches");
  if (!(state->delta > 0.0)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: trust radius must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  hipLaunchKernelGGL(k_set_delta, dim3(1), dim3(64), 0, s, w, state->delta);
  HIP_TRY(hipGetLastError());
  return acopf_sqp_step_batch(g, x, d, rho_g, rho_l, p, workspace, stream, state);
}

acopf_status acopf_sqp_outcome_batch(const acopf_grid* g, void* workspace, void* stream, acopf_sqp_outcome* out) {
  if (!grid_ok(g) || !workspace || !out) return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_outcome_batch: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  std::vector<ScenState> sc(w.n_scen);
  HIP_TRY(hipMemcpyAsync(sc.data(), w.scen, w.n_scen * sizeof(ScenState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int dev = 0, khz = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return fail(ACOPF_ERR_HIP, "acopf_sqp_outcome_batch: no device wall-clock rate");
  for (int k = 0; k < w.n_scen; ++k) {
    out[k].done = sc[k].sqp_done;
    out[k].reason = sc[k].sqp_reason;
    out[k].iterations = sc[k].sqp_iters;
    out[k].reserved = 0;
    out[k].seconds = sc[k].sqp_done ? (double)(sc[k].t_done - sc[k].t_start) / (1e3 * (double)khz) : 0.0;
  }
  return ACOPF_OK;
}

acopf_status acopf_residuals_batch(const acopf_grid* g, const acopf_iterate* x, void* workspace, void* stream,
                                   acopf_residuals_report* out) {
  if (!grid_ok(g) || !iterate_ok(x) || !workspace || !out)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_residuals: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int bs = 256;
  const int nb = blocks_for(std::max(std::max(g->n_line, g->n_bus), g->n_gen), bs);
  const int K = red_blocks(g, w.n_scen);
  hipLaunchKernelGGL(k_residual_parts, dim3(nb), dim3(bs), 0, s, *g, *x, w);
  hipLaunchKernelGGL(k_residual_partial, dim3(w.n_scen * K), dim3(256), 0, s, w, K);
  hipLaunchKernelGGL(k_residual_reduce, dim3(w.n_scen), dim3(64), 0, s, w, K);
  HIP_TRY(hipGetLastError());
  std::vector<ResidualReport> r(w.n_scen);
  HIP_TRY(hipMemcpyAsync(r.data(), w.report, w.n_scen * sizeof(ResidualReport), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < w.n_scen; ++k) {
    out[k].balance = r[k].balance;
    out[k].c11 = r[k].c11;
    out[k].c12 = r[k].c12;
    out[k].limit = r[k].limit;
    out[k].bounds = r[k].bounds;
    out[k].primal = std::max(std::max(std::max(r[k].balance, r[k].c11), std::max(r[k].c12, r[k].limit)), r[k].bounds);
    out[k].dual = r[k].dual / std::max(1.0, r[k].gradf);
  }
  return ACOPF_OK;
}

acopf_status acopf_linfeas(const acopf_grid* g, const acopf_iterate* x, double rho, const acopf_admm_params* p,
                           void* workspace, void* stream, acopf_admm_result* result) {
  if (!grid_ok(g) || !iterate_ok(x) || !p || !workspace)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_linfeas: null argument");
  if (!(rho > 0.0)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_linfeas: rho must be > 0");
  if (p->sweep_mode == ACOPF_SWEEP_PERSISTENT)
    return fail(ACOPF_ERR_UNSUPPORTED, "acopf_linfeas: the projection runs in the launch-per-phase modes");
  if (p->trace || p->balance_every != 0)
    return fail(ACOPF_ERR_UNSUPPORTED, "acopf_linfeas: no trace sums or residual balancing for the projection");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int bs = kDefaultBlock;
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, w, kModeLinfeas);
  set_hessian_mode(workspace, kModeLinfeas);
  hipLaunchKernelGGL(k_build_lines_linfeas, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, *g, *x, w);
  if (g->n_gen > 0)
    hipLaunchKernelGGL(k_build_gens_linfeas, dim3(blocks_for(g->n_gen, bs)), dim3(bs), 0, s, *g, *x, w);
  hipLaunchKernelGGL(k_build_buses, dim3(blocks_for(g->n_bus, bs)), dim3(bs), 0, s, *g, *x, w);
  HIP_TRY(hipGetLastError());
  acopf_status rc = admm_init_impl(g, nullptr, nullptr, nullptr, nullptr, false, workspace, stream, rho);
  if (rc != ACOPF_OK) return rc;
  rc = acopf_admm_solve(g, p, workspace, stream, nullptr);
  if (rc != ACOPF_OK) return rc;
  const int n = g->n_gen + g->n_bus + g->n_line;
  hipLaunchKernelGGL(k_apply_linfeas, dim3(blocks_for(n, bs)), dim3(bs), 0, s, *g, *x, w);
  HIP_TRY(hipGetLastError());
  if (result) return acopf_admm_result_get(g, workspace, stream, result);
  return ACOPF_OK;
}

acopf_status acopf_residuals(const acopf_grid* g, const acopf_iterate* x, void* workspace, void* stream,
                             acopf_residuals_report* out) {
  if (!grid_ok(g) || !out) return fail(ACOPF_ERR_INVALID_ARG, "acopf_residuals: null argument");
  if (n_scen_of(g) != 1) return fail(ACOPF_ERR_INVALID_ARG, "acopf_residuals: use acopf_residuals_batch for batches");
  return acopf_residuals_batch(g, x, workspace, stream, out);
}

acopf_status acopf_features(const acopf_grid* g, const acopf_iterate* x, void* workspace, int32_t first,
                            float* line_x, int64_t ld_line, float* gen_x, int64_t ld_gen, void* stream) {
  if (!grid_ok(g) || !iterate_ok(x) || !workspace || !line_x || (g->n_gen > 0 && !gen_x))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_features: null argument");
  if (ld_line < g->n_line || (g->n_gen > 0 && ld_gen < g->n_gen))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_features: leading dimension below the component count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = std::max(g->n_line, g->n_gen);
  Workspace w = ws_of(g, workspace);
  hipLaunchKernelGGL(k_features, dim3(blocks_for(n, 256)), dim3(256), 0, s, *g, *x, w, (int)(first != 0), line_x,
                     (long long)ld_line, gen_x, (long long)ld_gen);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_warm_targets(const acopf_grid* g, void* workspace, float* line_t, int64_t ld_line, float* gen_t,
                                int64_t ld_gen, void* stream) {
  if (!grid_ok(g) || !workspace || !line_t || (g->n_gen > 0 && !gen_t))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_warm_targets: null argument");
  if (ld_line < g->n_line || (g->n_gen > 0 && ld_gen < g->n_gen))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_warm_targets: leading dimension below the component count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int n = std::max(g->n_line, g->n_gen);
  hipLaunchKernelGGL(k_targets, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, line_t, (long long)ld_line, gen_t,
                     (long long)ld_gen);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_warm_decode(const acopf_grid* g, void* workspace, const float* line_y, int64_t ld_line,
                               const float* gen_y, int64_t ld_gen, double rho_l0, double rho_g0, int32_t first,
                               int32_t use_lam, int32_t use_rho, double* lam_l, double* lam_g, double* rho_l,
                               double* rho_g, void* stream) {
  if (!grid_ok(g) || !workspace || !line_y || !lam_l || !rho_l ||
      (g->n_gen > 0 && (!gen_y || !lam_g || !rho_g)))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_warm_decode: null argument");
  if (ld_line < g->n_line || (g->n_gen > 0 && ld_gen < g->n_gen))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_warm_decode: leading dimension below the component count");
  if (!(rho_l0 > 0.0) || !(rho_g0 > 0.0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_warm_decode: base penalties must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int n = std::max(g->n_line, g->n_gen);
  hipLaunchKernelGGL(k_decode, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, line_y, (long long)ld_line, gen_y,
                     (long long)ld_gen, rho_l0, rho_g0, (int)(first != 0), (int)(use_lam != 0), (int)(use_rho != 0),
                     lam_l, lam_g, rho_l, rho_g);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

}  // extern "C"
