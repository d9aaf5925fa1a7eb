// MI355X (gfx950) kernels and C ABI of the ADMM QP solver for the SQP
// method for ACOPF (arXiv 2310.13143, Sections III-IV).
//
// One thread per component: the line update (the only non-closed-form
// subproblem) runs one 4-variable QP per lane; buses gather the couplings of
// their incident line ends and generators through CSR tables.  A sweep is
// phase A (lines) -> grid barrier -> phase B (generators, buses,
// multipliers, residual partials) -> grid barrier, the last block to arrive
// summing the partials in a fixed order and deciding the stop.  The
// persistent kernel keeps every block resident for all sweeps; the
// "launches" mode runs the same phases as three kernels per sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "components.h"

using namespace acopf;

namespace {

thread_local std::string g_last_error = "no error";

acopf_status fail(acopf_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(ACOPF_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
  } while (0)

constexpr int kDefaultBlock = 256;
constexpr long long kSpinLimit = 1LL << 25;

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

// ---------------------------------------------------------------- QP build
__global__ void k_build_lines(acopf_grid g, acopf_iterate x, double delta, int mode, Workspace w) {
  for (int l = gtid(); l < g.n_line; l += gstride())
    if (!build_line(g, x, delta, mode, w, l)) atomicAdd(&w.sync->numeric_error, 1);
}

__global__ void k_build_gens(acopf_grid g, acopf_iterate x, double delta, Workspace w) {
  for (int k = gtid(); k < g.n_gen; k += gstride()) build_gen(g, x, delta, w, k);
}

__global__ void k_build_buses(acopf_grid g, acopf_iterate x, Workspace w) {
  for (int i = gtid(); i < g.n_bus; i += gstride()) build_bus(g, x, w, i);
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

__global__ void k_prep_lines(Workspace w) {
  for (int l = gtid(); l < w.n_line; l += gstride())
    if (!prep_line(w, l)) atomicAdd(&w.sync->nonconvex, 1);
}

__global__ void k_reset_sync(Workspace w, int blocks) {
  for (int b = gtid(); b < w.max_partials; b += gstride()) w.arrive[b * kArriveStride] = 0u;
  if (gtid() == 0) {
    SyncState* s = w.sync;
    s->go = 0u;
    s->converged = 0;
    s->blocks = blocks;
    s->count = 0;
    s->gen = 0;
    s->done = 0;
    s->sweeps = 0;
    s->barrier_error = 0;
    s->infeasible[0] = 0;
    s->infeasible[1] = 0;
    s->r_norm = 0.0;
    s->s_norm = 0.0;
  }
}

__global__ void k_clear_flags(Workspace w) {
  if (gtid() == 0) {
    w.sync->numeric_error = 0;
    w.sync->nonconvex = 0;
  }
}

// ---------------------------------------------------------------- sweeps
__device__ __forceinline__ void phase_lines(const acopf_grid& g, const Workspace& w, int* infeasible) {
  for (int l = gtid(); l < g.n_line; l += gstride())
    if (update_line(g, w, l) != 0) atomicAdd(infeasible, 1);
}

__device__ __forceinline__ void phase_buses(const acopf_grid& g, const Workspace& w, double* lds) {
  double r2 = 0.0, s2 = 0.0;
  for (int i = gtid(); i < g.n_bus; i += gstride()) update_bus(g, w, i, r2, s2);
  r2 = block_sum(r2, lds);
  s2 = block_sum(s2, lds);
  if (threadIdx.x == 0) {
    w.partials[blockIdx.x] = r2;
    w.partials[w.max_partials + blockIdx.x] = s2;
  }
}

// Sum of the per-block partials (fixed order), stop decision, sweep count.
__device__ void finish_sweep(const Workspace& w, int nparts, int max_sweeps, double eps_pri,
                             double eps_dual, double* lds) {
  double r2 = 0.0, s2 = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
    r2 += w.partials[b];
    s2 += w.partials[w.max_partials + b];
  }
  r2 = block_sum(r2, lds);
  s2 = block_sum(s2, lds);
  if (threadIdx.x == 0) {
    SyncState* s = w.sync;
    const int k = s->sweeps + 1;
    s->sweeps = k;
    const double r = sqrt(r2), sn = sqrt(s2);
    s->r_norm = r;
    s->s_norm = sn;
    const bool conv = (eps_pri > 0.0 || eps_dual > 0.0) && r <= eps_pri && sn <= eps_dual;
    s->converged = conv ? 1 : 0;
    s->done = (conv || k >= max_sweeps || s->barrier_error) ? 1 : 0;
    s->infeasible[k & 1] = 0;  // counter of the next sweep
  }
}

__global__ void __launch_bounds__(256) k_line_phase(acopf_grid g, Workspace w) {
  if (__hip_atomic_load(&w.sync->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int k = w.sync->sweeps;
  phase_lines(g, w, &w.sync->infeasible[k & 1]);
}

__global__ void __launch_bounds__(256) k_bus_phase(acopf_grid g, Workspace w) {
  __shared__ double lds[16];
  if (__hip_atomic_load(&w.sync->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  phase_buses(g, w, lds);
}

__global__ void k_finish_phase(Workspace w, int nparts, int max_sweeps, double eps_pri, double eps_dual) {
  __shared__ double lds[16];
  if (w.sync->done) return;
  finish_sweep(w, nparts, max_sweeps, eps_pri, eps_dual, lds);
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
  // block 0: wait for every other block
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

__global__ void __launch_bounds__(256) k_sweep_persistent(acopf_grid g, Workspace w, int max_sweeps,
                                                          double eps_pri, double eps_dual) {
  __shared__ double lds[16];
  __shared__ int s_stop;
  SyncState* sy = w.sync;
  for (int k = 0; k < max_sweeps; ++k) {
    phase_lines(g, w, &sy->infeasible[k & 1]);
    grid_barrier(w, 2u * k + 1u, [] {});
    phase_buses(g, w, lds);
    grid_barrier(w, 2u * k + 2u, [&] { finish_sweep(w, gridDim.x, max_sweeps, eps_pri, eps_dual, lds); });
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
__global__ void k_step_lines(acopf_grid g, acopf_iterate x, Workspace w, acopf_iterate d) {
  for (int l = gtid(); l < g.n_line; l += gstride()) step_line(g, x, w, d, l);
}

__global__ void k_step_nodes(acopf_grid g, Workspace w, acopf_iterate d) {
  for (int i = gtid(); i < g.n_bus; i += gstride()) {
    d.w[i] = w.dw[i];
    d.th[i] = w.dth[i];
  }
  for (int k = gtid(); k < g.n_gen; k += gstride()) {
    d.pg[k] = w.xg[k];
    d.qg[k] = w.xg[g.n_gen + k];
  }
}

// ---------------------------------------------------------------- SQP step
// Block-wise sums of the merit pieces and the maximum step component.
__global__ void __launch_bounds__(256) k_merit(acopf_grid g, acopf_iterate x, Workspace w, acopf_iterate d) {
  __shared__ double lds[16];
  double acc[kMeritFields];
#pragma unroll
  for (int k = 0; k < kMeritFields; ++k) acc[k] = 0.0;
  for (int l = gtid(); l < g.n_line; l += gstride()) {
    double o[4];
    merit_line(g, x, w, d, l, o);
    acc[3] += o[0];
    acc[4] += o[1];
    acc[5] += o[2];
    acc[6] += o[3];
  }
  double smax = 0.0;
  for (int k = gtid(); k < g.n_gen; k += gstride()) {
    double o[3];
    merit_gen(g, x, d, k, o);
    acc[0] += o[0];
    acc[1] += o[1];
    acc[2] += o[2];
    smax = fmax(smax, fmax(fabs(d.pg[k]), fabs(d.qg[k])));
  }
  for (int i = gtid(); i < g.n_bus; i += gstride()) smax = fmax(smax, fmax(fabs(d.w[i]), fabs(d.th[i])));
#pragma unroll
  for (int k = 0; k < kMeritFields - 1; ++k) acc[k] = block_sum(acc[k], lds);
  // block maximum of the step (order independent)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = smax;
  __syncthreads();
  double m = 0.0;
  for (int k = 0; k < (int)((blockDim.x + 63) >> 6); ++k) m = fmax(m, lds[k]);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kMeritFields - 1; ++k) w.merit_partials[k * w.max_partials + blockIdx.x] = acc[k];
    w.merit_partials[(kMeritFields - 1) * w.max_partials + blockIdx.x] = m;
  }
}

// Acceptance test and trust-radius update of Algorithm 1 (one block).
__global__ void k_decide(Workspace w, int nparts, double mu, double delta, double delta_max, double grow) {
  __shared__ double lds[16];
  double acc[kMeritFields];
#pragma unroll
  for (int k = 0; k < kMeritFields; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kMeritFields - 1; ++k) acc[k] += w.merit_partials[k * w.max_partials + b];
    acc[kMeritFields - 1] = fmax(acc[kMeritFields - 1], w.merit_partials[(kMeritFields - 1) * w.max_partials + b]);
  }
#pragma unroll
  for (int k = 0; k < kMeritFields - 1; ++k) acc[k] = block_sum(acc[k], lds);
  double smax = acc[kMeritFields - 1];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = smax;
  __syncthreads();
  double m = 0.0;
  for (int k = 0; k < (int)((blockDim.x + 63) >> 6); ++k) m = fmax(m, lds[k]);
  if (threadIdx.x == 0) {
    SqpDecision* dc = w.decision;
    dc->f_x = acc[0];
    dc->f_xd = acc[1];
    dc->h_x = acc[3];
    dc->h_xd = acc[4];
    dc->m_d = acc[5];
    dc->quad = acc[2] + acc[6];
    const double ared = (acc[0] + mu * acc[3]) - (acc[1] + mu * acc[4]);
    const double pred = -(acc[2] + acc[6]) + mu * (acc[3] - acc[5]);
    dc->ared = ared;
    dc->pred = pred;
    dc->step_inf = m;
    dc->delta_in = delta;
    const bool acc_ok = ared > 0.0 && pred > 0.0;
    double dn = delta;
    if (acc_ok) {
      if (m >= 0.99 * delta && ared >= grow * pred) dn = fmin(2.0 * delta, delta_max);
    } else {
      dn = 0.5 * fmin(delta, m);
    }
    dc->delta_out = dn;
    dc->accepted = acc_ok ? 1 : 0;
  }
}

// x <- x + d and pi <- new estimates, if the step was accepted.
__global__ void k_apply(acopf_grid g, acopf_iterate x, acopf_iterate d, Workspace w) {
  if (!w.decision->accepted) return;
  for (int k = gtid(); k < g.n_gen; k += gstride()) {
    x.pg[k] += d.pg[k];
    x.qg[k] += d.qg[k];
  }
  for (int i = gtid(); i < g.n_bus; i += gstride()) {
    x.w[i] += d.w[i];
    x.th[i] += d.th[i];
  }
  for (int l = gtid(); l < g.n_line; l += gstride()) {
    x.wR[l] += d.wR[l];
    x.wI[l] += d.wI[l];
    x.pi[l] = d.pi[l];
    x.pi[g.n_line + l] = d.pi[g.n_line + l];
    x.pi[2 * g.n_line + l] = d.pi[2 * g.n_line + l];
    x.pi[3 * g.n_line + l] = d.pi[3 * g.n_line + l];
  }
}

// ---------------------------------------------------------------- residuals
__device__ double block_max(double v, double* lds) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = 0.0;
  for (int k = 0; k < (int)((blockDim.x + 63) >> 6); ++k) m = fmax(m, lds[k]);
  __syncthreads();
  return m;
}

__global__ void __launch_bounds__(256) k_residuals(acopf_grid g, acopf_iterate x, Workspace w) {
  __shared__ double lds[16];
  double acc[kResidFields];
#pragma unroll
  for (int k = 0; k < kResidFields; ++k) acc[k] = 0.0;
  for (int l = gtid(); l < g.n_line; l += gstride()) {
    double pr[5] = {0, 0, 0, 0, 0}, du = 0.0;
    residual_line(g, x, w, l, pr, du);
    acc[1] = fmax(acc[1], pr[1]);
    acc[2] = fmax(acc[2], pr[2]);
    acc[3] = fmax(acc[3], pr[3]);
    acc[5] = fmax(acc[5], du);
  }
  for (int i = gtid(); i < g.n_bus; i += gstride()) {
    double pr[5] = {0, 0, 0, 0, 0}, du = 0.0;
    residual_bus(g, x, w, i, pr, du);
    acc[0] = fmax(acc[0], pr[0]);
    acc[4] = fmax(acc[4], pr[4]);
    acc[5] = fmax(acc[5], du);
  }
  for (int k = gtid(); k < g.n_gen; k += gstride()) {
    double bnd, du, gf;
    residual_gen(g, x, w, k, bnd, du, gf);
    acc[4] = fmax(acc[4], bnd);
    acc[5] = fmax(acc[5], du);
    acc[6] = fmax(acc[6], gf);
  }
#pragma unroll
  for (int k = 0; k < kResidFields; ++k) acc[k] = block_max(acc[k], lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kResidFields; ++k) w.resid_partials[k * w.max_partials + blockIdx.x] = acc[k];
  }
}

__global__ void k_residuals_final(Workspace w, int nparts) {
  __shared__ double lds[16];
  double acc[kResidFields];
#pragma unroll
  for (int k = 0; k < kResidFields; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kResidFields; ++k) acc[k] = fmax(acc[k], w.resid_partials[k * w.max_partials + b]);
  }
#pragma unroll
  for (int k = 0; k < kResidFields; ++k) acc[k] = block_max(acc[k], lds);
  if (threadIdx.x == 0) {
    ResidualReport* r = w.report;
    r->balance = acc[0];
    r->c11 = acc[1];
    r->c12 = acc[2];
    r->limit = acc[3];
    r->bounds = acc[4];
    r->dual = acc[5];
    r->gradf = acc[6];
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

bool grid_ok(const acopf_grid* g) {
  return g && g->n_bus > 0 && g->n_line > 0 && g->n_gen >= 0 && g->ref_bus >= 0 &&
         g->ref_bus < g->n_bus && g->vmin && g->vmax && g->pd && g->qd && g->gsh && g->bsh &&
         g->line_from && g->line_to && g->gii && g->bii && g->gij && g->bij && g->gji && g->bji &&
         g->gjj && g->bjj && g->smax_ij && g->smax_ji &&
         (g->n_gen == 0 || (g->gen_bus && g->pmin && g->pmax && g->qmin && g->qmax && g->cost2 && g->cost1));
}

bool iterate_ok(const acopf_iterate* x) {
  return x && x->pg && x->qg && x->w && x->th && x->wR && x->wI && x->pi;
}

Workspace ws_of(const acopf_grid* g, void* base) {
  Workspace w;
  layout_workspace(base, g->n_bus, g->n_line, g->n_gen, &w);
  return w;
}

acopf_status read_sync(void* ws_base, const acopf_grid* g, hipStream_t s, SyncState* out) {
  Workspace w = ws_of(g, ws_base);
  HIP_TRY(hipMemcpyAsync(out, w.sync, sizeof(SyncState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return ACOPF_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char* acopf_last_error(void) { return g_last_error.c_str(); }

size_t acopf_workspace_bytes(int32_t n_bus, int32_t n_line, int32_t n_gen) {
  if (n_bus <= 0 || n_line <= 0 || n_gen < 0) return 0;
  return layout_workspace(nullptr, n_bus, n_line, n_gen, nullptr);
}

acopf_status acopf_setup(const acopf_grid* g, void* workspace, size_t bytes, void* stream) {
  if (!grid_ok(g)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: incomplete grid description");
  if (!workspace) return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: null workspace");
  const size_t need = acopf_workspace_bytes(g->n_bus, g->n_line, g->n_gen);
  if (bytes < need)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: workspace of " + std::to_string(bytes) +
                                           " bytes, need " + std::to_string(need));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = g->n_bus, nl = g->n_line, ng = g->n_gen;
  std::vector<int32_t> from(nl), to(nl), gb(ng);
  HIP_TRY(hipMemcpyAsync(from.data(), g->line_from, nl * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(to.data(), g->line_to, nl * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  if (ng > 0) HIP_TRY(hipMemcpyAsync(gb.data(), g->gen_bus, ng * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int32_t> deg(nb, 0), gdeg(nb, 0);
  for (int l = 0; l < nl; ++l) {
    if (from[l] < 0 || from[l] >= nb || to[l] < 0 || to[l] >= nb || from[l] == to[l])
      return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: line " + std::to_string(l) + " has a bad end bus");
    deg[from[l]]++;
    deg[to[l]]++;
  }
  for (int k = 0; k < ng; ++k) {
    if (gb[k] < 0 || gb[k] >= nb)
      return fail(ACOPF_ERR_INVALID_ARG, "acopf_setup: generator " + std::to_string(k) + " has a bad bus");
    gdeg[gb[k]]++;
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
  for (int k = 0; k < ng; ++k) gens[gfill[gb[k]]++] = k;
  Workspace w = ws_of(g, workspace);
  HIP_TRY(hipMemcpy(w.bus_end_ptr, eptr.data(), (nb + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.bus_end, ends.data(), 2 * (size_t)nl * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.bus_gen_ptr, gptr.data(), (nb + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  if (ng > 0) HIP_TRY(hipMemcpy(w.bus_gen, gens.data(), ng * sizeof(int32_t), hipMemcpyHostToDevice));
  SyncState zero;
  std::memset(&zero, 0, sizeof(zero));
  HIP_TRY(hipMemcpy(w.sync, &zero, sizeof(zero), hipMemcpyHostToDevice));
  return ACOPF_OK;
}

acopf_status acopf_qp_build(const acopf_grid* g, const acopf_iterate* x, double delta, int32_t mode,
                            void* workspace, void* stream) {
  if (!grid_ok(g) || !iterate_ok(x) || !workspace)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_qp_build: null argument");
  if (!(delta > 0.0)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_qp_build: trust radius must be > 0");
  if (mode != ACOPF_HESSIAN_PSD && mode != ACOPF_HESSIAN_RAW)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_qp_build: unknown Hessian mode");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int bs = kDefaultBlock;
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, w);
  hipLaunchKernelGGL(k_build_lines, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, *g, *x, delta, (int)mode, w);
  if (g->n_gen > 0)
    hipLaunchKernelGGL(k_build_gens, dim3(blocks_for(g->n_gen, bs)), dim3(bs), 0, s, *g, *x, delta, w);
  hipLaunchKernelGGL(k_build_buses, dim3(blocks_for(g->n_bus, bs)), dim3(bs), 0, s, *g, *x, w);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

static acopf_status admm_init_impl(const acopf_grid* g, const double* rho_g, const double* rho_l,
                            const double* lam_g, const double* lam_l, bool keep_lam, void* workspace,
                            void* stream) {
  if (!grid_ok(g) || !workspace || !rho_l || (g->n_gen > 0 && !rho_g))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_init: null argument");
  if ((lam_g == nullptr) != (lam_l == nullptr))
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
  copy(w.rho_g, rho_g, G2);
  copy(w.rho_l, rho_l, L8);
  if (keep_lam) {
    // multipliers of the previous solve stay in place (previous-iterate warm start)
  } else if (lam_l) {
    copy(w.lam_g, lam_g, G2);
    copy(w.lam_l, lam_l, L8);
  } else {
    fill(w.lam_g, G2, 0.0);
    fill(w.lam_l, L8, 0.0);
  }
  fill(w.xg, G2, 0.0);
  fill(w.xbar_g, G2, 0.0);
  fill(w.xl, L8, 0.0);
  fill(w.xbar_f, 4LL * g->n_line, 0.0);
  fill(w.dw, g->n_bus, 0.0);
  fill(w.dth, g->n_bus, 0.0);
  fill(w.nu, 2LL * g->n_bus, 0.0);
  fill(w.mu, 2LL * g->n_line, 0.0);
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, w.line_mask,
                     (long long)g->n_line, 0);
  hipLaunchKernelGGL(k_prep_lines, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, w);
  hipLaunchKernelGGL(k_reset_sync, dim3(blocks_for(w.max_partials, 256)), dim3(256), 0, s, w, 0);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_admm_init(const acopf_grid* g, const double* rho_g, const double* rho_l,
                             const double* lam_g, const double* lam_l, void* workspace, void* stream) {
  return admm_init_impl(g, rho_g, rho_l, lam_g, lam_l, false, workspace, stream);
}

acopf_status acopf_admm_solve(const acopf_grid* g, const acopf_admm_params* p, void* workspace,
                              void* stream, acopf_admm_result* result) {
  if (!grid_ok(g) || !p || !workspace) return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: null argument");
  if (p->max_sweeps < 0 || !(p->eps_pri >= 0.0) || !(p->eps_dual >= 0.0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: bad parameters");
  const int bs = p->block_size > 0 ? p->block_size : kDefaultBlock;
  if (bs % 64 != 0 || bs > 256) return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: block_size must be a multiple of 64, <= 256");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  // errors recorded by the QP build and the factorisation
  SyncState st;
  acopf_status rs = read_sync(workspace, g, s, &st);
  if (rs != ACOPF_OK) return rs;
  if (st.numeric_error) return fail(ACOPF_ERR_NUMERIC, "acopf_admm_solve: the QP build met a vanishing elimination pivot or non-finite data");
  if (st.nonconvex) return fail(ACOPF_ERR_NONCONVEX_LINE, "acopf_admm_solve: a line subproblem matrix is not positive definite");
  if (p->max_sweeps == 0) {
    hipLaunchKernelGGL(k_reset_sync, dim3(blocks_for(w.max_partials, 256)), dim3(256), 0, s, w, 0);
    HIP_TRY(hipGetLastError());
    if (result) return acopf_admm_result_get(g, workspace, stream, result);
    return ACOPF_OK;
  }
  if (p->sweep_mode == ACOPF_SWEEP_LAUNCHES) {
    const int nbl = blocks_for(g->n_line, bs), nbb = blocks_for(g->n_bus, bs);
    if (nbb > w.max_partials) return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: too many bus blocks");
    hipLaunchKernelGGL(k_reset_sync, dim3(blocks_for(w.max_partials, 256)), dim3(256), 0, s, w, nbb);
    for (int k = 0; k < p->max_sweeps; ++k) {
      hipLaunchKernelGGL(k_line_phase, dim3(nbl), dim3(bs), 0, s, *g, w);
      hipLaunchKernelGGL(k_bus_phase, dim3(nbb), dim3(bs), 0, s, *g, w);
      hipLaunchKernelGGL(k_finish_phase, dim3(1), dim3(256), 0, s, w, nbb, p->max_sweeps, p->eps_pri, p->eps_dual);
    }
    HIP_TRY(hipGetLastError());
  } else if (p->sweep_mode == ACOPF_SWEEP_PERSISTENT) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int cus = 0, coop = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: device has no cooperative launch");
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_persistent, bs, 0));
    if (per_cu < 1) return fail(ACOPF_ERR_UNSUPPORTED, "acopf_admm_solve: persistent kernel does not fit a CU");
    long long want = std::max(blocks_for(g->n_line, bs), blocks_for(g->n_bus, bs));
    long long nblk = std::min<long long>(want, (long long)per_cu * cus);
    if (p->max_blocks > 0) nblk = std::min<long long>(nblk, p->max_blocks);
    nblk = std::min<long long>(nblk, w.max_partials);
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_reset_sync, dim3(blocks_for(w.max_partials, 256)), dim3(256), 0, s, w, (int)nblk);
    acopf_grid gg = *g;
    int ms = p->max_sweeps;
    double ep = p->eps_pri, ed = p->eps_dual;
    void* args[] = {&gg, &w, &ms, &ep, &ed};
    HIP_TRY(hipLaunchCooperativeKernel((const void*)k_sweep_persistent, dim3((unsigned)nblk), dim3(bs), args, 0, s));
  } else {
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_solve: unknown sweep mode");
  }
  if (result) return acopf_admm_result_get(g, workspace, stream, result);
  return ACOPF_OK;
}

acopf_status acopf_admm_result_get(const acopf_grid* g, void* workspace, void* stream,
                                   acopf_admm_result* result) {
  if (!grid_ok(g) || !workspace || !result)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_result_get: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  SyncState st;
  HIP_TRY(hipMemcpyAsync(&st, w.sync, sizeof(SyncState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  result->sweeps = st.sweeps;
  result->r_norm = st.r_norm;
  result->s_norm = st.s_norm;
  result->infeasible_lines = st.sweeps > 0 ? st.infeasible[(st.sweeps - 1) & 1] : 0;
  result->blocks = st.blocks;
  result->outcome = st.converged ? ACOPF_ADMM_CONVERGED : ACOPF_ADMM_MAX_SWEEPS;
  if (st.barrier_error) return fail(ACOPF_ERR_BARRIER, "acopf_admm_solve: grid barrier timed out");
  return ACOPF_OK;
}

acopf_status acopf_admm_state_get(const acopf_grid* g, void* workspace, const acopf_admm_state* o,
                                  void* stream) {
  if (!grid_ok(g) || !workspace || !o) return fail(ACOPF_ERR_INVALID_ARG, "acopf_admm_state_get: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const size_t D = sizeof(double);
  const size_t G2 = 2 * (size_t)g->n_gen, L8 = 8 * (size_t)g->n_line, L4 = 4 * (size_t)g->n_line;
  auto cp = [&](double* dst, const double* src, size_t n) -> hipError_t {
    if (!dst || n == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, n * D, hipMemcpyDeviceToDevice, s);
  };
  HIP_TRY(cp(o->xg, w.xg, G2));
  HIP_TRY(cp(o->xbar_g, w.xbar_g, G2));
  HIP_TRY(cp(o->lam_g, w.lam_g, G2));
  HIP_TRY(cp(o->rho_g, w.rho_g, G2));
  HIP_TRY(cp(o->xl, w.xl, L8));
  HIP_TRY(cp(o->xbar_f, w.xbar_f, L4));
  HIP_TRY(cp(o->lam_l, w.lam_l, L8));
  HIP_TRY(cp(o->rho_l, w.rho_l, L8));
  HIP_TRY(cp(o->dw, w.dw, g->n_bus));
  HIP_TRY(cp(o->dth, w.dth, g->n_bus));
  HIP_TRY(cp(o->nu, w.nu, 2 * (size_t)g->n_bus));
  HIP_TRY(cp(o->mu, w.mu, 2 * (size_t)g->n_line));
  return ACOPF_OK;
}

acopf_status acopf_step(const acopf_grid* g, const acopf_iterate* x, void* workspace, const acopf_iterate* d,
                        void* stream) {
  if (!grid_ok(g) || !iterate_ok(x) || !iterate_ok(d) || !workspace)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_step: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int bs = kDefaultBlock;
  hipLaunchKernelGGL(k_step_lines, dim3(blocks_for(g->n_line, bs)), dim3(bs), 0, s, *g, *x, w, *d);
  hipLaunchKernelGGL(k_step_nodes, dim3(blocks_for(std::max(g->n_bus, g->n_gen), bs)), dim3(bs), 0, s, *g, w, *d);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_sqp_step(const acopf_grid* g, const acopf_iterate* x, const acopf_iterate* d,
                            const double* rho_g, const double* rho_l, const acopf_sqp_params* p, void* workspace,
                            void* stream, acopf_sqp_state* state) {
  if (!grid_ok(g) || !iterate_ok(x) || !iterate_ok(d) || !p || !workspace || !state)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: null argument");
  if (!(state->delta > 0.0) || !(p->mu > 0.0) || !(p->delta_max > 0.0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_sqp_step: trust radius, penalty and radius cap must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  acopf_status rc = acopf_qp_build(g, x, state->delta, p->hessian_mode, workspace, stream);
  if (rc != ACOPF_OK) return rc;
  rc = admm_init_impl(g, rho_g, rho_l, nullptr, nullptr, p->warm_start != 0, workspace, stream);
  if (rc != ACOPF_OK) return rc;
  // the solve checks the build's error flags first (a synchronising read),
  // so the events bracket the sweep launches only
  SyncState pre;
  rc = read_sync(workspace, g, s, &pre);
  if (rc != ACOPF_OK) return rc;
  EventPair ev;
  HIP_TRY(ev.create());
  HIP_TRY(hipEventRecord(ev.a, s));
  rc = acopf_admm_solve(g, &p->admm, workspace, stream, nullptr);
  if (rc != ACOPF_OK) return rc;
  HIP_TRY(hipEventRecord(ev.b, s));
  rc = acopf_step(g, x, workspace, d, stream);
  if (rc != ACOPF_OK) return rc;
  const int bs = 256;
  const int nb = std::min(blocks_for(std::max(std::max(g->n_line, g->n_bus), g->n_gen), bs), w.max_partials);
  hipLaunchKernelGGL(k_merit, dim3(nb), dim3(bs), 0, s, *g, *x, w, *d);
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, s, w, nb, p->mu, state->delta, p->delta_max, p->grow_ratio);
  hipLaunchKernelGGL(k_apply, dim3(blocks_for(std::max(std::max(g->n_line, g->n_bus), g->n_gen), bs)), dim3(bs), 0, s,
                     *g, *x, *d, w);
  HIP_TRY(hipGetLastError());
  SqpDecision dc;
  HIP_TRY(hipMemcpyAsync(&dc, w.decision, sizeof(dc), hipMemcpyDeviceToHost, s));
  acopf_admm_result ar;
  rc = acopf_admm_result_get(g, workspace, stream, &ar);
  if (rc != ACOPF_OK) return rc;
  state->accepted = dc.accepted;
  state->ared = dc.ared;
  state->pred = dc.pred;
  state->step_inf = dc.step_inf;
  state->delta = dc.delta_out;
  state->objective = dc.accepted ? dc.f_xd : dc.f_x;
  state->merit = dc.accepted ? dc.f_xd + p->mu * dc.h_xd : dc.f_x + p->mu * dc.h_x;
  state->admm_sweeps = ar.sweeps;
  state->admm_r = ar.r_norm;
  state->admm_s = ar.s_norm;
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
  state->admm_ms = ms;
  return ACOPF_OK;
}

acopf_status acopf_residuals(const acopf_grid* g, const acopf_iterate* x, void* workspace, void* stream,
                             acopf_residuals_report* out) {
  if (!grid_ok(g) || !iterate_ok(x) || !workspace || !out)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_residuals: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = ws_of(g, workspace);
  const int bs = 256;
  const int nb = std::min(blocks_for(std::max(std::max(g->n_line, g->n_bus), g->n_gen), bs), w.max_partials);
  hipLaunchKernelGGL(k_residuals, dim3(nb), dim3(bs), 0, s, *g, *x, w);
  hipLaunchKernelGGL(k_residuals_final, dim3(1), dim3(256), 0, s, w, nb);
  HIP_TRY(hipGetLastError());
  ResidualReport r;
  HIP_TRY(hipMemcpyAsync(&r, w.report, sizeof(r), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->balance = r.balance;
  out->c11 = r.c11;
  out->c12 = r.c12;
  out->limit = r.limit;
  out->bounds = r.bounds;
  out->primal = std::max(std::max(std::max(r.balance, r.c11), std::max(r.c12, r.limit)), r.bounds);
  out->dual = r.dual / std::max(1.0, r.gradf);
  return ACOPF_OK;
}

}  // extern "C"
