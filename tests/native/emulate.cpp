// Host build of the library's per-component arithmetic (the device code in
// paper_2310_13143_amd/csrc compiled as plain C++), used by CPU tests to
// check the kernels' arithmetic against the oracle before any GPU run.  The
// loops below stand in for the kernels' thread grids, in component order.
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../paper_2310_13143_amd/csrc/components.h"
#include "../../paper_2310_13143_amd/csrc/launch_order.h"
#include "../../paper_2310_13143_amd/csrc/linfeas.h"

using namespace acopf;

extern "C" {

// Logical block of each of the xcd_grid(bound) workgroups of a launch that
// uses n blocks (out: xcd_grid(bound) entries); returns the workgroup count.
int emu_xcd_blocks(int n, int bound, int* out) {
  const int g = (int)xcd_grid(bound);
  for (int b = 0; b < g; ++b) out[b] = xcd_block(b, n);
  return g;
}

// warm: per-instance starting working sets (NULL = none); mask_out
// (optional): the returned working sets.
void emu_line_qp(int n, const double* P, const double* c, const double* lo, const double* hi,
                 const double* G, const double* h, double* z, double* mu, int* status, const int* warm,
                 int* mask_out) {
  for (int k = 0; k < n; ++k) {
    double Gk[2][4] = {{G[8 * k + 0], G[8 * k + 1], G[8 * k + 2], G[8 * k + 3]},
                       {G[8 * k + 4], G[8 * k + 5], G[8 * k + 6], G[8 * k + 7]}};
    LineQPResult r = solve_line_qp(P + 10 * k, c + 4 * k, lo + 4 * k, hi + 4 * k, Gk, h + 2 * k,
                                   warm ? warm[k] : 0);
    for (int i = 0; i < 4; ++i) z[4 * k + i] = r.z[i];
    mu[2 * k] = r.mu[0];
    mu[2 * k + 1] = r.mu[1];
    status[k] = r.status;
    if (mask_out) mask_out[k] = r.mask;
  }
}

// Limit-row shift of the QP build for n lines (lo, hi (n,4), G (n,2,4), h (n,2)).
void emu_limit_relaxation(int n, const double* lo, const double* hi, const double* G, const double* h,
                          double* out) {
  for (int k = 0; k < n; ++k) {
    const double Gk[2][4] = {{G[8 * k + 0], G[8 * k + 1], G[8 * k + 2], G[8 * k + 3]},
                             {G[8 * k + 4], G[8 * k + 5], G[8 * k + 6], G[8 * k + 7]}};
    limit_relaxation(lo + 4 * k, hi + 4 * k, Gk, h + 2 * k, out + 2 * k);
  }
}

// Slot of coupling k in a line's 8-entry record.
int emu_slot8(int k) { return slot8(k); }

// Neighbouring working sets of the line phase's wave search.
int emu_neighbour_mask(int base, int idx) { return neighbour_mask(base, idx); }

void emu_psd_project(int n, double* m) {
  for (int k = 0; k < n; ++k) {
    double a[4][4];
    std::memcpy(a, m + 16 * k, sizeof(a));
    psd_project4(a);
    std::memcpy(m + 16 * k, a, sizeof(a));
  }
}

// Bus phase used by emu_run: 0 = update_bus per bus, 1 = the per-item
// decomposition of the launch-mode kernel (items of a bus: generators, then
// line ends in CSR order), summed in item order; 2 = the kernel's one-thread
// walk over a bus wider than an item block.
static int g_bus_items = 0;
void emu_set_bus_items(int on) { g_bus_items = on; }

static void bus_by_items(const acopf_grid& g, const Workspace& w, int i, double& r2, double& s2) {
  std::vector<int> codes;
  for (int e = w.bus_gen_ptr[i]; e < w.bus_gen_ptr[i + 1]; ++e) codes.push_back(-(w.bus_gen[e] + 1));
  for (int e = w.bus_end_ptr[i]; e < w.bus_end_ptr[i + 1]; ++e) codes.push_back(w.bus_end[e]);
  const size_t n = codes.size();
  std::vector<double> v(14 * n), a(8 * n);
  double bc[7];
  bus_item_consts(g, w, i, bc);
  for (size_t j = 0; j < n; ++j) bus_item_terms(w, codes[j], &v[14 * j], &a[8 * j]);
  double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0}, out[6];
  for (size_t j = 0; j < n; ++j)
    for (int m = 0; m < 8; ++m) sum[m] += a[8 * j + m];
  bus_item_solve(sum, bc, out);
  w.dw[i] = out[2];
  w.dth[i] = out[3];
  w.nu[i] = out[0];
  w.nu[w.n_bus + i] = out[1];
  for (size_t j = 0; j < n; ++j) bus_item_update(w, codes[j], &v[14 * j], out, r2, s2);
}

// Full solve emulation: setup tables, QP build, init, `sweeps` sweeps, step.
// The workspace is a host buffer of acopf_workspace_bytes-equivalent size.
size_t emu_workspace_bytes(int nb, int nl, int ng) { return layout_workspace(nullptr, nb, nl, ng, 1, nullptr); }

}  // extern "C"

// Workspace of one scenario with the tables of acopf_setup.
static Workspace emu_setup(const acopf_grid* g, void* ws_base) {
  const int nb = g->n_bus, nl = g->n_line, ng = g->n_gen;
  Workspace w;
  layout_workspace(ws_base, nb, nl, ng, 1, &w);
  // one scenario: tables of acopf_setup
  w.scen_bus_off[0] = 0; w.scen_bus_off[1] = nb;
  w.scen_line_off[0] = 0; w.scen_line_off[1] = nl;
  w.scen_gen_off[0] = 0; w.scen_gen_off[1] = ng;
  for (int i = 0; i < nb; ++i) { w.bus_scen[i] = 0; w.bus_flags[i] = (i == g->ref_bus) ? BUS_REF : 0; }
  // incidence tables (same construction as acopf_setup)
  std::vector<int> deg(nb, 0), gdeg(nb, 0);
  for (int l = 0; l < nl; ++l) { deg[g->line_from[l]]++; deg[g->line_to[l]]++; }
  for (int k = 0; k < ng; ++k) gdeg[g->gen_bus[k]]++;
  w.bus_end_ptr[0] = 0;
  w.bus_gen_ptr[0] = 0;
  for (int i = 0; i < nb; ++i) {
    w.bus_end_ptr[i + 1] = w.bus_end_ptr[i] + deg[i];
    w.bus_gen_ptr[i + 1] = w.bus_gen_ptr[i] + gdeg[i];
  }
  std::vector<int> fe(w.bus_end_ptr, w.bus_end_ptr + nb), fg(w.bus_gen_ptr, w.bus_gen_ptr + nb);
  for (int l = 0; l < nl; ++l) {
    w.bus_end[fe[g->line_from[l]]++] = 2 * l;
    w.bus_end[fe[g->line_to[l]]++] = 2 * l + 1;
  }
  for (int k = 0; k < ng; ++k) w.bus_gen[fg[g->gen_bus[k]]++] = k;
  return w;
}

extern "C" {

int emu_run(const acopf_grid* g, const acopf_iterate* x, double delta, int mode, const double* rho_g,
            const double* rho_l, const double* lam_g, const double* lam_l, int sweeps, void* ws_base,
            const acopf_iterate* d, double* rs_out) {
  const int nb = g->n_bus, nl = g->n_line, ng = g->n_gen;
  Workspace w = emu_setup(g, ws_base);
  w.scen[0].delta = delta;
  int bad = 0;
  w.sync->hessian_mode = mode;
  for (int l = 0; l < nl; ++l) bad += build_line(*g, *x, delta, mode, w, l) ? 0 : 1;
  for (int k = 0; k < ng; ++k) build_gen(*g, *x, delta, w, k, mode == kModeRestore);
  for (int i = 0; i < nb; ++i) build_bus(*g, *x, w, i);
  std::memcpy(w.rho_g, rho_g, sizeof(double) * 2 * ng);
  // caller layout [field][line] -> the workspace's line-by-line state
  for (int l = 0; l < nl; ++l)
    for (int k = 0; k < 8; ++k) w.rho_l[lc8(l, k)] = rho_l[k * nl + l];
  if (lam_l) {
    std::memcpy(w.lam_g, lam_g, sizeof(double) * 2 * ng);
    for (int l = 0; l < nl; ++l)
      for (int k = 0; k < 8; ++k) w.lam_l[lc8(l, k)] = lam_l[k * nl + l];
  } else {
    std::memset(w.lam_g, 0, sizeof(double) * 2 * ng);
    std::memset(w.lam_l, 0, sizeof(double) * 8 * nl);
  }
  std::memset(w.xg, 0, sizeof(double) * 2 * ng);
  std::memset(w.xbar_g, 0, sizeof(double) * 2 * ng);
  std::memset(w.xl, 0, sizeof(double) * 8 * nl);
  std::memset(w.xbar_f, 0, sizeof(double) * 4 * nl);
  std::memset(w.xbar_v, 0, sizeof(double) * 4 * nl);
  std::memset(w.dw, 0, sizeof(double) * nb);
  std::memset(w.dth, 0, sizeof(double) * nb);
  std::memset(w.nu, 0, sizeof(double) * 2 * nb);
  std::memset(w.mu, 0, sizeof(double) * 2 * nl);
  std::memset(w.line_mask, 0, sizeof(int32_t) * nl);
  for (int l = 0; l < nl; ++l) bad += prep_line(w, l) ? 0 : 1000;
  int infeasible = 0;
  for (int k = 0; k < sweeps; ++k) {
    infeasible = 0;
    for (int l = 0; l < nl; ++l)
      infeasible += (mode == ACOPF_HESSIAN_RAW_LOCAL ? update_line_local(w, l) : update_line(*g, w, l)) != 0;
    double r2 = 0.0, s2 = 0.0;
    for (int i = 0; i < nb; ++i) {
      if (g_bus_items == 2)
        bus_whole_update(*g, w, i, r2, s2);
      else if (g_bus_items)
        bus_by_items(*g, w, i, r2, s2);
      else
        update_bus(*g, w, i, r2, s2);
    }
    rs_out[2 * k] = r2;
    rs_out[2 * k + 1] = s2;
  }
  if (d) {
    for (int l = 0; l < nl; ++l) step_line(*g, *x, w, *d, l);
    for (int i = 0; i < nb; ++i) { d->w[i] = w.dw[i]; d->th[i] = w.dth[i]; }
    for (int k = 0; k < ng; ++k) { d->pg[k] = w.xg[k]; d->qg[k] = w.xg[ng + k]; }
  }
  return bad * 10000 + infeasible;
}

// Linear feasibility projection (acopf_linfeas) on the host: build, cold
// start with every penalty rho, `sweeps` sweeps, x <- x + d (x modified).
// rs_out: ||r||^2, ||s||^2 per sweep.  Returns the number of line solves
// that did not succeed in the last sweep.
int emu_linfeas_run(const acopf_grid* g, const acopf_iterate* x, double rho, int sweeps, void* ws_base,
                    double* rs_out) {
  const int nb = g->n_bus, nl = g->n_line, ng = g->n_gen;
  Workspace w = emu_setup(g, ws_base);
  w.sync->hessian_mode = kModeLinfeas;
  for (int l = 0; l < nl; ++l) build_line_linfeas(*g, *x, w, l);
  for (int k = 0; k < ng; ++k) build_gen_linfeas(*g, *x, w, k);
  for (int i = 0; i < nb; ++i) build_bus(*g, *x, w, i);
  for (int k = 0; k < 2 * ng; ++k) w.rho_g[k] = rho;
  for (int k = 0; k < 8 * nl; ++k) w.rho_l[k] = rho;
  std::memset(w.lam_g, 0, sizeof(double) * 2 * ng);
  std::memset(w.lam_l, 0, sizeof(double) * 8 * nl);
  std::memset(w.xg, 0, sizeof(double) * 2 * ng);
  std::memset(w.xbar_g, 0, sizeof(double) * 2 * ng);
  std::memset(w.xl, 0, sizeof(double) * 8 * nl);
  std::memset(w.xbar_f, 0, sizeof(double) * 4 * nl);
  std::memset(w.xbar_v, 0, sizeof(double) * 4 * nl);
  std::memset(w.dw, 0, sizeof(double) * nb);
  std::memset(w.dth, 0, sizeof(double) * nb);
  std::memset(w.nu, 0, sizeof(double) * 2 * nb);
  std::memset(w.mu, 0, sizeof(double) * 2 * nl);
  std::memset(w.line_mask, 0, sizeof(int32_t) * nl);
  for (int l = 0; l < nl; ++l) prep_line(w, l);
  int bad = 0;
  for (int k = 0; k < sweeps; ++k) {
    bad = 0;
    for (int l = 0; l < nl; ++l) bad += update_line_linfeas(w, l) != 0;
    double r2 = 0.0, s2 = 0.0;
    for (int i = 0; i < nb; ++i) update_bus(*g, w, i, r2, s2);
    rs_out[2 * k] = r2;
    rs_out[2 * k + 1] = s2;
  }
  for (int k = 0; k < ng; ++k) { x->pg[k] += w.xg[k]; x->qg[k] += w.xg[ng + k]; }
  for (int i = 0; i < nb; ++i) { x->w[i] += w.dw[i]; x->th[i] += w.dth[i]; }
  for (int l = 0; l < nl; ++l) { x->wR[l] += w.mu[l]; x->wI[l] += w.mu[nl + l]; }
  return bad;
}

// Addresses of the ADMM state arrays inside a host workspace, in the order
// xl, lam_l, xbar_f, xg, lam_g, dw, dth, nu (xl, lam_l: 8 slots per line,
// emu_slot8 maps a coupling to its slot; xbar_f: 4 per line).
void emu_state_ptrs(void* base, int nb, int nl, int ng, double** out) {
  Workspace w;
  layout_workspace(base, nb, nl, ng, 1, &w);
  out[0] = w.xl; out[1] = w.lam_l; out[2] = w.xbar_f; out[3] = w.xg;
  out[4] = w.lam_g; out[5] = w.dw; out[6] = w.dth; out[7] = w.nu;
}

// Merit sums of an SQP step (order: f_x, f_xd, quad_gen, h_x, h_xd, m_d,
// quad_line, step max) from a workspace holding the QP of x.
void emu_merit(const acopf_grid* g, const acopf_iterate* x, const acopf_iterate* d, void* base, double* out) {
  Workspace w;
  layout_workspace(base, g->n_bus, g->n_line, g->n_gen, 1, &w);
  for (int k = 0; k < 8; ++k) out[k] = 0.0;
  for (int l = 0; l < g->n_line; ++l) {
    double o[4];
    merit_line(*g, *x, w, *d, l, o);
    out[3] += o[0]; out[4] += o[1]; out[5] += o[2]; out[6] += o[3];
  }
  for (int k = 0; k < g->n_gen; ++k) {
    double o[3];
    merit_gen(*g, *x, *d, k, o);
    out[0] += o[0]; out[1] += o[1]; out[2] += o[2];
    out[7] = fmax(out[7], fmax(fabs(d->pg[k]), fabs(d->qg[k])));
  }
  for (int i = 0; i < g->n_bus; ++i) out[7] = fmax(out[7], fmax(fabs(d->w[i]), fabs(d->th[i])));
}

// Residual maxima (balance, c11, c12, limit, bounds, dual, gradf) at x with
// the workspace's balance multipliers.
void emu_residuals(const acopf_grid* g, const acopf_iterate* x, void* base, double* out) {
  Workspace w;
  layout_workspace(base, g->n_bus, g->n_line, g->n_gen, 1, &w);
  for (int k = 0; k < 7; ++k) out[k] = 0.0;
  for (int l = 0; l < g->n_line; ++l) {
    double pr[5] = {0, 0, 0, 0, 0}, du = 0.0;
    residual_line(*g, *x, w, l, pr, du);
    out[1] = fmax(out[1], pr[1]); out[2] = fmax(out[2], pr[2]); out[3] = fmax(out[3], pr[3]);
    out[5] = fmax(out[5], du);
  }
  for (int i = 0; i < g->n_bus; ++i) {
    double pr[5] = {0, 0, 0, 0, 0}, du = 0.0;
    residual_bus(*g, *x, w, i, pr, du);
    out[0] = fmax(out[0], pr[0]); out[4] = fmax(out[4], pr[4]); out[5] = fmax(out[5], du);
  }
  for (int k = 0; k < g->n_gen; ++k) {
    double b, du, gf;
    residual_gen(*g, *x, w, k, b, du, gf);
    out[4] = fmax(out[4], b); out[5] = fmax(out[5], du); out[6] = fmax(out[6], gf);
  }
}

}  // extern "C"
