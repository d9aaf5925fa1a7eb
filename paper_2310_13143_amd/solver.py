"""Device-side handle of one grid: argument marshalling for the C ABI.

Every step of the method runs in the HIP library; this module only moves
arrays to the device (torch tensors), fills the ABI structs with their
addresses and the current stream, and copies results back.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import (AdmmParams, AdmmResult, AdmmState, Grid, Iterate, ResidualsReport, SqpParams, SqpState,
                   check)


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _col_ptr(t: torch.Tensor, col: int) -> int:
    """Address of column col of a row-major 2-D tensor."""
    return t.data_ptr() + int(col) * t.element_size()


def _pack(grids):
    """Concatenate the arrays of several grids (a batch of independent
    scenarios) and offset their bus indices; returns (arrays, offsets)."""
    nb = np.cumsum([0] + [int(g.n_bus) for g in grids])
    nl = np.cumsum([0] + [int(g.n_line) for g in grids])
    ng = np.cumsum([0] + [int(g.n_gen) for g in grids])
    arrays = {}
    for n in _abi.GRID_BUS_FIELDS + _abi.GRID_LINE_FIELDS + _abi.GRID_GEN_FIELDS:
        arrays[n] = np.concatenate([np.asarray(getattr(g, n), dtype=np.float64) for g in grids])
    arrays["line_from"] = np.concatenate([np.asarray(g.f) + nb[k] for k, g in enumerate(grids)])
    arrays["line_to"] = np.concatenate([np.asarray(g.t) + nb[k] for k, g in enumerate(grids)])
    arrays["gen_bus"] = np.concatenate([np.asarray(g.gbus) + nb[k] for k, g in enumerate(grids)])
    refs = np.array([int(g.ref) + nb[k] for k, g in enumerate(grids)], dtype=np.int32)
    return arrays, (nb.astype(np.int32), nl.astype(np.int32), ng.astype(np.int32), refs)


def _admm_params(max_sweeps, eps_pri, eps_dual, sweep_mode, block_size, max_blocks, trace, balance,
                 norm_inf=False) -> AdmmParams:
    p = AdmmParams(int(max_sweeps), float(eps_pri), float(eps_dual), int(sweep_mode), int(block_size),
                   int(max_blocks), int(bool(trace)))
    if balance is not None:
        p.balance_every, p.balance_mu, p.balance_tau = int(balance[0]), float(balance[1]), float(balance[2])
    p.norm_inf = int(bool(norm_inf))
    return p


class DeviceGrid:
    """The network arrays of a grid, or of a batch of independent scenario
    grids packed one after another (pass a list), resident on one device,
    plus its workspace.  Grids are objects with the attributes of
    ``acopf_grid`` (n_bus, n_line, n_gen, ref, f, t, gbus and the data)."""

    def __init__(self, grid, device: str = "cuda:0"):
        self.lib = _abi.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the ADMM solver runs on a HIP device only")
        grids = list(grid) if isinstance(grid, (list, tuple)) else [grid]
        self.n_scen = len(grids)
        arrays, (bo, lo, go, refs) = _pack(grids)
        self.offsets = {"bus": bo, "line": lo, "gen": go}
        self.n_bus, self.n_line, self.n_gen = int(bo[-1]), int(lo[-1]), int(go[-1])
        self.ref = int(refs[0])
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).to(self.device)
        t = {n: f64(arrays[n]) for n in _abi.GRID_BUS_FIELDS + _abi.GRID_LINE_FIELDS + _abi.GRID_GEN_FIELDS}
        for n in _abi.GRID_LINE_INT + _abi.GRID_GEN_INT:
            t[n] = i32(arrays[n])
        self.tensors = t
        self.cgrid = Grid(self.n_bus, self.n_line, self.n_gen, self.ref, self.n_scen, 0,
                          *[t[n].data_ptr() for n in _abi.GRID_BUS_FIELDS + _abi.GRID_LINE_INT
                            + _abi.GRID_LINE_FIELDS + _abi.GRID_GEN_INT + _abi.GRID_GEN_FIELDS])
        nbytes = self.lib.acopf_workspace_bytes(self.n_bus, self.n_line, self.n_gen, self.n_scen)
        if nbytes == 0:
            raise ValueError("bad grid sizes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ws = ctypes.c_void_p(self.workspace.data_ptr())
        if self.n_scen == 1:
            check(self.lib.acopf_setup(ctypes.byref(self.cgrid), self.ws, nbytes, self.stream))
        else:
            self._offs = [np.ascontiguousarray(a, dtype=np.int32) for a in (bo, lo, go, refs)]
            check(self.lib.acopf_setup_batch(ctypes.byref(self.cgrid), *[a.ctypes.data for a in self._offs],
                                             self.ws, nbytes, self.stream))

    @property
    def stream(self):
        return ctypes.c_void_p(_stream_handle(self.device))

    # ------------------------------------------------------------ iterates
    def iterate(self, pg, qg, w, th, wR, wI, pi=None) -> dict:
        f64 = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64) if not torch.is_tensor(a) else a,
                                        dtype=torch.float64).to(self.device).contiguous()
        it = {"pg": f64(pg), "qg": f64(qg), "w": f64(w), "th": f64(th), "wR": f64(wR), "wI": f64(wI)}
        if pi is None:
            it["pi"] = torch.zeros(4 * self.n_line, dtype=torch.float64, device=self.device)
        else:
            p = torch.as_tensor(pi, dtype=torch.float64)
            if p.dim() == 2:  # (n_line, 4) -> field-major
                p = p.t()
            it["pi"] = p.reshape(-1).to(self.device).contiguous()
        return it

    def empty_iterate(self) -> dict:
        z = lambda n: torch.zeros(n, dtype=torch.float64, device=self.device)
        return {"pg": z(self.n_gen), "qg": z(self.n_gen), "w": z(self.n_bus), "th": z(self.n_bus),
                "wR": z(self.n_line), "wI": z(self.n_line), "pi": z(4 * self.n_line)}

    @staticmethod
    def c_iterate(it: dict) -> Iterate:
        return Iterate(*[it[n].data_ptr() for n in _abi.ITERATE_FIELDS])

    # ------------------------------------------------------------ ABI calls
    def qp_build(self, x: dict, delta: float, hessian_mode: int = _abi.HESSIAN_PSD):
        cx = self.c_iterate(x)
        check(self.lib.acopf_qp_build(ctypes.byref(self.cgrid), ctypes.byref(cx), float(delta),
                                      int(hessian_mode), self.ws, self.stream))

    def admm_init(self, rho_g, rho_l, lam_g=None, lam_l=None):
        f64 = lambda a: torch.as_tensor(a, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        self._rho_g, self._rho_l = f64(rho_g), f64(rho_l)
        if lam_g is None:
            lg = ll = None
        else:
            self._lam_g, self._lam_l = f64(lam_g), f64(lam_l)
            lg, ll = self._lam_g.data_ptr(), self._lam_l.data_ptr()
        check(self.lib.acopf_admm_init(ctypes.byref(self.cgrid), self._rho_g.data_ptr(),
                                       self._rho_l.data_ptr(), lg, ll, self.ws, self.stream))

    def rho_scalar(self, rho: float):
        return (torch.full((2 * self.n_gen,), float(rho), dtype=torch.float64),
                torch.full((8 * self.n_line,), float(rho), dtype=torch.float64))

    def admm_solve(self, max_sweeps: int, eps_pri: float = 0.0, eps_dual: float = 0.0,
                   sweep_mode: int = _abi.SWEEP_PERSISTENT, block_size: int = 0, max_blocks: int = 0,
                   sync: bool = True, trace: bool = False, balance=None, norm_inf: bool = False):
        """balance = (every, mu, tau): residual balancing of the penalties;
        norm_inf: stop test and reported norms on infinity norms."""
        p = _admm_params(max_sweeps, eps_pri, eps_dual, sweep_mode, block_size, max_blocks, trace, balance,
                         norm_inf)
        res = AdmmResult()
        check(self.lib.acopf_admm_solve(ctypes.byref(self.cgrid), ctypes.byref(p), self.ws, self.stream,
                                        ctypes.byref(res) if sync else None))
        return self._result_dict(res) if sync else None

    def admm_result(self) -> dict:
        res = AdmmResult()
        check(self.lib.acopf_admm_result_get(ctypes.byref(self.cgrid), self.ws, self.stream, ctypes.byref(res)))
        return self._result_dict(res)

    def admm_results(self) -> list:
        """Per-scenario results of the last solve."""
        res = (AdmmResult * self.n_scen)()
        check(self.lib.acopf_admm_result_batch(ctypes.byref(self.cgrid), self.ws, self.stream, res))
        return [self._result_dict(r) for r in res]

    def set_delta(self, delta):
        """Per-scenario trust radii (scalar or one value per scenario)."""
        d = torch.as_tensor(np.broadcast_to(np.asarray(delta, dtype=np.float64), (self.n_scen,)).copy()).to(self.device)
        self._delta = d
        check(self.lib.acopf_set_delta(ctypes.byref(self.cgrid), d.data_ptr(), self.ws, self.stream))

    @staticmethod
    def _result_dict(res: AdmmResult) -> dict:
        return {"sweeps": res.sweeps, "outcome": res.outcome, "r": res.r_norm, "s": res.s_norm,
                "infeasible_lines": res.infeasible_lines, "blocks": res.blocks, "status": res.status,
                "relaxed_lines": res.relaxed_lines,
                "converged": res.outcome == _abi.ADMM_CONVERGED}

    def admm_state(self) -> dict:
        """Copy of the ADMM state as device tensors in the line-major layout."""
        G, L, B = self.n_gen, self.n_line, self.n_bus
        sizes = {"xg": 2 * G, "xbar_g": 2 * G, "lam_g": 2 * G, "rho_g": 2 * G, "xl": 8 * L, "xbar_f": 4 * L,
                 "lam_l": 8 * L, "rho_l": 8 * L, "dw": B, "dth": B, "nu": 2 * B, "mu": 2 * L,
                 "sum_r_g": 2 * G, "sum_s_g": 2 * G, "sum_r_l": 8 * L, "sum_s_l": 8 * L}
        out = {k: torch.empty(n, dtype=torch.float64, device=self.device) for k, n in sizes.items()}
        st = AdmmState(*[out[n].data_ptr() for n in _abi.STATE_FIELDS])
        check(self.lib.acopf_admm_state_get(ctypes.byref(self.cgrid), self.ws, ctypes.byref(st), self.stream))
        return out

    def step(self, x: dict) -> dict:
        """Trial step d (generator side p, q; bus side w, th; eliminated wR, wI)
        and the new multiplier estimates in d['pi']."""
        d = self.empty_iterate()
        cx, cd = self.c_iterate(x), self.c_iterate(d)
        check(self.lib.acopf_step(ctypes.byref(self.cgrid), ctypes.byref(cx), self.ws, ctypes.byref(cd),
                                  self.stream))
        return d

    def _sqp_params(self, mu, delta_max, grow_ratio, hessian_mode, warm_start, admm: AdmmParams, lam, pi_update,
                    soc=False, stop=None, restore=False):
        start = int(warm_start) if not isinstance(warm_start, bool) else int(warm_start)
        p = SqpParams(float(mu), float(delta_max), float(grow_ratio), int(hessian_mode), start, admm)
        p.pi_update = int(pi_update)
        p.soc = int(bool(soc))
        p.restore = int(bool(restore))
        if stop is not None:
            p.stop = 1
            p.tol_primal, p.tol_dual, p.tol_step, p.delta_min = (float(v) for v in stop)
        if start == _abi.START_GIVEN:
            if lam is None:
                raise ValueError("warm_start=START_GIVEN needs lam=(lam_g, lam_l)")
            f64 = lambda a: torch.as_tensor(a, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
            self._lam0 = (f64(lam[0]), f64(lam[1]))
            p.lam_g0, p.lam_l0 = self._lam0[0].data_ptr(), self._lam0[1].data_ptr()
        return p

    def sqp_step(self, x: dict, delta: float, rho_g, rho_l, mu: float = 1e5, delta_max: float = 10.0,
                 grow_ratio: float = 0.75, hessian_mode: int = _abi.HESSIAN_PSD, warm_start=False,
                 max_sweeps: int = 20000, eps: float = 1e-4, sweep_mode: int = _abi.SWEEP_PERSISTENT,
                 block_size: int = 0, max_blocks: int = 0, d: dict | None = None, lam=None,
                 trace: bool = False, pi_update: int = _abi.PI_ALWAYS, soc: bool = False,
                 balance=None, restore: bool = False) -> dict:
        """One trust-region SQP iteration on the device; x is updated in place
        when the step is accepted.  warm_start: False/True (zero / previous
        multipliers) or one of _abi.START_*; lam = (lam_g, lam_l) for
        START_GIVEN; soc: second-order correction of a rejected step;
        restore: a feasibility restoration step instead (accepted iff it
        lowers the constraint violation h; radius and pi unchanged).
        Returns the host-side decision record."""
        if d is None:
            d = self.empty_iterate()
        self._d = d
        f64 = lambda a: torch.as_tensor(a, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        self._rho_g, self._rho_l = f64(rho_g), f64(rho_l)
        p = self._sqp_params(mu, delta_max, grow_ratio, hessian_mode, warm_start,
                             _admm_params(max_sweeps, eps, eps, sweep_mode, block_size, max_blocks, trace, balance),
                             lam, pi_update, soc, restore=restore)
        st = SqpState()
        st.delta = float(delta)
        cx, cd = self.c_iterate(x), self.c_iterate(d)
        check(self.lib.acopf_sqp_step(ctypes.byref(self.cgrid), ctypes.byref(cx), ctypes.byref(cd),
                                      self._rho_g.data_ptr(), self._rho_l.data_ptr(), ctypes.byref(p), self.ws,
                                      self.stream, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in SqpState._fields_}

    def sqp_step_batch(self, x: dict, rho_g, rho_l, mu: float = 1e5, delta_max: float = 10.0,
                       grow_ratio: float = 0.75, hessian_mode: int = _abi.HESSIAN_PSD, warm_start=False,
                       max_sweeps: int = 20000, eps: float = 1e-4, block_size: int = 0, d: dict | None = None,
                       sync: bool = True, lam=None, trace: bool = False, pi_update: int = _abi.PI_ALWAYS,
                       sweep_mode: int = _abi.SWEEP_LAUNCHES, soc: bool = False, balance=None, stop=None):
        """One SQP iteration for every scenario of the batch (radii held on
        the device, see set_delta); per-scenario decisions if sync.  stop =
        (tol_primal, tol_dual, tol_step, delta_min): device-side stop of each
        scenario's run (see sqp_outcomes)."""
        if d is None:
            d = self.empty_iterate()
        self._d = d
        f64 = lambda a: torch.as_tensor(a, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        self._rho_g, self._rho_l = f64(rho_g), f64(rho_l)
        p = self._sqp_params(mu, delta_max, grow_ratio, hessian_mode, warm_start,
                             _admm_params(max_sweeps, eps, eps, sweep_mode, block_size, 0, trace, balance),
                             lam, pi_update, soc, stop)
        sts = (SqpState * self.n_scen)() if sync else None
        cx, cd = self.c_iterate(x), self.c_iterate(d)
        check(self.lib.acopf_sqp_step_batch(ctypes.byref(self.cgrid), ctypes.byref(cx), ctypes.byref(cd),
                                            self._rho_g.data_ptr(), self._rho_l.data_ptr(), ctypes.byref(p),
                                            self.ws, self.stream, sts))
        if not sync:
            return None
        return [{k: getattr(st, k) for k, _ in SqpState._fields_} for st in sts]

    def sqp_outcomes(self) -> list:
        """Per-scenario state of device-stopped runs (done, reason,
        iterations, seconds from set_delta to the stop)."""
        out = (_abi.SqpOutcome * self.n_scen)()
        check(self.lib.acopf_sqp_outcome_batch(ctypes.byref(self.cgrid), self.ws, self.stream, out))
        return [{k: getattr(o, k) for k, _ in _abi.SqpOutcome._fields_} for o in out]

    # ------------------------------------------------------------ learned warm start
    def features(self, x: dict, first: bool, out=None, cols=(0, 0)):
        """Line and generator features at x (FP32, feature-major; the
        workspace's multipliers as the previous ones; first = first QP of a
        run).  With out = (line_x, gen_x) (2-D tensors, row stride = leading
        dimension) they are written from columns cols = (line column, gen
        column); otherwise new tensors are returned."""
        if out is None:
            out = (torch.empty(_abi.LINE_FEATURES, self.n_line, dtype=torch.float32, device=self.device),
                   torch.empty(_abi.GEN_FEATURES, max(self.n_gen, 1), dtype=torch.float32, device=self.device))
        fl, fg = out
        cx = self.c_iterate(x)
        check(self.lib.acopf_features(ctypes.byref(self.cgrid), ctypes.byref(cx), self.ws, int(bool(first)),
                                      _col_ptr(fl, cols[0]), fl.stride(0), _col_ptr(fg, cols[1]), fg.stride(0),
                                      self.stream))
        return fl, fg

    def warm_targets(self, out=None, cols=(0, 0)):
        """Training targets of the last (traced) solve, FP32 feature-major
        (columns as in features)."""
        if out is None:
            out = (torch.empty(_abi.LINE_OUTPUTS, self.n_line, dtype=torch.float32, device=self.device),
                   torch.empty(_abi.GEN_OUTPUTS, max(self.n_gen, 1), dtype=torch.float32, device=self.device))
        tl, tg = out
        check(self.lib.acopf_warm_targets(ctypes.byref(self.cgrid), self.ws, _col_ptr(tl, cols[0]), tl.stride(0),
                                          _col_ptr(tg, cols[1]), tg.stride(0), self.stream))
        return tl, tg

    def warm_decode(self, yl, yg, rho_l0: float, rho_g0: float, first: bool, use_lam: bool = True,
                    use_rho: bool = True):
        """ADMM start (lam_g, lam_l, rho_g, rho_l; FP64, layout of the ADMM
        state) from network outputs yl [16][n_line], yg [4][n_gen]: the plain
        start (the workspace's multipliers, zero if first) corrected by the
        outputs (if use_lam), the base penalties scaled by them (if use_rho)."""
        G, L = self.n_gen, self.n_line
        z = lambda n: torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        lam_g, lam_l, rho_g, rho_l = z(2 * G), z(8 * L), z(2 * G), z(8 * L)
        check(self.lib.acopf_warm_decode(ctypes.byref(self.cgrid), self.ws, yl.data_ptr(), yl.stride(0),
                                         yg.data_ptr(), yg.stride(0), float(rho_l0), float(rho_g0), int(bool(first)),
                                         int(bool(use_lam)), int(bool(use_rho)), lam_l.data_ptr(), lam_g.data_ptr(),
                                         rho_l.data_ptr(), rho_g.data_ptr(), self.stream))
        return lam_g[:2 * G], lam_l, rho_g[:2 * G], rho_l

    def linfeas(self, x: dict, rho: float = 1.0, max_sweeps: int = 20000, eps: float = 1e-8,
                sweep_mode: int = _abi.SWEEP_GRAPH, block_size: int = 0) -> dict:
        """Linear feasibility projection of the iterate x, in place
        (acopf_linfeas); returns the ADMM result of the projection."""
        p = _admm_params(max_sweeps, eps, eps, sweep_mode, block_size, 0, False, None)
        res = AdmmResult()
        cx = self.c_iterate(x)
        check(self.lib.acopf_linfeas(ctypes.byref(self.cgrid), ctypes.byref(cx), float(rho), ctypes.byref(p),
                                     self.ws, self.stream, ctypes.byref(res)))
        return self._result_dict(res)

    def residuals_batch(self, x: dict) -> list:
        r = (ResidualsReport * self.n_scen)()
        cx = self.c_iterate(x)
        check(self.lib.acopf_residuals_batch(ctypes.byref(self.cgrid), ctypes.byref(cx), self.ws, self.stream, r))
        return [{k: getattr(e, k) for k, _ in ResidualsReport._fields_} for e in r]

    def residuals(self, x: dict) -> dict:
        r = ResidualsReport()
        cx = self.c_iterate(x)
        check(self.lib.acopf_residuals(ctypes.byref(self.cgrid), ctypes.byref(cx), self.ws, self.stream,
                                       ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in ResidualsReport._fields_}


_TUNED = {}


def autotune_block(dg: DeviceGrid, x: dict, delta: float = 0.05, rho: float = 2e4, sweeps: int = 128,
                   candidates=(64, 128, 256), sweep_mode: int = _abi.SWEEP_GRAPH, cache: bool = True):
    """Block size of the line phase that runs fastest on this grid or batch
    in the given sweep mode, timed with HIP events over a few sweeps of the
    QP at x (after one untimed pass per candidate); cached per (buses, lines,
    scenarios, mode) for the process.  Returns (block size, {candidate: ms})."""
    key = (dg.n_bus, dg.n_line, dg.n_scen, sweep_mode)
    if cache and key in _TUNED:
        return _TUNED[key]
    stream = torch.cuda.current_stream(dg.device)
    dg.qp_build(x, delta)
    times = {}
    for bs in candidates:
        dg.admm_init(*dg.rho_scalar(rho))
        dg.admm_solve(sweeps, sweep_mode=sweep_mode, block_size=bs, sync=False)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        dg.admm_init(*dg.rho_scalar(rho))
        a.record(stream)
        dg.admm_solve(sweeps, sweep_mode=sweep_mode, block_size=bs, sync=False)
        b.record(stream)
        b.synchronize()
        times[bs] = a.elapsed_time(b)
    best = min(times, key=times.get)
    if cache:
        _TUNED[key] = (best, times)
    return best, times


# Segment schedules: orders of the scenario segments in a packed batch.
# The sweep kernels' blocks follow the packing (each XCD runs a contiguous
# run of them), so the order decides which scenarios share an XCD and how
# evenly the work of mixed sizes spreads.
SCHEDULES = ("given", "largest_first", "interleaved")


def schedule_order(grids, kind: str) -> list:
    """Permutation of the scenarios for a schedule: 'given' (as passed),
    'largest_first' (by line count, stable), 'interleaved' (one scenario of
    each size in turn, largest size first)."""
    n = [g.n_line for g in grids]
    idx = list(range(len(grids)))
    if kind == "given":
        return idx
    if kind == "largest_first":
        return sorted(idx, key=lambda k: -n[k])
    if kind == "interleaved":
        queues = [[k for k in idx if n[k] == c] for c in sorted(set(n), reverse=True)]
        out = []
        while any(queues):
            for q in queues:
                if q:
                    out.append(q.pop(0))
        return out
    raise ValueError(f"unknown schedule {kind!r}")


def autotune_schedule(grids, starts, delta: float = 0.05, rho: float = 2e4, sweeps: int = 128,
                      schedules=SCHEDULES, blocks=(64, 128, 256), sweep_mode: int = _abi.SWEEP_GRAPH,
                      device: str = "cuda:0"):
    """Segment schedule x line block size of a batch that runs fastest: for
    each schedule the batch is packed in that order and its block size tuned
    (autotune_block, timed sweeps of the QP at the given starts).  Returns
    (order, block, {"schedule/block": ms}); a caller packs
    [grids[k] for k in order] and maps per-scenario results back with order."""
    times, best = {}, None
    for kind in schedules:
        order = schedule_order(grids, kind)
        dg = DeviceGrid([grids[k] for k in order], device)
        cat = lambda name: np.concatenate([starts[k][name] for k in order])
        x = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)
        bs, tb = autotune_block(dg, x, delta, rho, sweeps, blocks, sweep_mode, cache=False)
        for b, ms in tb.items():
            times[f"{kind}/{b}"] = ms
        if best is None or tb[bs] < best[2]:
            best = (order, bs, tb[bs])
        del dg, x
    return best[0], best[1], times
