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


class DeviceGrid:
    """The network arrays of a grid (any object with the attributes of
    ``acopf_grid``) resident on one device, plus its workspace."""

    def __init__(self, grid, device: str = "cuda:0"):
        self.lib = _abi.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the ADMM solver runs on a HIP device only")
        self.n_bus, self.n_line, self.n_gen = int(grid.n_bus), int(grid.n_line), int(grid.n_gen)
        self.ref = int(grid.ref)
        t = {}
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).to(self.device)
        for n in _abi.GRID_BUS_FIELDS + _abi.GRID_LINE_FIELDS + _abi.GRID_GEN_FIELDS:
            t[n] = f64(getattr(grid, n))
        t["line_from"] = i32(grid.f)
        t["line_to"] = i32(grid.t)
        t["gen_bus"] = i32(grid.gbus)
        self.tensors = t
        self.cgrid = Grid(self.n_bus, self.n_line, self.n_gen, self.ref,
                          *[t[n].data_ptr() for n in _abi.GRID_BUS_FIELDS + _abi.GRID_LINE_INT
                            + _abi.GRID_LINE_FIELDS + _abi.GRID_GEN_INT + _abi.GRID_GEN_FIELDS])
        nbytes = self.lib.acopf_workspace_bytes(self.n_bus, self.n_line, self.n_gen)
        if nbytes == 0:
            raise ValueError("bad grid sizes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ws = ctypes.c_void_p(self.workspace.data_ptr())
        check(self.lib.acopf_setup(ctypes.byref(self.cgrid), self.ws, nbytes, self.stream))

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
                   sync: bool = True):
        p = AdmmParams(int(max_sweeps), float(eps_pri), float(eps_dual), int(sweep_mode), int(block_size),
                       int(max_blocks))
        res = AdmmResult()
        check(self.lib.acopf_admm_solve(ctypes.byref(self.cgrid), ctypes.byref(p), self.ws, self.stream,
                                        ctypes.byref(res) if sync else None))
        return self._result_dict(res) if sync else None

    def admm_result(self) -> dict:
        res = AdmmResult()
        check(self.lib.acopf_admm_result_get(ctypes.byref(self.cgrid), self.ws, self.stream, ctypes.byref(res)))
        return self._result_dict(res)

    @staticmethod
    def _result_dict(res: AdmmResult) -> dict:
        return {"sweeps": res.sweeps, "outcome": res.outcome, "r": res.r_norm, "s": res.s_norm,
                "infeasible_lines": res.infeasible_lines, "blocks": res.blocks,
                "converged": res.outcome == _abi.ADMM_CONVERGED}

    def admm_state(self) -> dict:
        """Copy of the ADMM state as device tensors in the line-major layout."""
        G, L, B = self.n_gen, self.n_line, self.n_bus
        sizes = {"xg": 2 * G, "xbar_g": 2 * G, "lam_g": 2 * G, "rho_g": 2 * G, "xl": 8 * L, "xbar_f": 4 * L,
                 "lam_l": 8 * L, "rho_l": 8 * L, "dw": B, "dth": B, "nu": 2 * B, "mu": 2 * L}
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

    def sqp_step(self, x: dict, delta: float, rho_g, rho_l, mu: float = 1e5, delta_max: float = 10.0,
                 grow_ratio: float = 0.75, hessian_mode: int = _abi.HESSIAN_PSD, warm_start: bool = False,
                 max_sweeps: int = 20000, eps: float = 1e-4, sweep_mode: int = _abi.SWEEP_PERSISTENT,
                 block_size: int = 0, max_blocks: int = 0, d: dict | None = None) -> dict:
        """One trust-region SQP iteration on the device; x is updated in place
        when the step is accepted.  Returns the host-side decision record."""
        if d is None:
            d = self.empty_iterate()
        self._d = d
        f64 = lambda a: torch.as_tensor(a, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        self._rho_g, self._rho_l = f64(rho_g), f64(rho_l)
        p = SqpParams(float(mu), float(delta_max), float(grow_ratio), int(hessian_mode), int(bool(warm_start)),
                      AdmmParams(int(max_sweeps), float(eps), float(eps), int(sweep_mode), int(block_size),
                                 int(max_blocks)))
        st = SqpState()
        st.delta = float(delta)
        cx, cd = self.c_iterate(x), self.c_iterate(d)
        check(self.lib.acopf_sqp_step(ctypes.byref(self.cgrid), ctypes.byref(cx), ctypes.byref(cd),
                                      self._rho_g.data_ptr(), self._rho_l.data_ptr(), ctypes.byref(p), self.ws,
                                      self.stream, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in SqpState._fields_}

    def residuals(self, x: dict) -> dict:
        r = ResidualsReport()
        cx = self.c_iterate(x)
        check(self.lib.acopf_residuals(ctypes.byref(self.cgrid), ctypes.byref(cx), self.ws, self.stream,
                                       ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in ResidualsReport._fields_}
