"""Learned ADMM warm start: per-component networks trained on the solver's
own traces (an extension of the paper's method, which starts each ADMM
solve from a fixed or the previous point).

Everything numeric runs in the HIP library: features, targets and the
decoding of outputs (acopf_features / acopf_warm_targets /
acopf_warm_decode), the network's forward pass, back-propagation and Adam
(acopf_mlp_*).  This module holds the FP32 parameter vectors and Adam
moments as device tensors and sequences the calls.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import _abi
from ._abi import check


def _f32(t: torch.Tensor, rows: int, name: str) -> torch.Tensor:
    """Check a device FP32 array of `rows` rows with unit column stride."""
    if t.dtype != torch.float32 or t.device.type != "cuda":
        raise TypeError(f"{name}: expected a float32 device tensor, got {t.dtype} on {t.device}")
    if t.dim() == 1:
        if rows != 1 or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous vector")
    elif t.dim() != 2 or t.shape[0] != rows or t.stride(1) != 1:
        raise ValueError(f"{name}: expected shape [{rows}][n] with unit column stride, got {tuple(t.shape)}")
    return t


class MLP:
    """One network: theta (FP32), Adam moments m, v and the step count."""

    def __init__(self, n_in: int, n_out: int, device="cuda:0", seed: int = 0):
        self.lib = _abi.load()
        self.n_in, self.n_out = int(n_in), int(n_out)
        self.count = int(self.lib.acopf_mlp_param_count(self.n_in, self.n_out))
        if self.count == 0:
            raise ValueError("unsupported network size")
        self.device = torch.device(device)
        self.theta = torch.as_tensor(init_params(self.n_in, self.n_out, seed)).to(self.device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.t = 0
        self._scratch = None

    @property
    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, X: torch.Tensor, n: int | None = None) -> torch.Tensor:
        """Outputs [n_out][n] of samples X [n_in][ld] (columns 0..n-1)."""
        _f32(X, self.n_in, "X")
        n = X.shape[1] if n is None else int(n)
        if n > X.shape[1]:
            raise ValueError("n exceeds the sample array")
        Y = torch.empty(self.n_out, max(n, 1), dtype=torch.float32, device=self.device)
        check(self.lib.acopf_mlp_forward(self.theta.data_ptr(), self.n_in, self.n_out, X.data_ptr(), X.stride(0),
                                         n, Y.data_ptr(), Y.stride(0), self.stream))
        return Y[:, :n]

    def gradient(self, X: torch.Tensor, T: torch.Tensor, n: int | None = None):
        """(gradient, loss) of the mean squared error over n samples; the
        loss is a one-element device tensor."""
        _f32(X, self.n_in, "X")
        _f32(T, self.n_out, "T")
        n = X.shape[1] if n is None else int(n)
        if n > X.shape[1] or n > T.shape[1]:
            raise ValueError("n exceeds the sample arrays")
        need = int(self.lib.acopf_mlp_scratch_bytes(self.n_in, self.n_out, n))
        if self._scratch is None or self._scratch.numel() < need:
            self._scratch = torch.empty(need, dtype=torch.uint8, device=self.device)
        grad = torch.empty(self.count, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check(self.lib.acopf_mlp_gradient(self.theta.data_ptr(), self.n_in, self.n_out, X.data_ptr(), X.stride(0),
                                          T.data_ptr(), T.stride(0), n, grad.data_ptr(), loss.data_ptr(),
                                          self._scratch.data_ptr(), self._scratch.numel(), self.stream))
        return grad, loss

    def adam(self, grad: torch.Tensor, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _f32(grad, 1, "grad")
        if grad.numel() != self.count:
            raise ValueError("gradient size differs from the parameter count")
        self.t += 1
        check(self.lib.acopf_mlp_adam(self.theta.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                      grad.data_ptr(), self.count, self.t, float(lr), float(beta1), float(beta2),
                                      float(eps), self.stream))

    def fit_standardized(self, X: torch.Tensor, T: torch.Tensor, steps: int, lr: float = 3e-3,
                         lr_end: float | None = None, log_every: int = 0, out_clip: float = 5.0):
        """Train on standardised copies of X and T (per-row mean and
        deviation of the training set; targets clipped to +-out_clip
        deviations), then fold the two maps into the network so that it takes
        raw features and returns raw outputs.  Returns the loss log."""
        stats = {}
        for name, A, rows in (("in", X, self.n_in), ("out", T, self.n_out)):
            mean = torch.empty(rows, dtype=torch.float64, device=self.device)
            std = torch.empty(rows, dtype=torch.float64, device=self.device)
            check(self.lib.acopf_mlp_feature_stats(A.data_ptr(), rows, A.stride(0), A.shape[1], mean.data_ptr(),
                                                   std.data_ptr(), self.stream))
            stats[name] = (mean, std)
        Xs, Ts = X.clone(), T.clone()
        check(self.lib.acopf_mlp_standardize(Xs.data_ptr(), self.n_in, Xs.stride(0), Xs.shape[1],
                                             stats["in"][0].data_ptr(), stats["in"][1].data_ptr(), 0.0, self.stream))
        check(self.lib.acopf_mlp_standardize(Ts.data_ptr(), self.n_out, Ts.stride(0), Ts.shape[1],
                                             stats["out"][0].data_ptr(), stats["out"][1].data_ptr(), float(out_clip),
                                             self.stream))
        hist = self.fit(Xs, Ts, steps, lr, lr_end, log_every)
        check(self.lib.acopf_mlp_fold(self.theta.data_ptr(), self.n_in, self.n_out, stats["in"][0].data_ptr(),
                                      stats["in"][1].data_ptr(), stats["out"][0].data_ptr(),
                                      stats["out"][1].data_ptr(), self.stream))
        self.stats = stats
        return hist

    def fit(self, X: torch.Tensor, T: torch.Tensor, steps: int, lr: float = 3e-3, lr_end: float | None = None,
            log_every: int = 0):
        """Full-batch Adam for `steps` steps (learning rate decayed
        geometrically to lr_end); returns the loss at every logged step."""
        hist = []
        decay = 1.0 if lr_end is None or steps < 2 else (lr_end / lr) ** (1.0 / (steps - 1))
        for k in range(steps):
            grad, loss = self.gradient(X, T)
            self.adam(grad, lr * decay ** k)
            if log_every and (k % log_every == 0 or k == steps - 1):
                hist.append((k, float(loss.item())))
        return hist


def init_params(n_in: int, n_out: int, seed: int, n_h: int = _abi.MLP_HIDDEN) -> np.ndarray:
    """Seeded initial parameters, uniform +-1/sqrt(fan_in) per layer, in the
    flat order W1, b1, W2, b2, W3, b3."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, shape in ((n_in, (n_h, n_in)), (n_in, (n_h,)), (n_h, (n_h, n_h)), (n_h, (n_h,)),
                          (n_h, (n_out, n_h)), (n_h, (n_out,))):
        b = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, shape).ravel())
    return np.concatenate(parts).astype(np.float32)


class WarmStart:
    """The line and generator networks of the learned start."""

    def __init__(self, device="cuda:0", seed: int = 0):
        self.line = MLP(_abi.LINE_FEATURES, _abi.LINE_OUTPUTS, device, seed)
        self.gen = MLP(_abi.GEN_FEATURES, _abi.GEN_OUTPUTS, device, seed + 1)

    def fit(self, data, steps: int, lr: float = 3e-3, lr_end: float = 3e-5, log_every: int = 0):
        """Train both networks on collected samples (see collect)."""
        Xl, Tl, Xg, Tg = data
        hl = self.line.fit_standardized(Xl, Tl, steps, lr, lr_end, log_every)
        hg = self.gen.fit_standardized(Xg, Tg, steps, lr, lr_end, log_every)
        return hl, hg

    def start(self, dg, x: dict, first: bool, rho0: float, use_lam: bool = True, use_rho: bool = True):
        """(lam_g, lam_l, rho_g, rho_l) for the QP at iterate x of grid dg
        (the workspace holds the plain start's multipliers)."""
        fl, fg = dg.features(x, first)
        yl = self.line.forward(fl, dg.n_line)
        yg = self.gen.forward(fg, dg.n_gen) if dg.n_gen > 0 else fg[:_abi.GEN_OUTPUTS]
        return dg.warm_decode(yl, yg, rho0, rho0, first, use_lam, use_rho)


def collect(dg, x: dict, iters: int, rho: float, delta0: float, max_sweeps: int, eps: float, block_size: int = 64,
            **sqp_kw):
    """Run `iters` batched SQP iterations from x with the plain start (zero,
    then the previous multipliers; scalar rho), tracing every ADMM solve; return the
    samples (line features, line targets, gen features, gen targets), one
    column block per iteration."""
    L, G = dg.n_line, dg.n_gen
    f32 = lambda r, c: torch.empty(r, max(c, 1), dtype=torch.float32, device=dg.device)
    Xl, Tl = f32(_abi.LINE_FEATURES, iters * L), f32(_abi.LINE_OUTPUTS, iters * L)
    Xg, Tg = f32(_abi.GEN_FEATURES, iters * G), f32(_abi.GEN_OUTPUTS, iters * G)
    rho_g, rho_l = dg.rho_scalar(rho)
    dg.set_delta(delta0)
    for it in range(iters):
        dg.features(x, it == 0, (Xl, Xg), (it * L, it * G))
        start = _abi.START_ZERO if it == 0 else _abi.START_PREVIOUS
        dg.sqp_step_batch(x, rho_g, rho_l, warm_start=start, max_sweeps=max_sweeps, eps=eps,
                          block_size=block_size, sync=False, trace=True, **sqp_kw)
        dg.warm_targets((Tl, Tg), (it * L, it * G))
    return Xl, Tl, Xg, Tg


def run_sqp(dg, x: dict, iters: int, rho: float, delta0: float, max_sweeps: int, eps: float,
            net: WarmStart | None = None, lam_policy: str = "first", use_rho: bool = True, block_size: int = 64,
            tol: float = 1e-4, device_stop: bool = False, **sqp_kw):
    """Batched SQP from x for up to `iters` iterations, with the plain start
    (net=None: zero, then the previous multipliers) or the learned start:
    penalties from the network if use_rho, multipliers corrected by the
    network at the first QP (lam_policy "first"), at every QP ("all") or
    never ("none").  Returns per-scenario records: ADMM sweeps per
    iteration, primal infeasibility after each iteration, the iteration and
    wall time at which it first reached tol, and the total wall time.  With
    device_stop, each scenario stops on the device once its primal
    infeasibility is <= tol (its iterate is then frozen) and "t_device" holds
    its stop time read from the device clock (NaN if it did not stop)."""
    if device_stop:
        sqp_kw = dict(sqp_kw, stop=(tol, 1e300, 0.0, 0.0))
    S = dg.n_scen
    rho_g, rho_l = dg.rho_scalar(rho)
    dg.set_delta(delta0)
    sweeps = np.zeros((iters, S), dtype=np.int64)
    primal = np.zeros((iters, S))
    t_hit = np.full(S, np.nan)
    it_hit = np.full(S, -1)
    torch.cuda.synchronize(dg.device)
    t0 = time.perf_counter()
    for it in range(iters):
        if net is None:
            start = _abi.START_ZERO if it == 0 else _abi.START_PREVIOUS
            outs = dg.sqp_step_batch(x, rho_g, rho_l, warm_start=start, max_sweeps=max_sweeps,
                                     eps=eps, block_size=block_size, **sqp_kw)
        else:
            use_lam = lam_policy == "all" or (lam_policy == "first" and it == 0)
            lam_g, lam_l, rg, rl = net.start(dg, x, it == 0, rho, use_lam, use_rho)
            outs = dg.sqp_step_batch(x, rg, rl, warm_start=_abi.START_GIVEN, lam=(lam_g, lam_l),
                                     max_sweeps=max_sweeps, eps=eps, block_size=block_size, **sqp_kw)
        rep = dg.residuals_batch(x)
        now = time.perf_counter() - t0
        for k in range(S):
            sweeps[it, k] = outs[k]["admm_sweeps"]
            primal[it, k] = rep[k]["primal"]
            if it_hit[k] < 0 and rep[k]["primal"] <= tol:
                it_hit[k], t_hit[k] = it, now
    torch.cuda.synchronize(dg.device)
    out = {"sweeps": sweeps, "primal": primal, "it_hit": it_hit, "t_hit": t_hit, "wall": time.perf_counter() - t0}
    if device_stop:
        oc = dg.sqp_outcomes()
        out["t_device"] = np.array([o["seconds"] if o["done"] else np.nan for o in oc])
        out["it_device"] = np.array([o["iterations"] if o["done"] else -1 for o in oc])
    return out
