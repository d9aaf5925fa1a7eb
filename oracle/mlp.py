"""Learned warm start for the ADMM solve (not in the paper): a small
per-component MLP that predicts, from local data, the correction to the
plain start of a component's coupling multipliers (at the first QP of an
SQP run, where the plain start is zero) and a factor on each coupling's
penalty, trained on traces the method itself produces.  Plain FP64 NumPy
restatement of what the HIP path computes (the network in FP32).

Network: x -> relu(W1 x + b1) -> relu(W2 h1 + b2) -> W3 h2 + b3, loss the
mean squared error over samples and outputs, optimiser Adam (Kingma and Ba,
2015) with bias correction.  Training runs on standardised inputs and
outputs (per-column mean and standard deviation of the training set,
outputs clipped to +-5 deviations); the affine maps are then folded into
the first and last layers, so the trained network takes raw features and
returns raw outputs.

Features (per component, from the grid, the loads, the SQP iterate and the
multipliers of the previous solve):
  line (25): p_d, q_d at both ends; g_ij, b_ij, g_ii, b_ii, g_jj, b_jj
             scaled by 1/100; w_i, w_j, wR, wI; sin of the angle
             difference; s_max_ij; the 8 previous multipliers / 1e3; 1 at
             the first QP of a run, else 0;
  gen (11):  p_d, q_d of its bus; cost2 / 1e4; cost1 / 1e3; p_g, q_g;
             p_max, q_max; the 2 previous multipliers / 1e3; the flag.
Targets: (final multiplier - starting multiplier) / 1e3 of each coupling
(8 per line, 2 per generator), then the log penalty factors.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

LAM_SCALE = 1e3
N_LINE_FEAT = 25
N_GEN_FEAT = 11
STD_FLOOR = 1e-4
OUT_CLIP = 5.0


def line_features(grid, x, lam_prev_l, first) -> np.ndarray:
    """lam_prev_l: (L, 8) multipliers the plain start would use; first: bool."""
    f, t = grid.f, grid.t
    ph = x.th[f] - x.th[t]
    cols = [grid.pd[f], grid.qd[f], grid.pd[t], grid.qd[t],
            grid.gij / 100, grid.bij / 100, grid.gii / 100, grid.bii / 100, grid.gjj / 100, grid.bjj / 100,
            x.w[f], x.w[t], x.wR, x.wI, np.sin(ph), grid.smax_ij]
    cols += [lam_prev_l[:, c] / LAM_SCALE for c in range(8)]
    cols += [np.full(grid.n_line, 1.0 if first else 0.0)]
    return np.stack(cols, 1)


def gen_features(grid, x, lam_prev_g, first) -> np.ndarray:
    b = grid.gbus
    cols = [grid.pd[b], grid.qd[b], grid.cost2 / 1e4, grid.cost1 / 1e3, x.pg, x.qg, grid.pmax, grid.qmax,
            lam_prev_g[:, 0] / LAM_SCALE, lam_prev_g[:, 1] / LAM_SCALE, np.full(grid.n_gen, 1.0 if first else 0.0)]
    return np.stack(cols, 1)


@dataclass
class Params:
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    W3: np.ndarray
    b3: np.ndarray

    def flat(self) -> np.ndarray:
        return np.concatenate([a.ravel() for a in (self.W1, self.b1, self.W2, self.b2, self.W3, self.b3)])

    @staticmethod
    def unflat(v, n_in, n_h, n_out) -> "Params":
        shapes = [(n_h, n_in), (n_h,), (n_h, n_h), (n_h,), (n_out, n_h), (n_out,)]
        out, o = [], 0
        for s in shapes:
            n = int(np.prod(s))
            out.append(np.asarray(v[o:o + n], dtype=np.float64).reshape(s))
            o += n
        return Params(*out)


def n_params(n_in, n_h, n_out) -> int:
    return n_h * n_in + n_h + n_h * n_h + n_h + n_out * n_h + n_out


def forward(p: Params, X: np.ndarray):
    z1 = X @ p.W1.T + p.b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p.W2.T + p.b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p.W3.T + p.b3
    return y, (X, z1, h1, z2, h2)


def loss(p: Params, X, T) -> float:
    y, _ = forward(p, X)
    return float(np.mean((y - T) ** 2))


def gradients(p: Params, X, T) -> Params:
    """Gradient of the mean squared error by back-propagation."""
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n, m = T.shape
    d3 = 2.0 * (y - T) / (n * m)
    gW3 = d3.T @ h2
    gb3 = d3.sum(0)
    d2 = (d3 @ p.W3) * (z2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ p.W2) * (z1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(0)
    return Params(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the flat parameter vector (t counts from 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def column_stats(X):
    """Per-column mean and standard deviation (population) of samples X
    (n, F); deviations below STD_FLOOR are raised to it."""
    X = np.asarray(X, dtype=np.float64)
    mean = X.mean(0)
    std = np.sqrt(np.mean((X - mean) ** 2, 0))
    return mean, np.maximum(std, STD_FLOOR)


def standardize(X, mean, std, clip=0.0):
    """(X - mean) / std per column, clipped to +-clip if clip > 0."""
    Z = (np.asarray(X, dtype=np.float64) - mean) / std
    return np.clip(Z, -clip, clip) if clip > 0 else Z


def fold(p: Params, in_mean, in_std, out_mean, out_std) -> Params:
    """The network x -> out_std * net((x - in_mean) / in_std) + out_mean as
    one network: the input map folded into W1, b1, the output map into W3, b3."""
    W1 = p.W1 / in_std[None, :]
    b1 = p.b1 - W1 @ in_mean
    W3 = p.W3 * out_std[:, None]
    b3 = p.b3 * out_std + out_mean
    return Params(W1, b1, p.W2.copy(), p.b2.copy(), W3, b3)


# ---------------------------------------------------------------------------
# Training targets and the decoding of network outputs into an ADMM start.
#
# Line output row layout: 8 multipliers (coupling order p_ij, q_ij, p_ji,
# q_ji, w_i, th_i, w_j, th_j) divided by LAM_SCALE, then 8 log penalty
# factors; generator rows: 2 multipliers (p, q) / LAM_SCALE, then 2 log
# penalty factors.  The penalty factor of a coupling is the residual-
# balancing ratio over a traced solve, rho* = rho * clip(sqrt((rho sum|r_c|
# + RHO_REG) / (sum|s_c| + RHO_REG)), 0.1, 10), where r_c = x_c - xbar_c and
# s_c = rho (xbar_c^new - xbar_c^old) are the coupling's primal and dual
# residuals of each sweep (Section IV-B5); the factor raises rho where the
# primal residual dominates and lowers it where the dual one does (residual
# balancing, Boyd et al., 2011, Section 3.4.1).  RHO_REG (multiplier units,
# far below the sums of a coupling that moves) makes couplings with
# vanishing sums, such as the fixed reference angle, get factor 1 whatever
# rounding noise their sums hold.

RHO_CLIP = 10.0
RHO_REG = 1e-6


def _xbar_line(grid, st):
    f, t = grid.f, grid.t
    return np.concatenate([st.xbar_f, np.stack([st.dw[f], st.dth[f], st.dw[t], st.dth[t]], 1)], 1)


def trace_sums(grid, rho, start, states):
    """Per-coupling sums of |r_c| and |s_c| over the sweeps of a solve, from
    its start state and the recorded state after every sweep.  Returns
    (sum_r_g (G, 2), sum_s_g (G, 2), sum_r_l (L, 8), sum_s_l (L, 8))."""
    G, L = grid.n_gen, grid.n_line
    rg, sg = np.zeros((G, 2)), np.zeros((G, 2))
    rl, sl = np.zeros((L, 8)), np.zeros((L, 8))
    prev_g, prev_l = start.xbar_g, _xbar_line(grid, start)
    for st in states:
        xb_l = _xbar_line(grid, st)
        rg += np.abs(st.xg - st.xbar_g)
        rl += np.abs(st.xl - xb_l)
        sg += np.abs(rho.g * (st.xbar_g - prev_g))
        sl += np.abs(rho.l * (xb_l - prev_l))
        prev_g, prev_l = st.xbar_g, xb_l
    return rg, sg, rl, sl


def log_rho_factor(rho, sum_r, sum_s):
    """log of clip(sqrt((rho sum|r| + RHO_REG) / (sum|s| + RHO_REG)),
    1/RHO_CLIP, RHO_CLIP)."""
    ratio = (rho * sum_r + RHO_REG) / (sum_s + RHO_REG)
    return np.log(np.clip(np.sqrt(ratio), 1.0 / RHO_CLIP, RHO_CLIP))


def targets(rho, lam_g, lam_l, lam0_g, lam0_l, sums):
    """Training targets of one traced solve that started from (lam0_g,
    lam0_l) and ended at (lam_g, lam_l): (line rows (L, 16), gen rows (G, 4))."""
    rg, sg, rl, sl = sums
    tl = np.concatenate([(lam_l - lam0_l) / LAM_SCALE, log_rho_factor(rho.l, rl, sl)], 1)
    tg = np.concatenate([(lam_g - lam0_g) / LAM_SCALE, log_rho_factor(rho.g, rg, sg)], 1)
    return tl, tg


def decode(out_l, out_g, rho_l0, rho_g0, lam_l_prev, lam_g_prev, use_lam, use_rho):
    """ADMM start from network outputs: multipliers lam_prev + out *
    LAM_SCALE if use_lam (else lam_prev, the plain start), penalties rho0
    exp(out) with out clipped to +-log(RHO_CLIP) if use_rho (else rho0).  A
    non-finite output falls back to the plain start of that coupling.
    Returns (lam_l, lam_g, rho_l, rho_g)."""
    def lam(out, prev):
        v = prev + np.asarray(out, dtype=np.float64) * LAM_SCALE
        return np.where(np.isfinite(v) & bool(use_lam), v, prev)

    def rho(out, r0):
        o = np.asarray(out, dtype=np.float64)
        c = np.clip(o, -np.log(RHO_CLIP), np.log(RHO_CLIP))
        v = r0 * np.exp(c)
        return np.where(np.isfinite(o) & bool(use_rho), v, r0)

    return (lam(out_l[:, :8], lam_l_prev), lam(out_g[:, :2], lam_g_prev),
            rho(out_l[:, 8:], rho_l0), rho(out_g[:, 2:], rho_g0))
