"""Writes tests/golden/rgg2000_500sweeps.npz: the oracle's serial ADMM
(Algorithm 2) on the first QP of the 2,000-bus grid, 500 sweeps from the
cold start at delta = 0.05, rho = 2e4, the iterate and multipliers of the
GPU parity test (power-flow start, line multipliers pi of scale 20, seed 2).
Stored: the state after 100 and after 500 sweeps for a seeded sample of 400
lines and every generator and bus, and the residual norms of every sweep.

Calls only the oracle; run from the repository root:
    python tests/golden/make_rgg2000_sweeps.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth.grids import grid_2000  # noqa: E402
from oracle import admm, qp as qpm  # noqa: E402
from tests._util import start_point  # noqa: E402

SWEEPS = (100, 500)
DELTA, RHO = 0.05, 2e4


def main():
    g = grid_2000()
    x, pi = start_point(g, pi_scale=20.0, seed=2)
    Q = qpm.build_qp(g, x, pi, DELTA, "psd")
    rho = admm.Rho.scalar(g, RHO)
    sample = np.sort(np.random.default_rng(2000).choice(g.n_line, 400, replace=False))
    out = {"lines": sample, "delta": DELTA, "rho": RHO, "sweeps": np.array(SWEEPS)}
    st = admm.cold_state(g)
    Qm = admm.line_matrices(Q, rho)
    hist = []
    for k in range(1, SWEEPS[-1] + 1):
        st, r, s, feas = admm.sweep(g, Q, st, rho, Qm)
        assert feas.all()
        hist.append((r, s))
        if k in SWEEPS:
            for name in ("xl", "lam_l", "xbar_f"):
                out[f"{name}_{k}"] = getattr(st, name)[sample]
            for name in ("xg", "lam_g", "xbar_g", "dw", "dth", "nu"):
                out[f"{name}_{k}"] = getattr(st, name)
            print(f"sweep {k}: r = {r:.6e}, s = {s:.6e}", flush=True)
    out["rs"] = np.array(hist)
    np.savez_compressed(os.path.join(ROOT, "tests", "golden", "rgg2000_500sweeps.npz"), **out)


if __name__ == "__main__":
    main()
