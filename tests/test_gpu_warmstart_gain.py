"""What the trained warm-start network gains over the plain start.

The line and generator networks are trained on the device, by the
library's own kernels, on ADMM traces of SQP runs over perturbed-load
scenarios of the 14-bus grid; held-out scenarios are then solved by the
batched SQP with the plain start (zero multipliers, then the previous
solve's; scalar penalty) and with the network's per-coupling penalties.
Both must bring every held-out scenario to primal infeasibility <= 1e-4,
and the learned start must need clearly fewer ADMM sweeps on average.

The workload is the 14-bus grid because its SQP converges; the configured
2,000-bus grid's QPs have no feasible point, so their traces carry no
converged multipliers or penalties to learn from."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

RHO, DELTA0, MAX_SWEEPS, EPS = 1e3, 0.05, 20000, 1e-4
TRACE_ITERS, SQP_ITERS = 6, 10


def _batch(seeds):
    from synth.grids import grid_14, perturb_loads, power_flow_start
    from paper_2310_13143_amd.solver import DeviceGrid
    grids = [perturb_loads(grid_14(), int(s)) for s in seeds]
    starts = [power_flow_start(g) for g in grids]
    dg = DeviceGrid(grids, "cuda:0")
    cat = lambda k: np.concatenate([st[k] for st in starts])
    return dg, dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)


def test_learned_penalties_need_fewer_sweeps_than_the_plain_start():
    import torch
    from paper_2310_13143_amd import warmstart as W
    sq = dict(rho=RHO, delta0=DELTA0, max_sweeps=MAX_SWEEPS, eps=EPS)
    print("[gpu] warm-start gain: tracing 96 training scenarios", flush=True)
    dg, x = _batch(50000 + np.arange(96))
    Xl, Tl, Xg, Tg = W.collect(dg, x, TRACE_ITERS, **sq)
    torch.cuda.synchronize()
    print("[gpu] warm-start gain: training", flush=True)
    net = W.WarmStart("cuda:0", seed=7)
    hl = net.line.fit_standardized(Xl, Tl, 1500, lr=3e-3, lr_end=3e-5, log_every=500)
    hg = net.gen.fit_standardized(Xg, Tg, 1500, lr=3e-3, lr_end=3e-5, log_every=500)
    assert hl[-1][1] < hl[0][1] and hg[-1][1] < hg[0][1]
    held = 60000 + np.arange(32)
    print("[gpu] warm-start gain: 32 held-out scenarios, plain start", flush=True)
    dg, x = _batch(held)
    plain = W.run_sqp(dg, x, SQP_ITERS, **sq)
    print("[gpu] warm-start gain: 32 held-out scenarios, learned penalties", flush=True)
    dg, x = _batch(held)
    learned = W.run_sqp(dg, x, SQP_ITERS, **sq, net=net, lam_policy="none", use_rho=True)
    assert (plain["it_hit"] >= 0).all() and (learned["it_hit"] >= 0).all()
    # ADMM sweeps of each scenario up to the SQP iteration that reached 1e-4
    upto = lambda r: np.array([r["sweeps"][:k + 1, s].sum() for s, k in enumerate(r["it_hit"])])
    sp, sl = upto(plain), upto(learned)
    print(f"[gpu] mean sweeps to 1e-4: plain {sp.mean():.0f}, learned {sl.mean():.0f}; "
          f"iterations to 1e-4: plain {plain['it_hit'].mean() + 1:.2f}, learned {learned['it_hit'].mean() + 1:.2f}",
          flush=True)
    assert sl.mean() <= 0.85 * sp.mean()
