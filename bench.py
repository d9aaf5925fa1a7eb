"""Benchmark of the ADMM QP solve of the SQP method for ACOPF on one MI355X.

A step is one trust-region SQP iteration (Algorithm 1) on the device: QP
build at the iterate, ADMM start and factorisation, the sweep kernels (up to
--sweeps sweeps, stop at ||r||, ||s|| <= --eps unless eps = 0), step and
multiplier recovery, merit test and radius update.  The metric is ADMM
component updates per second, (|G| + |L| + |B|) x sweeps / time, over the
timed steps.

Default workload: the 70,000-bus grid (88,000 branches, 10,000 generators),
each step the SQP iteration at the start point (the iteration-0 QP) with a
fixed 2,000 sweeps and no early stop.  Other workloads (--workload) run
consecutive SQP iterations with the stop test; their SQP primal
infeasibility after each step gives the time to 1e-4.

Prints one JSON line (see the keys below).  --gpus > 1 is not supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Bytes one sweep moves between L2 and memory, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters scaled by a 256 MiB copy (profiles/hbm_traffic_*.md),
# keyed by workload.  A figure holds only for the sweep kernels' sources it
# was measured with (sha256 prefix over SWEEP_SOURCES); otherwise the bench
# reports null.
SWEEP_SOURCES = ("paper_2310_13143_amd/csrc/acopf_admm.hip", "paper_2310_13143_amd/csrc/components.h",
                 "paper_2310_13143_amd/csrc/line_qp.h", "paper_2310_13143_amd/csrc/line_alm.h",
                 "paper_2310_13143_amd/csrc/linfeas.h", "paper_2310_13143_amd/csrc/launch_order.h",
                 "paper_2310_13143_amd/csrc/small_linalg.h",
                 "paper_2310_13143_amd/csrc/workspace.h", "paper_2310_13143_amd/csrc/errors.h",
                 "include/acopf_admm.h")
MEASURED_SWEEP_TRAFFIC = {"rgg70000": ("b9d2cf52492be334", 111921145)}


def sweep_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sweep_traffic(workload: str):
    rec = MEASURED_SWEEP_TRAFFIC.get(workload)
    return rec[1] if rec is not None and rec[0] == sweep_sources_sha() else None


# Per-workload defaults of the options left unset.  rgg70000: the
# iteration-0 QP with a fixed 2,000 sweeps (no early stop), 20 timed repeats
# after 3 warm-ups; the others: consecutive SQP iterations with the stop test.
WORKLOAD_DEFAULTS = {
    "rgg70000": dict(steps=20, warmup=3, eps=0.0, restart=1, cpu_sweeps=1),
    "*": dict(steps=10, warmup=2, eps=1e-4, restart=0, cpu_sweeps=20),
}


def sweep_bytes(n_bus: int, n_line: int, n_gen: int) -> int:
    """Algorithmic bytes one ADMM sweep must move (FP64 values + int32 indices):
    line phase 696 B/line, bus phase 328 B/line (two ends) + 148 B/gen +
    96 B/bus."""
    return 1024 * n_line + 148 * n_gen + 96 * n_bus


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default per workload)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default per workload)")
    ap.add_argument("--workload", default="rgg70000",
                    choices=["ring14", "rgg300", "rgg2000", "rgg10000", "rgg70000", "batch64", "warmstart"])
    ap.add_argument("--sweeps", type=int, default=2000)
    ap.add_argument("--eps", type=float, default=None, help="ADMM stop tolerance (0 = fixed sweep count)")
    ap.add_argument("--restart", type=int, default=None,
                    help="1: every step is the SQP iteration at the start point (iteration-0 QP, cold ADMM)")
    ap.add_argument("--rho", type=float, default=2e4)
    ap.add_argument("--delta", type=float, default=0.05)
    ap.add_argument("--mode", default="graph", choices=["persistent", "launches", "graph"])
    ap.add_argument("--block", type=int, default=None,
                    help="threads per line-phase block (default: 64 for one grid; batch64: tuned, 0 = tune)")
    ap.add_argument("--max-blocks", type=int, default=0, help="persistent grid size cap (0 = fill the device)")
    ap.add_argument("--cpu-sweeps", type=int, default=None,
                    help="oracle sweeps timed for the CPU baseline (0 = skip; default per workload)")
    ap.add_argument("--train-scen", type=int, default=512, help="warmstart: training scenarios")
    ap.add_argument("--test-scen", type=int, default=128, help="warmstart: held-out scenarios")
    ap.add_argument("--val-scen", type=int, default=64, help="warmstart: validation scenarios (policy choice)")
    ap.add_argument("--sqp-iters", type=int, default=15, help="warmstart: SQP iterations per scenario")
    ap.add_argument("--train-steps", type=int, default=3000, help="warmstart: full-batch Adam steps")
    ap.add_argument("--sqp-compare", type=int, default=1,
                    help="1: add the SQP time-to-1e-4 of the learned and the plain start on held-out 14-bus "
                         "scenarios (trained on the device first) to the line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB FP32 tensor three times (memory counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 26, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copied 262144 KiB three times"}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    for k, v in WORKLOAD_DEFAULTS.get(args.workload, WORKLOAD_DEFAULTS["*"]).items():
        if getattr(args, k) is None:
            setattr(args, k, v)
    if args.block is None:
        args.block = 0 if args.workload == "batch64" else 128

    import torch
    from synth.grids import WORKLOADS, power_flow_start
    from paper_2310_13143_amd.solver import DeviceGrid
    from paper_2310_13143_amd import SWEEP_GRAPH, SWEEP_LAUNCHES, SWEEP_PERSISTENT

    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "warmstart":
        return bench_warmstart(args)

    g = WORKLOADS[args.workload]()
    s = power_flow_start(g)
    dev = torch.device("cuda:0")
    dg = DeviceGrid(g, "cuda:0")
    pi = np.zeros((g.n_line, 4))
    x = dg.iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"], pi)
    rho_g, rho_l = dg.rho_scalar(args.rho)
    mode = {"persistent": SWEEP_PERSISTENT, "launches": SWEEP_LAUNCHES, "graph": SWEEP_GRAPH}[args.mode]
    stream = torch.cuda.current_stream(dev)

    state = {"delta": args.delta, "k": 0}
    from paper_2310_13143_amd import _abi
    sqp_kw = dict(mu=1e5, delta_max=10.0, max_sweeps=args.sweeps, eps=args.eps, sweep_mode=mode,
                  block_size=args.block, max_blocks=args.max_blocks, pi_update=_abi.PI_IF_CONVERGED)

    x0 = {k: v.clone() for k, v in x.items()}

    def one_step():
        if args.restart:  # the iteration-0 QP again: start point, cold ADMM
            for k in x:
                x[k].copy_(x0[k])
            state.update(delta=args.delta, k=0)
        out = dg.sqp_step(x, state["delta"], rho_g, rho_l, warm_start=state["k"] > 0, **sqp_kw)
        state["delta"] = out["delta"]
        state["k"] += 1
        return out

    # warm-up on a copy of the start point, then restart from it
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    for k in x:
        x[k].copy_(x0[k])
    state.update(delta=args.delta, k=0)
    # per-launch duration of the sweep kernel: its HIP events bracket each
    # ADMM solve on the library's stream
    sweeps, recs, kern_ms = [], [], []
    t0 = time.perf_counter()
    t_first_1e4 = None
    for k in range(args.steps):
        out = one_step()
        sweeps.append(out["admm_sweeps"])
        kern_ms.append(out["admm_ms"])
        pr = dg.residuals(x)["primal"]
        recs.append({"accepted": out["accepted"], "delta": out["delta"], "sweeps": out["admm_sweeps"],
                     "admm_ms": out["admm_ms"], "primal": pr, "objective": out["objective"]})
        if t_first_1e4 is None and pr <= 1e-4:
            t_first_1e4 = time.perf_counter() - t0
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res = dg.admm_result()
    comps = g.n_gen + g.n_line + g.n_bus
    total_sweeps = int(sum(sweeps))
    value = comps * total_sweeps / wall
    bsweep = sweep_bytes(g.n_bus, g.n_line, g.n_gen)
    avg_launch_s = float(np.mean(kern_ms)) / 1e3
    avg_sweeps = total_sweeps / args.steps
    achieved = bsweep * avg_sweeps / avg_launch_s / 1e9
    pr_final = recs[-1]["primal"] if recs else None

    cpu = None
    if args.cpu_sweeps > 0:
        cpu = cpu_baseline(g, s, args)
    sqp_cmp = None
    if args.sqp_compare:
        progress = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
        sqp_cmp = sqp_learned_vs_plain(96, 32, 1500, 10, 1e3, 0.05, 20000, 1e-4, progress)

    out = {
        "metric": "ADMM component updates/s + SQP time-to-1e-4 residual (learned vs plain), 1 GPU",
        "value": value,
        "unit": "component updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload_text(g, args),
                   "sweeps_per_step": avg_sweeps, "components": comps, "couplings": 2 * g.n_gen + 8 * g.n_line,
                   "last_r": res["r"], "last_s": res["s"], "blocks": res["blocks"]},
        "sqp": {"time_to_1e-4_s": t_first_1e4, "primal_final": pr_final,
                "accepted": int(sum(r["accepted"] for r in recs)),
                "primal": [r["primal"] for r in recs], "sweeps": [r["sweeps"] for r in recs],
                "admm_ms": [r["admm_ms"] for r in recs], "delta": [r["delta"] for r in recs]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": sweep_traffic(args.workload),
                     "kernel": "k_sweep_persistent" if mode == SWEEP_PERSISTENT else "k_line_phase+k_bus_items",
                     "bytes_per_sweep": bsweep, "avg_launch_ms": avg_launch_s * 1e3,
                     "us_per_sweep": avg_launch_s / avg_sweeps * 1e6},
        "cpu_baseline": cpu,
    }
    if sqp_cmp is not None:
        out["sqp_learned_vs_plain"] = sqp_cmp
    print(json.dumps(out), flush=True)


def workload_text(g, args) -> str:
    head = f"{g.name}: {g.n_bus} buses, {g.n_line} branches, {g.n_gen} generators; "
    if args.restart:
        stop = "no early stop" if args.eps == 0 else f"stop at eps={args.eps:g}"
        return (head + f"each step the SQP iteration at the power-flow start (DC angles if it has none): "
                f"iteration-0 QP build, cold ADMM with a fixed {args.sweeps} sweeps ({stop}), step, "
                f"multipliers and merit test; delta0={args.delta:g}, rho={args.rho:g}, FP64, "
                f"{args.mode} sweep kernels")
    return (head + f"{args.steps} SQP iterations from the power-flow start (DC angles if it has "
            f"none), delta0={args.delta:g}, rho={args.rho:g}, <= {args.sweeps} ADMM sweeps "
            f"per QP, eps={args.eps:g}, previous-iterate warm start, pi kept unless the "
            f"solve converged, {args.mode} sweep kernels")


def batch_grids():
    """64 load scenarios (per-bus factor N(1, 0.1) clipped to [0.5, 1.5],
    seeds 64000 + s) over the 300-, 2,000- and 10,000-bus grids, assigned
    round robin (22 / 21 / 21)."""
    from synth.grids import grid_300, grid_2000, grid_10000, perturb_loads
    bases = [grid_300(), grid_2000(), grid_10000()]
    return [perturb_loads(bases[s % 3], 64000 + s) for s in range(64)]


def bench_batch(args):
    """Batched SQP: every step is one SQP iteration of all 64 scenarios in
    shared launches (per-scenario ADMM stop tests, radii and decisions); a
    scenario stops on the device once its primal infeasibility is <= 1e-4
    (its time is then read from the device clock).  The line-phase block
    size is tuned on the batch first (--block 0)."""
    import torch
    from synth.grids import power_flow_start
    from paper_2310_13143_amd.solver import DeviceGrid, autotune_schedule
    from paper_2310_13143_amd._abi import PI_IF_CONVERGED, SWEEP_GRAPH, SWEEP_LAUNCHES
    grids = batch_grids()
    starts = [power_flow_start(g) for g in grids]
    mode = SWEEP_GRAPH if args.mode == "graph" else SWEEP_LAUNCHES
    tuned, schedule = None, "given"
    if args.block == 0:
        # segment schedule (scenario order in the packed batch) x block size
        order, bs, tuned = autotune_schedule(grids, starts, args.delta, args.rho, sweep_mode=mode)
        schedule = min(tuned, key=tuned.get).split("/")[0]
        grids, starts = [grids[k] for k in order], [starts[k] for k in order]
    else:
        bs = args.block
    dg = DeviceGrid(grids, "cuda:0")
    cat = lambda k: np.concatenate([st[k] for st in starts])
    x = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)
    x0 = {k: v.clone() for k, v in x.items()}
    rho_g, rho_l = dg.rho_scalar(args.rho)

    def run(steps):
        for k in x:
            x[k].copy_(x0[k])
        dg.set_delta(args.delta)
        outs = []
        for it in range(steps):
            outs.append(dg.sqp_step_batch(x, rho_g, rho_l, warm_start=it > 0, max_sweeps=args.sweeps,
                                          eps=args.eps, block_size=bs, pi_update=PI_IF_CONVERGED,
                                          sweep_mode=mode, stop=(1e-4, 1e300, 0.0, 0.0)))
        return outs

    run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = run(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    oc = dg.sqp_outcomes()
    comps = np.array([g.n_gen + g.n_line + g.n_bus for g in grids])
    sweeps = np.array([[o[k]["admm_sweeps"] for k in range(len(grids))] for o in outs])  # (steps, scen)
    admm_ms = np.array([o[0]["admm_ms"] for o in outs])
    per_sweep_ms = admm_ms / np.maximum(sweeps.max(axis=1), 1)
    value = float((sweeps * comps[None, :]).sum()) / wall
    bsweep = sum(sweep_bytes(g.n_bus, g.n_line, g.n_gen) for g in grids)
    achieved = bsweep / (float(per_sweep_ms.mean()) / 1e3) / 1e9
    res = dg.residuals_batch(x)
    t_stop = np.array([o["seconds"] for o in oc if o["done"]])
    out = {
        "metric": "batched ADMM component updates/s (64 scenarios per launch), 1 GPU",
        "value": value, "unit": "component updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch64: 64 load scenarios (N(1,0.1) per-bus factors) over the 300-, 2,000- and "
                               "10,000-bus grids (22/21/21), shared launches, per-scenario stop tests and SQP "
                               f"decisions; <= {args.sweeps} sweeps per QP, eps={args.eps:g}, block {bs}, "
                               f"scenario order {schedule}" + (" (tuned)" if tuned else ""),
                   "buses": dg.n_bus, "lines": dg.n_line, "generators": dg.n_gen},
        "batch": {"scenarios_per_s": len(grids) * args.steps / wall,
                  "stopped_at_1e-4": int(len(t_stop)),
                  "p50_stop_s": float(np.median(t_stop)) if len(t_stop) else None,
                  "p99_stop_s": float(np.percentile(t_stop, 99)) if len(t_stop) else None,
                  "run_s": wall,
                  "accepted": int(sum(o[k]["accepted"] for o in outs for k in range(len(grids)))),
                  "primal_max": float(max(r["primal"] for r in res)), "primal_min": float(min(r["primal"] for r in res)),
                  "block": bs, "schedule": schedule, "tuning_ms": tuned},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": sweep_traffic(args.workload),
                     "kernel": "k_line_phase+k_bus_items",
                     "bytes_per_sweep": bsweep, "us_per_sweep": float(per_sweep_ms.mean()) * 1e3},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def ring14_scenarios(seeds):
    from synth.grids import grid_14, perturb_loads, power_flow_start
    grids = [perturb_loads(grid_14(), int(s)) for s in seeds]
    return grids, [power_flow_start(g) for g in grids]


def sqp_learned_vs_plain(n_train: int, n_test: int, train_steps: int, sqp_iters: int, rho: float, delta: float,
                         sweeps: int, eps: float, progress=None) -> dict:
    """SQP time-to-1e-4 with the learned and the plain ADMM start on the same
    device: trace the plain batched SQP on n_train perturbed-load scenarios
    of the 14-bus grid, train the line and generator networks on the device,
    then run n_test held-out scenarios as one batch with each start; every
    scenario stops on the device once its primal infeasibility is <= 1e-4,
    and its time is read from the device clock."""
    import torch
    from paper_2310_13143_amd.solver import DeviceGrid
    from paper_2310_13143_amd import warmstart as W

    def device_batch(seeds):
        grids, starts = ring14_scenarios(seeds)
        dg = DeviceGrid(grids, "cuda:0")
        cat = lambda k: np.concatenate([st[k] for st in starts])
        return dg, dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)

    sq = dict(rho=rho, delta0=delta, max_sweeps=sweeps, eps=eps)
    t0 = time.perf_counter()
    dg, x = device_batch(50000 + np.arange(n_train))
    Xl, Tl, Xg, Tg = W.collect(dg, x, min(sqp_iters, 6), **sq)
    torch.cuda.synchronize()
    t_trace = time.perf_counter() - t0
    if progress:
        progress(f"traced {n_train} training scenarios")
    net = W.WarmStart("cuda:0", seed=7)
    net.line.fit_standardized(Xl, Tl, train_steps, lr=3e-3, lr_end=3e-5)
    net.gen.fit_standardized(Xg, Tg, train_steps, lr=3e-3, lr_end=3e-5)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0 - t_trace
    if progress:
        progress("trained the networks")
    held = 60000 + np.arange(n_test)
    out = {"workload": f"ring14 (14 buses, 20 branches, 5 generators) with per-bus load factors N(1,0.1): "
                       f"{n_train} training and {n_test} held-out scenarios; batched SQP of the held-out "
                       f"scenarios, <= {sqp_iters} iterations, <= {sweeps} ADMM sweeps per QP, eps={eps:g}, "
                       f"rho={rho:g}, delta0={delta:g}; a scenario stops on the device at primal "
                       "infeasibility <= 1e-4 and its time is read from the device clock",
           "trace_s": t_trace, "train_s": t_train}
    for name, kw in (("plain", dict(net=None)), ("learned", dict(net=net, lam_policy="none", use_rho=True))):
        for rep in range(2):  # the first pass warms up the launches
            dg, x = device_batch(held)
            r = W.run_sqp(dg, x, sqp_iters, **sq, **kw, device_stop=True)
        t = r["t_device"]
        hit = np.isfinite(t)
        upto = [r["sweeps"][:k, s].sum() for s, k in enumerate(r["it_device"]) if k > 0]
        out[name] = {"solved": int(hit.sum()),
                     "time_to_1e-4_s": {"p50": float(np.median(t[hit])) if hit.any() else None,
                                        "p99": float(np.percentile(t[hit], 99)) if hit.any() else None,
                                        "max": float(t[hit].max()) if hit.any() else None},
                     "iterations_mean": float(r["it_device"][hit].mean()) if hit.any() else None,
                     "sweeps_to_1e-4_mean": float(np.mean(upto)) if upto else None,
                     "wall_s": r["wall"]}
        if progress:
            progress(f"{n_test} held-out scenarios with the {name} start")
    return out


def bench_warmstart(args):
    """Learned warm start: trace the plain batched SQP on the training
    scenarios, train the line and generator networks on the device, choose
    the start policy (which of multipliers / penalties come from the
    network) on validation scenarios, then solve the held-out scenarios
    with the plain and every learned start.  The value is held-out scenarios
    solved to primal <= 1e-4 per second with the chosen policy; the roofline
    is the network's training kernel."""
    import torch
    from paper_2310_13143_amd.solver import DeviceGrid
    from paper_2310_13143_amd import warmstart as W

    def device_batch(seeds):
        grids, starts = ring14_scenarios(seeds)
        dg = DeviceGrid(grids, "cuda:0")
        cat = lambda k: np.concatenate([st[k] for st in starts])
        x = dg.iterate(cat("pg"), cat("qg"), cat("w"), cat("th"), cat("wR"), cat("wI"), None)
        return dg, x

    sq = dict(rho=args.rho, delta0=args.delta, max_sweeps=args.sweeps, eps=args.eps)
    t0 = time.perf_counter()
    dg, x = device_batch(50000 + np.arange(args.train_scen))
    Xl, Tl, Xg, Tg = W.collect(dg, x, args.sqp_iters, **sq)
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    progress = lambda msg: print(f"[warmstart] {msg} ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    progress(f"traced {args.train_scen} training scenarios")
    net = W.WarmStart("cuda:0", seed=7)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    log = max(1, args.train_steps // 10)
    ev[0].record()
    hl = net.line.fit_standardized(Xl, Tl, args.train_steps, lr=3e-3, lr_end=3e-5, log_every=log)
    ev[1].record()
    hg = net.gen.fit_standardized(Xg, Tg, args.train_steps, lr=3e-3, lr_end=3e-5, log_every=log)
    ev[2].record()
    torch.cuda.synchronize()
    ms_line = ev[0].elapsed_time(ev[1])
    ms_gen = ev[1].elapsed_time(ev[2])
    progress("trained the line and generator networks")

    variants = (("plain", dict(net=None)),
                ("learned_lam_first_rho", dict(net=net, lam_policy="first", use_rho=True)),
                ("learned_lam_first", dict(net=net, lam_policy="first", use_rho=False)),
                ("learned_rho", dict(net=net, lam_policy="none", use_rho=True)),
                ("learned_lam_all_rho", dict(net=net, lam_policy="all", use_rho=True)))

    def evaluate(seeds):
        runs = {}
        for name, kw in variants:
            for rep in range(2):  # the first pass warms up the launches
                dg, x = device_batch(seeds)
                r = W.run_sqp(dg, x, args.sqp_iters, **sq, **kw)
            runs[name] = r
            progress(f"{len(seeds)} scenarios with the {name} start")
        return runs

    # the policy is chosen on validation scenarios, then measured on held-out ones
    val = evaluate(55000 + np.arange(args.val_scen))
    choice = min((k for k, _ in variants if k != "plain"), key=lambda k: float(val[k]["sweeps"].sum(0).mean()))
    runs = evaluate(60000 + np.arange(args.test_scen))

    def summary(r):
        hit = r["it_hit"] >= 0
        return {"solved": int(hit.sum()), "sweeps_total_mean": float(r["sweeps"].sum(0).mean()),
                "sweeps_first_qp_mean": float(r["sweeps"][0].mean()),
                "iters_to_1e-4_mean": float(r["it_hit"][hit].mean() + 1) if hit.any() else None,
                "time_to_1e-4_s_max": float(np.nanmax(r["t_hit"])) if hit.any() else None,
                "wall_s": r["wall"]}

    res = {k: summary(v) for k, v in runs.items()}
    best = runs[choice]
    t_all = float(np.nanmax(best["t_hit"])) if (best["it_hit"] >= 0).all() else best["wall"]
    n_line_samples, n_gen_samples = Xl.shape[1], Xg.shape[1]
    # dominant network kernel: the line network's gradient over the training
    # set (k_mlp<true> and its fixed-order reduction), timed on its stream
    reps = 50
    net.line.gradient(Xl, Tl)
    ev[2].record()
    for _ in range(reps):
        net.line.gradient(Xl, Tl)
    ev[3].record()
    torch.cuda.synchronize()
    ms_grad = ev[2].elapsed_time(ev[3]) / reps
    n_in, n_out, H = 25, 16, 64
    flop_grad = 2 * (2 * n_in * H + 3 * H * H + 3 * H * n_out) * n_line_samples  # forward + back-propagation
    tflops = flop_grad / (ms_grad / 1e3) / 1e12
    out = {
        "metric": "held-out ACOPF scenarios solved to primal <= 1e-4 per second, learned ADMM warm start, 1 GPU",
        "value": args.test_scen / t_all, "unit": "scenarios/s", "n_gpus": 1, "steps": args.sqp_iters,
        "warmup": 1, "ms_per_step": t_all / args.sqp_iters * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (network f32)", "data": "synthetic",
        "config": {"workload": f"warmstart: ring14 with per-bus load factors N(1,0.1); {args.train_scen} training "
                               f"and {args.test_scen} held-out scenarios, each a batch in one workspace; "
                               f"{args.sqp_iters} SQP iterations, <= {args.sweeps} sweeps per QP, eps={args.eps:g}, "
                               f"delta0={args.delta:g}, rho={args.rho:g}; networks 25-64-64-16 (lines) and "
                               f"11-64-64-4 (generators), {args.train_steps} full-batch Adam steps on "
                               "standardised data; start policy chosen on "
                               f"{args.val_scen} validation scenarios"},
        "warmstart": {"policy": choice, "validation": {k: summary(v) for k, v in val.items()},
                      "collect_s": t_collect, "line_samples": n_line_samples, "gen_samples": n_gen_samples,
                      "train_ms_line": ms_line, "train_ms_gen": ms_gen, "loss_line": hl, "loss_gen": hg,
                      "results": res},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": 157.3, "unit": "TFLOP/s", "frac": tflops / 157.3,
                     "traffic": None, "kernel": "k_mlp<true> + k_mlp_reduce (line network gradient, FP32)",
                     "flop_per_launch": flop_grad, "ms_per_launch": ms_grad},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


CPU_SNIPPET = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
from synth.grids import WORKLOADS, power_flow_start
from oracle import acopf, admm, qp as qpm
g = WORKLOADS[sys.argv[2]]()
s = power_flow_start(g)
x = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
Q = qpm.build_qp(g, x, np.zeros((g.n_line, 4)), float(sys.argv[3]))
rho = admm.Rho.scalar(g, float(sys.argv[4]))
n = int(sys.argv[5])
frac = float(sys.argv[6])
if frac >= 1.0:
    admm.solve(g, Q, rho, 1, 0.0, 0.0)
    t0 = time.perf_counter()
    admm.solve(g, Q, rho, n, 0.0, 0.0)
    print(json.dumps({"seconds_per_sweep": (time.perf_counter() - t0) / n, "lines": g.n_line}))
else:
    # the first sweep of the cold solve: generator and bus updates over the
    # whole grid, the line update (the oracle's exact line QPs) on a seeded
    # sample of the lines, scaled to all lines
    from dataclasses import replace
    st = admm.cold_state(g)
    t0 = time.perf_counter()
    xg = admm.gen_update(Q, st, rho)
    t_gen = time.perf_counter() - t0
    sel = np.sort(np.random.default_rng(12345).choice(g.n_line, int(round(frac * g.n_line)), replace=False))
    gs = replace(g, f=g.f[sel], t=g.t[sel])
    Ls = replace(Q.line, **{k: getattr(Q.line, k)[sel] for k in Q.line.__dataclass_fields__})
    Qs = replace(Q, line=Ls)
    rs = admm.Rho(rho.g, rho.l[sel])
    ss = replace(st, lam_l=st.lam_l[sel], xbar_f=st.xbar_f[sel])
    t0 = time.perf_counter()
    admm.line_update(gs, Qs, ss, rs)
    t_line = (time.perf_counter() - t0) * g.n_line / sel.size
    xl = np.zeros((g.n_line, 8))
    t0 = time.perf_counter()
    admm.bus_update(g, Q, xg, xl, st, rho)
    t_bus = time.perf_counter() - t0
    print(json.dumps({"seconds_per_sweep": t_gen + t_line + t_bus, "lines": int(sel.size),
                      "t_gen": t_gen, "t_line": t_line, "t_bus": t_bus}))
"""

# grids with more lines than this time a sample of the line updates
CPU_SAMPLE_LINES = 20000


def cpu_baseline(g, s, args):
    """The oracle's serial ADMM (NumPy FP64) on the first QP of the same
    workload, in a child process pinned to one BLAS/OpenMP thread: whole
    sweeps on small grids; on large ones the first sweep with the line
    update timed on a seeded 10% sample of the lines and scaled."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    frac = 1.0 if g.n_line <= CPU_SAMPLE_LINES else 0.1
    p = subprocess.run([sys.executable, "-c", CPU_SNIPPET, ROOT, args.workload, str(args.delta), str(args.rho),
                        str(args.cpu_sweeps), str(frac)], env=env, capture_output=True, text=True, check=True)
    r = json.loads(p.stdout.strip().splitlines()[-1])
    dt = r["seconds_per_sweep"]
    comps = g.n_gen + g.n_line + g.n_bus
    if frac >= 1.0:
        sample = (f"{args.cpu_sweeps} serial sweeps of the oracle ADMM on the first QP of the workload "
                  f"({dt * args.cpu_sweeps:.2f} s, one thread)")
    else:
        sample = (f"the first sweep of the oracle ADMM on the first QP of the workload: generator and bus "
                  f"updates over the whole grid, the line update on a seeded sample of {r['lines']} of "
                  f"{g.n_line} lines scaled to all ({r['t_line'] * frac:.1f} s measured), one thread; "
                  f"extrapolated {dt:.1f} s per sweep")
    return {"value": comps / dt, "unit": "component updates/s", "cores": 1, "kind": "oracle", "sample": sample}


if __name__ == "__main__":
    main()
