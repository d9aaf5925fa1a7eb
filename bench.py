"""Benchmark of the ADMM QP solve of the SQP method for ACOPF on one MI355X.

A step is one pass of the hot path over the workload's QP: QP build at the
iterate, ADMM start (cold) and factorisation, the persistent sweep kernel
(up to --sweeps sweeps, stop at ||r||, ||s|| <= --eps), and the step /
multiplier recovery.  The metric is ADMM component updates per second,
(|G| + |L| + |B|) x sweeps / time, over the timed steps.

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


def sweep_bytes(n_bus: int, n_line: int, n_gen: int) -> int:
    """Algorithmic bytes one ADMM sweep must move (FP64 values + int32 indices):
    line phase 696 B/line, bus phase 328 B/line (two ends) + 148 B/gen +
    96 B/bus."""
    return 1024 * n_line + 148 * n_gen + 96 * n_bus


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rgg2000", choices=["ring14", "rgg300", "rgg2000", "rgg10000", "rgg70000"])
    ap.add_argument("--sweeps", type=int, default=2000)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--rho", type=float, default=2e4)
    ap.add_argument("--delta", type=float, default=0.05)
    ap.add_argument("--mode", default="persistent", choices=["persistent", "launches"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-sweeps", type=int, default=5, help="oracle sweeps timed for the CPU baseline (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from synth.grids import WORKLOADS, power_flow_start
    from paper_2310_13143_amd.solver import DeviceGrid
    from paper_2310_13143_amd import SWEEP_LAUNCHES, SWEEP_PERSISTENT

    g = WORKLOADS[args.workload]()
    s = power_flow_start(g)
    dev = torch.device("cuda:0")
    dg = DeviceGrid(g, "cuda:0")
    pi = np.zeros((g.n_line, 4))
    x = dg.iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"], pi)
    rho_g, rho_l = dg.rho_scalar(args.rho)
    mode = SWEEP_PERSISTENT if args.mode == "persistent" else SWEEP_LAUNCHES
    stream = torch.cuda.current_stream(dev)

    def one_step(events=None):
        dg.qp_build(x, args.delta)
        dg.admm_init(rho_g, rho_l)
        if events:
            events[0].record(stream)
        dg.admm_solve(args.sweeps, args.eps, args.eps, sweep_mode=mode, block_size=args.block, sync=False)
        if events:
            events[1].record(stream)
        dg.step(x)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    sweeps = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(ev[k])
        sweeps.append(dg.admm_result()["sweeps"])  # synchronises: the step's sweep count
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res = dg.admm_result()
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    comps = g.n_gen + g.n_line + g.n_bus
    total_sweeps = int(sum(sweeps))
    value = comps * total_sweeps / wall
    bsweep = sweep_bytes(g.n_bus, g.n_line, g.n_gen)
    avg_launch_s = float(np.mean(kern_ms)) / 1e3
    avg_sweeps = total_sweeps / args.steps
    achieved = bsweep * avg_sweeps / avg_launch_s / 1e9

    cpu = None
    if args.cpu_sweeps > 0:
        cpu = cpu_baseline(g, s, args)

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
        "config": {"workload": f"{g.name}: {g.n_bus} buses, {g.n_line} branches, {g.n_gen} generators; "
                               f"QP at a power-flow start, rho={args.rho:g}, delta={args.delta:g}, cold start, "
                               f"<= {args.sweeps} sweeps, eps={args.eps:g}, {args.mode} sweep kernel",
                   "sweeps_per_step": avg_sweeps, "components": comps, "couplings": 2 * g.n_gen + 8 * g.n_line,
                   "last_r": res["r"], "last_s": res["s"], "blocks": res["blocks"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_sweep_persistent" if mode == SWEEP_PERSISTENT else "k_line_phase+k_bus_phase",
                     "bytes_per_sweep": bsweep, "avg_launch_ms": avg_launch_s * 1e3,
                     "us_per_sweep": avg_launch_s / avg_sweeps * 1e6},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(g, s, args):
    """The oracle's serial ADMM on the same QP, timed for a few sweeps."""
    import threading
    from oracle import acopf, admm, qp as qpm
    x = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    Q = qpm.build_qp(g, x, np.zeros((g.n_line, 4)), args.delta)
    rho = admm.Rho.scalar(g, args.rho)
    admm.solve(g, Q, rho, 1, 0.0, 0.0)  # warm caches / imports
    t0 = time.perf_counter()
    admm.solve(g, Q, rho, args.cpu_sweeps, 0.0, 0.0)
    dt = time.perf_counter() - t0
    comps = g.n_gen + g.n_line + g.n_bus
    threads = os.environ.get("OMP_NUM_THREADS", "")
    return {"value": comps * args.cpu_sweeps / dt, "unit": "component updates/s",
            "cores": int(threads) if threads.isdigit() else (os.cpu_count() or 1), "kind": "oracle",
            "sample": f"{args.cpu_sweeps} serial sweeps of the oracle ADMM (NumPy FP64) on the same QP, "
                      f"{dt:.2f} s"}


if __name__ == "__main__":
    main()
