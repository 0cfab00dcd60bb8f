#!/usr/bin/env python3
"""Throughput of the MUSTA-FORCE step on one MI355X.

Default workload: 256^3 hot-spot grid (40 seeded Gaussian hot spots on e = 0.1,
v = 0, box [-12.8, 12.8]^3), FP64, p = e/3, MC limiter, k = 3 MUSTA stages, RK2,
dt = 0.03, outflow boundaries.  A "step" is one full Runge-Kutta step (two
stages, each an x, y and z sweep with reconstruction, Hancock half step,
MUSTA-FORCE fluxes, con2prim, flux-difference accumulation, the RK combine and
the speed reduction).  Inputs are resident in HBM before timing starts.

Prints one JSON line.  `roofline` is for the axis-sweep kernel (the only kernel
in the step), from HIP events around every sweep launch on the library's stream.
`cpu_baseline` times the FP64 CPU oracle on the host cores on the first steps of
the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per 3D step + % HBM roofline; batched/learned vs plain"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (FMA = 2 flops)
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector

# Algorithmic operation counts (add, sub, mul, div, sqrt, min/max each 1 flop).
C2P_FLUX = 24   # ideal-EoS con2prim + physical flux along one axis
LIMITER_OPS = {0: 2, 1: 1, 2: 5, 3: 6, 4: 4, 5: 7}


def flops_per_cell_axis(k: int, limiter: int) -> int:
    """Reconstruction + Hancock half step + k-stage MUSTA-FORCE + flux difference, per cell and axis."""
    recon = 4 * (2 + LIMITER_OPS[limiter] + 3)
    hancock = 2 * C2P_FLUX + 4 * 4
    musta = k * (3 * C2P_FLUX + 4 * 12) + (k - 1) * 4 * 6
    return recon + hancock + musta + 4 * 2


def flops_per_cell_stage(k: int, limiter: int) -> int:
    """Three axis sweeps, two L accumulations and the RK combine (12 on average)."""
    return 3 * flops_per_cell_axis(k, limiter) + 8 + 12


def bytes_per_cell_step(rk: int, elem: int) -> int:
    """Algorithmic HBM bytes: RK2 reads U^n, writes U1, reads U1 and U^n, writes U^{n+1} (5 passes of 4 comps)."""
    passes = 5 if rk == 2 else 8
    return passes * 4 * elem


def cpu_baseline(w, U, budget_s: float):
    import oracle
    prob = oracle.Problem.from_workload(w)
    steps, t_total = 0, 0.0
    V = U
    while steps < 20:
        t0 = time.perf_counter()
        V, _ = oracle.step(prob, V, w.dt, 1, steps * w.dt)
        t_total += time.perf_counter() - t0
        steps += 1
        if t_total >= budget_s:
            break
    return {
        "value": w.cells * steps / t_total,
        "unit": "cell-updates/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"first {steps} RK2 step(s) of the same {w.n[0]}x{w.n[1]}x{w.n[2]} workload, FP64 C oracle, "
                  f"OpenMP over grid lines, {t_total:.1f} s",
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis of the hot-spot grid")
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--seg", type=int, nargs=3, default=None, help="cells per thread along x, y, z")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before timing, copy this many MiB device-to-device (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU layout is described in DESIGN.md", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1510_06340_amd import inputs as I
    from paper_1510_06340_amd import mf

    torch.cuda.set_device(0)
    w = I.hotspot_workload(n=args.n)
    U = I.initial_state(w)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    dev = [torch.from_numpy(np.ascontiguousarray(U[c]).ravel()).to(device="cuda", dtype=tdt) for c in range(4)]
    desc = mf.desc_from_workload(w, mf.MF_F64 if args.dtype == "f64" else mf.MF_F32)
    g = mf.Grid([desc], [dev])
    g.set_eos_ideal(w.cs2)
    if args.seg is not None or args.block != 256:
        g.set_tuning(args.seg or (0, 0, 0), args.block)

    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.warmup > 0:
        g.step(w.dt, args.warmup, stats=False)
    torch.cuda.synchronize()
    g.set_profiling(True)
    g.get_profile()  # reset
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    g.step(w.dt, args.steps, stats=False)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    kms, klaunch = g.get_profile()
    g.set_profiling(False)
    st = g.step(w.dt, 1, stats=True)[0]  # one more step for the end-of-run diagnostics
    g.free()

    elem = 8 if args.dtype == "f64" else 4
    cell_updates = w.cells * args.steps
    value = cell_updates / (ms_total / 1e3)
    fl_axis = flops_per_cell_axis(w.k, w.limiter)
    n_launch = sum(klaunch)
    avg_launch_ms = sum(kms) / max(n_launch, 1)
    achieved_tflops = fl_axis * w.cells / (avg_launch_ms / 1e3) / 1e12
    peak = FP64_PEAK_TFLOPS if args.dtype == "f64" else FP32_PEAK_TFLOPS
    hbm_bytes = bytes_per_cell_step(w.rk, elem)
    hbm_gbs = value * hbm_bytes / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"hotspot {w.n[0]}x{w.n[1]}x{w.n[2]} (40 seeded Gaussian hot spots, seed {w.seed}), "
                        f"p=e/3, MC limiter, k={w.k}, RK{w.rk}, dt={w.dt:g}, outflow",
            "cells": w.cells,
            "wall_s": wall,
        },
        "roofline": {
            "kernel": "k_sweep (x, y and z axis sweeps)",
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / peak,
            "traffic": None,
            "flops_per_cell_axis": fl_axis,
            "avg_launch_ms": avg_launch_ms,
            "launches": n_launch,
            "per_axis_ms": [m / max(c, 1) for m, c in zip(kms, klaunch)],
        },
        "hbm_roofline": {
            "algorithmic_bytes_per_cell_step": hbm_bytes,
            "achieved_GBs": hbm_gbs,
            "peak_GBs": HBM_PEAK_GBS,
            "frac": hbm_gbs / HBM_PEAK_GBS,
        },
        "end_state": {"smax": st["smax"], "n_floor": st["n_floor"], "n_bad": st["n_bad"], "E_total": st["totals"][0]},
    }
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(w, U, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
