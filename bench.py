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

# HBM bytes per axis-sweep launch (average of x, y, z) of the 256^3 FP64 hot-spot
# configuration with the default launch shapes, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a 1 GiB device copy (FETCH x 2, WRITE x 1); see
# profiles/k_sweep_hotspot256_fp64.md.  Other configurations report null.
TRAFFIC_HOTSPOT256_F64 = 1.585e9

# Algorithmic operation counts (add, sub, mul, div, sqrt, min/max each 1 flop).
C2P_FLUX = 22   # ideal-EoS con2prim + physical flux along one axis (energy flux = M_d)
LIMITER_OPS = {0: 2, 1: 1, 2: 5, 3: 5, 4: 4, 5: 7}   # MC computes phi / 2 directly (below)


def flops_per_cell_axis(k: int, limiter: int) -> int:
    """Reconstruction + Hancock half step + k-stage MUSTA-FORCE + flux difference, per cell and axis."""
    # 2 differences, the limiter, phi / 2 (folded into MC's terms) and the two face values
    recon = 4 * (2 + LIMITER_OPS[limiter] + (0 if limiter == 3 else 1) + 2)
    hancock = 2 * C2P_FLUX + 4 * 4
    # per stage: Richtmyer state (5 per component) and F_lw + F_lf (6), then the predictor (6)
    musta = k * (3 * C2P_FLUX + 4 * 11) + (k - 1) * 4 * 6
    return recon + hancock + musta + 4 * 2


def flops_per_cell_stage(k: int, limiter: int) -> int:
    """Three axis sweeps, two L accumulations and the RK combine (12 on average)."""
    return 3 * flops_per_cell_axis(k, limiter) + 8 + 12


def bytes_per_cell_step(rk: int, elem: int) -> int:
    """Algorithmic HBM bytes: RK2 reads U^n, writes U1, reads U1 and U^n, writes U^{n+1} (5 passes of 4 comps)."""
    passes = 5 if rk == 2 else 8
    return passes * 4 * elem


def cpu_baseline(w, U, budget_s: float, table=None):
    import oracle
    prob = oracle.Problem.from_workload(w, table=table)
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


def upload(U, tdt):
    import numpy as np
    import torch
    return [torch.from_numpy(np.ascontiguousarray(U[c]).ravel()).to(device="cuda", dtype=tdt) for c in range(4)]


def run_single(args, w, U, table=None, jet_x0=None):
    """One grid through mf_step; returns (ms_total, per-axis kernel ms and launches, end stats)."""
    import torch
    from paper_1510_06340_amd import mf
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    dev = upload(U, tdt)
    flags = mf.MF_FLAG_UNSPLIT_HANCOCK if args.unsplit_hancock else 0
    g = mf.Grid([mf.desc_from_workload(w, mf.MF_F64 if args.dtype == "f64" else mf.MF_F32, flags)], [dev])
    if table is None:
        g.set_eos_ideal(w.cs2)
    else:
        g.set_eos_table(*table)
    if jet_x0 is not None:
        g.set_jet(0, jet_x0, w.jet["v"], w.jet["dedx"], w.jet["sigma"])
    if args.seg is not None or args.block != 256:
        g.set_tuning(args.seg or (0, 0, 0), args.block)
    calibration_copy(args)
    if args.warmup > 0:
        g.step(w.dt, args.warmup, stats=False)
    torch.cuda.synchronize()
    g.set_profiling(True)
    g.get_profile()  # reset
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    g.step(w.dt, args.steps, stats=False)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    kms, klaunch = g.get_profile()
    g.set_profiling(False)
    st = g.step(w.dt, 1, stats=True)[0]  # one more step for the end-of-run diagnostics
    g.free()
    return ms_total, kms, klaunch, st


def run_events(args, ws, Us, batched, table=None, seed_net=None):
    """Many events: one batched handle (mf_batch_step) or one mf_step call per event in turn."""
    import torch
    from paper_1510_06340_amd import mf
    devs = [upload(U, torch.float64) for U in Us]
    g = None
    if batched:
        g = mf.Grid([mf.desc_from_workload(w) for w in ws], devs)
        if table is None:
            g.set_eos_ideal()
        else:
            g.set_eos_table(*table, surrogate=seed_net)
    dts = [w.dt for w in ws]
    per = []
    if not batched:
        for w, d in zip(ws, devs):
            h = mf.Grid([mf.desc_from_workload(w)], [d])
            if table is None:
                h.set_eos_ideal()
            else:
                h.set_eos_table(*table)
            per.append(h)

    def advance(n):
        if batched:
            g.batch_step(dts, n, stats=False)
        else:
            for h, dt in zip(per, dts):
                h.step(dt, n, stats=False)

    advance(max(args.warmup, 1))  # includes the autotuner and graph capture for the batched form
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    advance(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = g.batch_step(dts, 1) if batched else [h.step(dt, 1)[0] for h, dt in zip(per, dts)]
    for h in per:
        h.free()
    if g is not None:
        g.free()
    return ms, st


def calibration_copy(args):
    import torch
    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's own count)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["hotspot", "shock", "jet", "ensemble", "crossover"], default="hotspot")
    ap.add_argument("--n", type=int, default=None, help="cells per axis (hotspot / jet)")
    ap.add_argument("--events", type=int, default=None, help="events (ensemble / crossover)")
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--eos", choices=["ideal", "table"], default="ideal",
                    help="hotspot only: p = e/3, or the tabulated crossover EoS")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--seg", type=int, nargs=3, default=None, help="x chunks per wavefront, y and z cells per thread")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before timing, copy this many MiB device-to-device (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    ap.add_argument("--unsplit-hancock", action="store_true",
                    help="hotspot / shock: the unsplit Hancock reading (one correction per cell from all three "
                         "axes, computed by a pre-pass each stage) instead of the per-axis half step")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); events shard across "
              "GPUs by event and one large grid by z slabs, which is not built", file=sys.stderr)
        return 2

    if args.unsplit_hancock and args.workload not in ("hotspot", "shock"):
        print("bench.py: --unsplit-hancock applies to the hotspot and shock workloads", file=sys.stderr)
        return 2

    import torch

    from paper_1510_06340_amd import inputs as I

    torch.cuda.set_device(0)
    elem = 8 if args.dtype == "f64" else 4
    peak = FP64_PEAK_TFLOPS if args.dtype == "f64" else FP32_PEAK_TFLOPS
    if args.workload in ("ensemble", "crossover"):
        return bench_events(args, I)

    table = None
    jet_x0 = None
    if args.workload == "hotspot":
        w = I.hotspot_workload(n=args.n or 256)
        eos_desc = "p=e/3"
        if args.eos == "table":
            if args.dtype != "f64":
                print("bench.py: the tabulated EoS runs in FP64 only", file=sys.stderr)
                return 2
            table = I.crossover_table()
            w.eos = I.EOS_TABLE
            eos_desc = "tabulated crossover EoS"
        desc = (f"hotspot {w.n[0]}x{w.n[1]}x{w.n[2]} (40 seeded Gaussian hot spots, seed {w.seed}), {eos_desc}, "
                f"MC limiter, k={w.k}, RK{w.rk}, dt={w.dt:g}, outflow")
    elif args.workload == "jet":
        w = I.jet_workload(n=args.n or 512)
        jet_x0 = I.jet_start(w)
        desc = (f"jet {w.n[0]}^3 hot spots (seed {w.seed}) + point jet v=0.999 dE/dx=5 sigma=0.3, superbee, "
                f"k={w.k}, RK{w.rk}, dt={w.dt:g}")
    else:
        w = I.shock_workload()
        desc = "shock tube 200x16x16, e=10|1, minmod, k=2, RK2, dt=0.03"
    if args.unsplit_hancock:
        w.extra["unsplit_hancock"] = True
        desc += "; unsplit Hancock reading (a correction pre-pass over the grid and one ghost layer each stage)"
    if args.steps is None:
        args.steps = w.steps
    U = I.initial_state(w)
    ms_total, kms, klaunch, st = run_single(args, w, U, table, jet_x0)

    value = w.cells * args.steps / (ms_total / 1e3)
    fl_axis = flops_per_cell_axis(w.k, w.limiter)
    n_launch = sum(klaunch)
    avg_launch_ms = sum(kms) / max(n_launch, 1)
    achieved_tflops = fl_axis * w.cells / (avg_launch_ms / 1e3) / 1e12
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
        "config": {"workload": desc, "cells": w.cells},
        "roofline": {
            "kernel": "k_sweep / k_sweep_x (x, y and z axis sweeps)",
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / peak,
            "traffic": (TRAFFIC_HOTSPOT256_F64 if (args.workload == "hotspot" and w.n == (256, 256, 256)
                                                    and args.dtype == "f64" and table is None and args.seg is None
                                                    and args.block == 256 and not args.unsplit_hancock) else None),
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
    if args.unsplit_hancock:
        out["roofline"]["prepass_and_gaps_ms_per_step"] = (ms_total - sum(kms)) / args.steps
    if table is not None:
        out["roofline"]["note"] = ("algorithmic flops counted as for p = e/3; the table lookups and Newton "
                                   "iterations of the tabulated EoS are not counted")
    if args.cpu_budget > 0 and args.workload != "jet":
        out["cpu_baseline"] = cpu_baseline(w, U, args.cpu_budget, table)
    print(json.dumps(out), flush=True)
    return 0


def bench_events(args, I):
    """Ensemble (64 uneven events, p = e/3) or crossover (32 x 192^3, tabulated EoS): batched vs per-event."""
    if args.workload == "ensemble":
        ws = I.ensemble_workloads(n_events=args.events or 64)
        table = None
        desc = "ensemble: 64 events, sizes per axis from {96..192}, hot spots (seeds 1000+j), MC, k=3, RK2, dt=0.03"
    else:
        ws = I.crossover_workloads(n_events=args.events or 32)
        table = I.crossover_table()
        desc = "crossover: 32 events of 192^3 (seeds 2000+j), tabulated crossover EoS, MC, k=3, RK2, dt=0.03"
    if args.steps is None:
        args.steps = ws[0].steps
    Us = [I.initial_state(w) for w in ws]
    cells = sum(w.cells for w in ws)
    seeded = None
    if args.workload == "crossover":
        import time
        from paper_1510_06340_amd import surrogate
        t0 = time.perf_counter()
        E, M = surrogate.collect_states(n_samples=1 << 22, seed=42, n=128)
        e, pr = surrogate.label_states(E, M, table)
        seeded = {"collect_label_seconds": time.perf_counter() - t0}
        for name, output in (("ln_e", 0), ("bracket_fraction", 1)):
            t0 = time.perf_counter()
            net = surrogate.train(E, M, e, pr, epochs=30, output=output)
            err = surrogate.relative_error(net, E, M, e)
            train_s = time.perf_counter() - t0
            ms_s, st_s = run_events(args, ws, Us, batched=True, table=table, seed_net=net.network())
            seeded[name] = {"value": cells * args.steps / (ms_s / 1e3), "ms_per_step": ms_s / args.steps,
                            "newton_iters": sum(s["newton_iters"] for s in st_s),
                            "guesses_outside_bracket": sum(s["n_fallback"] for s in st_s),
                            "train": {"states": int(E.numel()), "epochs": 30, "seconds": train_s,
                                      "val_loss": net.history[-1][2], "seed_rel_err_median": float(err.median()),
                                      "seed_rel_err_p99": float(err.quantile(0.99))}}
    ms_b, st_b = run_events(args, ws, Us, batched=True, table=table)
    ms_p, st_p = run_events(args, ws, Us, batched=False, table=table)
    value = cells * args.steps / (ms_b / 1e3)
    plain = cells * args.steps / (ms_p / 1e3)
    fl_axis = flops_per_cell_axis(ws[0].k, ws[0].limiter)
    achieved = 3 * 2 * fl_axis * cells * args.steps / (ms_b / 1e3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_b / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "cells": cells, "form": "batched (persistent tile queue, graph replay)"},
        "plain_per_event": {"value": plain, "ms_per_step": ms_p / args.steps, "speedup_batched": value / plain},
        "batched_seeded": seeded,
        "roofline": {"kernel": "k_batch_sweep (all sweeps of the step)", "bound": "alu", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": None, "note": "whole-step average (graph replay, no per-launch events)"},
        "end_state": {"n_floor": sum(s["n_floor"] for s in st_b), "n_bad": sum(s["n_bad"] for s in st_b),
                      "newton_iters": sum(s["newton_iters"] for s in st_b)},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
