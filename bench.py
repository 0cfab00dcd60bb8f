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

The default line also carries `batched_vs_plain`: a few timed steps of the
64-event ensemble (one persistent launch per sweep over all events, replayed
from a HIP graph, against one mf_step call per event) and of the 32 x 192^3
crossover workload under the tabulated EoS (batched plain, batched with the
learned ln e seed trained in the run, and per-event plain), each with its own
whole-step roofline (Newton iterations counted) and a bounded oracle sample.
"""
from __future__ import annotations

import argparse
import json
import math
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


# Tabulated EoS: con2prim + flux along one axis without Newton iterations: |M|^2 (5), the
# bracket [E - |M|^2/E, E] and its midpoint (4), one piece lookup of p and dp/de (the
# piece's t (2), the cubic (6), its derivative (7) and the piece index (1)), then
# v = M / (E + p) and the momentum fluxes (11).
C2P_FLUX_TABLE = 5 + 4 + 16 + 11
# One safeguarded Newton iteration: g and g' (9), the step and its acceptance test (6),
# the bracket update (3) and the lookup at the new iterate (16).
NEWTON_ITER_FLOPS = 34
# Ideal gas p = (gamma - 1)(e - n) with the charge: |M|^2 (5), the residual f(p), f'(p) at p = 0
# (1 / (E + p), v^2, sqrt(1 - v^2), e, f, f': 18) and the start (1), then v_d and the five fluxes (7).
C2P_FLUX_GAS = 5 + 18 + 1 + 7
# One safeguarded Newton iteration on f(p): the residual (18), the step (2), its test (2) and the bracket (2).
NEWTON_ITER_FLOPS_GAS = 24
# The y and z sweeps start every solve but one per cell and axis (the Hancock pair's first
# state) from a neighbouring pressure and take the first step before the cold-gas test, which
# a converged step makes unnecessary: those solves skip the residual at p = 0 and the start.
GAS_WARM_SKIP = 18 + 1


def flops_per_cell_axis(k: int, limiter: int, c2p_flux: int = C2P_FLUX, nc: int = 4) -> int:
    """Reconstruction + Hancock half step + k-stage MUSTA-FORCE + flux difference, per cell and axis
    (nc conserved components: 4, or 5 with the charge)."""
    # 2 differences, the limiter, phi / 2 (folded into MC's terms) and the two face values
    recon = nc * (2 + LIMITER_OPS[limiter] + (0 if limiter == 3 else 1) + 2)
    hancock = 2 * c2p_flux + nc * 4
    # per stage: Richtmyer state (5 per component) and F_lw + F_lf (6), then the predictor (6)
    musta = k * (3 * c2p_flux + nc * 11) + (k - 1) * nc * 6
    return recon + hancock + musta + nc * 2


def gas_flops_per_cell_axis(k: int, limiter: int) -> float:
    """The ideal gas with the charge, mean over the x, y and z sweeps: in y and z all solves per cell
    but the Hancock pair's first (1 + 3k of 2 + 3k) skip the residual at p = 0 and the start."""
    fx = flops_per_cell_axis(k, limiter, C2P_FLUX_GAS, nc=5)
    return (fx + 2 * (fx - (1 + 3 * k) * GAS_WARM_SKIP)) / 3


def flops_per_cell_stage(k: int, limiter: int) -> int:
    """Three axis sweeps, two L accumulations and the RK combine (12 on average)."""
    return 3 * flops_per_cell_axis(k, limiter) + 8 + 12


def bytes_per_cell_step(rk: int, elem: int, nc: int = 4) -> int:
    """Algorithmic HBM bytes: RK2 reads U^n, writes U1, reads U1 and U^n, writes U^{n+1} (5 passes of nc
    components; RK3: 8)."""
    passes = 5 if rk == 2 else 8
    return passes * nc * elem


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
        "sample": f"first {steps} RK{w.rk} step(s) of the same {w.n[0]}x{w.n[1]}x{w.n[2]} workload, FP64 C oracle, "
                  f"OpenMP over grid lines, {t_total:.1f} s",
    }


def upload(U, tdt):
    import numpy as np
    import torch
    return [torch.from_numpy(np.ascontiguousarray(U[c]).ravel()).to(device="cuda", dtype=tdt)
            for c in range(U.shape[0])]


def run_single(args, w, U, table=None, jet_x0=None):
    """One grid through mf_step; returns (ms_total, per-axis kernel ms and launches, end stats)."""
    import torch
    from paper_1510_06340_amd import mf
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    dev = upload(U, tdt)
    flags = mf.MF_FLAG_UNSPLIT_HANCOCK if args.unsplit_hancock else 0
    g = mf.Grid([mf.desc_from_workload(w, mf.MF_F64 if args.dtype == "f64" else mf.MF_F32, flags)], [dev])
    if "gamma" in w.extra:
        g.set_eos_gamma(w.extra["gamma"])
    elif table is None:
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


def run_events(ws, Us, batched, steps, warmup, table=None, seed_net=None):
    """Many events: one batched handle (mf_batch_step) or one mf_step call per event in turn.
    Returns (ms over the timed steps, per-event stats of one more step)."""
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

    advance(max(warmup, 1))  # includes the autotuner and graph capture for the batched form
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    advance(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = g.batch_step(dts, 1) if batched else [h.step(dt, 1)[0] for h, dt in zip(per, dts)]
    for h in per:
        h.free()
    if g is not None:
        g.free()
    del devs
    torch.cuda.empty_cache()
    return ms, st


def cpu_baseline_events(ws, Us, budget_s, table=None, crop=None):
    """The oracle on event 0 (or on a central crop^3 block of it, outflow at the block's faces),
    one step at a time until the budget is spent."""
    import oracle
    w, U = ws[0], Us[0]
    what = f"event 0 ({w.n[0]}x{w.n[1]}x{w.n[2]})"
    if crop is not None:
        import copy
        lo = [(w.n[d] - crop) // 2 for d in range(3)]
        U = U[:, lo[2]:lo[2] + crop, lo[1]:lo[1] + crop, lo[0]:lo[0] + crop].copy()
        w = copy.copy(w)
        w.xlo = tuple(w.xlo[d] + lo[d] * w.dx[d] for d in range(3))
        w.n = (crop, crop, crop)
        what = f"the central {crop}^3 block of event 0 (outflow at its faces; the hot spots lie there)"
    prob = oracle.Problem.from_workload(w, table=table)
    steps, t_total, V = 0, 0.0, U
    while steps < 20:
        t0 = time.perf_counter()
        V, _ = oracle.step(prob, V, w.dt, 1, steps * w.dt)
        t_total += time.perf_counter() - t0
        steps += 1
        if t_total >= budget_s:
            break
    return {"value": w.cells * steps / t_total, "unit": "cell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {steps} RK2 step(s) of {what}, FP64 C oracle"
                      f"{' (bisection con2prim on the table)' if table is not None else ''}, {t_total:.1f} s"}


def event_compare(I, kind, steps, warmup, n_events=None, cpu_budget=0.0):
    """Batched vs per-event throughput of the ensemble (64 uneven events, p = e/3) or of the
    crossover workload (32 x 192^3, tabulated EoS; batched plain, batched with the learned
    ln e seed, per-event plain).  Returns a dict (one block of the JSON line)."""
    if kind == "ensemble":
        ws = I.ensemble_workloads(n_events=n_events or 64)
        table = None
        desc = (f"ensemble: {len(ws)} events, sizes per axis from {{96..192}}, hot spots (seeds 1000+j), MC, k=3, "
                "RK2, dt=0.03, p=e/3")
    else:
        ws = I.crossover_workloads(n_events=n_events or 32)
        table = I.crossover_table()
        desc = (f"crossover: {len(ws)} events of 192^3 (seeds 2000+j), tabulated crossover EoS, MC, k=3, RK2, "
                "dt=0.03")
    Us = [I.initial_state(w) for w in ws]
    cells = sum(w.cells for w in ws)
    k, lim = ws[0].k, ws[0].limiter
    c2p = C2P_FLUX if table is None else C2P_FLUX_TABLE
    fl_step = 3 * 2 * flops_per_cell_axis(k, lim, c2p) * cells   # 3 axes x 2 RK stages

    def form(ms, st, extra=None):
        iters = sum(x["newton_iters"] for x in st)   # of the one step after the timed ones
        fl = fl_step + NEWTON_ITER_FLOPS * iters
        achieved = fl * steps / (ms / 1e3) / 1e12
        d = {"value": cells * steps / (ms / 1e3), "ms_per_step": ms / steps,
             "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                          "flops_per_step": fl, "newton_iters_per_step": iters}}
        if extra:
            d.update(extra)
        return d

    out = {"workload": desc, "cells": cells, "steps": steps, "warmup": max(warmup, 1),
           "note": (f"{steps} timed steps of the workload's {ws[0].steps}; whole-step times (graph replay "
                    "has no per-launch events); Newton iterations per step measured on the step after the "
                    "timed ones and counted at " + str(NEWTON_ITER_FLOPS) + " flops each")}
    ms_b, st_b = run_events(ws, Us, True, steps, warmup, table)
    out["batched"] = form(ms_b, st_b)
    ms_p, st_p = run_events(ws, Us, False, steps, warmup, table)
    out["per_event"] = form(ms_p, st_p)
    out["speedup_batched_vs_per_event"] = out["batched"]["value"] / out["per_event"]["value"]
    if kind == "crossover":
        from paper_1510_06340_amd import surrogate
        t0 = time.perf_counter()
        E, M = surrogate.collect_states(n_samples=1 << 22, seed=42, n=128)
        e, pr = surrogate.label_states(E, M, table)
        t_collect = time.perf_counter() - t0
        t0 = time.perf_counter()
        net = surrogate.train(E, M, e, pr, epochs=30, output=0)
        t_train = time.perf_counter() - t0
        err = surrogate.relative_error(net, E, M, e)
        del E, M, e, pr
        ms_s, st_s = run_events(ws, Us, True, steps, warmup, table, seed_net=net.network())
        out["batched_seeded"] = form(ms_s, st_s, {
            "seeds_outside_bracket_per_step": sum(x["n_fallback"] for x in st_s),
            "seed": {"output": "ln e", "states": 1 << 22, "epochs": 30, "collect_label_s": t_collect,
                     "train_s": t_train, "val_loss": net.history[-1][2],
                     "rel_err_median": float(err.median()), "rel_err_p99": float(err.quantile(0.99))}})
        out["seeded_vs_per_event_plain"] = out["batched_seeded"]["value"] / out["per_event"]["value"]
        out["seeded_vs_batched_plain"] = out["batched_seeded"]["value"] / out["batched"]["value"]
    if cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline_events(ws, Us, cpu_budget, table, crop=64 if table is not None else None)
    return out


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
    ap.add_argument("--workload", choices=["hotspot", "shock", "jet", "ensemble", "crossover", "seed", "sod"],
                    default="hotspot",
                    help="seed: the learned seed's kernels alone (network forward, gradient, Adam, seeded con2prim); "
                         "sod: the Sod tube of the ideal gas with the conserved charge, 500 cells along x, "
                         "extended to n x n cells across (periodic)")
    ap.add_argument("--n", type=int, default=None, help="cells per axis (hotspot / jet), across the tube (sod)")
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
    ap.add_argument("--compare-steps", type=int, default=5,
                    help="hotspot line: timed steps of the batched-vs-per-event and learned-seed comparisons "
                         "(ensemble and crossover workloads) carried in the same JSON line; 0 = leave them out")
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
    if args.workload == "seed":
        return bench_seed(args, I)

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
    elif args.workload == "sod":
        if args.dtype != "f64":
            print("bench.py: the charge runs in FP64 only", file=sys.stderr)
            return 2
        nt = args.n or 96
        w = I.sod_workload(ny=nt, nz=nt)
        desc = (f"Sod tube {w.n[0]}x{w.n[1]}x{w.n[2]} (500 cells of 0.02 along x, n=10|1, p=13.33|0 at rest, "
                f"periodic across), ideal gas gamma=5/3 with the conserved charge, minmod, k={w.k}, RK{w.rk}, "
                f"dt={w.dt:g}")
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
    n_launch = sum(klaunch)
    avg_launch_ms = sum(kms) / max(n_launch, 1)
    newton_flops = None
    if "gamma" in w.extra:
        # Newton iterations per sweep launch: those of the step after the timed ones, over its sweeps
        fl_axis = gas_flops_per_cell_axis(w.k, w.limiter)
        fl_launch = fl_axis * w.cells + NEWTON_ITER_FLOPS_GAS * st["newton_iters"] / (3 * w.rk)
        newton_flops = NEWTON_ITER_FLOPS_GAS
    elif table is None:
        fl_axis = flops_per_cell_axis(w.k, w.limiter)
        if args.unsplit_hancock:
            # the sweeps add the pre-pass's correction to both faces (8) instead of the per-axis
            # Hancock half step (two flux evaluations and 16); the pre-pass is timed apart
            fl_axis = fl_axis - (2 * C2P_FLUX + 4 * 4) + 8
        fl_launch = fl_axis * w.cells
    else:
        # Newton iterations per sweep launch: those of the step after the timed ones, over its 6 sweeps
        fl_axis = flops_per_cell_axis(w.k, w.limiter, C2P_FLUX_TABLE)
        fl_launch = fl_axis * w.cells + NEWTON_ITER_FLOPS * st["newton_iters"] / (3 * w.rk)
        newton_flops = NEWTON_ITER_FLOPS
    achieved_tflops = fl_launch / (avg_launch_ms / 1e3) / 1e12
    hbm_bytes = bytes_per_cell_step(w.rk, elem, 5 if w.extra.get("charge") else 4)
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
            "flops_per_cell_axis": round(fl_axis, 1),
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
        out["roofline"]["newton_iters_per_step"] = st["newton_iters"]
        out["roofline"]["note"] = (f"tabulated EoS: {C2P_FLUX_TABLE} flops per con2prim + flux (bracket, one "
                                   f"piece lookup of p and dp/de, velocity, fluxes) and {NEWTON_ITER_FLOPS} per "
                                   "Newton iteration, iterations measured on the step after the timed ones")
    elif newton_flops is not None:
        out["roofline"]["newton_iters_per_step"] = st["newton_iters"]
        out["roofline"]["note"] = (f"ideal gas with the charge (5 components): {C2P_FLUX_GAS} flops per con2prim + "
                                   f"flux (the residual at p = 0, velocity, fluxes; in y and z {C2P_FLUX_GAS - GAS_WARM_SKIP} "
                                   "for the warm-started solves, all but one per cell and axis) and "
                                   f"{NEWTON_ITER_FLOPS_GAS} per Newton iteration on f(p), iterations measured on the "
                                   "step after the timed ones")
    if args.cpu_budget > 0 and args.workload != "jet":
        out["cpu_baseline"] = cpu_baseline(w, U, args.cpu_budget, table)
    if (args.compare_steps > 0 and args.workload == "hotspot" and table is None and args.dtype == "f64"
            and w.n == (256, 256, 256) and not args.unsplit_hancock):
        del U
        budget = min(args.cpu_budget, 4.0)
        out["batched_vs_plain"] = {kind: event_compare(I, kind, args.compare_steps, 1, cpu_budget=budget)
                                   for kind in ("ensemble", "crossover")}
    print(json.dumps(out), flush=True)
    return 0


def bench_events(args, I):
    """--workload ensemble | crossover: the line's value is the configured batched form (the
    crossover workload's with the learned seed), with the other forms beside it."""
    steps = args.steps if args.steps is not None else 10
    blk = event_compare(I, args.workload, steps, args.warmup, args.events, args.cpu_budget)
    main_form = blk["batched_seeded"] if args.workload == "crossover" else blk["batched"]
    out = {
        "metric": METRIC,
        "value": main_form["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": blk["warmup"],
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": blk["workload"], "cells": blk["cells"],
                   "form": "batched (persistent tile queue, graph replay)"
                           + (" with the learned ln e seed" if args.workload == "crossover" else "")},
        "roofline": dict(main_form["roofline"], kernel="k_batch_sweep (all sweeps of the step)"),
        "forms": blk,
    }
    if "cpu_baseline" in blk:
        out["cpu_baseline"] = blk["cpu_baseline"]
    print(json.dumps(out), flush=True)
    return 0


def bench_seed(args, I):
    """The seed network's kernels on their own: forward over 2^20 states, one epoch of
    gradients and Adam steps at the training batch (4096), and con2prim of 2^20 crossover
    states plain and seeded (network per state).  Network: Glorot initialisation (the
    arithmetic per sample does not depend on the weights)."""
    import torch
    from paper_1510_06340_amd import mf, surrogate
    reps = args.steps or 20
    n = 1 << 20
    batch = 4096
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    P = torch.from_numpy(surrogate.init_params(0)).cuda()
    X = torch.randn((n, 2), generator=gen, device="cuda")
    T = torch.randn(n, generator=gen, device="cuda")
    y = torch.empty(n, device="cuda")
    grad, loss = torch.zeros_like(P), torch.zeros(1, device="cuda")
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    work = torch.empty(mf.mlp_workspace(batch), device="cuda")

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms_fwd = timed(lambda: mf.mlp_forward(P, X, y), reps)

    def epoch():
        for b in range(n // batch):
            mf.mlp_grad(P, X[b * batch:(b + 1) * batch], T[b * batch:(b + 1) * batch], grad, loss, work)
            mf.mlp_adam(P, grad, m, v, b + 1, 1e-3)

    ms_epoch = timed(epoch, max(1, reps // 10))
    ms_adam = timed(lambda: mf.mlp_adam(P, grad, m, v, 1, 1e-3), reps)
    # crossover states: E log-uniform in [1e-2, 1e2], |M|/E uniform in [0, 0.99)
    E = torch.exp(torch.empty(n, dtype=torch.float64, device="cuda").uniform_(math.log(1e-2), math.log(1e2),
                                                                              generator=gen))
    Ma = E * torch.empty(n, dtype=torch.float64, device="cuda").uniform_(0.0, 0.99, generator=gen)
    U = [E, Ma, torch.zeros_like(E), torch.zeros_like(E)]
    prim = [torch.empty_like(E) for _ in range(5)]
    g = mf.Grid([mf.make_desc((n, 1, 1), (1, 1, 1), (0, 0, 0), (0, 0, 0))], [U])
    net = mf.SeedNetwork(P.cpu().numpy(), (0.0, 0.0), (1.0, 1.0), 0.0, 1.0, 0)
    g.set_eos_table(*I.crossover_table(), surrogate=net)
    ms_plain = timed(lambda: g.con2prim(U, prim, None, mf.MF_C2P_PLAIN), reps)
    ms_seeded = timed(lambda: g.con2prim(U, prim, None, mf.MF_C2P_SEEDED), reps)
    g.free()
    H = mf.MF_MLP_HIDDEN
    mm_flops = 2 * H * H   # layer 2 per sample, on the matrix cores
    fwd = n / (ms_fwd / 1e3)
    out = {
        "metric": "seed-network samples/s (forward)",
        "value": fwd,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": 1,
        "ms_per_step": ms_fwd,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (FP32 accumulation)",
        "data": "synthetic",
        "config": {"workload": "seed network 2-64-64-1 tanh: forward of 2^20 states, one epoch of 256 "
                               "gradient + Adam steps at batch 4096, con2prim of 2^20 crossover states"},
        "forward": {"ms": ms_fwd, "samples_per_s": fwd, "layer2_mfma_TFLOPs": mm_flops * fwd / 1e12},
        "train_epoch": {"ms": ms_epoch, "samples_per_s": n / (ms_epoch / 1e3),
                        "layer2_mfma_TFLOPs": 3 * mm_flops * n / (ms_epoch / 1e3) / 1e12},
        "adam_ms": ms_adam,
        "con2prim": {"plain_ms": ms_plain, "seeded_ms": ms_seeded, "states": n},
        "roofline": {"bound": "mfma", "kernel": "k_mlp_forward", "achieved": mm_flops * fwd / 1e12,
                     "peak": 2500.0, "unit": "TFLOP/s", "frac": mm_flops * fwd / 1e12 / 2500.0, "traffic": None,
                     "note": "layer-2 matrix flops against the dense BF16 matrix peak; the kernel's time goes to "
                             "the 128 tanh per sample on the vector ALUs"},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
