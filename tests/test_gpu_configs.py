"""GPU parity at the workloads' stated sizes (FP64 max relative error <= 1e-10 per cell with
momenta measured against E; FP32 relative L1 of E <= 1e-5), each against the FP64 oracle.

What is compared, per workload:

* hot spots, 256^3 (dx = 0.1, MC, k = 3, RK2): the first 10 steps on the full grid, FP64 and
  FP32 against one oracle run; the same workload at 128^3 on a 12.8 box (the same dx = 0.1
  and dt = 0.03) for all 200 steps, FP64.
* jet, 512^3 (dx = 0.05, superbee, k = 3): the seeded jet start, the first 10 steps, compared
  on oracle blocks around the jet, the centre and two opposite corners (the block oracle is
  the full run's arithmetic on each cell's domain of dependence); and the same generator at
  128^3 for all 150 steps on the full grid.
* ensemble, 64 events of sizes {96, ..., 192}^3: one batched step (the persistent tile-queue
  launches replayed from the HIP graph) and a second replay, every event against the oracle.

The crossover workload in its batched, surrogate-seeded form is compared in
test_gpu_surrogate.py, where the trained network is at hand.
"""
import numpy as np
import pytest

import oracle
from paper_1510_06340_amd import inputs as I
from paper_1510_06340_amd import mf
from helpers import from_dev, gpu_run, max_rel_err, oracle_block, rel_l1_E, to_dev

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def oracle_run(w, U, nsteps, jet_x0=None, t0=0.0):
    prob = oracle.Problem.from_workload(w, jet_x0=jet_x0)
    return oracle.step(prob, U, w.dt, nsteps, t0)


@pytest.fixture(scope="module")
def hotspot256():
    w = I.hotspot_workload()
    U = I.initial_state(w)
    print(f"\nhot spots 256^3: oracle, 10 steps on {oracle.num_threads()} threads", flush=True)
    Uo, sto = oracle_run(w, U, 10)
    return w, U, Uo, sto


def test_hotspot_256_fp64_ten_steps(hotspot256):
    w, U, Uo, sto = hotspot256
    Ug, st = gpu_run(w, U, nsteps=10)
    err = max_rel_err(Ug, Uo)
    print(f"\nFP64 256^3, 10 steps: max rel err {err:.2e}")
    assert err <= TOL64
    assert st["n_floor"] == sto["n_floor"] and st["n_bad"] == 0
    assert st["smax"] == pytest.approx(sto["smax"], rel=1e-10)


def test_hotspot_256_fp32_ten_steps(hotspot256):
    w, U, Uo, _ = hotspot256
    Ug, st = gpu_run(w, U, dtype="f32", nsteps=10)
    l1 = rel_l1_E(Ug, Uo)
    print(f"\nFP32 256^3, 10 steps: relative L1 of E {l1:.2e}")
    assert l1 <= 1e-5
    assert st["n_bad"] == 0


def test_hotspot_dx01_full_run():
    """All 200 steps of the hot-spot workload at its dx = 0.1 and dt = 0.03, on a 128^3 grid
    (box 12.8, which still holds the ball of hot-spot centres)."""
    w = I.hotspot_workload(n=128, box=12.8)
    assert w.dx[0] == pytest.approx(0.1) and w.dt == pytest.approx(0.03) and w.steps == 200
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U)
    Uo, sto = oracle_run(w, U, w.steps)
    err = max_rel_err(Ug, Uo)
    print(f"\nhot spots 128^3 dx 0.1, 200 steps: max rel err {err:.2e}")
    assert err <= TOL64
    assert st["n_floor"] == sto["n_floor"] and st["n_bad"] == 0
    assert st["smax"] == pytest.approx(sto["smax"], rel=1e-10)


def test_jet_512_seeded_start_sampled_blocks():
    """The jet workload at its stated size, from the seeded jet start, 10 steps."""
    w = I.jet_workload()
    U = I.initial_state(w)
    x0 = I.jet_start(w)
    nsteps = 10
    Ug, st = gpu_run(w, U, jet_x0=x0, nsteps=nsteps)
    assert st["n_bad"] == 0 and st["t"] == pytest.approx(nsteps * w.dt)
    # the jet's cell after the steps
    xj = [x0[0] + w.jet["v"] * nsteps * w.dt, x0[1], x0[2]]
    ij = [int((xj[d] - w.xlo[d]) / w.dx[d]) for d in range(3)]
    blocks = [([ij[0] - 14, ij[1] - 10, ij[2] - 10], (24, 20, 20)),
              ([246, 246, 246], (20, 20, 20)), ([0, 0, 0], (16, 16, 16)), ([496, 496, 496], (16, 16, 16))]
    dep = 0.0
    for lo, size in blocks:
        Ub, sl = oracle_block(w, U, lo, size, nsteps, jet_x0=x0)
        Gb = Ug[(slice(None),) + sl]
        err = max_rel_err(Gb, Ub)
        print(f"\njet 512^3 block {lo} + {size}: max rel err {err:.2e}", flush=True)
        assert err <= TOL64, (lo, err)
        dep = max(dep, float((Ub[0] - U[(0,) + sl]).max()))
    assert dep > 0.2   # the block at the jet holds its deposit


def test_jet_128_all_steps():
    """The jet workload's generator at 128^3 (dx = 0.2, dt = 0.06) for all 150 steps: the jet
    crosses from x = -5 to x = 4."""
    w = I.jet_workload(n=128)
    U = I.initial_state(w)
    x0 = I.jet_start(w)
    Ug, st = gpu_run(w, U, jet_x0=x0)
    Uo, sto = oracle_run(w, U, w.steps, jet_x0=x0)
    err = max_rel_err(Ug, Uo)
    print(f"\njet 128^3, 150 steps: max rel err {err:.2e}")
    assert err <= TOL64
    assert st["n_floor"] == sto["n_floor"] and st["n_bad"] == sto["n_bad"]


def test_ensemble_64_events_full_size():
    """The 64-event ensemble at its stated sizes: two batched steps (the HIP graph is built on
    the first and replayed on the second); every event against the oracle."""
    import torch
    ws = I.ensemble_workloads()
    Us = [I.initial_state(w) for w in ws]
    devs = [to_dev(U) for U in Us]
    g = mf.Grid([mf.desc_from_workload(w) for w in ws], devs)
    try:
        g.set_eos_ideal()
        g.batch_step([w.dt for w in ws], 1)
        st = g.batch_step([w.dt for w in ws], 1)
        torch.cuda.synchronize()
        worst = 0.0
        for j, w in enumerate(ws):
            Uo, sto = oracle_run(w, Us[j], 2)
            err = max_rel_err(from_dev(devs[j], Us[j].shape[1:]), Uo)
            worst = max(worst, err)
            assert err <= TOL64, (j, err)
            assert st[j]["steps"] == 2 and st[j]["n_floor"] == sto["n_floor"]
            assert st[j]["smax"] == pytest.approx(sto["smax"], rel=1e-12)
        print(f"\n64 events, 2 batched steps: worst max rel err {worst:.2e}")
    finally:
        g.free()
