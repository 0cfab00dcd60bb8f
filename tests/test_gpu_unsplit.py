"""GPU parity of the unsplit Hancock ablation (MF_FLAG_UNSPLIT_HANCOCK) against the oracle's
unsplit_hancock option: one correction per cell from the limited faces of all three axes on the
grid extended by one ghost layer, added to the faces of every sweep."""
import math

import numpy as np
import pytest

import oracle
from paper_1510_06340_amd import inputs as I
from paper_1510_06340_amd import mf
from helpers import gpu_run, max_rel_err, rel_l1_E

pytestmark = pytest.mark.gpu


def moving_state(rng, n, mfrac=0.6):
    U = np.zeros((4,) + tuple(n[::-1]))
    U[0] = 1.0 + rng.uniform(0, 4, size=n[::-1])
    U[1:] = rng.uniform(-1, 1, size=(3,) + tuple(n[::-1])) * (mfrac / math.sqrt(3)) * U[0]
    return U


def unsplit_workload(n, lim, rk, bc, eos=I.EOS_IDEAL):
    w = I.Workload("t", n, (0.1, 0.12, 0.09), (0.0, 0.0, 0.0), bc, lim, 3, rk, 0.02, 3, eos=eos)
    w.extra["unsplit_hancock"] = True
    return w


@pytest.mark.parametrize("lim,rk,bc", [(I.LIM_MC, 2, (0, 1, 0)), (I.LIM_MINMOD, 3, (1, 0, 1)),
                                       (I.LIM_VANALBADA, 2, (1, 1, 1))])
def test_unsplit_matches_oracle(lim, rk, bc):
    rng = np.random.default_rng(11 + lim)
    n = (20, 17, 13)
    U = moving_state(rng, n)
    w = unsplit_workload(n, lim, rk, bc)
    Ug, st = gpu_run(w, U, flags=mf.MF_FLAG_UNSPLIT_HANCOCK)
    Uo, sto = oracle.step(oracle.Problem.from_workload(w), U, w.dt, w.steps)
    assert max_rel_err(Ug, Uo) <= 1e-10
    assert st["n_floor"] == sto["n_floor"] and st["n_bad"] == 0
    # the reading changes the result: the per-axis step differs far above rounding
    Up, _ = gpu_run(w, U)
    assert max_rel_err(Ug, Up) > 1e-6


def test_unsplit_thin_and_ragged_grids():
    """Lines of 1 and 2 cells (ghost indices wrap or clamp on every side), a ragged x extent, and
    42 x 62 extended columns: 11 chunks of 256, two per XCD group, five idle blocks."""
    rng = np.random.default_rng(5)
    for n in [(1, 9, 7), (2, 1, 11), (67, 3, 2), (40, 60, 9)]:
        U = moving_state(rng, n, 0.4)
        w = unsplit_workload(n, I.LIM_SUPERBEE, 2, (1, 0, 1))
        Ug, _ = gpu_run(w, U, flags=mf.MF_FLAG_UNSPLIT_HANCOCK)
        Uo, _ = oracle.step(oracle.Problem.from_workload(w), U, w.dt, w.steps)
        assert max_rel_err(Ug, Uo) <= 1e-10, n


def test_unsplit_table_eos_and_fp32():
    table = I.crossover_table()
    rng = np.random.default_rng(8)
    n = (17, 15, 13)
    U = np.zeros((4,) + n[::-1])
    U[0] = np.exp(rng.uniform(-2, 4, size=n[::-1]))
    U[1:] = rng.uniform(-0.3, 0.3, size=(3,) + n[::-1]) * U[0]
    w = unsplit_workload(n, I.LIM_MC, 2, (1, 0, 1), eos=I.EOS_TABLE)
    Ug, st = gpu_run(w, U, eos_table=table, flags=mf.MF_FLAG_UNSPLIT_HANCOCK)
    Uo, _ = oracle.step(oracle.Problem.from_workload(w, table=table), U, w.dt, w.steps)
    assert max_rel_err(Ug, Uo) <= 1e-10
    assert st["newton_iters"] > 0
    # FP32 against the FP64 oracle (ideal EoS)
    w = unsplit_workload(n, I.LIM_MC, 2, (0, 0, 0))
    U = moving_state(rng, n)
    Ug, _ = gpu_run(w, U, dtype="f32", flags=mf.MF_FLAG_UNSPLIT_HANCOCK)
    Uo, _ = oracle.step(oracle.Problem.from_workload(w), U, w.dt, w.steps)
    assert rel_l1_E(Ug, Uo) <= 1e-5


def test_unsplit_is_refused_by_batched_stepping():
    import torch
    from helpers import to_dev
    n = (8, 7, 6)
    U = moving_state(np.random.default_rng(1), n)
    w = unsplit_workload(n, I.LIM_MC, 2, (0, 0, 0))
    dev = to_dev(U)
    g = mf.Grid([mf.desc_from_workload(w, flags=mf.MF_FLAG_UNSPLIT_HANCOCK)], [dev])
    g.set_eos_ideal()
    with pytest.raises(mf.MFError) as ei:
        g.batch_step([w.dt], 1)
    assert ei.value.code == mf.MF_ERR_ARG
    torch.cuda.synchronize()
    g.free()


def test_unsplit_with_jet_source():
    """The unsplit reading with the jet source (the z sweep's jet and unsplit variant), from a nonzero time."""
    w = I.jet_workload(n=32, steps=4, box=8.0)
    w.extra["unsplit_hancock"] = True
    x0 = (-2.0, 0.3, -0.2)
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U, jet_x0=x0, t0=0.5, flags=mf.MF_FLAG_UNSPLIT_HANCOCK)
    prob = oracle.Problem.from_workload(w, jet_x0=x0)
    Uo, sto = oracle.step(prob, U, w.dt, w.steps, 0.5)
    assert max_rel_err(Ug, Uo) <= 1e-10
    assert st["n_floor"] == sto["n_floor"] and st["n_bad"] == 0
