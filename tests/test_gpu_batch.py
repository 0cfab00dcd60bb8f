"""Batched stepping (persistent tile-queue sweeps replayed from a HIP graph).

Results must equal the per-event path bitwise (same arithmetic per cell; the
sweeps are independent of launch shape), and the oracle to 1e-10.  The graph
is replayed several times with eager work and synchronisation in between, and
every replay is checked against the eager per-event result.
"""
import numpy as np
import pytest

import oracle
from paper_1510_06340_amd import inputs as I
from paper_1510_06340_amd import mf
from helpers import from_dev, max_rel_err, to_dev

pytestmark = pytest.mark.gpu

SIZES = [(20, 17, 13), (33, 8, 21), (16, 16, 16), (9, 30, 12), (25, 25, 5)]


def events(sizes, rk=2, jet=False, eos=I.EOS_IDEAL):
    out = []
    for j, n in enumerate(sizes):
        w = I.Workload("ensemble", n, (0.1, 0.1, 0.1), tuple(-0.05 * s for s in n), (0, j % 2, 0), I.LIM_MC,
                       2 + (j % 2), rk, 0.02 + 0.002 * j, 3, eos=eos, seed=1000 + j)
        if jet:
            w.jet = dict(v=0.999, dedx=5.0, sigma=0.3, x_start=-0.5)
        out.append(w)
    return out


def make_grid(ws, Us, table=None, jets=None, dtype="f64"):
    devs = [to_dev(U, dtype) for U in Us]
    g = mf.Grid([mf.desc_from_workload(w, mf.MF_F32 if dtype == "f32" else mf.MF_F64) for w in ws], devs)
    if table is None:
        g.set_eos_ideal()
    else:
        g.set_eos_table(*table)
    for j, w in enumerate(ws):
        if jets is not None:
            g.set_jet(j, jets[j], w.jet["v"], w.jet["dedx"], w.jet["sigma"])
    return g, devs


def initial(ws):
    return [I.at_rest(I.hotspot_energy(w.n, w.dx, w.xlo, I.draw_event(w.seed))) for w in ws]


@pytest.mark.parametrize("rk", [2, 3])
def test_batch_equals_per_event_every_replay(rk):
    import torch
    ws = events(SIZES, rk=rk)
    Us = initial(ws)
    gb, devb = make_grid(ws, Us)
    gp, devp = make_grid(ws, Us)
    dts = [w.dt for w in ws]
    for rep in range(3):
        stb = gb.batch_step(dts, 1)
        torch.cuda.synchronize()
        # the per-event path: one event at a time, same step
        for j, w in enumerate(ws):
            gj = mf.Grid([mf.desc_from_workload(w)], [devp[j]])
            gj.set_eos_ideal()
            gj.set_time(0, rep * w.dt if rep else 0.0, rep)
            stj = gj.step(w.dt, 1)[0]
            gj.free()
            assert stb[j]["steps"] == rep + 1
            assert stb[j]["t"] == pytest.approx(stj["t"], rel=1e-15)
            assert stb[j]["n_floor"] == stj["n_floor"]
        torch.cuda.synchronize()
        for j, w in enumerate(ws):
            a = from_dev(devb[j], Us[j].shape[1:])
            b = from_dev(devp[j], Us[j].shape[1:])
            assert np.array_equal(a, b), (rep, j)
        # eager work between replays
        x = torch.randn(1000, device="cuda")
        (x * 2).sum().item()
    gb.free()
    gp.free()


def test_batch_matches_oracle_and_rebuilds_on_new_dt():
    import torch
    ws = events(SIZES[:3])
    Us = initial(ws)
    g, dev = make_grid(ws, Us)
    g.batch_step([w.dt for w in ws], 2)
    dts2 = [0.5 * w.dt for w in ws]
    st = g.batch_step(dts2, 2)
    torch.cuda.synchronize()
    for j, w in enumerate(ws):
        prob = oracle.Problem.from_workload(w)
        Uo, _ = oracle.step(prob, Us[j], w.dt, 2)
        Uo, _ = oracle.step(prob, Uo, dts2[j], 2, 2 * w.dt)
        Ug = from_dev(dev[j], Us[j].shape[1:])
        assert max_rel_err(Ug, Uo) <= 1e-10
        assert st[j]["t"] == pytest.approx(2 * w.dt + 2 * dts2[j])
    g.free()


def test_batch_jet_events_match_oracle():
    import torch
    ws = events(SIZES[:2], jet=True)
    Us = initial(ws)
    x0 = [(-0.5, 0.1, -0.05), (-0.3, -0.2, 0.1)]
    g, dev = make_grid(ws, Us, jets=x0)
    g.batch_step([w.dt for w in ws], 3)
    torch.cuda.synchronize()
    for j, w in enumerate(ws):
        Uo, _ = oracle.step(oracle.Problem.from_workload(w, jet_x0=x0[j]), Us[j], w.dt, 3)
        assert max_rel_err(from_dev(dev[j], Us[j].shape[1:]), Uo) <= 1e-10
    g.free()


def test_batch_table_eos_matches_oracle():
    import torch
    table = I.crossover_table()
    ws = events(SIZES[1:3], eos=I.EOS_TABLE)
    Us = initial(ws)
    g, dev = make_grid(ws, Us, table=table)
    st = g.batch_step([w.dt for w in ws], 2)
    torch.cuda.synchronize()
    for j, w in enumerate(ws):
        Uo, _ = oracle.step(oracle.Problem.from_workload(w, table=table), Us[j], w.dt, 2)
        assert max_rel_err(from_dev(dev[j], Us[j].shape[1:]), Uo) <= 1e-10
        assert st[j]["newton_iters"] > 0
    g.free()


def test_batch_table_eos_with_jets_matches_oracle():
    """The tabulated EoS with the jet source (the z sweep's jet variant of the table kernels), batched."""
    import torch
    table = I.crossover_table()
    ws = events(SIZES[:2], jet=True, eos=I.EOS_TABLE)
    Us = initial(ws)
    x0 = [(-0.5, 0.1, -0.05), (-0.3, -0.2, 0.1)]
    g, dev = make_grid(ws, Us, table=table, jets=x0)
    st = g.batch_step([w.dt for w in ws], 3)
    torch.cuda.synchronize()
    for j, w in enumerate(ws):
        Uo, sto = oracle.step(oracle.Problem.from_workload(w, table=table, jet_x0=x0[j]), Us[j], w.dt, 3)
        assert max_rel_err(from_dev(dev[j], Us[j].shape[1:]), Uo) <= 1e-10
        assert st[j]["newton_iters"] > 0 and st[j]["n_bad"] == 0 and st[j]["n_floor"] == sto["n_floor"]
    g.free()


def test_batch_f32_equals_per_event_and_oracle():
    """FP32 events, batched: bitwise the per-event FP32 result, and the FP64 oracle to FP32 accuracy."""
    import torch
    ws = events(SIZES[:3])
    Us = initial(ws)
    gb, devb = make_grid(ws, Us, dtype="f32")
    gb.batch_step([w.dt for w in ws], 3)
    torch.cuda.synchronize()
    for j, w in enumerate(ws):
        devp = to_dev(Us[j], "f32")
        gj = mf.Grid([mf.desc_from_workload(w, mf.MF_F32)], [devp])
        gj.set_eos_ideal()
        gj.step(w.dt, 3)
        torch.cuda.synchronize()
        gj.free()
        a = from_dev(devb[j], Us[j].shape[1:])
        assert np.array_equal(a, from_dev(devp, Us[j].shape[1:])), j
        Uo, _ = oracle.step(oracle.Problem.from_workload(w), Us[j], w.dt, 3)
        assert float(np.abs(a[0] - Uo[0]).sum() / np.abs(Uo[0]).sum()) <= 1e-5
    gb.free()


def test_batch_rejects_mixed_limiters():
    ws = events(SIZES[:2])
    ws[1].limiter = I.LIM_MINMOD
    g, _ = make_grid(ws, initial(ws))
    with pytest.raises(mf.MFError) as ei:
        g.batch_step([w.dt for w in ws], 1)
    assert ei.value.code == mf.MF_ERR_ARG
    g.free()
