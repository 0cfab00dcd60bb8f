"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 max over cells of max_c |U_gpu - U_oracle| / E_oracle <= 1e-10;
FP32 relative L1 of E <= 1e-5.  Invariants (uniform state, planar and mirror
symmetry) are checked on the GPU alone.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1510_06340_amd import inputs as I
from helpers import gpu_run, max_rel_err, rel_l1_E, to_dev, from_dev

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def oracle_run(w, U, nsteps=None, jet_x0=None, table=None, t0=0.0):
    prob = oracle.Problem.from_workload(w, table=table, jet_x0=jet_x0)
    return oracle.step(prob, U, w.dt, w.steps if nsteps is None else nsteps, t0)


def test_con2prim_matches_oracle():
    import torch
    from paper_1510_06340_amd import mf
    rng = np.random.default_rng(0)
    n = 100_000
    e = np.exp(rng.uniform(math.log(1e-3), math.log(1e3), n))
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    v = d * 0.999 * rng.uniform(0, 1, n) ** 0.5
    g2 = 1 / (1 - (v ** 2).sum(0))
    p = e / 3
    U = np.concatenate([((e + p) * g2 - p)[None], ((e + p) * g2)[None] * v]).reshape(4, 1, 1, n)
    prim_o, _ = oracle.con2prim(oracle.Problem(), U)
    dev = to_dev(U)
    out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(5)]
    it = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    g = mf.Grid([mf.make_desc((n, 1, 1), (1, 1, 1), (0, 0, 0), (0, 0, 0))], [dev])
    g.set_eos_ideal()
    g.con2prim(dev, out, it)
    torch.cuda.synchronize()
    prim_g = np.stack([t.cpu().numpy() for t in out])
    g.free()
    pg = prim_g.reshape(5, -1)
    po = prim_o.reshape(5, -1)
    # e = E - M.v loses digits as v -> 1 (relative conditioning ~ E / e): compare on the scale of E
    E = U[0].ravel()
    assert np.all(np.abs(pg[:2] - po[:2]) <= 1e-14 * E)
    np.testing.assert_allclose(pg[2:], po[2:], rtol=0, atol=1e-14)
    assert int(it.min()) == 0 and int(it.max()) == 0


def test_shock_tube_full_config_parity():
    """200x16x16 planar shock tube, minmod, k = 2, RK2, 100 steps (t = 3)."""
    w = I.shock_workload()
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U)
    Uo, sto = oracle_run(w, U)
    assert max_rel_err(Ug, Uo) <= TOL64
    assert st["n_floor"] == 0 and st["n_bad"] == 0
    # planar invariance on the GPU: every (y, z) pencil is bitwise the same
    assert np.all(Ug == Ug[:, :1, :1, :])
    assert st["smax"] == pytest.approx(sto["smax"], rel=1e-10)
    assert st["steps"] == 100 and st["t"] == pytest.approx(3.0)


@pytest.mark.parametrize("lim", range(6))
def test_shock_tube_paper_setting(lim):
    """The paper's experimental setting (RK3, 4 MUSTA stages) on the shock tube, every limiter, 100 steps."""
    w = I.shock_workload(ny=4, nz=4, limiter=lim, k=4, rk=3)
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U)
    Uo, sto = oracle_run(w, U)
    assert max_rel_err(Ug, Uo) <= TOL64
    assert np.all(Ug == Ug[:, :1, :1, :])
    assert st["n_floor"] == sto["n_floor"] and st["n_bad"] == sto["n_bad"]


def test_predictor_alpha_ablation_parity():
    """MF_FLAG_PREDICTOR_ALPHA (alpha dt/dx in the MUSTA predictor) against the oracle's alternative reading."""
    from paper_1510_06340_amd import mf
    w = I.shock_workload(ny=4, nz=4, k=4, rk=3)
    w.extra["predictor_alpha"] = True
    U = I.initial_state(w)
    Ug, _ = gpu_run(w, U, flags=mf.MF_FLAG_PREDICTOR_ALPHA)
    Uo, _ = oracle_run(w, U)
    assert max_rel_err(Ug, Uo) <= TOL64
    w.extra["predictor_alpha"] = False
    Ul, _ = oracle_run(w, U)
    assert max_rel_err(Ul, Uo) > 1e-4   # the readings differ


@pytest.mark.parametrize("bc", [I.BC_OUTFLOW, I.BC_PERIODIC])
def test_hotspot_parity_ragged_grid(bc):
    """Hot spots on a 67x45x38 grid (ragged against every segment and block shape), MC, k = 3."""
    w = I.hotspot_workload(n=64, box=12.8, steps=12)
    w.n = (67, 45, 38)
    w.bc = (bc,) * 3
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U)
    Uo, sto = oracle_run(w, U)
    assert max_rel_err(Ug, Uo) <= TOL64
    assert st["n_bad"] == 0 and st["n_floor"] == sto["n_floor"]
    assert st["smax"] == pytest.approx(sto["smax"], rel=1e-10)


def random_state(rng, n, mfrac=0.6):
    U = np.zeros((4,) + tuple(n[::-1]))
    U[0] = 1.0 + rng.uniform(0, 4, size=n[::-1])
    U[1:] = rng.uniform(-1, 1, size=(3,) + tuple(n[::-1])) * (mfrac / math.sqrt(3)) * U[0]
    return U


@pytest.mark.parametrize("lim", range(6))
def test_every_limiter_stage_count_and_rk(lim):
    rng = np.random.default_rng(lim)
    n = (21, 18, 15)
    U = random_state(rng, n)
    for k in (1, 2, 3, 4):
        for rk in (2, 3):
            w = I.Workload("t", n, (0.1, 0.12, 0.09), (0, 0, 0), (0, 1, 0), lim, k, rk, 0.02, 3)
            Ug, st = gpu_run(w, U)
            Uo, sto = oracle_run(w, U)
            err = max_rel_err(Ug, Uo)
            assert err <= 1e-12, (lim, k, rk, err)
            assert st["n_floor"] == sto["n_floor"] and st["n_bad"] == sto["n_bad"]


def test_zero_steps_and_empty_calls():
    """nsteps = 0 leaves the state untouched; zero-length con2prim and network calls are no-ops."""
    import torch
    from paper_1510_06340_amd import mf
    w = I.shock_workload(nx=20, ny=3, nz=2)
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U, nsteps=0)
    assert np.array_equal(Ug, U) and st["steps"] == 0 and st["t"] == 0.0
    dev = to_dev(U)
    g = mf.Grid([mf.desc_from_workload(w)], [dev])
    try:
        g.set_eos_ideal(w.cs2)
        empty = [torch.empty(0, dtype=torch.float64, device="cuda") for _ in range(5)]
        g.con2prim(empty[:4], empty)
        sts = g.batch_step([w.dt], 0)
        assert sts[0]["steps"] == 0
    finally:
        g.free()
    params = torch.zeros(mf.MF_MLP_PARAMS, device="cuda")
    mf.mlp_forward(params, torch.empty((0, 2), device="cuda"), torch.empty(0, device="cuda"))
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [(1, 1, 1), (2, 1, 1), (1, 5, 1), (1, 1, 7), (3, 1, 130), (130, 2, 3), (65, 66, 1)])
def test_degenerate_and_thin_grids(n):
    rng = np.random.default_rng(sum(n))
    U = random_state(rng, n)
    for bc in (0, 1):
        w = I.Workload("t", n, (0.1, 0.1, 0.1), (0, 0, 0), (bc, 1 - bc, bc), I.LIM_MC, 3, 2, 0.02, 4)
        Ug, _ = gpu_run(w, U)
        Uo, _ = oracle_run(w, U)
        assert max_rel_err(Ug, Uo) <= 1e-12


@pytest.mark.parametrize("n,bc", [((256, 256, 2), (0, 0, 1)), ((256, 2, 256), (0, 1, 0)), ((64, 2, 2), (1, 1, 1))])
def test_two_cell_periodic_axes(n, bc):
    """Periodic axes only two cells thick on wide planes: the y/z march's look-ahead stays
    inside the line (the last iteration's load is clamped to the last ghost cell)."""
    rng = np.random.default_rng(n[0] + 3 * n[1] + 7 * n[2])
    U = random_state(rng, n)
    w = I.Workload("t", n, (0.1, 0.1, 0.1), (0, 0, 0), bc, I.LIM_MC, 3, 2, 0.02, 2)
    Ug, st = gpu_run(w, U)
    Uo, sto = oracle_run(w, U)
    assert max_rel_err(Ug, Uo) <= 1e-12
    assert st["n_floor"] == sto["n_floor"] and st["n_bad"] == 0


@pytest.mark.parametrize("seg,block", [((1, 1, 1), 64), ((5, 7, 3), 128), ((1000, 1000, 1000), 256), ((2, 16, 16), 64)])
def test_launch_shapes_agree(seg, block):
    """Every segment length and block size gives the same result (bitwise) and matches the oracle."""
    rng = np.random.default_rng(7)
    n = (40, 33, 29)
    U = random_state(rng, n)
    w = I.Workload("t", n, (0.1, 0.1, 0.1), (0, 0, 0), (0, 0, 1), I.LIM_SUPERBEE, 3, 2, 0.02, 3)
    Ug, st = gpu_run(w, U, tuning=(seg, block))
    Ua, sta = gpu_run(w, U)
    assert np.array_equal(Ug, Ua)
    assert st["n_floor"] == sta["n_floor"]
    Uo, _ = oracle_run(w, U)
    assert max_rel_err(Ug, Uo) <= 1e-12


def test_uniform_state_bitwise_on_gpu():
    n = (9, 7, 5)
    U = np.empty((4,) + n[::-1])
    U[0], U[1], U[2], U[3] = 2.5, 0.9, -0.7, 1.3
    for lim in range(6):
        for bc in (0, 1):
            w = I.Workload("t", n, (0.1, 0.2, 0.3), (0, 0, 0), (bc,) * 3, lim, 3, 2, 0.02, 3)
            Ug, _ = gpu_run(w, U)
            assert np.array_equal(Ug, U), (lim, bc)


def test_mirror_symmetry_on_gpu():
    rng = np.random.default_rng(11)
    n = (12, 10, 8)
    U = random_state(rng, n, 0.3)

    def mirror(V, ax):
        W = np.flip(V, axis=3 - ax).copy()
        W[1 + ax] = -W[1 + ax]
        return W

    for ax in range(3):
        U = (U + mirror(U, ax)) / 2.0
    w = I.Workload("t", n, (0.1, 0.1, 0.1), (0, 0, 0), (0, 0, 0), I.LIM_MC, 3, 2, 0.03, 4)
    Ug, _ = gpu_run(w, U)
    for ax in range(3):
        assert max_rel_err(mirror(Ug, ax), Ug) <= 1e-14


def test_jet_source_parity():
    w = I.jet_workload(n=48, steps=6, box=12.0)
    x0 = (-2.0, 0.3, -0.2)
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U, jet_x0=x0, t0=0.5)
    Uo, sto = oracle_run(w, U, jet_x0=x0, t0=0.5)
    assert max_rel_err(Ug, Uo) <= TOL64
    assert st["t"] == pytest.approx(0.5 + 6 * w.dt)


def test_fp32_against_fp64_oracle():
    w = I.hotspot_workload(n=64, box=12.8, steps=20)
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U, dtype="f32")
    Uo, _ = oracle_run(w, U)
    assert rel_l1_E(Ug, Uo) <= 1e-5
    assert st["n_bad"] == 0


def test_fp32_jet_against_fp64_oracle():
    """FP32 with the jet source (the FP32 jet variant of the z sweep) against the FP64 oracle."""
    w = I.jet_workload(n=48, steps=6, box=12.0)
    x0 = (-2.0, 0.3, -0.2)
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U, dtype="f32", jet_x0=x0, t0=0.5)
    Uo, _ = oracle_run(w, U, jet_x0=x0, t0=0.5)
    assert rel_l1_E(Ug, Uo) <= 1e-5
    assert st["n_bad"] == 0


def test_totals_match_oracle():
    from paper_1510_06340_amd import mf
    w = I.hotspot_workload(n=40, box=8.0, steps=3)
    w.bc = (1, 1, 1)
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U)
    Uo, _ = oracle_run(w, U)
    prob = oracle.Problem.from_workload(w)
    To = oracle.totals(prob, Uo)
    T0 = oracle.totals(prob, U)
    np.testing.assert_allclose(st["totals"][0], To[0], rtol=1e-13)
    np.testing.assert_allclose(st["totals"][1:], To[1:], atol=1e-12 * To[0])
    # periodic: conserved
    assert abs(st["totals"][0] - T0[0]) <= 1e-13 * T0[0]


def test_strict_mode_reports_unphysical_states():
    from paper_1510_06340_amd import mf
    n = (16, 8, 8)
    U = np.zeros((4,) + n[::-1])
    U[0] = 1.0
    U[0, 3, 4, 5] = -1.0        # E < 0
    U[1, 5, 2, 9] = 2.0         # |M| > E
    w = I.Workload("t", n, (0.1,) * 3, (0, 0, 0), (1, 1, 1), I.LIM_MINMOD, 2, 2, 0.01, 1)
    Ug, st = gpu_run(w, U)
    Uo, sto = oracle_run(w, U)
    assert st["n_bad"] > 0 and st["n_floor"] > 0
    assert st["n_bad"] == sto["n_bad"] and st["n_floor"] == sto["n_floor"]
    with pytest.raises(mf.MFError) as ei:
        gpu_run(w, U, flags=mf.MF_FLAG_STRICT)
    assert ei.value.code == mf.MF_ERR_UNPHYSICAL


def test_hotspot_256_full_size_one_step():
    """The bench workload itself (256^3, MC, k = 3, RK2, launch shape as timed): one full step vs the oracle."""
    w = I.hotspot_workload()
    U = I.initial_state(w)
    Ug, st = gpu_run(w, U, nsteps=1)
    Uo, sto = oracle_run(w, U, nsteps=1)
    assert max_rel_err(Ug, Uo) <= TOL64
    assert st["n_floor"] == 0 and st["n_bad"] == 0
    assert st["smax"] == pytest.approx(sto["smax"], rel=1e-12)
