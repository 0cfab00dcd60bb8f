"""Pins for the oracle with the conserved charge R (Sec. 2.1: U = (E, M, R), flux R v_d;
Sec. 2.6: n = R sqrt(1 - v^2)) and the ideal-gas EoS p = (gamma - 1)(e - n) of the paper's
Sod shock tube (Sec. 3.2 and its parameter table).

* the exact Riemann solver: the lab-frame jump conditions of all three conserved
  quantities hold across its shock, and its fan satisfies the simple-wave relation
  dv / (1 - v^2) = -dp / ((e + p) cs) (checked by finite differences, independent of the
  closed-form invariant it is built from);
* con2prim: prim -> cons -> prim round trips (Sec. 2.1 relations) for the ideal gas,
  including cold gas (p = 0), and for p = e/3 with a passive charge;
* with p = e/3 the charge is passive: E and M are bitwise those of the run without it,
  R is conserved exactly on a periodic grid, uniform states stay bitwise, mirror
  symmetry holds bitwise;
* the scheme converges to the exact Sod solution (L1 of n and v fall with resolution).
"""
import math

import numpy as np
import pytest

import oracle
from oracle.riemann_gas import GasShockTube, enthalpy, prim_to_cons, sound_speed
from paper_1510_06340_amd import inputs as I

G = 5.0 / 3.0


def lab_state(n, p, v, gamma):
    """Conserved densities (R, M, E) and their x fluxes (R v, M v + p, M) of a state."""
    E, M, R = prim_to_cons(n, p, v, gamma)
    return np.array([R, M, E]), np.array([R * v, M * v + p, M])


@pytest.mark.parametrize("pars", [(10.0, 40.0 / 3.0, 1.0, 0.0, G), (1.0, 1000.0, 1.0, 0.01, G),
                                  (5.0, 3.0, 1.0, 1.0, 4.0 / 3.0)])
def test_gas_riemann_solver_jump_conditions_and_fan(pars):
    s = GasShockTube(*pars)
    g = s.g
    # shock: V (U_b - U_a) = F_b - F_a for R, M and E
    Ua, Fa = lab_state(s.nR, s.pR, 0.0, g)
    Ub, Fb = lab_state(s.n_star_right, s.p_star, s.v_star, g)
    np.testing.assert_allclose(s.shock_speed * (Ub - Ua), Fb - Fa, rtol=0, atol=1e-12 * np.abs(Fb).max())
    # contact: pressure and velocity continuous, the left plateau on the left isentrope
    assert s.n_star_left == pytest.approx(s.nL * (s.p_star / s.pL) ** (1 / g), rel=1e-13)
    assert s.head == pytest.approx(-s.csL, rel=1e-15) and s.head < s.tail < s.v_star < s.shock_speed < 1.0
    # fan: simple-wave relation by finite differences in xi
    t = 1.0
    xs = np.linspace(s.head, s.tail, 1602)[1:-1]
    n, p, v = s.sample(xs, t)
    e = n + p / (g - 1.0)
    cs = sound_speed(n, p, g)
    dv, dp = np.gradient(v, xs), np.gradient(p, xs)
    lhs = dv / (1 - v * v)
    rhs = -dp / ((e + p) * cs)
    np.testing.assert_allclose(lhs[2:-2], rhs[2:-2], rtol=1e-4)
    # the fan's characteristic is x / t
    np.testing.assert_allclose((v - cs) / (1 - v * cs), xs, atol=1e-12)


def test_gas_riemann_paper_sod_values():
    """The Sod parameters of the paper's table: the plateau lies between the two states."""
    s = GasShockTube()
    assert 0.0 < s.p_star < s.pL and 0.6 < s.v_star < 0.8
    assert s.nR < s.n_star_right < 4 * s.nR * (G + 1) / (G - 1) and s.n_star_left < s.nL
    assert enthalpy(s.nR, 0.0, G) == 1.0


def _prob(n, charge=True, gamma=G, **kw):
    return oracle.Problem(n=n, dx=(0.1, 0.1, 0.1), charge=charge, gamma=gamma, **kw)


def test_con2prim_round_trip_ideal_gas():
    rng = np.random.default_rng(5)
    m = 20000
    n = np.exp(rng.uniform(-3, 3, m))
    p = n * np.exp(rng.uniform(-8, 4, m))
    p[:2000] = 0.0  # cold gas
    d = rng.normal(size=(3, m))
    d /= np.linalg.norm(d, axis=0)
    speed = 0.995 * rng.uniform(0, 1, m) ** 0.5
    vv = d * speed
    E, Mabs, R = prim_to_cons(n, p, speed, G)
    U = np.concatenate([E[None], (Mabs * d), R[None]]).reshape(5, 1, 1, m)
    prim, cnt = oracle.con2prim(_prob((m, 1, 1)), U)
    prim = prim.reshape(6, m)
    e = n + p / (G - 1)
    assert cnt["n_bad"] == 0 and cnt["n_floor"] == 0
    np.testing.assert_allclose(prim[2:5], vv, rtol=0, atol=2e-13)
    # n = R sqrt(1 - v^2): relative error about v dv / (1 - v^2)
    assert np.all(np.abs(prim[5] - n) <= 1e-13 * n / (1 - speed ** 2))
    # e and p from the root: relative to E (e = E - M.v loses digits as v -> 1)
    assert np.all(np.abs(prim[0] - e) <= 1e-11 * E)
    assert np.all(np.abs(prim[1] - p) <= 1e-11 * E)
    assert np.all(prim[1][:2000] <= 1e-11 * E[:2000])
    # at rest: v = 0, e = E, n = R exactly
    U0 = np.array([30.0, 0.0, 0.0, 0.0, 10.0]).reshape(5, 1, 1, 1)
    pr0, _ = oracle.con2prim(_prob((1, 1, 1)), U0)
    assert pr0.ravel().tolist() == [30.0, (G - 1) * 20.0, 0.0, 0.0, 0.0, 10.0]


def test_con2prim_passive_charge_and_dust():
    """p = e/3 with the charge: e, p, v as without it, n = R sqrt(1 - v^2); gamma = 1
    (pressureless dust): p = 0 and v = M / E."""
    rng = np.random.default_rng(6)
    m = 5000
    U = np.empty((5, 1, 1, m))
    U[0] = 1 + rng.uniform(0, 3, m)
    U[1:4] = rng.uniform(-1, 1, (3, 1, 1, m)) * 0.55 * U[0]
    U[4] = rng.uniform(0.1, 2.0, m)
    pr4, _ = oracle.con2prim(oracle.Problem(n=(m, 1, 1)), U[:4])
    pr5, _ = oracle.con2prim(oracle.Problem(n=(m, 1, 1), charge=True), U)
    assert np.array_equal(pr4, pr5[:5])
    v2 = (pr5[2:5] ** 2).sum(0)
    np.testing.assert_allclose(pr5[5], U[4] * np.sqrt(1 - v2), rtol=1e-15)
    U[4] = np.sqrt(U[0] ** 2 - (U[1:4] ** 2).sum(0)) * rng.uniform(0.2, 1.0, m)   # E^2 >= M^2 + R^2
    dust, _ = oracle.con2prim(_prob((m, 1, 1), gamma=1.0), U)
    assert np.all(dust[1] == 0.0)
    np.testing.assert_allclose(dust[2:5], U[1:4] / U[0], rtol=1e-15)


def random_charged(rng, n, mfrac=0.5):
    U = np.zeros((5,) + tuple(n[::-1]))
    U[0] = 1.0 + rng.uniform(0, 4, size=n[::-1])
    U[1:4] = rng.uniform(-1, 1, size=(3,) + tuple(n[::-1])) * (mfrac / math.sqrt(3)) * U[0]
    U[4] = rng.uniform(0.2, 0.9, size=n[::-1]) * np.sqrt(U[0] ** 2 - (U[1:4] ** 2).sum(0))
    return U


@pytest.mark.parametrize("lim", [I.LIM_MC, I.LIM_VANALBADA])
def test_passive_charge_leaves_the_flow_bitwise(lim):
    rng = np.random.default_rng(7)
    n = (10, 8, 6)
    U = random_charged(rng, n)
    kw = dict(n=n, dx=(0.1, 0.12, 0.09), bc=(1, 1, 1), limiter=lim, k=3, rk=3)
    V4, _ = oracle.step(oracle.Problem(**kw), U[:4], 0.02, 4)
    p5 = oracle.Problem(charge=True, **kw)
    V5, _ = oracle.step(p5, U, 0.02, 4)
    assert np.array_equal(V4, V5[:4])
    T0, T1 = oracle.totals(p5, U), oracle.totals(p5, V5)
    assert abs(T1[4] - T0[4]) <= 1e-13 * abs(T0[4])
    assert np.max(np.abs(V5[4] - U[4])) > 1e-3   # the charge moved


def test_ideal_gas_conservation_uniform_and_mirror():
    rng = np.random.default_rng(8)
    n = (9, 8, 7)
    U = random_charged(rng, n, 0.3)
    prob = _prob(n, bc=(1, 1, 1), limiter=I.LIM_MINMOD, k=2, rk=2)
    V, st = oracle.step(prob, U, 0.02, 3)
    assert st["n_bad"] == 0
    T0, T1 = oracle.totals(prob, U), oracle.totals(prob, V)
    np.testing.assert_allclose(T1, T0, rtol=0, atol=1e-13 * T0[0])
    # uniform moving state: unchanged bitwise
    Uu = np.empty((5,) + n[::-1])
    Uu[0], Uu[1], Uu[2], Uu[3], Uu[4] = 3.0, 0.8, -0.5, 0.4, 1.7
    for lim in range(6):
        Vu, _ = oracle.step(_prob(n, bc=(0, 1, 0), limiter=lim, k=3, rk=2), Uu, 0.02, 2)
        assert np.array_equal(Vu, Uu), lim
    # mirror symmetry in x (R even, Mx odd): bitwise

    def mirror(W):
        W = np.flip(W, axis=3).copy()
        W[1] = -W[1]
        return W

    Us = (U + mirror(U)) / 2
    Vs, _ = oracle.step(_prob(n, bc=(0, 0, 0), limiter=I.LIM_MC, k=3, rk=2), Us, 0.02, 3)
    assert np.array_equal(mirror(Vs), Vs)


def test_sod_converges_to_exact_solution():
    """The paper's Sod data on [-2, 2] to t = 1 (RK2, k = 2, minmod): L1 of n and v fall with
    resolution; at the finest grid the plateau velocity and the shock position match."""
    ex = GasShockTube()
    errs = []
    for nx in (100, 200, 400):
        dx = 4.0 / nx
        w = I.sod_workload(nx=nx, dx=dx, dt=0.25 * dx, steps=int(round(4.0 / dx)), k=2, rk=2)
        w.xlo = (-2.0, -0.5 * dx, -0.5 * dx)
        prob = oracle.Problem.from_workload(w)
        V, st = oracle.step(prob, I.initial_state(w), w.dt, w.steps)
        assert st["n_bad"] == 0 and st["n_floor"] == 0
        prim, _ = oracle.con2prim(prob, V)
        x = I.cell_centres(nx, dx, w.xlo[0])
        n_ex, _, v_ex = ex.sample(x, w.steps * w.dt)
        errs.append((np.abs(prim[5, 0, 0] - n_ex).sum() * dx, np.abs(prim[2, 0, 0] - v_ex).sum() * dx))
    for q in range(2):
        ratios = [errs[i][q] / errs[i + 1][q] for i in range(2)]
        assert all(r > 1.4 for r in ratios), (errs, ratios)
    v = prim[2, 0, 0]
    plateau = v[(x > 0.4) & (x < 0.65)]
    assert np.all(np.abs(plateau - ex.v_star) < 0.03)
    i_shock = np.argmax((x > 0.5) & (v < 0.5 * ex.v_star))
    assert abs(x[i_shock] - ex.shock_speed * 1.0) < 0.06


def close(a, b, rtol, atol):
    assert np.all(np.abs(a - b) <= rtol * np.abs(b) + atol), float(np.max(np.abs(a - b) / (rtol * np.abs(b) + atol)))


def test_charge_flux_is_the_covariant_current():
    """The charge flux R v_d equals N^d = n u^d = n W v_d of the charge current, computed from the
    primitive state (n, v); the other components are as without the charge."""
    rng = np.random.default_rng(9)
    m = 3000
    n = np.exp(rng.uniform(-2, 2, m))
    p = n * np.exp(rng.uniform(-5, 2, m))
    d = rng.normal(size=(3, m))
    d /= np.linalg.norm(d, axis=0)
    speed = 0.99 * rng.uniform(0, 1, m)
    E, Mabs, R = prim_to_cons(n, p, speed, G)
    U = np.concatenate([E[None], Mabs * d, R[None]]).reshape(5, 1, 1, m)
    W = 1.0 / np.sqrt(1.0 - speed ** 2)
    for ax in range(3):
        F = oracle.flux(_prob((m, 1, 1)), ax, U).reshape(5, m)
        close(F[4], n * W * speed * d[ax], 1e-12, 1e-14 * R)
        # T^{0d} and T^{jd} of the ideal gas
        e = n + p / (G - 1)
        u0, ud = W, W * speed * d[ax]
        close(F[0], (e + p) * u0 * ud, 1e-11, 1e-13 * E)
        for j in range(3):
            Tjd = (e + p) * (W * speed * d[j]) * ud + (p if j == ax else 0.0)
            close(F[1 + j], Tjd, 1e-11, 1e-12 * E)


def test_max_speed_ideal_gas():
    """The characteristic-speed diagnostic with the ideal gas: the sound speed sqrt(gamma p / (n h))
    at rest, and relativistic velocity addition (v + cs) / (1 + v cs) for flow along an axis."""
    s = GasShockTube()
    U = np.zeros((5, 1, 1, 1))
    U[0], U[4] = 30.0, 10.0
    prob = _prob((1, 1, 1))
    assert oracle.max_speed(prob, U) == pytest.approx(s.csL, rel=1e-13)
    v = 0.6
    E, M, R = prim_to_cons(2.0, 0.7, v, G)
    U[0], U[1], U[4] = E, M, R
    cs = float(sound_speed(2.0, 0.7, G))
    assert oracle.max_speed(prob, U) == pytest.approx((v + cs) / (1 + v * cs), rel=1e-12)
    # cold gas: no sound, the flow speed itself
    E, M, R = prim_to_cons(2.0, 0.0, v, G)
    U[0], U[1], U[4] = E, M, R
    assert oracle.max_speed(prob, U) == pytest.approx(v, rel=1e-12)


def test_ellipsoidal_flow_converges_to_exact_solution():
    """The paper's ellipsoidal flow (Sec. 3.2; pressureless dust with the charge, gamma = 1) from
    the exact state at t0 = 2 to t = 2.4 on [-2, 2]^3: in the central region r < 1 the oracle
    follows the exact e, n and v, and the error falls with resolution.  The state is formed
    from (e, n, v) and the oracle's con2prim returns them where there is matter."""
    errs = []
    for N in (24, 48):
        dx = 4.0 / N
        dt = 0.2 * dx
        steps = int(round(0.4 / dt))
        w = I.ellipsoidal_workload(n=N, dx=dx, dt=dt, steps=steps)
        U = I.initial_state(w)
        prob = oracle.Problem.from_workload(w)
        p0, _ = oracle.con2prim(prob, U)
        e0, n0, v0 = I.ellipsoidal_prim(w.n, w.dx, w.xlo, 2.0)
        m = U[0] > 0
        assert np.abs(p0[0][m] - e0[m]).max() <= 1e-13 * e0.max() and np.all(p0[1] == 0.0)
        assert np.abs(p0[5][m] - n0[m]).max() <= 1e-13 * n0.max()
        V, st = oracle.step(prob, U, dt, steps, 2.0)
        prim, _ = oracle.con2prim(prob, V)
        e, nn, v = I.ellipsoidal_prim(w.n, w.dx, w.xlo, 2.0 + steps * dt)
        x = I.cell_centres(N, dx, w.xlo[0])
        c = np.sqrt(x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2) < 1.0
        errs.append((np.abs(prim[0][c] - e[c]).max() / e[c].max(), np.abs(prim[5][c] - nn[c]).max() / nn[c].max(),
                     np.abs(prim[2:5][:, c] - v[:, c]).max()))
    (e1, n1, v1), (e2, n2, v2) = errs
    assert e1 < 6e-3 and n1 < 6e-3 and v1 < 3e-3, errs
    assert e1 / e2 > 1.4 and n1 / n2 > 1.3 and v1 / v2 > 1.4, errs
