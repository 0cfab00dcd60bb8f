"""Pins for the oracle's pointwise parts: con2prim, flux, limiters, MUSTA, EoS table.

Each check compares against something other than the oracle's own formula:
brute-force root finding of the paper's fixed-point equation, the covariant
stress tensor, the paper's ratio-form limiters, library interpolation, and
invariants (consistency, mirror symmetry).
"""
import math

import numpy as np
import pytest

from paper_1510_06340_amd import inputs as I

CS2 = 1.0 / 3.0


def prim_to_cons(e, v, p):
    """E = (e+p) g^2 - p, M_i = (e+p) g^2 v_i (Sec. 2.1)."""
    v2 = (v ** 2).sum(axis=0)
    g2 = 1.0 / (1.0 - v2)
    return np.concatenate([((e + p) * g2 - p)[None], ((e + p) * g2)[None] * v])


def random_prim(rng, n, vmax=0.95, emin=0.01, emax=100.0):
    e = np.exp(rng.uniform(math.log(emin), math.log(emax), n))
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    vm = vmax * rng.uniform(0, 1, n) ** 0.5
    return e, d * vm


def brute_force_v(E, M, pfun):
    """Bisection on v in [0, 1) of v (E + p(E - M v)) = M (the paper's fixed point for v)."""
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        h = mid * (E + pfun(E - M * mid)) - M
        if h > 0:
            hi = mid
        else:
            lo = mid
        if hi - lo < 1e-17:
            break
    return 0.5 * (lo + hi)


# ---------------------------------------------------------------- con2prim


def test_con2prim_ideal_matches_brute_force_fixed_point(ora):
    rng = np.random.default_rng(1)
    e, v = random_prim(rng, 300)
    U = prim_to_cons(e, v, CS2 * e)
    prim, cnt = ora.con2prim(ora.Problem(), U)
    assert cnt["n_floor"] == 0 and cnt["n_bad"] == 0
    for i in range(U.shape[1]):
        E, Mv = U[0, i], U[1:, i]
        M = float(np.linalg.norm(Mv))
        vb = brute_force_v(E, M, lambda ee: CS2 * ee)
        assert np.linalg.norm(prim[2:, i]) == pytest.approx(vb, rel=1e-13, abs=1e-16)
        assert prim[0, i] == pytest.approx(E - M * vb, rel=1e-12)


def test_con2prim_round_trip(ora):
    rng = np.random.default_rng(2)
    e, v = random_prim(rng, 2000, vmax=0.99)
    U = prim_to_cons(e, v, CS2 * e)
    prim, _ = ora.con2prim(ora.Problem(), U)
    np.testing.assert_allclose(prim[0], e, rtol=1e-12)
    np.testing.assert_allclose(prim[1], CS2 * e, rtol=1e-12)
    np.testing.assert_allclose(prim[2:], v, rtol=0, atol=1e-14)


def test_con2prim_at_rest_is_exact(ora):
    E = np.array([1e-3, 0.1, 1.0, 7.25, 1e4])
    U = np.stack([E, 0 * E, 0 * E, 0 * E])
    prim, _ = ora.con2prim(ora.Problem(), U)
    assert np.array_equal(prim[0], E) and np.array_equal(prim[1], CS2 * E)
    assert np.all(prim[2:] == 0.0)


def test_con2prim_guards_count(ora):
    U = np.array([[1.0, 1.0, 2.0, -1.0, np.nan, 1.0],
                  [0.5, 1.0, 2.5, 0.0, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 0.0, 0.0, np.inf],
                  [0.0, 0.0, 0.0, 0.0, 0.0, 0.0]])
    prim, cnt = ora.con2prim(ora.Problem(), U)
    # |M| >= E clamps (cells 1 and 2); E <= 0, NaN or inf are bad (cells 3, 4, 5)
    assert cnt["n_floor"] == 2 and cnt["n_bad"] == 3
    v = np.linalg.norm(prim[2:, :3], axis=0)
    assert np.all(v < 1.0) and np.all(prim[0, 1:3] > 0)
    assert np.all(prim[:, 3:] == 0.0)


def test_pchip_matches_scipy_on_crossover_table(ora):
    from scipy.interpolate import PchipInterpolator
    e, p = I.crossover_table()
    prob = ora.Problem(table=(e, p))
    ref = PchipInterpolator(e, p)
    rng = np.random.default_rng(3)
    x = 10 ** rng.uniform(-3, 3, 5000)
    pv, dv = ora.eos(prob, x)
    np.testing.assert_allclose(pv, ref(x), rtol=1e-13)
    np.testing.assert_allclose(dv, ref(x, 1), rtol=1e-10)
    # nodes are reproduced exactly and the interpolant is monotone
    pn, _ = ora.eos(prob, e)
    np.testing.assert_allclose(pn, p, rtol=2e-16)
    xs = np.sort(x)
    assert np.all(np.diff(ora.eos(prob, xs)[0]) >= 0)
    # extrapolation: linear through the origin below, with the end slope above
    lo, dlo = ora.eos(prob, np.array([1e-4]))
    assert lo[0] == pytest.approx(p[0] * 1e-4 / e[0], rel=1e-15) and dlo[0] == pytest.approx(p[0] / e[0])
    hi, _ = ora.eos(prob, np.array([2e3]))
    assert hi[0] == pytest.approx(p[-1] + ref(e[-1], 1) * (2e3 - e[-1]), rel=1e-12)


def test_table_con2prim_matches_brute_force(ora):
    from scipy.interpolate import PchipInterpolator
    e_t, p_t = I.crossover_table()
    prob = ora.Problem(table=(e_t, p_t))
    ref = PchipInterpolator(e_t, p_t)
    rng = np.random.default_rng(4)
    e, v = random_prim(rng, 200, vmax=0.95, emin=0.01, emax=500.0)
    U = prim_to_cons(e, v, ref(e))
    prim, cnt = ora.con2prim(prob, U)
    assert cnt["n_iter"] > 0 and cnt["n_bad"] == 0
    np.testing.assert_allclose(prim[0], e, rtol=1e-12)
    np.testing.assert_allclose(prim[2:], v, atol=1e-13)
    for i in range(20):
        M = float(np.linalg.norm(U[1:, i]))
        vb = brute_force_v(U[0, i], M, lambda ee: float(ref(ee)))
        assert np.linalg.norm(prim[2:, i]) == pytest.approx(vb, rel=1e-12, abs=1e-15)


def test_linear_table_reduces_to_ideal(ora):
    e_t = I.crossover_nodes()
    prob_t = ora.Problem(table=(e_t, e_t / 3.0))
    rng = np.random.default_rng(5)
    e, v = random_prim(rng, 500, emin=0.01, emax=500.0)
    U = prim_to_cons(e, v, CS2 * e)
    a, _ = ora.con2prim(prob_t, U)
    b, _ = ora.con2prim(ora.Problem(), U)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- flux


def test_flux_equals_stress_tensor(ora):
    """F_d = (T^{0d}, T^{xd}, T^{yd}, T^{zd}) with T = (e+p) u u - p g."""
    rng = np.random.default_rng(6)
    e, v = random_prim(rng, 400)
    p = CS2 * e
    U = prim_to_cons(e, v, p)
    g2 = 1.0 / (1.0 - (v ** 2).sum(axis=0))
    w = (e + p) * g2
    for d in range(3):
        F = ora.flux(ora.Problem(), d, U)
        T0 = w * v[d]
        Tj = w * v * v[d]
        Tj[d] += p
        np.testing.assert_allclose(F[0], T0, rtol=1e-12, atol=1e-14 * w.max())
        np.testing.assert_allclose(F[1:], Tj, rtol=1e-12, atol=1e-12 * w.max())


# ---------------------------------------------------------------- limiters

XI = {
    I.LIM_MINMOD: lambda r: max(0.0, min(1.0, r)),
    I.LIM_SUPERBEE: lambda r: max(0.0, min(2 * r, 1.0), min(r, 2.0)),
    I.LIM_MC: lambda r: max(0.0, min(2 * r, 0.5 * (1 + r), 2.0)),
    I.LIM_VANLEER: lambda r: (r + abs(r)) / (1 + abs(r)),
    I.LIM_VANALBADA: lambda r: (r * r + r) / (r * r + 1),
}


@pytest.mark.parametrize("lim", sorted(XI))
def test_two_argument_limiter_equals_ratio_form(ora, lim):
    rng = np.random.default_rng(10 + lim)
    a = rng.normal(size=4000) * 10 ** rng.uniform(-6, 3, 4000)
    b = rng.normal(size=4000) * 10 ** rng.uniform(-6, 3, 4000)
    phi = ora.limiter(lim, a, b)
    ref = np.array([XI[lim](bb / aa) * aa for aa, bb in zip(a, b)])
    np.testing.assert_allclose(phi, ref, rtol=1e-14, atol=1e-300)
    # symmetric limiters treat forward and backward differences alike: phi(a,b) = phi(b,a)
    np.testing.assert_allclose(ora.limiter(lim, b, a), phi, rtol=1e-15, atol=1e-300)
    # odd: phi(-a,-b) = -phi(a,b)
    assert np.array_equal(ora.limiter(lim, -a, -b), -phi)


@pytest.mark.parametrize("lim", sorted(XI))
def test_limiter_symmetry_property(lim):
    for r in np.geomspace(1e-3, 1e3, 61):
        assert XI[lim](1 / r) == pytest.approx(XI[lim](r) / r, rel=1e-13)


def test_limiters_in_tvd_region(ora):
    r = np.geomspace(1e-3, 1e3, 400)
    a = np.ones_like(r)
    mb = ora.limiter(I.LIM_MINMOD, a, r)
    sb = ora.limiter(I.LIM_SUPERBEE, a, r)
    for lim in (I.LIM_MC, I.LIM_VANLEER, I.LIM_VANALBADA):
        phi = ora.limiter(lim, a, r)
        assert np.all(phi >= mb * (1 - 1e-15)) and np.all(phi <= sb * (1 + 1e-15))
    # at extrema and flat neighbours the TVD limiters give no slope
    for lim in (I.LIM_MINMOD, I.LIM_SUPERBEE, I.LIM_MC, I.LIM_VANLEER):
        assert np.all(ora.limiter(lim, np.array([1.0, -2.0, 0.0, 3.0]), np.array([-1.0, 5.0, 4.0, 0.0])) == 0.0)
    # no limiter: central slope
    assert ora.limiter(I.LIM_NONE, np.array([1.0]), np.array([3.0]))[0] == 2.0


# ---------------------------------------------------------------- MUSTA


def random_states(rng, n):
    e, v = random_prim(rng, n, vmax=0.8, emin=0.1, emax=10.0)
    return prim_to_cons(e, v, CS2 * e)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_musta_consistency_bitwise(ora, k):
    rng = np.random.default_rng(20 + k)
    U = random_states(rng, 200)
    prob = ora.Problem(k=k)
    for d in range(3):
        F = ora.musta(prob, d, 0.3, U, U)
        assert np.array_equal(F, ora.flux(prob, d, U))


@pytest.mark.parametrize("k", [1, 3])
def test_musta_mirror_symmetry_bitwise(ora, k):
    rng = np.random.default_rng(30 + k)
    UL, UR = random_states(rng, 200), random_states(rng, 200)
    prob = ora.Problem(k=k)
    for d in range(3):
        P = np.ones((4, 1))
        P[1 + d] = -1.0
        F = ora.musta(prob, d, 0.3, UL, UR)
        Fm = ora.musta(prob, d, 0.3, P * UR, P * UL)
        assert np.array_equal(Fm, -P * F)


def test_musta_axis_rotation(ora):
    rng = np.random.default_rng(40)
    UL, UR = random_states(rng, 100), random_states(rng, 100)
    prob = ora.Problem(k=3)
    Fx = ora.musta(prob, 0, 0.3, UL, UR)
    for d in (1, 2):
        perm = [0, 1, 2, 3]
        perm[1], perm[1 + d] = perm[1 + d], perm[1]
        Fd = ora.musta(prob, d, 0.3, UL[perm], UR[perm])
        np.testing.assert_allclose(Fd[perm], Fx, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("lam", [0.1, 0.3])
def test_musta_linearised_about_rest(ora, k, lam):
    """Small perturbations of a state at rest: MUSTA-FORCE reduces to its linear form.

    About (E0, 0, 0, 0) with p = e/3 the flux along x is F(U0 + dU) = F(U0) + A dU
    + O(dU^2) with A = [[0,1,0,0],[1/3,0,0,0],[0,0,0,0],[0,0,0,0]] (dF/dU of the
    stress tensor at rest).  With a linear flux each stage is
      Fh = A (UL + UR)/2 - (alpha lam A^2 + I/(alpha lam)) (UR - UL)/4,
      UL <- UL - lam (Fh - A UL),  UR <- UR - lam (A UR - Fh),
    so k stages give an explicit matrix map of (dUL, dUR).
    """
    alpha, E0, eps = 3.0, 2.0, 1e-7
    A = np.zeros((4, 4))
    A[0, 1], A[1, 0] = 1.0, CS2
    rng = np.random.default_rng(50 + k)
    dL = rng.normal(size=4) * eps
    dR = rng.normal(size=4) * eps
    dL[2:] = 0.0
    dR[2:] = 0.0
    U0 = np.array([E0, 0.0, 0.0, 0.0])
    F = ora.musta(ora.Problem(k=k), 0, lam, (U0 + dL)[:, None], (U0 + dR)[:, None])[:, 0]
    F0 = np.array([0.0, CS2 * E0, 0.0, 0.0])
    uL, uR = dL.copy(), dR.copy()
    B = alpha * lam * A @ A + np.eye(4) / (alpha * lam)
    for l in range(1, k + 1):
        Fh = A @ (uL + uR) / 2 - B @ (uR - uL) / 4
        if l < k:
            uL, uR = uL - lam * (Fh - A @ uL), uR - lam * (A @ uR - Fh)
    np.testing.assert_allclose(F - F0, Fh, rtol=0, atol=1e-5 * eps)


def test_predictor_coefficient_ablation(ora):
    """Reading Q2 and its alternative (alpha dt/dx in the MUSTA predictor).

    k = 1 has no predictor step, so both readings give the same flux.  For the
    linearised problem about rest both readings converge, as k grows, to the
    same flux, the alternative in fewer stages; that limit has less viscosity
    than the upwind (Godunov) flux, so neither reading turns MUSTA into an
    exact Riemann solver."""
    cs = math.sqrt(1.0 / 3.0)
    d = 1e-7
    UL = np.array([1.0 + d, 0.0, 0.0, 0.0]).reshape(4, 1)
    UR = np.array([1.0, 0.0, 0.0, 0.0]).reshape(4, 1)

    def mass_flux(k, alt, lam=0.3):
        return float(ora.musta(ora.Problem(k=k, predictor_alpha=alt), 0, lam, UL, UR)[0, 0])

    assert mass_flux(1, False) == mass_flux(1, True)
    lim_lit, lim_alt = mass_flux(256, False), mass_flux(256, True)
    assert abs(lim_lit - lim_alt) <= 1e-6 * abs(lim_alt)   # rounding of a flux of O(d)
    assert abs(mass_flux(8, True) - lim_alt) < 0.1 * abs(mass_flux(8, False) - lim_lit)
    upwind = 0.5 * cs * d
    assert 0.7 < lim_alt / upwind < 0.9


def test_totals_are_compensated_sums(ora):
    """sum(U) dV by compensated summation: equal to the exactly rounded sum (math.fsum)
    even for terms of wildly mixed magnitude and sign, where naive summation fails."""
    rng = np.random.default_rng(11)
    n = (17, 9, 5)
    U = rng.normal(size=(4,) + n[::-1]) * np.exp(rng.uniform(-30, 30, size=(4,) + n[::-1]))
    U[0, 0, 0, 0], U[0, 1, 0, 0] = 1e300, -1e300   # exact cancellation of the two largest terms
    dx = (0.1, 0.2, 0.3)
    T = ora.totals(ora.Problem(n=n, dx=dx), U)
    dV = dx[0] * dx[1] * dx[2]
    for c in range(4):
        exact = math.fsum(U[c].ravel().tolist()) * dV
        assert abs(T[c] - exact) <= 4e-16 * abs(exact), (c, T[c], exact)
