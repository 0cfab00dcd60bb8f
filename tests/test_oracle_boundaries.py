"""Pins for the oracle's boundary handling (two ghost layers per side).

The ghost rule is fixed against explicit padding with numpy: the flux
divergence L(U) of a grid with outflow (zero-gradient copy of the edge cell)
or periodic (wrap) boundaries must equal, cell for cell and bitwise, that of
the grid padded by two cells per side with np.pad(mode="edge") or
np.pad(mode="wrap"), restricted to the original cells (the stencil of a cell
reaches two cells out, so the padded grid's own boundaries never matter).
A mirror ghost (U_-2 = U_1) gives the same result as the copy under every
limiter with phi(a, 0) = 0, so the unlimited (central) reconstruction is
included: it tells the two apart.

A wave leaving the box: the shock of the tube leaves through x = 10, and the
interior then matches the same run on a box three times wider (whose faces
stay quiet) until the small reflection of the zero-gradient boundary arrives.
"""
import numpy as np
import pytest

from paper_1510_06340_amd import inputs as I


def random_state(rng, n, mfrac=0.6):
    U = np.zeros((4,) + tuple(n[::-1]))
    U[0] = 1.0 + rng.uniform(0, 4, size=n[::-1])
    U[1:] = rng.uniform(-1, 1, size=(3,) + tuple(n[::-1])) * (mfrac / np.sqrt(3)) * U[0]
    return U


def pad(U, bc):
    """Two ghost cells per side along each axis (array axes are z, y, x)."""
    widths = [(0, 0)] + [(2, 2)] * 3
    V = U
    for ax in range(3):                      # grid axis ax = array axis 3 - ax
        w = [(0, 0)] * 4
        w[3 - ax] = (2, 2)
        V = np.pad(V, w, mode="wrap" if bc[ax] == I.BC_PERIODIC else "edge")
    assert V.shape[1:] == tuple(s + 4 for s in U.shape[1:])
    del widths
    return V


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (0, 1, 0), (1, 0, 1)])
@pytest.mark.parametrize("lim", [I.LIM_NONE, I.LIM_MC, I.LIM_VANALBADA])
def test_ghost_rule_equals_explicit_padding(ora, bc, lim):
    rng = np.random.default_rng(100 + 7 * lim + bc[0] + 2 * bc[1])
    n = (7, 5, 4)
    U = random_state(rng, n)
    prob = ora.Problem(n=n, dx=(0.1, 0.2, 0.15), bc=bc, limiter=lim, k=3)
    L, _ = ora.rhs(prob, U, 0.0, 0.02)
    P = pad(U, bc)
    ne = tuple(s + 4 for s in n)
    for pbc in ((0, 0, 0), (1, 1, 1)):        # the padded grid's own boundary rule is irrelevant
        probe = ora.Problem(n=ne, dx=(0.1, 0.2, 0.15), bc=pbc, limiter=lim, k=3)
        Lp, _ = ora.rhs(probe, P, 0.0, 0.02)
        assert np.array_equal(L, Lp[:, 2:-2, 2:-2, 2:-2]), (bc, lim, pbc)


def test_ghost_rule_on_one_and_two_cell_lines(ora):
    """Lines shorter than the stencil: the padding repeats the single cell, or wraps twice."""
    rng = np.random.default_rng(7)
    for n in ((1, 3, 2), (2, 1, 3), (3, 2, 1)):
        U = random_state(rng, n)
        for bc in ((0, 1, 0), (1, 0, 1)):
            prob = ora.Problem(n=n, dx=(0.1, 0.1, 0.1), bc=bc, limiter=I.LIM_NONE, k=2)
            L, _ = ora.rhs(prob, U, 0.0, 0.02)
            P = pad(U, bc)
            ne = tuple(s + 4 for s in n)
            Lp, _ = ora.rhs(ora.Problem(n=ne, dx=(0.1, 0.1, 0.1), bc=(1, 1, 1), limiter=I.LIM_NONE, k=2),
                            P, 0.0, 0.02)
            assert np.array_equal(L, Lp[:, 2:-2, 2:-2, 2:-2]), (n, bc)


def test_shock_leaves_through_the_outflow_face(ora):
    """Shock tube on [-10, 10] run to t = 13.5 (the shock, at speed 0.752, left at t = 13.3)
    against the same run on [-30, 30]: the interior [-9, 9] agrees to 1e-7 of the local E.
    A reflecting face would send the shock back (an O(1) difference)."""
    def run(nx, xlo, steps):
        w = I.shock_workload(nx=nx, ny=1, nz=1, dx=0.1, steps=steps)
        w.xlo = (xlo, -0.05, -0.05)
        U = I.at_rest(I.shock_tube_energy(w.n, w.dx, w.xlo))
        V, st = ora.step(ora.Problem.from_workload(w), U, w.dt, steps)
        return I.cell_centres(nx, 0.1, xlo), V, st
    x1, V1, st1 = run(200, -10.0, 450)
    x2, V2, _ = run(600, -30.0, 450)
    np.testing.assert_allclose(x2[200:400], x1, atol=1e-12)
    W = V2[..., 200:400]
    m = (x1 > -9.0) & (x1 < 9.0)
    err = (np.abs(V1[:, 0, 0, m] - W[:, 0, 0, m]) / W[0, 0, 0, m]).max()
    assert err <= 1e-7
    # the shock has left the narrow box: its right part holds the post-shock plateau
    # (E* = 4.2846, M* = 2.4704 of the exact solution) to 0.5%, not the right state (1, 0)
    right = (x1 > 5.0) & (x1 < 9.0)
    np.testing.assert_allclose(V1[0, 0, 0, right], 4.284551332569, rtol=5e-3)
    np.testing.assert_allclose(V1[1, 0, 0, right], 2.470361591409, rtol=5e-3)
    assert st1["n_bad"] == 0
