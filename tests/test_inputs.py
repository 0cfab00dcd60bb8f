"""Seeded input generators: RNG, hot spots, crossover EoS table."""
import math

import numpy as np
import pytest

from paper_1510_06340_amd import inputs as I


def test_splitmix64_reference_vector():
    # First outputs of SplitMix64 seeded with 1234567, as published with the
    # reference implementation by S. Vigna (prng.di.unimi.it, splitmix64.c).
    r = I.SplitMix64(1234567)
    assert [r.next_u64() for _ in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_uniform_and_normal_moments():
    r = I.SplitMix64(7)
    u = np.array([r.uniform() for _ in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    z = np.array([r.normal() for _ in range(20000)])
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1.0) < 0.05


def test_event_draw_is_deterministic_and_in_ball():
    a = I.draw_event(2)
    b = I.draw_event(2)
    assert np.array_equal(a.centres, b.centres) and np.array_equal(a.amplitudes, b.amplitudes)
    assert np.all(np.linalg.norm(a.centres, axis=1) <= 5.0)
    assert a.centres.shape == (40, 3)
    # the jet and the sizes are drawn after (jet) / before (sizes) the spots
    j = I.draw_event(2, draw_jet=True)
    assert np.array_equal(j.centres, a.centres) and j.jet_yz[0] ** 2 + j.jet_yz[1] ** 2 <= 25.0
    s = I.draw_event(1000, draw_sizes=True)
    assert all(v in range(96, 193, 16) for v in s.sizes)


def test_hotspot_energy_matches_direct_sum():
    w = I.hotspot_workload(n=12, box=12.0)
    ev = I.draw_event(w.seed)
    e = I.hotspot_energy(w.n, w.dx, w.xlo, ev)
    xs = I.cell_centres(12, w.dx[0], w.xlo[0])
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    ref = np.full(Z.shape, 0.1)
    for c, A in zip(ev.centres, ev.amplitudes):
        r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        ref += A * np.exp(-r2 / (2 * 0.4 ** 2))
    np.testing.assert_allclose(e, ref, rtol=1e-13, atol=1e-15)
    assert e.min() >= 0.1


def test_crossover_table_matches_quadrature():
    from scipy import integrate
    e, p = I.crossover_table()
    assert len(e) == 4096 and e[0] == pytest.approx(1e-3, rel=1e-15) and e[-1] == pytest.approx(1e3, rel=1e-13)
    f = lambda u: math.exp(u) / (1.0 + 4.0 * u * u)
    for i in [0, 1, 700, 2047, 3000, 4095]:
        I_ref, _ = integrate.quad(f, -np.inf, math.log(e[i]), epsabs=0, epsrel=2e-14, limit=400)
        assert p[i] == pytest.approx(e[i] / 3.0 - 0.2 * I_ref, rel=1e-12)
    # dp/de of the table follows the defining formula (centred differences)
    mid = slice(1, -1)
    dpde = (p[2:] - p[:-2]) / (e[2:] - e[:-2])
    ref = 1.0 / 3.0 - 0.2 / (1.0 + (np.log(e[mid]) / 0.5) ** 2)
    np.testing.assert_allclose(dpde, ref, rtol=1e-4)
    assert np.all(np.diff(p) > 0)
