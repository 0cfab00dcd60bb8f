"""Seeded synthetic inputs shared by the HIP path, the oracle and the bench.

This module holds none of the numerical method's steps: it draws random
numbers, lays out grids, builds initial energy-density fields of fluid at rest
(for v = 0 the conserved variables are E = e, M = 0), the exact Hubble-like
and ellipsoidal states (whose conserved variables it forms from e, n and v by
the standard relations E = (e + p) g^2 - p, M = (e + p) g^2 v, R = n g,
g^2 = 1 / (1 - v^2); tests check them against the oracle's inverse) and tabulates the crossover equation
of state, whose pressure is an input to the method.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) with the usual 53-bit mapping to
[0, 1) and the cosine branch of the Box-Muller transform.

Workloads (the paper's experiments use heavy-ion initial-condition generators
that are not available; seeded Gaussian hot spots stand in for them):

* ``shock``     200x16x16 planar shock tube along x (e = 10 | 1, v = 0),
                minmod, k = 2, RK2, dt = 0.03, 100 steps.
* ``hotspot``   256^3 on [-12.8, 12.8]^3, 40 Gaussian hot spots on e = 0.1,
                MC, k = 3, RK2, dt = 0.03, 200 steps, FP64 and FP32.
* ``jet``       512^3 on the same box (dx = 0.05), hot spots plus a moving
                point-jet source, superbee, k = 3, dt = 0.015, 150 steps.
* ``ensemble``  64 events with per-axis sizes drawn from {96, 112, ..., 192},
                dx = 0.1, hot spots, MC, k = 3, dt = 0.03, 100 steps.
* ``crossover`` 32 events of 192^3 under the tabulated crossover EoS.
* ``sod``       the paper's Sod tube of the ideal gas with the conserved
                charge: 500 cells of 0.02 along x, RK3, k = 4, 800 steps.
* ``ellipsoidal`` the paper's ellipsoidal flow of pressureless dust with the
                charge: 120^3 cells of 0.1 from t = 2, RK3, k = 4, 50 steps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1

# Boundary condition, limiter and EoS codes (the same integers as the C ABI).
BC_OUTFLOW, BC_PERIODIC = 0, 1
LIM_NONE, LIM_MINMOD, LIM_SUPERBEE, LIM_MC, LIM_VANLEER, LIM_VANALBADA = range(6)
LIMITER_NAMES = {
    "none": LIM_NONE, "minmod": LIM_MINMOD, "superbee": LIM_SUPERBEE,
    "mc": LIM_MC, "vanleer": LIM_VANLEER, "vanalbada": LIM_VANALBADA,
}
EOS_IDEAL, EOS_TABLE = 0, 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea, Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def normal(self) -> float:
        """Standard normal deviate, cosine branch of Box-Muller."""
        u1 = self.uniform()
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)


@dataclass
class HotSpots:
    centres: np.ndarray          # (n, 3) x, y, z
    amplitudes: np.ndarray       # (n,)
    sizes: tuple | None = None   # per-event grid size (ensemble workload)
    jet_yz: tuple | None = None  # transverse jet position (jet workload)


def draw_event(seed: int, n_spots: int = 40, ball_radius: float = 5.0,
               median: float = 5.0, log_sd: float = 0.5,
               draw_sizes: bool = False, draw_jet: bool = False,
               size_choices=tuple(range(96, 193, 16))) -> HotSpots:
    """Draw one event's random parameters in a fixed order.

    Order: grid sizes (Nx, Ny, Nz) if requested; then per hot spot a centre
    (rejection sampling in the cube [-R, R]^3 until inside the ball) and a
    normal deviate Z giving the amplitude median * exp(log_sd * Z); then the
    jet's transverse position (rejection in the disc of radius R).
    """
    rng = SplitMix64(seed)
    sizes = None
    if draw_sizes:
        m = len(size_choices)
        sizes = tuple(size_choices[min(int(rng.uniform() * m), m - 1)] for _ in range(3))
    centres = np.zeros((n_spots, 3))
    amps = np.zeros(n_spots)
    for k in range(n_spots):
        while True:
            c = [-ball_radius + 2.0 * ball_radius * rng.uniform() for _ in range(3)]
            if c[0] * c[0] + c[1] * c[1] + c[2] * c[2] <= ball_radius * ball_radius:
                break
        centres[k] = c
        amps[k] = median * math.exp(log_sd * rng.normal())
    jet = None
    if draw_jet:
        while True:
            y0 = -ball_radius + 2.0 * ball_radius * rng.uniform()
            z0 = -ball_radius + 2.0 * ball_radius * rng.uniform()
            if y0 * y0 + z0 * z0 <= ball_radius * ball_radius:
                break
        jet = (y0, z0)
    return HotSpots(centres, amps, sizes, jet)


def cell_centres(n: int, dx: float, xlo: float) -> np.ndarray:
    """Cell-centre coordinates xlo + (i + 1/2) dx, i = 0..n-1."""
    return xlo + (np.arange(n, dtype=np.float64) + 0.5) * dx


def hotspot_energy(n, dx, xlo, spots: HotSpots, width: float = 0.4,
                   background: float = 0.1) -> np.ndarray:
    """e(x) = background + sum_k A_k exp(-|x - c_k|^2 / (2 width^2)), shape (nz, ny, nx).

    The Gaussian factorises over the axes, so each z-slab is a small matrix
    product of per-axis factors (fixed order, deterministic).
    """
    nx, ny, nz = n
    xs = cell_centres(nx, dx[0], xlo[0])
    ys = cell_centres(ny, dx[1], xlo[1])
    zs = cell_centres(nz, dx[2], xlo[2])
    s = 1.0 / (2.0 * width * width)
    c = spots.centres
    gx = np.exp(-s * (xs[None, :] - c[:, 0:1]) ** 2)          # (K, nx)
    gy = np.exp(-s * (ys[None, :] - c[:, 1:2]) ** 2)          # (K, ny)
    gz = np.exp(-s * (zs[None, :] - c[:, 2:3]) ** 2)          # (K, nz)
    gyA = gy * spots.amplitudes[:, None]                       # (K, ny)
    e = np.empty((nz, ny, nx))
    for kz in range(nz):
        b = (gyA * gz[:, kz:kz + 1]).T                         # (ny, K)
        e[kz] = background + b @ gx
    return e


def shock_tube_energy(n, dx, xlo, e_left=10.0, e_right=1.0) -> np.ndarray:
    """Planar Riemann data along x: e_left where the cell centre x < 0."""
    nx, ny, nz = n
    xs = cell_centres(nx, dx[0], xlo[0])
    row = np.where(xs < 0.0, e_left, e_right)
    return np.broadcast_to(row, (nz, ny, nx)).copy()


def hubble_state(n, dx, xlo, t0=2.0, tau0=4.0, e0=1.0, cs2=1.0 / 3.0, edge=0.5) -> np.ndarray:
    """Hubble-like expansion (Sec. 3.2, the spherically symmetric test): v = r / t0 and
    e = e0 (tau0 / sqrt(t0^2 - r^2))^(3 (1 + cs2)) for r < t0 - edge, vacuum (e = v = 0)
    outside; conserved state (4, nz, ny, nx) at the cell centres."""
    nx, ny, nz = n
    x = cell_centres(nx, dx[0], xlo[0])[None, None, :]
    y = cell_centres(ny, dx[1], xlo[1])[None, :, None]
    z = cell_centres(nz, dx[2], xlo[2])[:, None, None]
    r2 = x * x + y * y + z * z
    inside = r2 < (t0 - edge) ** 2
    tau = np.sqrt(np.where(inside, t0 * t0 - r2, 1.0))
    e = np.where(inside, e0 * (tau0 / tau) ** (3.0 * (1.0 + cs2)), 0.0)
    p = cs2 * e
    g2 = np.where(inside, 1.0 / (1.0 - r2 / (t0 * t0)), 1.0)
    w = (e + p) * g2
    U = np.zeros((4, nz, ny, nx))
    U[0] = w - p
    U[1] = np.where(inside, w * x / t0, 0.0)
    U[2] = np.where(inside, w * y / t0, 0.0)
    U[3] = np.where(inside, w * z / t0, 0.0)
    return U


def at_rest(e: np.ndarray) -> np.ndarray:
    """Conserved state of fluid at rest: (E, Mx, My, Mz) = (e, 0, 0, 0), shape (4, ...)."""
    U = np.zeros((4,) + e.shape)
    U[0] = e
    return U


# --------------------------------------------------------------------------
# Crossover equation of state: dp/de = 1/3 - 0.2 / (1 + (ln e / 0.5)^2),
# p(0) = 0, tabulated on log-spaced nodes.
# --------------------------------------------------------------------------

def crossover_nodes(n: int = 4096, lo_exp: float = -3.0, hi_exp: float = 3.0) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * i / (n - 1))


def _crossover_integrand(u):
    return np.exp(u) / (1.0 + 4.0 * u * u)


def crossover_table(n: int = 4096, lo_exp: float = -3.0, hi_exp: float = 3.0):
    """Return (e_i, p_i) with p(e) = e/3 - 0.2 * I(ln e), I(y) = int_{-inf}^{y} e^u/(1+4u^2) du.

    I at the first node comes from adaptive quadrature over (-inf, y0]; each
    further node adds a 24-point Gauss-Legendre integral over its interval in
    u = ln e (intervals of width ~3.4e-3, where the rule is exact to rounding).
    """
    from scipy import integrate

    e = crossover_nodes(n, lo_exp, hi_exp)
    y = np.log(e)
    i0, _ = integrate.quad(_crossover_integrand, -np.inf, y[0], epsabs=0.0, epsrel=2e-14, limit=200)
    xg, wg = np.polynomial.legendre.leggauss(24)
    a, b = y[:-1], y[1:]
    mid, half = 0.5 * (a + b), 0.5 * (b - a)
    seg = (half[:, None] * wg[None, :] * _crossover_integrand(mid[:, None] + half[:, None] * xg[None, :])).sum(axis=1)
    I = np.empty(n)
    I[0] = i0
    I[1:] = i0 + np.cumsum(seg)
    p = e / 3.0 - 0.2 * I
    return e, p


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: tuple
    dx: tuple
    xlo: tuple
    bc: tuple
    limiter: int
    k: int
    rk: int
    dt: float
    steps: int
    alpha: float = 3.0
    eos: int = EOS_IDEAL
    cs2: float = 1.0 / 3.0
    jet: dict | None = None
    seed: int | None = None
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


def shock_workload(nx: int = 200, ny: int = 16, nz: int = 16, dx: float = 0.1,
                   dt: float | None = None, steps: int | None = None,
                   limiter: int = LIM_MINMOD, k: int = 2, rk: int = 2) -> Workload:
    """Planar shock tube on x in [-nx dx/2, nx dx/2], e = 10 | 1, outflow in x, periodic in y, z."""
    dt = 0.3 * dx if dt is None else dt
    steps = int(round(3.0 / dt)) if steps is None else steps
    return Workload("shock", (nx, ny, nz), (dx, dx, dx),
                    (-0.5 * nx * dx, -0.5 * ny * dx, -0.5 * nz * dx),
                    (BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC), limiter, k, rk, dt, steps)


def hotspot_workload(n: int = 256, seed: int = 2, steps: int = 200, limiter: int = LIM_MC,
                     k: int = 3, rk: int = 2, box: float = 25.6) -> Workload:
    dx = box / n
    return Workload("hotspot", (n, n, n), (dx, dx, dx), (-0.5 * box,) * 3,
                    (BC_OUTFLOW,) * 3, limiter, k, rk, 0.3 * dx, steps, seed=seed)


def jet_workload(n: int = 512, seed: int = 3, steps: int = 150, box: float = 25.6) -> Workload:
    dx = box / n
    return Workload("jet", (n, n, n), (dx, dx, dx), (-0.5 * box,) * 3,
                    (BC_OUTFLOW,) * 3, LIM_SUPERBEE, 3, 2, 0.3 * dx, steps, seed=seed,
                    jet=dict(v=0.999, dedx=5.0, sigma=0.3, x_start=-5.0))


def ensemble_workloads(n_events: int = 64, base_seed: int = 1000, steps: int = 100):
    out = []
    for j in range(n_events):
        ev = draw_event(base_seed + j, draw_sizes=True)
        n = ev.sizes
        out.append(Workload("ensemble", n, (0.1, 0.1, 0.1), tuple(-0.05 * s for s in n),
                            (BC_OUTFLOW,) * 3, LIM_MC, 3, 2, 0.03, steps, seed=base_seed + j))
    return out


def crossover_workloads(n_events: int = 32, base_seed: int = 2000, n: int = 192, steps: int = 100):
    return [Workload("crossover", (n, n, n), (0.1, 0.1, 0.1), (-0.05 * n,) * 3,
                     (BC_OUTFLOW,) * 3, LIM_MC, 3, 2, 0.03, steps, eos=EOS_TABLE,
                     seed=base_seed + j) for j in range(n_events)]


def sod_workload(nx: int = 500, dx: float = 0.02, dt: float = 0.005, steps: int = 800,
                 limiter: int = LIM_MINMOD, k: int = 4, rk: int = 3, ny: int = 1, nz: int = 1,
                 gamma: float = 5.0 / 3.0) -> Workload:
    """The paper's Sod shock tube (Sec. 3.2 and its parameter table): 500 cells of 0.02 along x
    (x in [-5, 5], the jump at 0), dt = 0.005, charge n_L = 10 | n_R = 1 and pressure
    p_L = 13 1/3 | p_R = 0 at rest, ideal gas p = (gamma - 1)(e - n) with gamma = 5/3, carried
    with the conserved charge R; 800 steps (t = 4, where the shock is inside the box); RK3
    and 4 MUSTA stages as in the paper's experiments; outflow in x, periodic in y, z."""
    return Workload("sod", (nx, ny, nz), (dx, dx, dx), (-0.5 * nx * dx, -0.5 * ny * dx, -0.5 * nz * dx),
                    (BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC), limiter, k, rk, dt, steps,
                    extra=dict(charge=True, gamma=gamma, n=(10.0, 1.0), p=(40.0 / 3.0, 0.0)))


def sod_state(n, dx, xlo, n_lr=(10.0, 1.0), p_lr=(40.0 / 3.0, 0.0), gamma=5.0 / 3.0) -> np.ndarray:
    """Conserved state (5, nz, ny, nx) of gas at rest with the charge and pressure jump at x = 0:
    E = e = n + p / (gamma - 1), M = 0, R = n (v = 0)."""
    nx, ny, nz = n
    xs = cell_centres(nx, dx[0], xlo[0])
    left = xs < 0.0
    nn = np.where(left, n_lr[0], n_lr[1])
    pp = np.where(left, p_lr[0], p_lr[1])
    U = np.zeros((5, nz, ny, nx))
    U[0] = np.broadcast_to(nn + pp / (gamma - 1.0), (nz, ny, nx))
    U[4] = np.broadcast_to(nn, (nz, ny, nx))
    return U


def ellipsoidal_workload(n: int = 120, dx: float = 0.1, dt: float = 0.02, steps: int = 50,
                         limiter: int = LIM_MINMOD, k: int = 4, rk: int = 3) -> Workload:
    """The paper's ellipsoidal flow (Sec. 3.2 and its parameter table): 120^3 cells of 0.1
    centred on the origin, dt = 0.02, from t0 = 2 with C_e = 2, C_n = 0.75, b_e = b_n = 1,
    T = (0.4, 0.6, 0.8); pressureless (p = 0: the ideal gas with gamma = 1) with the charge;
    RK3 and 4 MUSTA stages as in the paper's experiments; 50 steps (to t = 3)."""
    return Workload("ellipsoidal", (n, n, n), (dx, dx, dx), (-0.5 * n * dx,) * 3, (BC_OUTFLOW,) * 3,
                    limiter, k, rk, dt, steps,
                    extra=dict(charge=True, gamma=1.0, t0=2.0, Ce=2.0, Cn=0.75, be=1.0, bn=1.0,
                               T=(0.4, 0.6, 0.8)))


def ellipsoidal_prim(n, dx, xlo, t, Ce=2.0, Cn=0.75, be=1.0, bn=1.0, T=(0.4, 0.6, 0.8)):
    """Rest-frame e, n and velocity (3, ...) of the ellipsoidal flow at time t at the cell centres:
    v_i = a_i x_i / t with a_i = t / (t + T_i), tau^2 = t^2 - sum_i (a_i x_i)^2,
    e = C_e exp(-b_e^2 t^2 / tau^2) / prod_i (t + T_i), n likewise with C_n, b_n; outside
    tau^2 > 0 the exponential vanishes (e = n = 0, v = 0).  (The paper prints the velocity
    components as (a_1 x, a_3 y, a_2 z) / t; with tau built from a_i x_i the consistent reading
    is a_i x_i / t for every axis.)"""
    nx, ny, nz = n
    xs = [cell_centres(nx, dx[0], xlo[0])[None, None, :], cell_centres(ny, dx[1], xlo[1])[None, :, None],
          cell_centres(nz, dx[2], xlo[2])[:, None, None]]
    a = [t / (t + Ti) for Ti in T]
    v = [np.broadcast_to(a[i] * xs[i] / t, (nz, ny, nx)) for i in range(3)]
    tau2 = t * t - t * t * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    inside = tau2 > 0.0
    ratio = np.where(inside, t * t / np.where(inside, tau2, 1.0), np.inf)
    den = (t + T[0]) * (t + T[1]) * (t + T[2])
    e = Ce / den * np.exp(-be * be * ratio)
    nn = Cn / den * np.exp(-bn * bn * ratio)
    vv = np.stack([np.where(inside, vi, 0.0) for vi in v])
    return e, nn, vv


def ellipsoidal_state(n, dx, xlo, t, **kw) -> np.ndarray:
    """Conserved state (5, nz, ny, nx) of the ellipsoidal flow at time t (p = 0):
    E = e W^2, M = e W^2 v, R = n W."""
    e, nn, v = ellipsoidal_prim(n, dx, xlo, t, **kw)
    W2 = 1.0 / (1.0 - (v ** 2).sum(0))
    U = np.empty((5,) + e.shape)
    U[0] = e * W2
    U[1:4] = (e * W2)[None] * v
    U[4] = nn * np.sqrt(W2)
    return U


def hubble_workload(n: int = 120, dx: float = 0.1, dt: float = 0.03, steps: int = 20,
                    limiter: int = LIM_MINMOD, k: int = 4, rk: int = 3) -> Workload:
    """The paper's Hubble-like expansion test (Sec. 3.2 and its parameter table): 120^3
    cells of 0.1 centred on the origin, dt = 0.03, e0 = 1, tau0 = 4, t0 = 2, p = e/3,
    vacuum beyond r = t0 - 0.5; RK3 and 4 MUSTA stages as in the paper's experiments."""
    return Workload("hubble", (n, n, n), (dx, dx, dx), (-0.5 * n * dx,) * 3, (BC_OUTFLOW,) * 3,
                    limiter, k, rk, dt, steps, extra=dict(t0=2.0, tau0=4.0, e0=1.0, edge=0.5))


def initial_state(w: Workload) -> np.ndarray:
    """Conserved FP64 state (4, nz, ny, nx) for a workload ((5, ...) with the charge R)."""
    if w.name == "shock":
        return at_rest(shock_tube_energy(w.n, w.dx, w.xlo))
    if w.name == "sod":
        x = w.extra
        return sod_state(w.n, w.dx, w.xlo, x["n"], x["p"], x["gamma"])
    if w.name == "ellipsoidal":
        x = w.extra
        return ellipsoidal_state(w.n, w.dx, w.xlo, x["t0"], Ce=x["Ce"], Cn=x["Cn"], be=x["be"], bn=x["bn"], T=x["T"])
    if w.name == "hubble":
        x = w.extra
        return hubble_state(w.n, w.dx, w.xlo, x["t0"], x["tau0"], x["e0"], w.cs2, x["edge"])
    ev = draw_event(w.seed, draw_sizes=(w.name == "ensemble"), draw_jet=(w.jet is not None))
    return at_rest(hotspot_energy(w.n, w.dx, w.xlo, ev))


def jet_start(w: Workload) -> tuple:
    """Jet position at t = 0: (x_start, y0, z0) with (y0, z0) drawn from the event seed."""
    ev = draw_event(w.seed, draw_jet=True)
    return (w.jet["x_start"], ev.jet_yz[0], ev.jet_yz[1])
