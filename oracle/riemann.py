"""Exact solution of the planar Riemann problem for p = cs2 * e, both states at rest.

Test infrastructure only (reference for the shock-tube check of the scheme,
Sec. 3.2 "Sod shock tube": a left rarefaction and a right-moving shock).

With the high-energy state on the left, the solution is
  left state | rarefaction fan | uniform plateau (e*, v*) | shock | right state.

* Across the left-going rarefaction the Riemann invariant
  artanh(v) + (cs / (1 + cs2)) ln e is constant, so
  v(e) = tanh((cs / (1 + cs2)) ln(e_L / e)); inside the fan the
  characteristic (v - cs)/(1 - v cs) equals x/t.
* Across the shock into fluid at rest the relative velocity obeys
  v^2 = (p* - p_R)(e* - e_R) / ((e_R + p*)(e* + p_R)),
  and the shock speed follows from the energy jump, V = M* / (E* - E_R).
The plateau energy e* is the root where the two branches give the same v.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def prim_to_cons(e, v, cs2):
    """E = (e+p) g^2 - p, M = (e+p) g^2 v (Sec. 2.1, relations for E and M_i)."""
    p = cs2 * e
    g2 = 1.0 / (1.0 - v * v)
    return (e + p) * g2 - p, (e + p) * g2 * v


def rarefaction_velocity(e, e_left, cs2):
    cs = math.sqrt(cs2)
    return np.tanh(cs / (1.0 + cs2) * np.log(e_left / e))


def shock_velocity(e_star, e_right, cs2):
    p_s, p_r = cs2 * e_star, cs2 * e_right
    v2 = (p_s - p_r) * (e_star - e_right) / ((e_right + p_s) * (e_star + p_r))
    return math.sqrt(max(v2, 0.0))


class ShockTube:
    """Exact solution for (e_left, 0) | (e_right, 0) with e_left > e_right at x = x0, t = 0."""

    def __init__(self, e_left=10.0, e_right=1.0, cs2=1.0 / 3.0, x0=0.0):
        if not e_left > e_right > 0.0:
            raise ValueError("need e_left > e_right > 0")
        self.eL, self.eR, self.cs2, self.x0 = float(e_left), float(e_right), float(cs2), float(x0)
        self.cs = math.sqrt(cs2)
        f = lambda es: rarefaction_velocity(es, self.eL, cs2) - shock_velocity(es, self.eR, cs2)
        self.e_star = brentq(f, self.eR * (1 + 1e-15), self.eL, xtol=1e-15, rtol=1e-15, maxiter=500)
        self.v_star = float(rarefaction_velocity(self.e_star, self.eL, cs2))
        E, M = prim_to_cons(self.e_star, self.v_star, cs2)
        self.E_star, self.M_star = float(E), float(M)
        self.shock_speed = self.M_star / (self.E_star - self.eR)
        self.head = -self.cs
        self.tail = (self.v_star - self.cs) / (1.0 - self.v_star * self.cs)

    def momentum_jump_speed(self):
        """Shock speed from the momentum jump, V = (T^xx* - p_R) / M* (must equal shock_speed)."""
        p_s = self.cs2 * self.e_star
        Txx = (self.e_star + p_s) * self.v_star ** 2 / (1.0 - self.v_star ** 2) + p_s
        return (Txx - self.cs2 * self.eR) / self.M_star

    def sample(self, x, t):
        """Return (e, v) at positions x and time t > 0."""
        xi = (np.asarray(x, dtype=np.float64) - self.x0) / t
        e = np.empty_like(xi)
        v = np.empty_like(xi)
        left = xi < self.head
        fan = (xi >= self.head) & (xi < self.tail)
        plat = (xi >= self.tail) & (xi < self.shock_speed)
        right = xi >= self.shock_speed
        e[left], v[left] = self.eL, 0.0
        vf = (xi[fan] + self.cs) / (1.0 + xi[fan] * self.cs)
        v[fan] = vf
        # invert v = tanh(a ln(eL/e)), a = cs/(1+cs2)
        a = self.cs / (1.0 + self.cs2)
        e[fan] = self.eL * np.exp(-np.arctanh(vf) / a)
        e[plat], v[plat] = self.e_star, self.v_star
        e[right], v[right] = self.eR, 0.0
        return e, v
