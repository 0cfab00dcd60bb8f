"""Exact solution of the planar Riemann problem for the relativistic ideal gas
p = (gamma - 1)(e - n), both states at rest (test infrastructure only).

This is the reference for the paper's Sod shock tube (Sec. 3.2, its parameter
table: n_L = 10, p_L = 13 1/3, n_R = 1, p_R = 0), where n is the rest-frame
charge (rest-mass) density and e = n + p / (gamma - 1) the rest-frame energy
density.  With the higher pressure on the left the solution is
  left state | rarefaction fan | (n*_L, p*, v*) | contact | (n*_R, p*, v*) | shock | right state.

* Specific enthalpy h = (e + p) / n = 1 + gamma p / ((gamma - 1) n); sound
  speed cs^2 = gamma p / (n h).
* Rarefaction: isentropic, p / n^gamma fixed, and along the left-facing fan
  the Riemann invariant artanh(v) + (2 / sqrt(gamma - 1)) artanh(cs / sqrt(gamma - 1))
  is constant; inside the fan the characteristic (v - cs) / (1 - v cs) equals x / t.
* Shock into gas at rest (state a): the post-shock enthalpy h_b follows from
  the Taub adiabat h_b^2 - h_a^2 = (h_b / n_b + h_a / n_a)(p_b - p_a) with the
  EoS, the invariant mass flux from j^2 = -(p_b - p_a) / (h_b / n_b - h_a / n_a),
  the shock speed from V = j / sqrt(n_a^2 + j^2) and the post-shock velocity
  from v_b = W_s (p_b - p_a) / (j (h_a + (p_b - p_a) / n_a)), W_s = 1 / sqrt(1 - V^2)
  (the jump conditions of relativistic shocks, as in Marti and Mueller's
  exact Riemann solver, specialised to an upstream state at rest).
The plateau pressure p* is the root where the two branches give the same v*.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def enthalpy(n, p, gamma):
    return 1.0 + gamma * p / ((gamma - 1.0) * n)


def sound_speed(n, p, gamma):
    return np.sqrt(gamma * p / (n * enthalpy(n, p, gamma)))


def prim_to_cons(n, p, v, gamma):
    """(E, M, R) of a state (Sec. 2.1 relations): E = (e+p) W^2 - p, M = (e+p) W^2 v, R = n W."""
    e = n + p / (gamma - 1.0)
    W2 = 1.0 / (1.0 - v * v)
    return (e + p) * W2 - p, (e + p) * W2 * v, n * np.sqrt(W2)


class GasShockTube:
    """Exact solution for (n_L, p_L, v = 0) | (n_R, p_R, v = 0) at x = x0, p_L > p_R >= 0."""

    def __init__(self, n_left=10.0, p_left=40.0 / 3.0, n_right=1.0, p_right=0.0, gamma=5.0 / 3.0, x0=0.0):
        if not (p_left > p_right >= 0.0 and n_left > 0.0 and n_right > 0.0 and 1.0 < gamma <= 2.0):
            raise ValueError("need p_left > p_right >= 0, positive densities and 1 < gamma <= 2")
        self.nL, self.pL, self.nR, self.pR = float(n_left), float(p_left), float(n_right), float(p_right)
        self.g, self.x0 = float(gamma), float(x0)
        self.K = self.pL / self.nL ** self.g
        self.csL = float(sound_speed(self.nL, self.pL, self.g))
        f = lambda p: self.rarefaction_v(p) - self.shock(p)[0]
        self.p_star = brentq(f, self.pR + 1e-14 * self.pL, self.pL, xtol=1e-15, rtol=1e-15, maxiter=500)
        self.v_star = float(self.rarefaction_v(self.p_star))
        self.n_star_left = float(self.isentrope_n(self.p_star))
        _, self.n_star_right, self.shock_speed = self.shock(self.p_star)
        cs = float(sound_speed(self.n_star_left, self.p_star, self.g))
        self.head = -self.csL
        self.tail = (self.v_star - cs) / (1.0 - self.v_star * cs)

    # -- rarefaction
    def isentrope_n(self, p):
        return (np.asarray(p, dtype=np.float64) / self.K) ** (1.0 / self.g)

    def _B(self, cs):
        s = math.sqrt(self.g - 1.0)
        return 2.0 / s * np.arctanh(np.asarray(cs) / s)

    def rarefaction_v(self, p):
        """Velocity behind the left rarefaction at pressure p <= p_L."""
        cs = sound_speed(self.isentrope_n(p), p, self.g)
        return np.tanh(self._B(self.csL) - self._B(cs))

    # -- shock
    def shock(self, pb):
        """(v_b, n_b, V_s) behind a right-moving shock of post-shock pressure pb into the right state."""
        g, na, pa = self.g, self.nR, self.pR
        ha = float(enthalpy(na, pa, g))
        dp = pb - pa
        c = (g - 1.0) * dp / (g * pb)
        q = ha * ha + ha / na * dp
        hb = (-c + math.sqrt(c * c + 4.0 * (1.0 - c) * q)) / (2.0 * (1.0 - c))
        nb = g * pb / ((g - 1.0) * (hb - 1.0))
        j2 = -dp / (hb / nb - ha / na)
        j = math.sqrt(j2)
        V = j / math.sqrt(na * na + j2)
        Ws = 1.0 / math.sqrt(1.0 - V * V)
        vb = Ws * dp / (j * (ha + dp / na))
        return vb, nb, V

    def sample(self, x, t):
        """Return (n, p, v) at positions x and time t > 0."""
        xi = (np.asarray(x, dtype=np.float64) - self.x0) / t
        n, p, v = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
        left = xi < self.head
        fan = (xi >= self.head) & (xi < self.tail)
        plL = (xi >= self.tail) & (xi < self.v_star)
        plR = (xi >= self.v_star) & (xi < self.shock_speed)
        right = xi >= self.shock_speed
        n[left], p[left], v[left] = self.nL, self.pL, 0.0
        n[plL], p[plL], v[plL] = self.n_star_left, self.p_star, self.v_star
        n[plR], p[plR], v[plR] = self.n_star_right, self.p_star, self.v_star
        n[right], p[right], v[right] = self.nR, self.pR, 0.0
        for i in np.nonzero(fan)[0]:
            def char(pp):
                vv = float(self.rarefaction_v(pp))
                cs = float(sound_speed(self.isentrope_n(pp), pp, self.g))
                return (vv - cs) / (1.0 - vv * cs) - xi[i]
            pp = brentq(char, self.p_star, self.pL, xtol=1e-15, rtol=1e-15, maxiter=300)
            p[i] = pp
            n[i] = float(self.isentrope_n(pp))
            v[i] = float(self.rarefaction_v(pp))
        return n, p, v
