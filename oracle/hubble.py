"""Exact Hubble-like expansion for p = cs2 e (test infrastructure only).

Sec. 3.2 (the spherically symmetric test): matter expands uniformly with
v = r / t, and along each fluid line the proper time tau = sqrt(t^2 - r^2)
sets the energy density, e = e0 (tau0 / tau)^(3 (1 + cs2)) (for cs2 = 1/3
this is the tau^-4 cooling of a conformal fluid).  The solution holds for
r < t; the test starts from it inside r < t0 - 0.5 with vacuum outside, so it
stays exact in the central region until the rarefaction from the edge
arrives.
"""
from __future__ import annotations

import numpy as np


def exact(r, t, tau0=4.0, e0=1.0, cs2=1.0 / 3.0):
    """(e, |v|) at distance r < t from the centre at time t."""
    r = np.asarray(r, dtype=np.float64)
    tau = np.sqrt(t * t - r * r)
    return e0 * (tau0 / tau) ** (3.0 * (1.0 + cs2)), r / t
