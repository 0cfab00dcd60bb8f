"""The sampled-block oracle used by the full-size GPU parity tests (tests/helpers.py):
on grids the full oracle finishes quickly, the block result equals the full run's
cells bitwise -- interior blocks, blocks on faces and corners, for RK2 and RK3 (a
larger domain of dependence) -- and to 1e-13 with the jet source."""
import numpy as np
import pytest

import oracle
from paper_1510_06340_amd import inputs as I
from helpers import oracle_block


@pytest.mark.parametrize("rk,nsteps", [(2, 3), (3, 2)])
def test_block_equals_full_run(rk, nsteps):
    w = I.hotspot_workload(n=40, box=8.0, steps=nsteps, rk=rk)
    U = I.initial_state(w)
    x0 = (-1.0, 0.4, -0.3)
    w.jet = dict(v=0.999, dedx=5.0, sigma=0.3)
    full, _ = oracle.step(oracle.Problem.from_workload(w, jet_x0=x0), U, w.dt, nsteps, 0.2)
    for lo, size in (((16, 14, 12), (6, 7, 8)), ((0, 0, 0), (5, 5, 5)), ((33, 0, 30), (7, 9, 10)),
                     ((10, 35, 2), (20, 5, 3))):
        blk, sl = oracle_block(w, U, lo, size, nsteps, jet_x0=x0, t0=0.2)
        ref = full[(slice(None),) + sl]
        # the jet's cell centres are formed from the block's corner (an ulp of rounding)
        assert (np.abs(blk - ref) / ref[0]).max() <= 1e-13, (lo, size)
    w.jet = None
    full, _ = oracle.step(oracle.Problem.from_workload(w), U, w.dt, nsteps)
    for lo, size in (((16, 14, 12), (6, 7, 8)), ((0, 0, 0), (5, 5, 5)), ((33, 0, 30), (7, 9, 10))):
        blk, sl = oracle_block(w, U, lo, size, nsteps)
        assert np.array_equal(blk, full[(slice(None),) + sl]), (lo, size)


def test_block_margin_is_needed():
    """With a margin one cell short of the domain of dependence the block differs (the
    margin is not larger than it must be, so the test above is a real check)."""
    w = I.hotspot_workload(n=40, box=8.0, steps=2)
    U = I.initial_state(w)
    full, _ = oracle.step(oracle.Problem.from_workload(w), U, w.dt, 2)
    lo, size, m = (17, 17, 17), (6, 6, 6), 2 * 2 * 2 - 1
    sub = U[:, lo[2] - m:lo[2] + size[2] + m, lo[1] - m:lo[1] + size[1] + m, lo[0] - m:lo[0] + size[0] + m]
    prob = oracle.Problem(n=tuple(s + 2 * m for s in size), dx=w.dx,
                          xlo=tuple(w.xlo[d] + (lo[d] - m) * w.dx[d] for d in range(3)), bc=w.bc,
                          limiter=w.limiter, k=w.k, rk=w.rk)
    V, _ = oracle.step(prob, sub, w.dt, 2)
    inner = V[:, m:m + size[2], m:m + size[1], m:m + size[0]]
    assert not np.array_equal(inner, full[:, lo[2]:lo[2] + 6, lo[1]:lo[1] + 6, lo[0]:lo[0] + 6])
