"""The CPU reference of the seed network: analytic gradients against central finite differences."""
import numpy as np
import pytest

from oracle import mlp


@pytest.mark.parametrize("seed", [0, 1])
def test_reference_gradients_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    P = mlp.init_params(64, seed)
    for k in ("b1", "b2"):
        P[k] = rng.normal(size=64) * 0.1
    P["b3"] = 0.3
    X = rng.normal(size=(37, 2))
    t = rng.normal(size=37)
    _, g, _ = mlp.loss_and_grads(P, X, t, rnd=False)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        base = np.array(P[name], dtype=np.float64)
        flat = base.reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            for sgn, store in ((1, "p"), (-1, "m")):
                pert = flat.copy()
                pert[i] += sgn * h
                Q = dict(P)
                Q[name] = pert.reshape(base.shape) if base.shape else float(pert[0])
                val, _, _ = mlp.loss_and_grads(Q, X, t, rnd=False)
                if store == "p":
                    lp = val
                else:
                    lm = val
            fd = (lp - lm) / (2 * h)
            an = np.asarray(g[name], dtype=np.float64).reshape(-1)[i]
            assert an == pytest.approx(fd, rel=1e-6, abs=1e-9), (name, i)


def test_bf16_rounding_is_round_to_nearest_even():
    # 1 + 2^-8 lies halfway between the bfloat16 neighbours 1 and 1 + 2^-7: ties go to the even (1.0)
    assert mlp.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert mlp.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    assert mlp.bf16(np.array([-2.5]))[0] == -2.5
    x = np.random.default_rng(0).normal(size=1000)
    assert np.all(np.abs(mlp.bf16(x) - x) <= 2 ** -8 * np.abs(x))  # half an ulp of 8 significant bits
