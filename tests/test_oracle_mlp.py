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


def test_adam_reference_matches_torch_optimizer():
    """The float64 Adam step equals torch.optim.Adam (a library implementation of Kingma and
    Ba's Algorithm 1) over several steps with changing gradients, moments included."""
    import torch
    rng = np.random.default_rng(9)
    n = 301
    P0 = rng.normal(size=n)
    grads = [rng.normal(size=n) * s for s in (1.0, 0.3, 2.0, 0.01, 1.0, 5.0)]
    for lr, b1, b2, eps in ((1e-3, 0.9, 0.999, 1e-8), (3e-2, 0.8, 0.95, 1e-6)):
        p = torch.tensor(P0.copy(), dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([p], lr=lr, betas=(b1, b2), eps=eps)
        P, m, v = P0.copy(), np.zeros(n), np.zeros(n)
        for step, g in enumerate(grads, start=1):
            p.grad = torch.tensor(g, dtype=torch.float64)
            opt.step()
            P, m, v = mlp.adam(P, g, m, v, step, lr, b1, b2, eps)
            st = opt.state[p]
            np.testing.assert_allclose(P, p.detach().numpy(), rtol=1e-13, atol=1e-15)
            np.testing.assert_allclose(m, st["exp_avg"].numpy(), rtol=1e-12, atol=1e-16)
            np.testing.assert_allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-12, atol=1e-18)


def test_gradient_magnitudes_bound_the_gradients():
    """Each sum of |terms| bounds |gradient| (triangle inequality), with equality where every
    term has one sign (db3 when every residual y - t is positive)."""
    rng = np.random.default_rng(4)
    P = mlp.init_params(64, 4)
    X = rng.normal(size=(50, 2))
    t = rng.normal(size=50)
    _, g, _ = mlp.loss_and_grads(P, X, t)
    s = mlp.grad_magnitudes(P, X, t)
    for k in ("W1", "b1", "W2", "b2", "w3"):
        assert np.all(np.abs(g[k]) <= s[k] * (1 + 1e-12)), k
    y, _ = mlp.forward(P, X)
    _, g2, _ = mlp.loss_and_grads(P, X, y - 1.0)
    s2 = mlp.grad_magnitudes(P, X, y - 1.0)
    assert abs(g2["b3"]) == pytest.approx(s2["b3"], rel=1e-14)
