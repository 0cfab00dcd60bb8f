"""CPU reference of the con2prim-seed MLP (test infrastructure only).

A 2 -> H -> H -> 1 network with tanh hidden layers, evaluated in float64 with
the same bfloat16 rounding points as the GPU kernels, so that GPU outputs and
gradients can be compared element by element:

    z1 = bf(W1) x + b1,          h1 = tanh(z1),      h1b = bf(h1)
    z2 = bf(W2) h1b + b2,        h2 = tanh(z2)
    y  = bf(w3) . h2 + b3
    loss = mean((y - t)^2)

Backward (the mean squared error over the batch):

    dy  = 2 (y - t) / B
    dw3 = sum dy h2,             db3 = sum dy
    dz2 = dy bf(w3) (1 - h2^2),  dz2b = bf(dz2)
    dW2 = sum dz2b h1b^T,        db2 = sum dz2
    dz1 = (bf(W2)^T dz2b) (1 - h1^2)
    dW1 = sum dz1 x^T,           db1 = sum dz1

bf() rounds to the nearest bfloat16 (ties to even).  With round=False the
network is the plain float64 one (used for finite-difference checks).

grad_magnitudes() gives, for every gradient element, the sum of the absolute
values of the terms it sums (the scale of its rounding error), and adam() is
one Adam step (Kingma and Ba 2015, Algorithm 1) in float64.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round float values to the nearest bfloat16, ties to even (returned as float64)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def init_params(hidden=64, seed=0):
    """Glorot-uniform weights, zero biases (float64 masters)."""
    rng = np.random.default_rng(seed)

    def glorot(n_out, n_in):
        a = np.sqrt(6.0 / (n_in + n_out))
        return rng.uniform(-a, a, size=(n_out, n_in))

    return {"W1": glorot(hidden, 2), "b1": np.zeros(hidden), "W2": glorot(hidden, hidden), "b2": np.zeros(hidden),
            "w3": glorot(1, hidden)[0], "b3": 0.0}


def forward(P, X, rnd=True):
    """X: (B, 2) normalised inputs -> (y (B,), cache)."""
    r = bf16 if rnd else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, w3 = r(P["W1"]), r(P["W2"]), r(P["w3"])
    z1 = X @ W1.T + P["b1"]
    h1 = np.tanh(z1)
    h1b = r(h1)
    z2 = h1b @ W2.T + P["b2"]
    h2 = np.tanh(z2)
    y = h2 @ w3 + P["b3"]
    return y, dict(X=X, h1=h1, h1b=h1b, h2=h2, W2=W2, w3=w3)


def loss_and_grads(P, X, t, rnd=True):
    y, c = forward(P, X, rnd)
    B = X.shape[0]
    r = bf16 if rnd else (lambda a: np.asarray(a, dtype=np.float64))
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = float(dy.sum())
    dz2 = (dy[:, None] * c["w3"][None, :]) * (1.0 - c["h2"] ** 2)
    dz2b = r(dz2)
    g["W2"] = dz2b.T @ c["h1b"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2b @ c["W2"]) * (1.0 - c["h1"] ** 2)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return loss, g, y


def grad_magnitudes(P, X, t, rnd=True):
    """Per gradient element, the sum over the batch of |term| of the sum that defines it
    (the same structure as loss_and_grads, on absolute values)."""
    y, c = forward(P, X, rnd)
    B = X.shape[0]
    r = bf16 if rnd else (lambda a: np.asarray(a, dtype=np.float64))
    ady = np.abs(2.0 * (y - t) / B)
    s = {}
    s["w3"] = np.abs(c["h2"]).T @ ady
    s["b3"] = float(ady.sum())
    dz2 = (2.0 * (y - t)[:, None] / B * c["w3"][None, :]) * (1.0 - c["h2"] ** 2)
    adz2b = np.abs(r(dz2))
    s["W2"] = adz2b.T @ np.abs(c["h1b"])
    s["b2"] = np.abs(dz2).sum(axis=0)
    adz1 = (adz2b @ np.abs(c["W2"])) * (1.0 - c["h1"] ** 2)
    s["W1"] = adz1.T @ np.abs(X)
    s["b1"] = adz1.sum(axis=0)
    return s


def adam(P, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on flat float64 arrays: returns (P, m, v) after it.
    m <- beta1 m + (1 - beta1) g;  v <- beta2 v + (1 - beta2) g^2;
    P <- P - lr m_hat / (sqrt(v_hat) + eps), m_hat = m / (1 - beta1^step), v_hat = v / (1 - beta2^step)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return P - lr * mhat / (np.sqrt(vhat) + eps), m, v
