"""Training of the learned con2prim seed (crossover EoS) with the library's own kernels.

1. States: crossover-EoS runs of the hot-spot (seed 2), jet (seed 3, with its
   source) and ensemble (seeds 1000+j) workloads at reduced resolution are
   advanced on the GPU; the cell states (E, |M|) of snapshots taken every few
   steps form the stream from which ``n_samples`` states with 0 < |M| < E are
   reservoir-sampled (random keys from a seeded generator, smallest keys kept).
2. Labels: e and p from the plain bracketed-Newton con2prim (mf_con2prim, MF_C2P_PLAIN).
3. Network: 2 -> 64 -> 64 -> 1 tanh on x = ((ln E, |M|/E) - mean) / std,
   predicting the standardised ln e (as configured) or, optionally, the
   root's position in the bracket [E(1 - m^2), E]; trained with Adam on the mean squared
   error by the BF16 matrix-core kernels (mf_mlp_grad / mf_mlp_adam), 90/10
   train/validation split.

Every numerical step runs in libmf.so; this module only moves tensors around.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs as I
from . import mf


def _glorot(rng, n_out, n_in):
    a = math.sqrt(6.0 / (n_in + n_out))
    return rng.uniform(-a, a, size=(n_out, n_in))


def init_params(seed=0) -> np.ndarray:
    """Glorot-uniform weights, zero biases, in the library's parameter layout."""
    rng = np.random.default_rng(seed)
    H = mf.MF_MLP_HIDDEN
    return np.concatenate([_glorot(rng, H, 2).ravel(), np.zeros(H), _glorot(rng, H, H).ravel(), np.zeros(H),
                           _glorot(rng, 1, H).ravel(), np.zeros(1)]).astype(np.float32)


def _workloads(n):
    table = I.crossover_table()
    hs = I.hotspot_workload(n=n, seed=2, steps=60)
    hs.eos = I.EOS_TABLE
    jt = I.jet_workload(n=n, seed=3, steps=60)
    jt.eos = I.EOS_TABLE
    ens = I.ensemble_workloads(n_events=3, steps=60)
    for w in ens:
        w.eos = I.EOS_TABLE
    return table, [hs, jt] + ens


def collect_states(n_samples=1 << 22, seed=42, n=128, snap_every=6, steps=60):
    """Reservoir sample of (E, |M|) cell states with 0 < |M| < E from crossover-EoS runs (torch CUDA float64)."""
    import torch
    table, ws = _workloads(n)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    keys = torch.empty(0, device="cuda", dtype=torch.float64)
    E_s = torch.empty(0, device="cuda", dtype=torch.float64)
    M_s = torch.empty(0, device="cuda", dtype=torch.float64)
    for w in ws:
        U = I.initial_state(w)
        dev = [torch.from_numpy(np.ascontiguousarray(U[c]).ravel()).cuda() for c in range(4)]
        g = mf.Grid([mf.desc_from_workload(w)], [dev])
        g.set_eos_table(*table)
        if w.jet is not None:
            g.set_jet(0, I.jet_start(w), w.jet["v"], w.jet["dedx"], w.jet["sigma"])
        for _ in range(steps // snap_every):
            g.step(w.dt, snap_every, stats=False)
            Mabs = torch.sqrt(dev[1] ** 2 + dev[2] ** 2 + dev[3] ** 2)
            # states the solver sees as they are: moving and subluminal (the guards
            # clamp |M| >= E, whose root e << E would be a far outlier of ln e)
            sel = (Mabs > 0) & (Mabs < dev[0])
            k = torch.rand(int(sel.sum()), generator=gen, device="cuda", dtype=torch.float64)
            keys = torch.cat([keys, k])
            E_s = torch.cat([E_s, dev[0][sel]])
            M_s = torch.cat([M_s, Mabs[sel]])
            if keys.numel() > n_samples:
                idx = torch.topk(keys, n_samples, largest=False).indices
                keys, E_s, M_s = keys[idx], E_s[idx], M_s[idx]
        torch.cuda.synchronize()
        g.free()
    order = torch.argsort(keys)
    return E_s[order], M_s[order]


def label_states(E, Mabs, table=None):
    """Plain bracketed-Newton con2prim of states (E, |M| along x): returns (e, p) (torch float64)."""
    import torch
    table = I.crossover_table() if table is None else table
    n = E.numel()
    U = [E.contiguous(), Mabs.contiguous(), torch.zeros_like(E), torch.zeros_like(E)]
    prim = [torch.empty_like(E) for _ in range(5)]
    g = mf.Grid([mf.make_desc((n, 1, 1), (1, 1, 1), (0, 0, 0), (0, 0, 0))], [U])
    g.set_eos_table(*table)
    g.con2prim(U, prim)
    torch.cuda.synchronize()
    g.free()
    return prim[0], prim[1]


class Trained:
    def __init__(self, params, norm, history, output):
        self.params = params        # numpy float32 (MF_MLP_PARAMS,)
        self.norm = norm            # dict in_shift, in_scale, out_shift, out_scale
        self.history = history      # list of (epoch, train_loss, val_loss)
        self.output = output        # 0: ln e, 1: bracket fraction (E - e) E / |M|^2

    def network(self) -> mf.SeedNetwork:
        n = self.norm
        return mf.SeedNetwork(self.params, n["in_shift"], n["in_scale"], n["out_shift"], n["out_scale"], self.output)

    def predict_e(self, E, Mabs, y):
        """Guess e from the network output y (standardised)."""
        n = self.norm
        pred = y.double() * n["out_scale"] + n["out_shift"]
        if self.output == 1:
            return E - pred * Mabs * Mabs / E
        import torch
        return torch.exp(pred)


def train(E, Mabs, e, p, epochs=30, batch=4096, lr=2e-3, lr_min=2e-5, seed=0, val_frac=0.1, output=0):
    """Fit the seed from (ln E, |M|/E) with the matrix-core kernels; returns a Trained network.

    (e, p) are the labels from label_states.  output 0: the target is ln e (as
    configured); output 1: the target is the position of the root in the
    bracket [E(1 - m^2), E], phi = (E - e) E / |M|^2.  At the root
    E - e = |M|^2 / (E + p), so phi = E / (E + p), which is taken in that form
    (no cancellation near rest)."""
    import torch
    x0 = torch.log(E)
    x1 = Mabs / E
    y = torch.log(e) if output == 0 else E / (E + p)
    mu = [float(x0.mean()), float(x1.mean())]
    sd = [float(x0.std()), float(x1.std())]
    ym, ys = float(y.mean()), float(y.std())
    X = torch.stack([(x0 - mu[0]) / sd[0], (x1 - mu[1]) / sd[1]], dim=1).float().contiguous()
    T = ((y - ym) / ys).float().contiguous()
    n = X.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    perm = torch.randperm(n, generator=gen, device="cuda")
    nval = int(n * val_frac)
    Xv, Tv = X[perm[:nval]].contiguous(), T[perm[:nval]].contiguous()
    Xt, Tt = X[perm[nval:]].contiguous(), T[perm[nval:]].contiguous()
    P = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    grad = torch.zeros_like(P)
    loss = torch.zeros(1, device="cuda")
    work = torch.empty(mf.mlp_workspace(batch), device="cuda")
    nb = Xt.shape[0] // batch
    step = 0
    history = []
    yv = torch.empty(nval, device="cuda")
    for ep in range(epochs):
        order = torch.randperm(Xt.shape[0], generator=gen, device="cuda")
        Xs, Ts = Xt[order].contiguous(), Tt[order].contiguous()
        tr = torch.zeros((), device="cuda")
        for b in range(nb):
            step += 1
            frac = step / (epochs * nb)
            cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * frac))
            xb = Xs[b * batch:(b + 1) * batch]
            tb = Ts[b * batch:(b + 1) * batch]
            mf.mlp_grad(P, xb, tb, grad, loss, work)
            mf.mlp_adam(P, grad, m, v, step, cur)
            tr += loss[0]
        mf.mlp_forward(P, Xv, yv)
        vl = float(((yv - Tv) ** 2).mean())
        history.append((ep, float(tr) / max(nb, 1), vl))
    norm = dict(in_shift=mu, in_scale=[1.0 / sd[0], 1.0 / sd[1]], out_shift=ym, out_scale=ys)
    return Trained(P.cpu().numpy(), norm, history, output)


def relative_error(trained: Trained, E, Mabs, e):
    """|guess - e| / e on the given states (network via mf_mlp_forward)."""
    import torch
    n = trained.norm
    X = torch.stack([(torch.log(E) - n["in_shift"][0]) * n["in_scale"][0],
                     (Mabs / E - n["in_shift"][1]) * n["in_scale"][1]], dim=1).float().contiguous()
    y = torch.empty(X.shape[0], device="cuda")
    P = torch.from_numpy(trained.params).cuda()
    mf.mlp_forward(P, X, y)
    return (trained.predict_e(E, Mabs, y) - e).abs() / e
