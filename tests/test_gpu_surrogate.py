"""The learned con2prim seed on the GPU.

* Forward and gradients of the BF16 matrix-core kernels against the FP64 CPU
  reference with the same rounding points, element by element; Adam steps
  with changing gradients against the FP64 Adam reference.
* Training on solver-generated crossover-EoS states lowers the loss.
* Seeded con2prim (network on the matrix cores, and the prediction grid used
  by the sweeps) equals the plain bracketed Newton to 1e-12 per state, and a
  seeded run equals a plain run to 1e-10.
* The gain: Newton iterations and time, seeded vs plain vs the conformal guess.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as ref
from paper_1510_06340_amd import inputs as I
from paper_1510_06340_amd import mf, surrogate
from helpers import gpu_run, max_rel_err, to_dev

pytestmark = pytest.mark.gpu

TABLE = I.crossover_table()


def params_dict(flat):
    H = 64
    o = np.cumsum([0, 2 * H, H, H * H, H, H])
    f = np.asarray(flat, dtype=np.float64)
    return {"W1": f[o[0]:o[1]].reshape(H, 2), "b1": f[o[1]:o[2]], "W2": f[o[2]:o[3]].reshape(H, H),
            "b2": f[o[3]:o[4]], "w3": f[o[4]:o[5]], "b3": float(f[-1])}


def flat_grads(g):
    return np.concatenate([g["W1"].ravel(), g["b1"], g["W2"].ravel(), g["b2"], g["w3"], [g["b3"]]])


def random_net(seed):
    rng = np.random.default_rng(seed)
    p = surrogate.init_params(seed).astype(np.float64)
    p[128:192] = rng.normal(size=64) * 0.2           # b1
    p[192 + 4096:192 + 4096 + 64] = rng.normal(size=64) * 0.2  # b2
    p[-1] = 0.1
    return p.astype(np.float32)


@pytest.mark.parametrize("n", [64, 1000, 4096])
def test_mlp_forward_matches_reference(n):
    import torch
    rng = np.random.default_rng(n)
    p = random_net(1)
    X = rng.normal(size=(n, 2)).astype(np.float32)
    y = torch.empty(n, device="cuda")
    mf.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), y)
    yr, _ = ref.forward(params_dict(p), X.astype(np.float64), rnd=True)
    np.testing.assert_allclose(y.cpu().numpy(), yr, rtol=1e-3, atol=1e-3 * np.abs(yr).max())


@pytest.mark.parametrize("n", [64, 777, 4096])
def test_mlp_gradients_match_reference(n):
    """Every gradient element against the FP64 reference with the same bfloat16 rounding points.

    Bound per element: 1e-4 of the sum of the absolute values of the terms it sums (its
    rounding scale, oracle.mlp.grad_magnitudes).  The two sides differ by FP32 accumulation
    (at most about 4096 * 2^-24 of that sum) and by the rare bfloat16 roundings of h1 and
    dz2 that tie-break differently after FP32 vs FP64 arithmetic; the largest ratio
    measured is about 6e-6.  The targets sit at least 0.5 from the network's output, so
    y - t is never small and its relative error stays below about 2e-3.  A wrong element
    (a swapped W1 column, a missing tanh derivative, b3 off) moves an element by a large
    part of that sum."""
    import torch
    rng = np.random.default_rng(10 + n)
    p = random_net(2)
    X = rng.normal(size=(n, 2)).astype(np.float32)
    yr0, _ = ref.forward(params_dict(p), X.astype(np.float64), rnd=True)
    t = (yr0 + rng.choice([-1.0, 1.0], size=n) * (0.5 + np.abs(rng.normal(size=n)))).astype(np.float32)
    P = torch.from_numpy(p).cuda()
    grad = torch.zeros_like(P)
    loss = torch.zeros(1, device="cuda")
    work = torch.empty(mf.mlp_workspace(n), device="cuda")
    mf.mlp_grad(P, torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda(), grad, loss, work)
    Pd, Xd, td = params_dict(p), X.astype(np.float64), t.astype(np.float64)
    lr_, gr, _ = ref.loss_and_grads(Pd, Xd, td, rnd=True)
    mag = flat_grads(ref.grad_magnitudes(Pd, Xd, td, rnd=True))
    gg = grad.cpu().numpy().astype(np.float64)
    gref = flat_grads(gr)
    assert float(loss.cpu()[0]) == pytest.approx(lr_, rel=1e-3)
    H = 64
    o = np.cumsum([0, 2 * H, H, H * H, H, H, 1])
    worst = {}
    for name, a, b in zip(["W1", "b1", "W2", "b2", "w3", "b3"], o[:-1], o[1:]):
        ratio = np.abs(gg[a:b] - gref[a:b]) / np.maximum(mag[a:b], 1e-300)
        worst[name] = float(ratio.max())
        assert np.all(np.abs(gg[a:b] - gref[a:b]) <= 1e-4 * mag[a:b]), (name, worst[name], int(ratio.argmax()))
        err = np.linalg.norm(gg[a:b] - gref[a:b]) / max(np.linalg.norm(gref[a:b]), 1e-30)
        assert err <= 1e-3, (name, err)
    print("\nlargest |g_gpu - g_ref| / sum|terms| per group:", {k: f"{v:.1e}" for k, v in worst.items()})


@pytest.mark.parametrize("betas", [(0.9, 0.999), (0.8, 0.95)])
def test_adam_steps_match_reference(betas):
    """Five Adam steps with a different gradient each step against the FP64 reference
    (oracle.mlp.adam), element by element: parameters, first and second moments.  With
    changing gradients the bias-corrected moments differ from the gradient, so a swap of
    the two decay rates or a wrong bias correction is seen."""
    import torch
    # the kernel receives the rates as float: the reference takes the same values
    b1, b2 = (float(np.float32(b)) for b in betas)
    rng = np.random.default_rng(3)
    n = mf.MF_MLP_PARAMS
    p = rng.normal(size=n).astype(np.float32)
    P = torch.from_numpy(p.copy()).cuda()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    Pr, mr, vr = p.astype(np.float64), np.zeros(n), np.zeros(n)
    lr = 1e-2
    for step in range(1, 6):
        g = (rng.normal(size=n) * rng.uniform(0.1, 3.0, size=n)).astype(np.float32)
        mf.mlp_adam(P, torch.from_numpy(g).cuda(), m, v, step, lr, b1, b2, 1e-8)
        Pr, mr, vr = ref.adam(Pr, g.astype(np.float64), mr, vr, step, lr, b1, b2, 1e-8)
        Pg, mg, vg = (x.cpu().numpy().astype(np.float64) for x in (P, m, v))
        np.testing.assert_allclose(mg, mr, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(vg, vr, rtol=1e-5, atol=1e-9)
        # FP32 masters: a few ulp of P per step, plus the update's FP32 rounding
        np.testing.assert_allclose(Pg, Pr, rtol=4e-7 * step, atol=1e-5 * lr)
    # the steps moved the parameters by many times the tolerance
    assert np.median(np.abs(Pr - p)) > 100 * 1e-5 * lr


@pytest.fixture(scope="module")
def trained():
    E, M = surrogate.collect_states(n_samples=1 << 20, n=64, steps=30, snap_every=5)
    e, pr = surrogate.label_states(E, M)
    net = surrogate.train(E, M, e, pr, epochs=20, batch=4096)
    frac = surrogate.train(E, M, e, pr, epochs=20, batch=4096, output=1)
    return dict(E=E, M=M, e=e, net=net, frac=frac)


@pytest.mark.parametrize("which", ["net", "frac"])
def test_training_lowers_the_loss(trained, which):
    h = trained[which].history
    print("\nepoch, train loss, validation loss:", [(a, round(b, 6), round(c, 6)) for a, b, c in h[::4] + h[-1:]])
    assert h[-1][1] < 0.2 * h[0][1] and h[-1][2] < 0.2 * h[0][2]
    err = surrogate.relative_error(trained[which], trained["E"], trained["M"], trained["e"])
    print(f"relative error of the seed: median {float(err.median()):.2e}, 99% {float(err.quantile(0.99)):.2e}")
    assert float(err.median()) < 0.05


def run_c2p(E, M, mode, net=None):
    import torch
    n = E.numel()
    U = [E.contiguous(), M.contiguous(), torch.zeros_like(E), torch.zeros_like(E)]
    prim = [torch.empty_like(E) for _ in range(5)]
    it = torch.zeros(n, dtype=torch.int32, device="cuda")
    g = mf.Grid([mf.make_desc((n, 1, 1), (1, 1, 1), (0, 0, 0), (0, 0, 0))], [U])
    g.set_eos_table(*TABLE, surrogate=net)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.con2prim(U, prim, it, mode)  # warm-up
    start.record()
    g.con2prim(U, prim, it, mode)
    stop.record()
    torch.cuda.synchronize()
    stats = g.con2prim_stats()
    g.free()
    return prim[0], it, stats, start.elapsed_time(stop)


@pytest.mark.parametrize("which", ["net", "frac"])
def test_seeded_con2prim_equals_plain(trained, which):
    """P13: every seeded solution equals the plain one to 1e-12 (relative to E).

    The gain: near rest (|M|/E << 1) the bracket [E(1 - m^2), E] is so narrow
    that its midpoint is already closer than a guess of ln e can be (the guess
    then lies outside the bracket and the solve starts at the midpoint);
    where the flow is relativistic (m > 0.05) the root sits near 3/4 of the
    bracket, so the midpoint is off by about m^2/4: the network that predicts
    the root's position in the bracket ("frac") must then need fewer
    iterations than the midpoint start, and so must the one predicting ln e ("net",
    the configured output)."""
    net = trained[which].network()
    E, M = trained["E"], trained["M"]
    ep, itp, _, tp = run_c2p(E, M, mf.MF_C2P_PLAIN, net)
    es, its, sts, ts = run_c2p(E, M, mf.MF_C2P_SEEDED, net)
    ec, itc, stc, tc = run_c2p(E, M, mf.MF_C2P_CONFORMAL, net)
    # plain ignores an installed seed: same results and iterations as without one
    e0, it0, _, _ = run_c2p(E, M, mf.MF_C2P_PLAIN, None)
    assert bool((e0 == ep).all()) and bool((it0 == itp).all())
    # relative to E: g(e) = e - E + |M|^2 / (E + p) is known to a few ulp of E, so for
    # |M| -> E the root e << E is defined only to that absolute level
    for x in (es, ec):
        rel = ((x - ep).abs() / E).max().item()
        assert rel <= 1e-12, rel
    mp, ms, mc = float(itp.float().mean()), float(its.float().mean()), float(itc.float().mean())
    print(f"\nall {E.numel()} states: mean Newton iterations plain {mp:.3f}, learned seed {ms:.3f} "
          f"(guesses outside the bracket {sts[3]}), conformal {mc:.3f} (outside {stc[3]}); "
          f"time ms plain {tp:.3f} seeded {ts:.3f} conformal {tc:.3f}")
    # a wavefront iterates until its slowest lane has converged: the mean over wavefronts of
    # the largest count is what the time follows
    wp, ws, wc = (float(x.view(-1, 64).max(dim=1).values.float().mean()) for x in (itp, its, itc))
    print(f"mean over wavefronts of the largest iteration count: plain {wp:.3f}, learned seed {ws:.3f}, "
          f"conformal {wc:.3f}")
    fast = (M / E) > 0.05
    sp, ss, sc = (float(x[fast].float().mean()) for x in (itp, its, itc))
    print(f"{int(fast.sum())} states with |M|/E > 0.05: plain {sp:.3f}, learned seed {ss:.3f}, conformal {sc:.3f}")
    assert int(fast.sum()) > 1000
    # both outputs must beat the midpoint start where the flow is relativistic, and over all states
    assert ss < sp and ms < mp


@pytest.mark.parametrize("which", ["net", "frac"])
def test_seeded_run_equals_plain_run(trained, which):
    """A crossover-EoS run with the learned seed (prediction grid in the sweeps) equals the plain run to 1e-10."""
    net = trained[which].network()
    w = I.crossover_workloads(n_events=1, n=40, steps=5)[0]
    U = I.initial_state(w)
    Up, stp = gpu_run(w, U, eos_table=TABLE)
    import torch
    dev = to_dev(U)
    g = mf.Grid([mf.desc_from_workload(w)], [dev])
    g.set_eos_table(*TABLE, surrogate=net)
    sts = g.step(w.dt, w.steps)[0]
    torch.cuda.synchronize()
    Us = np.stack([t.cpu().numpy().reshape(U.shape[1:]) for t in dev])
    g.free()
    assert max_rel_err(Us, Up) <= 1e-10
    Uo, _ = oracle.step(oracle.Problem.from_workload(w, table=TABLE), U, w.dt, w.steps)
    assert max_rel_err(Us, Uo) <= 1e-10
    print(f"\nstep iterations: plain {stp['newton_iters']}, seeded {sts['newton_iters']} "
          f"(guesses outside the bracket {sts['n_fallback']})")
    assert sts["newton_iters"] <= 1.01 * stp["newton_iters"]


def test_crossover_batched_seeded_at_size(trained):
    """The crossover workload in its configured form: batched events of 192^3 under the
    tabulated EoS with the learned ln e seed installed, 2 steps.

    * batched seeded equals the per-event seeded run bitwise (the same arithmetic per cell);
    * batched seeded equals batched plain to 1e-10 over every cell, with equal floor counts;
    * both events against the oracle (bisection con2prim) on blocks around the hottest cell
      and at a corner, <= 1e-10."""
    import torch
    from helpers import from_dev, oracle_block
    net = trained["net"].network()
    assert net.output == 0
    ws = I.crossover_workloads(n_events=2, steps=2)
    Us = [I.initial_state(w) for w in ws]
    dts = [w.dt for w in ws]

    def batched(seed):
        devs = [to_dev(U) for U in Us]
        g = mf.Grid([mf.desc_from_workload(w) for w in ws], devs)
        try:
            g.set_eos_table(*TABLE, surrogate=net if seed else None)
            st = g.batch_step(dts, 2)
            torch.cuda.synchronize()
            return [from_dev(d, Us[0].shape[1:]) for d in devs], st
        finally:
            g.free()

    Gs, sts = batched(True)
    Gp, stp = batched(False)
    for j, w in enumerate(ws):
        dev = to_dev(Us[j])
        g = mf.Grid([mf.desc_from_workload(w)], [dev])
        g.set_eos_table(*TABLE, surrogate=net)
        g.step(w.dt, 2)
        torch.cuda.synchronize()
        g.free()
        assert np.array_equal(Gs[j], from_dev(dev, Us[j].shape[1:])), j
        assert max_rel_err(Gs[j], Gp[j]) <= 1e-10
        assert sts[j]["n_floor"] == stp[j]["n_floor"] and sts[j]["n_bad"] == 0
        hot = np.unravel_index(int(np.argmax(Us[j][0])), Us[j][0].shape)   # (z, y, x)
        lo_hot = [min(max(int(hot[2 - d]) - 8, 0), w.n[d] - 16) for d in range(3)]
        for lo in (lo_hot, [0, 0, w.n[2] - 16]):
            Ub, sl = oracle_block(w, Us[j], lo, (16, 16, 16), 2, table=TABLE)
            err = max_rel_err(Gs[j][(slice(None),) + sl], Ub)
            print(f"\nevent {j} block {lo}: max rel err {err:.2e}", flush=True)
            assert err <= 1e-10, (j, lo, err)
        print(f"event {j}: Newton iterations plain {stp[j]['newton_iters']}, seeded {sts[j]['newton_iters']} "
              f"(seeds outside the bracket {sts[j]['n_fallback']})")
