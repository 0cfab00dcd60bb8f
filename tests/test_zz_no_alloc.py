"""mf_mlp_grad_noalloc (partial gradients in the library's static device array) against
mf_mlp_grad (partials in a caller workspace), called through the C ABI: the same kernels
over the same partial layout, so gradient and loss must agree bitwise.  Two calls in a
row, the second with fewer samples (the array keeps the first call's partials, which the
second must not read), then a third at the largest size the array holds; sizes beyond it
are refused with MF_ERR_ARG."""

import numpy as np
import pytest

from paper_1510_06340_amd import mf

pytestmark = pytest.mark.gpu


def _net(seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=mf.MF_MLP_PARAMS) * 0.3).astype(np.float32)


def _grad_both(P, n, seed):
    import torch
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.normal(size=(n, 2)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.normal(size=n).astype(np.float32)).cuda()
    g_ref, l_ref = torch.zeros_like(P), torch.zeros(1, device="cuda")
    work = torch.empty(mf.mlp_workspace(n), device="cuda")
    mf.mlp_grad(P, X, t, g_ref, l_ref, work)
    g_na, l_na = torch.full_like(P, float("nan")), torch.full((1,), float("nan"), device="cuda")
    mf.mlp_grad_noalloc(P, X, t, g_na, l_na)
    torch.cuda.synchronize()
    return g_ref.cpu().numpy(), l_ref.cpu().numpy(), g_na.cpu().numpy(), l_na.cpu().numpy()


def test_noalloc_grad_equals_workspace_grad():
    import torch
    P = torch.from_numpy(_net(1)).cuda()
    for n, seed in ((5000, 1), (700, 2), (mf.MF_MLP_NOALLOC_MAX_N, 3), (1, 4)):
        g_ref, l_ref, g_na, l_na = _grad_both(P, n, seed)
        assert np.isfinite(g_na).all() and np.isfinite(l_na).all(), n
        assert np.array_equal(g_ref, g_na), (n, float(np.abs(g_ref - g_na).max()))
        assert np.array_equal(l_ref, l_na), n
        assert np.abs(g_ref).max() > 0


def test_noalloc_grad_refuses_sizes_beyond_its_array():
    import torch
    P = torch.zeros(mf.MF_MLP_PARAMS, device="cuda")
    n = mf.MF_MLP_NOALLOC_MAX_N + 1
    X = torch.zeros((n, 2), device="cuda")
    t = torch.zeros(n, device="cuda")
    g = torch.zeros_like(P)
    rc = mf.lib().mf_mlp_grad_noalloc(P.data_ptr(), X.data_ptr(), t.data_ptr(), n, g.data_ptr(), None, None)
    assert rc == mf.MF_ERR_ARG
    assert "MF_MLP_NOALLOC_MAX_N" in mf.last_error()
    rc = mf.lib().mf_mlp_grad_noalloc(P.data_ptr(), X.data_ptr(), t.data_ptr(), 0, g.data_ptr(), None, None)
    assert rc == mf.MF_ERR_ARG
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0
