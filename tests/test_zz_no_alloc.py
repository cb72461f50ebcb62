"""The allocation-free MLP backward entry point against the one that takes a
caller workspace: identical gradient and loss, bit for bit, on two calls in a
row (the second with fewer samples, so stale partials of the first call would
show), and sizes beyond the static array refused before any launch."""
import numpy as np
import pytest

import oracle.mlp as M

pytestmark = pytest.mark.gpu


def _data(n, seed):
    g = np.random.default_rng(seed)
    f = np.stack([g.lognormal(-3, 1.5, n), g.lognormal(3, 2, n), g.integers(0, 40, n).astype(float)], 1)
    y = np.stack([np.log(f[:, 0] * 1.3 + 1e-6), np.log(f[:, 1] * 2 + 1e-3)], 1) + g.normal(0, 0.3, (n, 2))
    return f.astype(np.float32), y.astype(np.float32)


def _params(seed=1):
    g = np.random.default_rng(seed)
    p = M.init_params(g, mu=(-3.0, 3.0, 2.5), sig=(1.5, 2.0, 1.0))
    p[M.OFF_B1:M.OFF_W2] = g.normal(0, 0.2, M.H)
    p[M.OFF_B2:M.OFF_W3] = g.normal(0, 0.2, M.H)
    return p.astype(np.float32)


def test_static_backward_equals_workspace_backward_on_consecutive_calls():
    import torch

    from paper_2307_03445_amd import _lib
    p = torch.tensor(_params(), device="cuda")
    grad = torch.empty_like(p)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    # the largest batch the static array holds, then a smaller one (ragged:
    # not a multiple of the 32-sample workgroup)
    for n, seed in ((_lib.MLP_STATIC_MAX_SAMPLES, 3), (1001, 4)):
        f, y = _data(n, seed)
        ft, yt = torch.tensor(f, device="cuda"), torch.tensor(y, device="cuda")
        g_ref, l_ref = _lib.mlp_backward(p, ft, yt, 0.99)
        grad.fill_(np.nan)
        loss.fill_(np.nan)
        _lib.mlp_backward_static(p, ft, yt, 0.99, grad, loss)
        torch.cuda.synchronize()
        assert torch.equal(grad, g_ref), f"n={n}: gradients differ"
        assert torch.equal(loss, l_ref), f"n={n}: losses differ"
        # and against the FP64 reference, as the workspace version is tested
        Lref, gref = M.loss_and_grad(p.cpu().numpy().astype(np.float64), f.astype(np.float64),
                                     y.astype(np.float64), 0.99)
        assert np.abs(grad.cpu().numpy() - gref).max() <= 1e-4 * np.abs(gref).max()
        assert abs(float(loss.item()) - Lref) <= 1e-4 * abs(Lref)


def test_static_backward_refuses_more_samples_than_it_holds():
    import torch

    from paper_2307_03445_amd import _lib
    n = _lib.MLP_STATIC_MAX_SAMPLES + 1
    p = torch.tensor(_params(), device="cuda")
    f = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    y = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    grad = torch.zeros_like(p)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.CdemError) as e:
        _lib.mlp_backward_static(p, f, y, 0.99, grad, loss)
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert not grad.any() and not loss.any()  # nothing was launched
