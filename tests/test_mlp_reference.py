"""Pins of the FP64 MLP reference: gradients against central finite
differences, closed forms of the loss, and the quantile property of the
pinball loss."""
import numpy as np
import pytest

from oracle import mlp as M


def _data(n=40, seed=0):
    g = np.random.default_rng(seed)
    f = np.stack([g.lognormal(-3, 1, n), g.lognormal(2, 2, n), g.integers(0, 30, n).astype(float)], 1)
    tgt = np.stack([np.log(f[:, 0] * 1.5 + 1e-4), np.log(f[:, 1] * 2 + 1e-2)], 1) + g.normal(0, 0.1, (n, 2))
    return f, tgt


def test_gradient_matches_central_differences():
    g = np.random.default_rng(1)
    p = M.init_params(g, mu=(-3.0, 2.0, 2.0), sig=(1.0, 2.0, 1.0))
    p[M.OFF_B1:M.OFF_W2] = g.normal(0, 0.1, M.H)      # move ReLU kinks away from samples
    p[M.OFF_B2:M.OFF_W3] = g.normal(0, 0.1, M.H)
    f, tgt = _data()
    tau = 0.9
    L, grad = M.loss_and_grad(p, f, tgt, tau)
    idx = np.r_[np.arange(M.OFF_W1, M.OFF_W1 + 20), np.arange(M.OFF_B1, M.OFF_B1 + 10),
                np.arange(M.OFF_W2, M.OFF_W2 + 30), np.arange(M.OFF_W3, M.N_PARAM)]
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (M.loss(pp, f, tgt, tau) - M.loss(pm, f, tgt, tau)) / (2 * eps)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), (i, fd, grad[i])
    assert np.all(grad[:6] == 0)  # standardisation is not trained


def test_zero_weights_output_is_bias():
    p = np.zeros(M.N_PARAM)
    p[M.OFF_SIG:M.OFF_SIG + 3] = 1.0
    p[M.OFF_B3:M.OFF_B3 + 2] = (0.7, -1.3)
    f, _ = _data(5)
    y, _ = M.forward(p, f)
    assert np.array_equal(y, np.tile([0.7, -1.3], (5, 1)))


def test_pinball_closed_form():
    """rho_tau(r) = tau r for r >= 0, (tau - 1) r for r < 0."""
    y = np.array([[0.0, 1.0]])
    t = np.array([[2.0, 0.5]])
    v = M.pinball(y, t, 0.99)
    assert np.allclose(v, [[0.99 * 2.0, 0.01 * 0.5]])


def test_pinball_minimiser_is_the_quantile():
    """For a constant predictor the mean pinball loss is minimised at the
    tau-quantile of the targets (checked by brute force over candidates)."""
    g = np.random.default_rng(3)
    t = g.normal(size=2001)
    tau = 0.99
    cands = np.sort(t)
    losses = [np.maximum(tau * (t - c), (tau - 1) * (t - c)).mean() for c in cands[1900:]]
    best = cands[1900 + int(np.argmin(losses))]
    assert best == np.quantile(t, tau, method="inverted_cdf")
