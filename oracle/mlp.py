"""FP64 reference of the envelope MLP and its quantile (pinball) loss.

TEST INFRASTRUCTURE ONLY (the HIP kernels are the product; this checks their
gradients).  Shares no code with the HIP path.

Network (per bin): x = standardised features (3) -> 64 ReLU -> 64 ReLU -> 2
(log speed envelope, log acceleration envelope).  Parameter vector layout
(float32 on the device, float64 here):
    mu[3], sigma[3]          feature standardisation (not trained)
    W1[64][3], b1[64]
    W2[64][64], b2[64]
    W3[2][64], b3[2]
Raw features f = (max sphere speed, max sphere acceleration, occupancy) of a
bin enter as u = (log(f0 + 1e-6), log(f1 + 1e-3), log(1 + f2)), then
x = (u - mu) / sigma.

Loss: mean over samples and both outputs of the pinball loss
rho_tau(r) = max(tau r, (tau - 1) r), r = target - prediction, so that the
prediction tracks the tau-quantile (tau near 1: envelopes err high).
"""
from __future__ import annotations

import numpy as np

H = 64
N_IN, N_OUT = 3, 2
OFF_MU, OFF_SIG = 0, 3
OFF_W1 = 6
OFF_B1 = OFF_W1 + H * N_IN
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + N_OUT * H
N_PARAM = OFF_B3 + N_OUT


def unpack(p):
    p = np.asarray(p, np.float64)
    return dict(mu=p[OFF_MU:OFF_MU + 3], sig=p[OFF_SIG:OFF_SIG + 3],
                W1=p[OFF_W1:OFF_B1].reshape(H, N_IN), b1=p[OFF_B1:OFF_W2],
                W2=p[OFF_W2:OFF_B2].reshape(H, H), b2=p[OFF_B2:OFF_W3],
                W3=p[OFF_W3:OFF_B3].reshape(N_OUT, H), b3=p[OFF_B3:OFF_B3 + N_OUT])


def features_to_input(f, mu, sig):
    f = np.asarray(f, np.float64)
    u = np.stack([np.log(f[:, 0] + 1e-6), np.log(f[:, 1] + 1e-3), np.log1p(f[:, 2])], 1)
    return (u - mu) / sig


def forward(p, f):
    """Raw features [n, 3] -> outputs [n, 2] (plus the activations)."""
    q = unpack(p)
    x = features_to_input(f, q["mu"], q["sig"])
    z1 = x @ q["W1"].T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ q["W3"].T + q["b3"]
    return y, (x, z1, h1, z2, h2)


def pinball(y, target, tau):
    r = np.asarray(target, np.float64) - y
    return np.maximum(tau * r, (tau - 1.0) * r)


def loss(p, f, target, tau):
    y, _ = forward(p, f)
    return pinball(y, target, tau).mean()


def loss_and_grad(p, f, target, tau):
    """Mean pinball loss and its gradient with respect to every parameter
    (zero for the standardisation entries)."""
    q = unpack(p)
    y, (x, z1, h1, z2, h2) = forward(p, f)
    n = y.shape[0]
    r = np.asarray(target, np.float64) - y
    # d rho / d y = -tau where r > 0, (1 - tau) where r <= 0; mean over n * 2 terms
    dy = np.where(r > 0, -tau, 1.0 - tau) / (n * N_OUT)
    g = np.zeros(N_PARAM)
    g[OFF_W3:OFF_B3] = (dy.T @ h2).ravel()
    g[OFF_B3:OFF_B3 + N_OUT] = dy.sum(0)
    dh2 = dy @ q["W3"]
    dz2 = dh2 * (z2 > 0)
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(0)
    dh1 = dz2 @ q["W2"]
    dz1 = dh1 * (z1 > 0)
    g[OFF_W1:OFF_B1] = (dz1.T @ x).ravel()
    g[OFF_B1:OFF_W2] = dz1.sum(0)
    return pinball(y, target, tau).mean(), g


def init_params(rng: np.random.Generator, mu=(0.0, 0.0, 0.0), sig=(1.0, 1.0, 1.0)):
    """He-initialised weights, zero biases."""
    p = np.zeros(N_PARAM)
    p[OFF_MU:OFF_MU + 3] = mu
    p[OFF_SIG:OFF_SIG + 3] = sig
    p[OFF_W1:OFF_B1] = rng.normal(0, np.sqrt(2.0 / N_IN), H * N_IN)
    p[OFF_W2:OFF_B2] = rng.normal(0, np.sqrt(2.0 / H), H * H)
    p[OFF_W3:OFF_B3] = rng.normal(0, np.sqrt(1.0 / H), N_OUT * H)
    return p
