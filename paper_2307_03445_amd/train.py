"""Training of the envelope MLP on trajectories of the plain method.

Data: a scene is run with per-step detection; at regular captures the
library records, for every occupied envelope region (2 x 2 x 2 bins), the
current features (max sphere speed, max acceleration envelope, occupancy)
and the largest speed and acceleration its spheres reach over the next
`horizon` steps
(``Scene.collect_envelopes``).  Fit: mean pinball loss at quantile tau (the
envelopes should err high), Adam, all arithmetic in the library's HIP kernels
(``cdem_mlp_backward`` / ``cdem_mlp_adam``); torch tensors only hold the data.

Run as a script to write ``envelope_mlp.npz`` next to this file.
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import inputs as I
from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "envelope_mlp.npz")
H = 64
N_PARAM = 6 + H * 3 + H + H * H + H + 2 * H + 2


def collect(desc, captures=6, horizon=20, gap=40, precision="fp32", log=None):
    """Features and labels of `captures` captures spaced `gap` steps apart."""
    sc = _lib.Scene(desc, precision=precision)
    F, Y = [], []
    for k in range(captures):
        sc.step(gap)
        f, y = sc.collect_envelopes(horizon)
        F.append(f)
        Y.append(y)
        if log:
            log(f"capture {k}: {len(f)} regions, label speed p50 {np.exp(np.median(y[:, 0])):.3g} "
                f"max {np.exp(y[:, 0].max()):.3g} m/s")
    sc.close()
    return np.concatenate(F), np.concatenate(Y)


def standardisation(F):
    u = np.stack([np.log(F[:, 0] + 1e-6), np.log(F[:, 1] + 1e-3), np.log1p(F[:, 2])], 1)
    mu = u.mean(0)
    sig = np.maximum(u.std(0), 1e-3)
    return mu, sig


def init_params(rng, mu, sig):
    p = np.zeros(N_PARAM, np.float32)
    p[0:3], p[3:6] = mu, sig
    o = 6
    p[o:o + 3 * H] = rng.normal(0, np.sqrt(2.0 / 3), 3 * H); o += 3 * H
    o += H
    p[o:o + H * H] = rng.normal(0, np.sqrt(2.0 / H), H * H); o += H * H
    o += H
    p[o:o + 2 * H] = rng.normal(0, np.sqrt(1.0 / H), 2 * H); o += 2 * H
    return p


def fit(F, Y, tau=0.99, steps=3000, batch=8192, lr=2e-3, seed=0, log=None):
    """Adam on the pinball loss; returns float32 parameters."""
    import torch
    assert _lib.mlp_param_count() == N_PARAM
    g = np.random.default_rng(seed)
    mu, sig = standardisation(F)
    p0 = init_params(g, mu, sig)
    # start the output biases at the label means (faster convergence)
    p0[-2:] = Y.mean(0)
    dev = torch.device("cuda")
    params = torch.tensor(p0, device=dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    Ft = torch.tensor(F, device=dev)
    Yt = torch.tensor(Y, device=dev)
    n = Ft.shape[0]
    t0 = time.perf_counter()
    hist = []
    for t in range(1, steps + 1):
        idx = torch.tensor(g.integers(0, n, min(batch, n)), device=dev)
        fb, yb = Ft[idx].contiguous(), Yt[idx].contiguous()
        grad, loss = _lib.mlp_backward(params, fb, yb, tau)
        _lib.mlp_adam(params, grad, m, v, t, lr=lr * (0.1 ** (t / steps)))
        if t % 500 == 0 or t == steps:
            hist.append(float(loss.item()))
            if log:
                log(f"adam step {t}: pinball loss {hist[-1]:.4f} ({time.perf_counter() - t0:.1f} s)")
    # coverage on all data: fraction of regions whose label the envelope covers
    out = _lib.mlp_forward(params, Ft).cpu().numpy()
    cover = (out >= Y).mean(0)
    return params.cpu().numpy(), dict(loss=hist, coverage_speed=float(cover[0]), coverage_acc=float(cover[1]),
                                      n=int(n), tau=tau)


def training_scenes(patch_x, patch_q):
    """A reduced rover bed with the wheel (the flow the envelopes must learn)
    and the contact-rich walled-box pile."""
    return [I.rover_bed(patch_x, patch_q, n_clumps=96 * patch_x.shape[0], bed=(0.8, 0.3), wheel_x=0.3),
            I.walled_box(dense=True)]


def train(patch_x, patch_q, log=None, captures=6, steps=3000):
    F, Y = [], []
    for d in training_scenes(patch_x, patch_q):
        f, y = collect(d, captures=captures, log=log)
        F.append(f)
        Y.append(y)
    F, Y = np.concatenate(F), np.concatenate(Y)
    return fit(F, Y, steps=steps, log=log)


def save(params, info, path=WEIGHTS):
    np.savez(path, params=np.asarray(params, np.float32), **{k: np.asarray(v) for k, v in info.items()})


def load_weights(path=WEIGHTS):
    if not os.path.exists(path):
        return None
    return np.load(path)["params"].astype(np.float32)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--patch", required=True, help="npz with the settled rover-bed patch (x, q)")
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args()
    z = np.load(a.patch)
    p, info = train(z["x"], z["q"], log=print)
    save(p, info, a.out)
    print(info)
