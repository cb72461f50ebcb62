"""Preparation of large beds with the simulator itself.

The paper prepares its large test beds by settling batches of clumps under
gravity and copying the settled base patch (Sec. 4.1).  ``settle_patch`` runs
that settling for one small patch on the GPU through the C ABI; the caller
tiles the result (``inputs.rover_bed``).
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from ._lib import Scene


def settle_patch(replica: int = 0, n_clumps: int = 6875, min_steps: int = 60000, max_steps: int = 300000,
                 chunk: int = 10000, v_stop: float = 0.05, log=None):
    """Settle the rover-bed preparation patch; returns (x, q, info)."""
    d = I.rover_patch_scene(replica, n_clumps=n_clumps)
    sc = Scene(d, precision="fp32")
    t0 = time.perf_counter()
    steps, vmax = 0, float("inf")
    while steps < max_steps:
        sc.step(chunk)
        steps += chunk
        st = sc.state()
        vmax = float(np.linalg.norm(st["v"], axis=1).max())
        if log:
            log(f"settle: {steps} steps, max speed {vmax:.3g} m/s, top {st['x'][:, 2].max():.3f} m, "
                f"{time.perf_counter() - t0:.1f} s")
        if steps >= min_steps and vmax < v_stop:
            break
    info = dict(steps=steps, h=d.h, max_speed=vmax, seconds=time.perf_counter() - t0,
                height=float(st["x"][:, 2].max()), n_clumps=d.n_clumps, n_spheres=d.n_spheres)
    sc.close()
    return st["x"], st["q"], info


def settle_funnels(desc, seconds: float = 0.05, h: float = 5e-6, chunk: int = 2000, log=None):
    """Run a batched funnel description for `seconds` of simulated time at a
    coarser step h (fixed-rule deferred detection, FP32 forces): the clumps
    drop off their spawn lattice, pack into the funnels and start to
    discharge through the outlets.  Returns the description with that state
    (positions, orientations, velocities) and its own time step, and info."""
    import dataclasses
    d = dataclasses.replace(desc, h=h)
    sc = Scene(d, precision="fp32")
    sc.set_detection("fixed", k_max=20, safety=1.5, margin_cap=2e-4, audit_period=0)
    n = int(round(seconds / h))
    t0 = time.perf_counter()
    done = 0
    while done < n:
        k = min(chunk, n - done)
        sc.step(k)
        done += k
        if log:
            log(f"funnel settle: {done}/{n} steps, {time.perf_counter() - t0:.1f} s")
    st = sc.state()
    info = dict(steps=n, h=h, seconds=time.perf_counter() - t0, contacts=sc.last_step_contacts(),
                max_speed=float(np.linalg.norm(st["v"], axis=1).max()))
    sc.close()
    out = dataclasses.replace(desc, x=st["x"], q=st["q"], v=st["v"], w=st["w"])
    return out, info
