"""Pins of the oracle's fixed-point positions (a state representation beyond
IEEE double: a clump's CoM is an integer k per axis, x = k 2^-E), against
what the encoding and the mathematics fix:

* the position update is the FP64 velocity update followed by
  k += rint(h v 2^E): the iterated closed form of a free fall, computed here
  with Python integers, matches bit for bit;
* sphere-to-sphere vectors are exact integer differences plus rotated
  offsets, so a pile translated by a multiple of the grid step (here a
  million metres) evolves bit for bit as the original, contact forces
  included; FP64 world positions cannot do this (their rounding grows with
  the distance from the origin), which the same test shows;
* the dynamics are those of FP64 positions up to the quantisation of
  positions: the force difference shrinks with the grid step, and at
  2^-52 m forces agree within 1e-9 and states after 200 steps within 1e-9
  of the smallest radius;
* out-of-range exponents and positions are refused."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2307_03445_amd import inputs as I


def _free_pile(n=300, replica=0):
    """A deposited pile of three-sphere clumps with its walls removed: every
    contact is sphere-sphere (gravity acts on all clumps alike)."""
    d = I.walled_box(replica=replica, n_clumps=n, dense=True)
    z = lambda *s: np.zeros(s)
    return dataclasses.replace(d, bnd_type=np.zeros(0, np.int32), bnd_param=z(0, I.BND_NPARAM), bnd_mat=z(0, 4),
                               bnd_vel=z(0, 3), bnd_omega=z(0, 3), bnd_scene=np.zeros(0, np.int32))


def _on_grid(d, E):
    """The same scene with CoMs already on the grid 2^-E."""
    return dataclasses.replace(d, x=np.ldexp(np.rint(np.ldexp(d.x, E)), -E), pos_exp=E)


def test_free_fall_position_update_closed_form():
    E, h, n = 40, 1e-6, 500
    t = I.sphere_template(1e-3)
    x0, v0, g = (0.0123, -0.004, 0.31), (0.2, -0.05, 0.0), (0.0, 0.0, -9.81)
    d = I.assemble([t], [0], [x0], [(1, 0, 0, 0)], [v0], [(0, 0, 0)], [(1e7, 0.3, 0.5, 0.5)], g,
                   (-1, -1, -1, 1, 1, 1), h)
    d = dataclasses.replace(d, pos_exp=E)
    o = oracle.Oracle(d)
    o.step(n)
    M = float(d.tmpl_mass[0])
    k = [int(np.rint(math.ldexp(c, E))) for c in x0]
    v = list(v0)
    for _ in range(n):
        for i in range(3):
            F = 0.0 + M * g[i]
            v[i] = v[i] + h * (F / M)
            k[i] += int(np.rint(math.ldexp(h * v[i], E)))
    assert o.fixed_positions()[0].tolist() == k
    st = o.state()
    assert st["v"][0].tolist() == v
    assert st["x"][0].tolist() == [math.ldexp(float(c), -E) for c in k]


@pytest.mark.parametrize("pos_exp", [32, 0])
def test_translation_by_a_grid_multiple(pos_exp):
    E = 32
    base = _on_grid(_free_pile(), E)
    T = np.array([2.0 ** 20, -(2.0 ** 19) + 0.25, 3 * 2.0 ** 18])
    far = dataclasses.replace(base, x=base.x + T, domain=base.domain + np.tile(T, 2))
    assert np.array_equal(far.x - T, base.x)  # the shift is exact in FP64
    base, far = (dataclasses.replace(s, pos_exp=pos_exp) for s in (base, far))
    a, b = oracle.Oracle(base), oracle.Oracle(far)
    a.eval(), b.eval()
    ca, cb = a.contacts(), b.contacts()
    assert len(ca["a"]) > 200
    a.step(100), b.step(100)
    a.eval(), b.eval()
    ca, cb = a.contacts(), b.contacts()
    sa, sb = a.state(), b.state()
    if pos_exp:
        dk = (b.fixed_positions() - a.fixed_positions()).astype(object)
        assert all(int(x) == int(np.ldexp(t, E)) for row in dk for x, t in zip(row, T))
        assert np.array_equal(ca["a"], cb["a"]) and np.array_equal(ca["b"], cb["b"])
        for k in ("delta", "F", "u", "Ta", "Tb"):
            assert np.array_equal(ca[k], cb[k]), k
        for k in ("q", "v", "w"):
            assert np.array_equal(sa[k], sb[k]), k
    else:
        # FP64 world positions round at a million metres: the pile does not
        # move as the one at the origin
        assert not np.array_equal(sa["v"], sb["v"])
        err = np.abs(sa["v"] - sb["v"]).max() / np.abs(sa["v"]).max()
        assert err > 1e-9, err


def test_fine_grid_follows_fp64_positions():
    """The fixed-point run differs from the FP64 one only by the quantisation
    of positions: the first step's force difference shrinks 16x per 4 more
    bits of grid, and at 2^-52 m forces agree within 1e-9 and states after
    200 steps within 1e-9 of the smallest radius."""
    d = I.walled_box(n_clumps=400, dense=True)
    a = oracle.Oracle(d)
    a.eval()
    ca = a.contacts()
    scale = np.abs(ca["F"]).max()
    diffs = []
    for E in (40, 44, 48, 52):
        b = oracle.Oracle(dataclasses.replace(d, pos_exp=E))
        b.eval()
        cb = b.contacts()
        assert np.array_equal(ca["a"], cb["a"]) and np.array_equal(ca["b"], cb["b"])
        diffs.append(np.abs(ca["F"] - cb["F"]).max() / scale)
    ratios = np.array(diffs[:-1]) / np.array(diffs[1:])
    assert np.all((ratios > 3) & (ratios < 100)), (diffs, ratios)
    assert diffs[-1] <= 1e-9
    assert np.abs(ca["Tb"] - cb["Tb"]).max() <= 1e-9 * np.abs(ca["Tb"]).max()
    a.step(200), b.step(200)
    sa, sb = a.state(), b.state()
    r = d.tmpl_radius.min()
    assert np.abs(sa["x"] - sb["x"]).max() <= 1e-9 * r
    assert np.abs(sa["v"] - sb["v"]).max() <= 1e-6 * np.abs(sa["v"]).max()


@pytest.mark.parametrize("pos_exp,x,msg", [(7, 0.0, "exponent"), (61, 0.0, "exponent"),
                                           (40, 2.0 ** 21, "range")])
def test_refused(pos_exp, x, msg):
    t = I.sphere_template(1e-3)
    d = I.assemble([t], [0], [(x, 0, 0)], [(1, 0, 0, 0)], [(0, 0, 0)], [(0, 0, 0)], [(1e7, 0.3, 0.5, 0.5)],
                   (0, 0, 0), (-1, -1, -1, 1, 1, 1), 1e-6)
    with pytest.raises(ValueError, match=msg):
        oracle.Oracle(dataclasses.replace(d, pos_exp=pos_exp))
