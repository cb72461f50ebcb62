"""The two precision modes against the FP64 oracle, error stated per
quantity (the FP32 force arithmetic extension: force arithmetic in FP32,
penetration, normal, tangential history, state and integration in FP64).

Per quantity: per-pair contact force (relative to its own magnitude, and to
max(|F|, its Hertz elastic scale)), per-clump force (relative to the sum of
the clump's contact-force magnitudes plus its weight) and torque (the same
scale times the clump's bounding radius), and after 100 steps from the same
start the clump states (position / smallest radius, velocity / largest
speed, angular velocity / largest angular velocity, rotation angle between
orientations).  Scenes: the contact-rich walled box (2,000 three-sphere
clumps), the rotating drum and the cone bed (scaled down: every step on the
oracle), and the drum at scale (R = 0.4 m, L = 3 m, 1.7M clumps, 5.4M
spheres: all the clumps of a CPU-deposited bed patch that fit the drum; the
oracle evaluates sampled spheres and clumps by brute force over every
partner).  The all-FP64 mode is bit-identical everywhere; the FP32-force mode
is held to the force and state tolerances, and its measured errors are
printed on lines starting PRECISION."""
import os

import numpy as np
import pytest

import oracle
from paper_2307_03445_amd import inputs as I
from paritylib import (FORCE_RTOL, STATE_TOL, check_pair_forces, compare_pairs, hertz_scale, pair_keys,
                       state_errors)

pytestmark = pytest.mark.gpu


def _scene(desc, prec):
    from paper_2307_03445_amd._lib import Scene
    return Scene(desc, precision=prec)


def _pair_errors(cg, co, desc):
    err = np.linalg.norm(cg["F"] - co["F"], axis=1)
    mag = np.linalg.norm(co["F"], axis=1)
    own = err / np.maximum(mag, 1e-300)
    scaled = err / np.maximum(np.maximum(mag, hertz_scale(desc, co)), 1e-300)
    return dict(pairs=len(err), own_max=float(own.max()), own_p99=float(np.quantile(own, 0.99)),
                own_p50=float(np.median(own)), scaled_max=float(scaled.max()),
                own_le_1e5=float((own <= FORCE_RTOL).mean()))


def _clump_scales(desc, co, clumps=None):
    """Sum of contact-force magnitudes on each clump plus its weight, and the
    clump's bounding radius."""
    sb = np.asarray(desc.sphere_begin(), np.int64)
    owner = np.repeat(np.arange(desc.n_clumps), np.diff(sb))
    mag = np.linalg.norm(co["F"], axis=1)
    s = np.zeros(desc.n_clumps)
    a, b = co["a"].astype(np.int64), co["b"].astype(np.int64)
    np.add.at(s, owner[a], mag)
    sph = b < desc.n_spheres
    np.add.at(s, owner[b[sph]], mag[sph])
    ct = np.asarray(desc.clump_template, np.int64)
    s += desc.tmpl_mass[ct] * 9.81
    tb = np.asarray(desc.tmpl_sphere_begin, np.int64)
    rad = np.array([I.bounding_radius(desc.tmpl_offset[tb[t]:tb[t + 1]], desc.tmpl_radius[tb[t]:tb[t + 1]])
                    for t in range(len(tb) - 1)])[ct]
    return s, rad


def _first_step(desc, prec):
    sc = _scene(desc, prec)
    sc.record_next_step()
    sc.step(1)
    cg = sc.contacts()
    F, T = sc.clump_forces()
    sc.close()
    return cg, F, T


SMALL = {"walled box": lambda: I.walled_box(dense=True), "drum": lambda: I.drum(), "cone bed": lambda: I.cone_bed()}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_errors_per_quantity_small_scenes(name):
    d = SMALL[name]()
    o = oracle.Oracle(d)
    o.eval()
    co = o.contacts()
    Fo, To = o.clump_forces()
    s, rad = _clump_scales(d, co)
    o.step(100)
    so = o.state()
    for prec in ("fp64", "fp32"):
        cg, Fg, Tg = _first_step(d, prec)
        compare_pairs(cg, co)
        ef = np.linalg.norm(Fg - Fo, axis=1) / s
        et = np.linalg.norm(Tg - To, axis=1) / (s * rad)
        sc = _scene(d, prec)
        sc.step(100)
        sg = sc.state()
        sc.close()
        es = state_errors(sg, so, d.tmpl_radius.min())
        pe = _pair_errors(cg, co, d)
        print(f"PRECISION {name} {prec}: pair {pe}; clump force max {ef.max():.3g}, clump torque max "
              f"{et.max():.3g}; 100-step state {es}", flush=True)
        if prec == "fp64":
            for k in ("F", "u", "Ta", "Tb", "delta"):
                assert np.array_equal(cg[k], co[k]), k
            assert np.array_equal(Fg, Fo) and np.array_equal(Tg, To)
            for k in ("x", "q", "v", "w"):
                assert np.array_equal(sg[k], so[k]), k
        else:
            check_pair_forces(cg, co, d)
            assert ef.max() <= FORCE_RTOL and et.max() <= FORCE_RTOL
            assert max(es.values()) <= STATE_TOL, es


def test_errors_per_quantity_drum_at_scale():
    x, q = I.rover_deposited_patch()
    d = I.drum_bed(x, q)
    assert d.n_spheres > 5_000_000
    g = np.random.default_rng(3445)
    sb = np.asarray(d.sphere_begin(), np.int64)
    clumps = np.sort(g.choice(d.n_clumps, 150, replace=False))
    clump_spheres = np.concatenate([np.arange(sb[c], sb[c + 1]) for c in clumps])
    ids = np.unique(np.r_[g.choice(d.n_spheres, 600, replace=False), clump_spheres])
    oracle.set_threads(min(16, os.cpu_count() or 1))
    o = oracle.Oracle(d)
    Fs, Ts, co = o.sample_spheres(ids)
    Fo, To = o.sample_clumps(clumps)
    ko, first = np.unique(pair_keys(co), return_index=True)
    cos = {k: v[first] for k, v in co.items() if k != "beg"}
    own = np.repeat(np.arange(len(ids)), np.diff(co["beg"]))
    mag = np.linalg.norm(co["F"], axis=1)
    fsum = np.bincount(own, weights=mag, minlength=len(ids))
    pos = np.searchsorted(ids, clump_spheres)
    cl_of = np.repeat(np.arange(len(clumps)), np.diff(sb)[clumps])
    scale = np.bincount(cl_of, weights=fsum[pos], minlength=len(clumps))
    ct = np.asarray(d.clump_template, np.int64)[clumps]
    scale = scale + d.tmpl_mass[ct] * 9.81
    tb = np.asarray(d.tmpl_sphere_begin, np.int64)
    rad = np.array([I.bounding_radius(d.tmpl_offset[tb[t]:tb[t + 1]], d.tmpl_radius[tb[t]:tb[t + 1]]) for t in ct])
    assert len(ko) > 300
    for prec in ("fp64", "fp32"):
        cg, Fg, Tg = _first_step(d, prec)
        m = np.isin(cg["a"], ids) | np.isin(cg["b"], ids)
        cgs = {k: v[m] for k, v in cg.items()}
        assert np.array_equal(pair_keys(cgs), ko)
        ef = np.linalg.norm(Fg[clumps] - Fo, axis=1) / scale
        et = np.linalg.norm(Tg[clumps] - To, axis=1) / (scale * rad)
        pe = _pair_errors(cgs, cos, d)
        print(f"PRECISION drum at scale ({d.n_clumps} clumps, {d.n_spheres} spheres, {len(cg['a'])} contacts) "
              f"{prec}: pair {pe}; clump force max {ef.max():.3g}, clump torque max {et.max():.3g}", flush=True)
        if prec == "fp64":
            for k in ("F", "delta"):
                assert np.array_equal(cgs[k], cos[k]), k
            assert np.array_equal(Fg[clumps], Fo) and np.array_equal(Tg[clumps], To)
        else:
            check_pair_forces(cgs, cos, d)
            assert ef.max() <= FORCE_RTOL and et.max() <= FORCE_RTOL
