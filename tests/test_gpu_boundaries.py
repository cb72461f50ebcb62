"""GPU parity of the boundary primitives that the walled box does not reach:
an inner cylinder and its end caps spinning about their axis (a rotating
drum, configuration 3 scaled down) and a cone with its shaft moving through
a bed (configuration 2 scaled down: contacts on the tip, the face, the rim
and the shaft).  FP64 trajectories are bit-identical to the oracle; FP32
force arithmetic is within the force and state tolerances; deferred
detection (the fixed rule and the learned envelopes, whose candidate margin
also covers the boundaries' own motion) is bit-identical to per-step
detection with zero misses at the audits."""
import numpy as np
import pytest

import oracle
from paper_2307_03445_amd import inputs as I
from paritylib import FORCE_RTOL, STATE_TOL, check_pair_forces, compare_pairs, state_errors

pytestmark = pytest.mark.gpu

SCENES = {"drum": lambda: I.drum(), "cone": lambda: I.cone_bed()}


@pytest.fixture(scope="module", params=sorted(SCENES))
def scene(request):
    return request.param, SCENES[request.param]()


def _gpu(desc, prec="fp64"):
    from paper_2307_03445_amd._lib import Scene
    return Scene(desc, precision=prec)


def _boundary_contacts(c, desc):
    return np.unique(c["b"][c["b"] >= desc.n_spheres] - desc.n_spheres)


def test_first_step_contacts_bitwise_fp64(scene):
    name, d = scene
    sc, o = _gpu(d), oracle.Oracle(d)
    sc.record_next_step()
    sc.step(1)
    o.eval()
    cg, co = sc.contacts(), o.contacts()
    compare_pairs(cg, co)
    # the drum's cylinder and both caps carry contacts; the cone bed's floor
    # and cone (tip, rim and shaft probes, and the face)
    bc = set(_boundary_contacts(co, d).tolist())
    if name == "drum":
        assert bc == {0, 1, 2}, bc
    else:
        assert 0 in bc and (co["b"] == d.n_spheres + d.n_bnd - 1).sum() >= 4
    for k in ("delta", "F", "u", "Ta", "Tb"):
        assert np.array_equal(cg[k], co[k]), k
    Fg, Tg = sc.clump_forces()
    Fo, To = o.clump_forces()
    assert np.array_equal(Fg, Fo) and np.array_equal(Tg, To)
    bg, bo = sc.boundary_forces(), o.boundary_forces()
    for g_, o_ in zip(bg, bo):
        scale = np.abs(o_).max() + 1e-300
        assert np.abs(g_ - o_).max() <= 1e-12 * scale


def test_hundred_steps_bitwise_fp64(scene):
    name, d = scene
    sc, o = _gpu(d), oracle.Oracle(d)
    sc.step(100)
    o.step(100)
    sg, so = sc.state(), o.state()
    for k in sg:
        assert np.array_equal(sg[k], so[k]), (name, k)


def test_fp32_force_tolerances(scene):
    name, d = scene
    sc, o = _gpu(d, "fp32"), oracle.Oracle(d)
    sc.record_next_step()
    sc.step(1)
    o.eval()
    cg, co = sc.contacts(), o.contacts()
    compare_pairs(cg, co)
    info = check_pair_forces(cg, co, d)
    print(name, "fp32 first step", info)
    sc.step(99)
    o.step(100)
    err = state_errors(sc.state(), o.state(), d.tmpl_radius.min())
    print(name, "fp32 state after 100 steps", err)
    assert max(err.values()) <= STATE_TOL, err


@pytest.mark.parametrize("mode", ["fixed", "learned"])
def test_deferred_detection_bitwise_equals_plain(scene, mode):
    name, d = scene
    from paper_2307_03445_amd import train
    plain, dfr = _gpu(d), _gpu(d)
    if mode == "learned":
        dfr.set_mlp(np.load(train.WEIGHTS)["params"].astype(np.float32))
    dfr.set_detection(mode, k_max=20, safety=1.5, margin_cap=1e-4, audit_period=10)
    plain.step(200)
    dfr.step(200)
    sp, sf = plain.state(), dfr.state()
    for k in sp:
        assert np.array_equal(sp[k], sf[k]), (name, mode, k)
    c = dfr.counts()
    assert c["detections"] < 100 and c["audits"] >= 19 and c["missed"] == 0, c
