"""A user force law compiled at run time into the pair kernel (hiprtc).

* The Hertz-Mindlin law written as a user law (tests/laws/hertz_mindlin.hip)
  reproduces the oracle bit for bit in the all-FP64 mode (first-step
  contacts, forces, histories and torques, and a 100-step trajectory of the
  contact-rich walled box), and in the FP32-force mode, where the user law
  runs in FP64, stays within the force tolerance of the oracle; restoring
  the built-in law gives the built-in path's trajectory again.
* A linear spring-dashpot law (tests/laws/linear_dashpot.hip: stiffness k,
  damping ratio zeta) reproduces its closed forms in a head-on collision of
  two spheres: restitution exp(-pi zeta / sqrt(1 - zeta^2)) and contact
  time pi / (omega_0 sqrt(1 - zeta^2)), omega_0 = sqrt(k / mbar), both
  independent of the impact speed.
* Deferred detection with a user law is bit-identical to per-step detection.
* A law that does not compile is refused and leaves the scene as it was."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2307_03445_amd import inputs as I
from paritylib import check_pair_forces, compare_pairs

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _law(name):
    with open(os.path.join(HERE, "laws", name)) as fh:
        return fh.read()


def _scene(desc, prec="fp64"):
    from paper_2307_03445_amd._lib import Scene
    return Scene(desc, precision=prec)


@pytest.fixture(scope="module")
def dense():
    return I.walled_box(dense=True)


def test_hertz_mindlin_user_law_matches_the_oracle_fp64(dense):
    sc, o = _scene(dense), oracle.Oracle(dense)
    sc.set_force_law(_law("hertz_mindlin.hip"))
    sc.record_next_step()
    sc.step(1)
    o.eval()
    cg, co = sc.contacts(), o.contacts()
    assert len(co["a"]) > 1000
    compare_pairs(cg, co)
    for k in ("delta", "F", "u", "Ta", "Tb"):
        assert np.array_equal(cg[k], co[k]), k
    Fg, Tg = sc.clump_forces()
    Fo, To = o.clump_forces()
    assert np.array_equal(Fg, Fo) and np.array_equal(Tg, To)
    sc.step(99)
    o.step(100)
    sg, so = sc.state(), o.state()
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(sg[k], so[k]), k


def test_hertz_mindlin_user_law_fp32_mode_and_restoring_the_builtin(dense):
    sc, o = _scene(dense, "fp32"), oracle.Oracle(dense)
    sc.set_force_law(_law("hertz_mindlin.hip"))
    sc.record_next_step()
    sc.step(1)
    o.eval()
    cg, co = sc.contacts(), o.contacts()
    compare_pairs(cg, co)
    info = check_pair_forces(cg, co, dense)
    print("user law in the FP32-force mode:", info, flush=True)
    # the built-in law back: the same trajectory as a scene that never had a user law
    sc.set_force_law(None)
    ref = _scene(dense, "fp32")
    ref.set_force_law(_law("hertz_mindlin.hip"))
    ref.step(1)
    ref.set_force_law(None)
    sc.step(50)
    ref.step(50)
    a, b = sc.state(), ref.state()
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(a[k], b[k]), k


def _headon_linear(v0, h=1e-6, r=1e-3):
    d = I.two_sphere_headon(r=r, v0=v0, h=h, gap=1e-9)
    sc = _scene(d)
    sc.set_force_law(_law("linear_dashpot.hip"))
    m = I.sphere_template(r)[2]
    mbar = m / 2.0
    steps, in_contact, t_c = 0, False, None
    chunk = 10
    while steps < 200000:
        sc.step(chunk)
        steps += chunk
        st = sc.state()
        gap = (st["x"][1, 0] - st["x"][0, 0]) - 2 * r
        if gap < 0:
            in_contact = True
        elif in_contact:
            t_c = steps * h
            break
    st = sc.state()
    vrel = st["v"][1, 0] - st["v"][0, 0]
    sc.close()
    return vrel / v0, t_c, mbar  # separation speed over approach speed


@pytest.mark.parametrize("v0", [0.05, 0.5])
def test_linear_spring_dashpot_user_law_closed_forms(v0):
    k, zeta = 1.0e3, 0.05  # as in tests/laws/linear_dashpot.hip
    e, t_c, mbar = _headon_linear(v0)
    e_exact = math.exp(-math.pi * zeta / math.sqrt(1 - zeta * zeta))
    w0 = math.sqrt(k / mbar)
    t_exact = math.pi / (w0 * math.sqrt(1 - zeta * zeta))
    print(f"v0 {v0}: e {e:.6f} (closed form {e_exact:.6f}), t_c {t_c:.6e} s (closed form {t_exact:.6e} s)",
          flush=True)
    assert abs(e - e_exact) <= 1e-4, (e, e_exact)
    assert abs(t_c - t_exact) <= 12e-6, (t_c, t_exact)  # sampled every 10 steps of 1 us


def test_deferred_detection_with_a_user_law_equals_per_step(dense):
    out = []
    for mode in ("plain", "fixed"):
        sc = _scene(dense)
        sc.set_force_law(_law("linear_dashpot.hip"))
        if mode == "fixed":
            sc.set_detection("fixed", k_max=10, safety=1.5, margin_cap=1e-4, audit_period=25)
        sc.step(100)
        out.append((sc.state(), sc.counts()))
        sc.close()
    (a, _), (b, cb) = out
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(a[k], b[k]), k
    assert cb["missed"] == 0 and cb["audits"] >= 3 and cb["detections"] < 50


def test_a_law_that_does_not_compile_leaves_the_scene_unchanged(dense):
    from paper_2307_03445_amd._lib import CdemError
    a, b = _scene(dense), _scene(dense)
    a.set_force_law(_law("linear_dashpot.hip"))
    b.set_force_law(_law("linear_dashpot.hip"))
    with pytest.raises(CdemError) as e:
        a.set_force_law("__device__ void cdem_user_law(const double *n) { nope; }")
    assert e.value.code == -1 and "nope" in str(e.value)
    a.step(30)
    b.step(30)
    sa, sb = a.state(), b.state()
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("pos_exp", [0, 40])
def test_user_law_on_meshes_and_fixed_point_positions(pos_exp):
    """The run-time compiled pair kernel takes every path of the built-in one:
    triangle contacts of moving meshes, and fixed-point positions.  With the
    Hertz-Mindlin law written as a user law, the mesh bin's contacts, forces,
    mesh forces and 60-step states are the oracle's, bit for bit."""
    import dataclasses
    d = dataclasses.replace(I.mesh_bin(n_clumps=300), pos_exp=pos_exp)
    sc, o = _scene(d), oracle.Oracle(d)
    sc.set_force_law(_law("hertz_mindlin.hip"))
    sc.step(60)
    o.step(60)
    sg, so = sc.state(), o.state()
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(sg[k], so[k]), k
    sc.record_next_step()
    sc.step(1)
    o.eval()
    cg, co = sc.contacts(), o.contacts()
    compare_pairs(cg, co)
    assert (cg["b"] >= d.n_spheres + d.n_bnd).sum() > 20
    for k in ("delta", "F", "u", "Ta", "Tb"):
        assert np.array_equal(cg[k], co[k]), k
    for x, y in zip(sc.mesh_forces(), o.mesh_forces()):
        assert np.array_equal(x, y)
