"""Pins of the oracle's triangle-mesh boundaries (rigid meshes with
prescribed motion), against what the mathematics fixes:

* a flat mesh (two triangles) is the same boundary as the analytic plane in
  its place: same contact, force, history, torque, and trajectories, up to
  the rounding of the different distance arithmetic; also when the mesh
  spins about its normal, against a plane with the same surface spin;
* the closest point and distance in a triangle's edge and vertex regions:
  the distance to the edge's line and to the vertex, the static Hertz force
  (4/3) E* sqrt(R delta) delta along the line from the closest point;
* prescribed motion: translation x0 + n h v, and a rotation whose angle per
  step is exactly 2 atan(h |w| / 2) (the first-order update renormalised);
* the force and torque the spheres exert on a mesh are minus the sum of its
  contact forces and r x (-F) about its reference point."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_03445_amd import inputs as I

MAT = (2e7, 0.25, 0.4, 0.6)


def _square(half=0.05, z=0.0):
    a, b, c, d = (-half, -half, z), (half, -half, z), (half, half, z), (-half, half, z)
    return [(a, b, c), (a, c, d)]


def _sphere_scene(p, v=(0, 0, 0), w=(0, 0, 0), r=1.5e-3, bnd=None, meshes=None, h=1e-6, g=(0, 0, 0)):
    t = I.sphere_template(r)
    return I.assemble([t], [0], [p], [(1, 0, 0, 0)], [v], [w], [MAT], g, (-0.1, -0.1, -0.1, 0.1, 0.1, 0.1), h,
                      bnd=bnd, meshes=meshes)


def _estar(E, nu):
    return 1.0 / (2 * (1 - nu * nu) / E)


def test_flat_mesh_is_the_analytic_plane():
    r, dl = 1.5e-3, 3e-6
    p = (0.013, -0.007, r - dl)
    v, w = (2e-3, -1e-3, -4e-3), (0.5, 0.2, -0.3)
    plane = _sphere_scene(p, v, w, bnd=[dict(type=I.BND_PLANE, param=(0, 0, 0, 0, 0, 1), mat=MAT)])
    mesh = _sphere_scene(p, v, w, meshes=[dict(vertices=_square(), mat=MAT)])
    op, om = oracle.Oracle(plane), oracle.Oracle(mesh)
    op.eval(), om.eval()
    cp, cm = op.contacts(), om.contacts()
    assert len(cp["a"]) == len(cm["a"]) == 1
    for k in ("delta", "F", "u", "Ta", "Tb"):
        assert np.allclose(cm[k], cp[k], rtol=1e-12, atol=1e-14 * np.abs(cp[k]).max()), k
    op.step(400), om.step(400)
    sp, sm = op.state(), om.state()
    for k in ("x", "v", "w"):
        assert np.allclose(sm[k], sp[k], rtol=1e-9, atol=1e-12), k


def test_spinning_mesh_is_a_plane_with_surface_spin():
    """A flat mesh spinning about its normal through the reference point, and
    an analytic plane with the same surface spin: the sphere sees the same
    surface velocity, so the same tangential force."""
    r, dl = 1.5e-3, 3e-6
    p = (0.02, 0.01, r - dl)
    om_ = (0.0, 0.0, 3.0)
    plane = _sphere_scene(p, bnd=[dict(type=I.BND_PLANE, param=(0, 0, 0, 0, 0, 1), mat=MAT, omega=om_)])
    mesh = _sphere_scene(p, meshes=[dict(vertices=_square(), mat=MAT, w=om_)])
    op, om = oracle.Oracle(plane), oracle.Oracle(mesh)
    op.eval(), om.eval()
    Fp, Fm = op.contacts()["F"][0], om.contacts()["F"][0]
    assert abs(Fp[0]) > 0 and np.allclose(Fm, Fp, rtol=1e-12, atol=1e-14 * np.abs(Fp).max())


@pytest.mark.parametrize("region", ["edge", "vertex"])
def test_edge_and_vertex_regions(region):
    """The sphere's centre lies beyond an edge (or a vertex) of a triangle:
    its distance is that to the edge's line (or to the vertex), the normal
    points from that closest point to the centre, and at rest the force is
    the static Hertz force along it."""
    r = 1.5e-3
    tri = [((0.0, 0.0, 0.0), (0.02, 0.0, 0.0), (0.0, 0.02, 0.0))]
    if region == "edge":   # beyond the hypotenuse x + y = 0.02, above the plane
        foot = np.array([0.012, 0.008, 0.0])
        out = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
        dirn = 0.6 * out + 0.8 * np.array([0, 0, 1.0])
    else:                  # beyond the vertex (0.02, 0, 0)
        foot = np.array([0.02, 0.0, 0.0])
        dirn = np.array([0.48, -0.6, 0.64])
    dirn = dirn / np.linalg.norm(dirn)
    dist = r - 2.5e-6
    p = foot + dist * dirn
    o = oracle.Oracle(_sphere_scene(tuple(p), meshes=[dict(vertices=tri, mat=MAT)]))
    o.eval()
    c = o.contacts()
    assert len(c["a"]) == 1 and c["b"][0] == 1  # the triangle: n_spheres + n_bnd + 0
    dl = r - dist
    assert abs(c["delta"][0] / dl - 1) < 1e-9
    F = c["F"][0]
    Fth = 4.0 / 3.0 * _estar(*MAT[:2]) * math.sqrt(r * dl) * dl
    assert np.allclose(F, Fth * dirn, rtol=1e-8, atol=1e-12 * Fth)
    # torque on the sphere about its centre: the force acts along the line through it
    assert np.abs(c["Tb"][0]).max() <= 1e-12 * Fth * r


def test_prescribed_translation_and_rotation():
    h, n = 1e-6, 5000
    v, w = np.array([0.03, -0.01, 0.02]), np.array([0.0, 2.0, 1.0])
    x0 = np.array([0.001, 0.002, -0.003])
    d = _sphere_scene((0, 0, 0.05), meshes=[dict(vertices=_square(), mat=MAT, x=tuple(x0), v=tuple(v), w=tuple(w))], h=h)
    o = oracle.Oracle(d)
    o.step(n)
    st = o.mesh_state()[0]
    xs = x0.copy()
    for _ in range(n):  # the closed form of the iterated update
        xs = xs + h * v
    assert np.array_equal(st[:3], xs)
    assert np.array_equal(st[7:10], v) and np.array_equal(st[10:13], w)
    q = st[3:7]
    assert abs(np.linalg.norm(q) - 1.0) < 1e-15
    ang = 2.0 * math.atan2(np.linalg.norm(q[1:]), q[0])
    wn = np.linalg.norm(w)
    assert abs(ang - 2.0 * n * math.atan(h * wn / 2.0)) < 1e-11
    assert np.allclose(q[1:] / np.linalg.norm(q[1:]), w / wn, rtol=0, atol=1e-12)


def test_mesh_force_and_torque_readout():
    """Two spheres on a flat mesh whose reference point is off to the side:
    the mesh receives minus their contact forces, and r x (-F) about its
    reference point."""
    r, dl = 1.5e-3, 3e-6
    t = I.sphere_template(r)
    ref = np.array([0.03, -0.02, 0.0])
    verts = [tuple(tuple(np.array(vv) - ref) for vv in tri) for tri in _square()]
    d = I.assemble([t, t], [0, 1], [(0.01, 0.0, r - dl), (-0.012, 0.007, r - 2 * dl)], [(1, 0, 0, 0)] * 2,
                   [(1e-3, 0, 0), (0, -2e-3, 0)], [(0, 0, 0)] * 2, [MAT, MAT], (0, 0, 0),
                   (-0.1, -0.1, -0.1, 0.1, 0.1, 0.1), 1e-6, meshes=[dict(vertices=verts, mat=MAT, x=tuple(ref))])
    o = oracle.Oracle(d)
    o.eval()
    c = o.contacts()
    assert len(c["a"]) == 2
    F, T = o.mesh_forces()
    Fexp = -c["F"].sum(0)
    xs = o.sphere_pos()
    Texp = np.zeros(3)
    for k in range(2):
        s = int(c["a"][k])
        pc = xs[s] - (r - 0.5 * c["delta"][k]) * np.array([0, 0, 1.0])  # contact point, normal +z
        Texp += np.cross(pc - ref, -c["F"][k])
    assert np.allclose(F[0], Fexp, rtol=1e-13)
    assert np.allclose(T[0], Texp, rtol=1e-9, atol=1e-15)
