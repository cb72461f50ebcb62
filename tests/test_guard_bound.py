"""The displacement guard's per-clump bound (deferred detection, Sec. 2.2):
every sphere of a clump moves by at most |x - x_det| + 2 sin(theta/2) r_ctr,
theta the rotation between the two orientations, whose |sin(theta/2)| is the
norm of the vector part of conj(q_det) q.  The reduction kernel skips the
per-sphere test when this bound clears the clump's smallest margin, so the
inequality (and its tightness) is checked here in plain numpy."""
import numpy as np


def rot(q):
    """Rotation matrix of a unit quaternion (w, x, y, z)."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def qmul(a, b):
    aw, av, bw, bv = a[0], np.asarray(a[1:]), b[0], np.asarray(b[1:])
    return np.r_[aw * bw - av @ bv, aw * bv + bw * av + np.cross(av, bv)]


def vec_norm(qd, q):
    """|vector part of conj(qd) q|, written out as in the kernel."""
    dw, dx, dy, dz = qd
    qw, qx, qy, qz = q
    vx = dw * qx - qw * dx - (dy * qz - dz * qy)
    vy = dw * qy - qw * dy - (dz * qx - dx * qz)
    vz = dw * qz - qw * dz - (dx * qy - dy * qx)
    return np.sqrt(vx * vx + vy * vy + vz * vz)


def unit(v):
    return v / np.linalg.norm(v)


def test_written_out_vector_part_matches_the_quaternion_product():
    g = np.random.default_rng(5)
    for _ in range(200):
        qd, q = unit(g.normal(size=4)), unit(g.normal(size=4))
        conj = np.r_[qd[0], -qd[1:]]
        assert np.isclose(vec_norm(qd, q), np.linalg.norm(qmul(conj, q)[1:]), rtol=1e-12, atol=1e-15)


def test_bound_covers_every_sphere_displacement():
    g = np.random.default_rng(7)
    worst = 0.0
    for _ in range(2000):
        qd = unit(g.normal(size=4))
        # small and large rotations since the detection, either quaternion sign
        ang = g.choice([1e-6, 1e-3, 0.3, 3.0]) * g.random()
        ax = unit(g.normal(size=3))
        dq = np.r_[np.cos(ang / 2), np.sin(ang / 2) * ax]
        q = qmul(qd, dq) * g.choice([1.0, -1.0])
        xd = g.uniform(-4, 4, 3)
        x = xd + g.normal(size=3) * g.choice([0.0, 1e-6, 1e-3])
        r_ctr = g.uniform(1e-3, 5e-3)
        bound = np.linalg.norm(x - xd) + 2.0 * vec_norm(qd, q) * r_ctr
        for o in unit(g.normal(size=(6, 3))) * (r_ctr * g.random((6, 1))):
            d = np.linalg.norm((x + rot(q) @ o) - (xd + rot(qd) @ o))
            assert d <= bound * (1 + 1e-9) + 1e-12, (d, bound)
            worst = max(worst, d / bound if bound > 0 else 0.0)
    assert worst > 0.5  # the bound is not vacuous


def test_bound_is_reached_by_a_pure_rotation():
    """x = x_det and an offset of length r_ctr perpendicular to the axis:
    the displacement equals the rotation term exactly (up to rounding)."""
    qd = unit(np.array([0.3, -0.2, 0.9, 0.1]))
    ax, ang, r_ctr = unit(np.array([0.0, 0.0, 1.0])), 0.2, 4e-3
    q = qmul(qd, np.r_[np.cos(ang / 2), np.sin(ang / 2) * ax])
    o = np.array([r_ctr, 0.0, 0.0])
    d = np.linalg.norm(rot(q) @ o - rot(qd) @ o)
    assert np.isclose(d, 2.0 * vec_norm(qd, q) * r_ctr, rtol=1e-12)
    assert np.isclose(d, 2.0 * np.sin(ang / 2) * r_ctr, rtol=1e-12)
