"""Comparison helpers shared by the parity tests (tolerances of the method's
accuracy targets: 1e-5 relative on per-step forces, 1e-4 on states after 100
steps, exact equality of contact-pair sets)."""
import numpy as np

FORCE_RTOL = 1e-5
STATE_TOL = 1e-4


def pair_keys(c):
    return c["a"].astype(np.uint64) << np.uint64(32) | c["b"].astype(np.uint64)


def compare_pairs(cg, co):
    """Contact sets must be identical; returns the index alignment (they are both sorted)."""
    kg, ko = pair_keys(cg), pair_keys(co)
    assert kg.shape == ko.shape and np.array_equal(kg, ko), \
        f"pair sets differ: gpu {len(kg)} oracle {len(ko)}; only-gpu {np.setdiff1d(kg, ko)[:5]} only-oracle {np.setdiff1d(ko, kg)[:5]}"


def pair_force_error(cg, co, Rbar):
    """Per-pair relative force error; pairs with delta/Rbar < 1e-6 are measured
    against the largest pair force instead of their own."""
    Fg, Fo = cg["F"], co["F"]
    err = np.linalg.norm(Fg - Fo, axis=1)
    mag = np.linalg.norm(Fo, axis=1)
    fmax = mag.max() if len(mag) else 1.0
    shallow = co["delta"] / Rbar < 1e-6
    denom = np.where(shallow, fmax, np.maximum(mag, 1e-300))
    return err / denom


def clump_force_error(Fg, Fo, scale):
    return np.linalg.norm(Fg - Fo, axis=1) / scale


def rotation_angle(qa, qb):
    """Angle of the rotation between unit quaternions qa and qb: four times
    the arcsine of half the chord between qa and +-qb (exact near zero, where
    an arccosine of their dot product loses half the digits)."""
    s = np.where((qa * qb).sum(1) < 0, -1.0, 1.0)[:, None]
    chord = np.linalg.norm(qa - s * qb, axis=1)
    return 4 * np.arcsin((chord / 2).clip(0, 1))


def state_errors(sg, so, r_min):
    vmax = np.linalg.norm(so["v"], axis=1).max()
    wmax = np.linalg.norm(so["w"], axis=1).max()
    wref = wmax if wmax > 0 else vmax / r_min
    return dict(
        x=np.linalg.norm(sg["x"] - so["x"], axis=1).max() / r_min,
        v=np.linalg.norm(sg["v"] - so["v"], axis=1).max() / max(vmax, 1e-300),
        w=np.linalg.norm(sg["w"] - so["w"], axis=1).max() / max(wref, 1e-300),
        q=rotation_angle(sg["q"], so["q"]).max(),
    )


def sphere_radii(desc):
    """Radius of every sphere instance (template radius of its clump's template)."""
    sb = np.asarray(desc.sphere_begin(), np.int64)
    owner = np.repeat(np.arange(desc.n_clumps), np.diff(sb))
    local = np.arange(desc.n_spheres) - sb[owner]
    tb = np.asarray(desc.tmpl_sphere_begin, np.int64)
    return np.asarray(desc.tmpl_radius)[tb[np.asarray(desc.clump_template, np.int64)[owner]] + local]


def hertz_scale(desc, c):
    """Elastic force scale (4/3) E* sqrt(Rbar delta) delta of every oracle contact
    (textbook Hertz with the pair's effective modulus), used to judge pairs whose
    net force is a near-cancellation of the spring and dashpot terms."""
    R = sphere_radii(desc)
    ns, nb = desc.n_spheres, desc.n_bnd
    a, b = c["a"].astype(np.int64), c["b"].astype(np.int64)
    wall = b >= ns
    # a wall's material: an analytic boundary's, or a triangle's mesh's
    wmat = np.concatenate([np.asarray(desc.bnd_mat, np.float64).reshape(-1, 4),
                           np.asarray(desc.mesh_mat, np.float64).reshape(-1, 4)[np.asarray(desc.tri_mesh, np.int64)]])
    mat_b = np.where(wall[:, None], wmat[np.clip(b - ns, 0, max(len(wmat) - 1, 0))] if len(wmat) else 0,
                     desc.sphere_mat[np.minimum(b, ns - 1)])
    mat_a = desc.sphere_mat[a]
    es = 1.0 / ((1 - mat_a[:, 1] ** 2) / mat_a[:, 0] + (1 - mat_b[:, 1] ** 2) / mat_b[:, 0])
    Rb = np.where(wall, np.inf, R[np.minimum(b, ns - 1)])
    Rbar = np.where(wall, R[a], R[a] * Rb / (R[a] + np.where(wall, 1.0, Rb)))
    dl = np.clip(c["delta"], 0, None)
    return 4.0 / 3.0 * es * np.sqrt(Rbar * dl) * dl


def check_pair_forces(cg, co, desc, rtol=FORCE_RTOL):
    """Per-pair force check: every pair within rtol of max(|F|, its Hertz scale),
    and at least 99 % of pairs within rtol of their own |F| (the rest are pairs
    whose net force is a near-cancellation of spring and dashpot)."""
    err = np.linalg.norm(cg["F"] - co["F"], axis=1)
    mag = np.linalg.norm(co["F"], axis=1)
    scale = np.maximum(mag, hertz_scale(desc, co))
    rel_scaled = err / np.maximum(scale, 1e-300)
    rel_own = err / np.maximum(mag, 1e-300)
    worst = int(np.argmax(rel_own)) if len(err) else 0
    info = dict(max_rel_scaled=float(rel_scaled.max()) if len(err) else 0.0,
                max_rel_own=float(rel_own.max()) if len(err) else 0.0,
                frac_own_ok=float((rel_own <= rtol).mean()) if len(err) else 1.0,
                worst=dict(a=int(co["a"][worst]), b=int(co["b"][worst]), delta=float(co["delta"][worst]),
                           F=co["F"][worst].tolist(), Fg=cg["F"][worst].tolist()) if len(err) else None)
    assert info["max_rel_scaled"] <= rtol and info["frac_own_ok"] >= 0.99, info
    return info
