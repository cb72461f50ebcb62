"""Long-run statistics of a settled bed and of a collapsed column, computed
the same way from any final state (GPU or oracle): the bulk packing fraction
and the angle of the deposit's free surface (angle of repose)."""
import numpy as np


def sphere_centres(desc, x, q):
    """Sphere centres and radii of a state (x [nc][3], q [nc][4] as w,x,y,z)."""
    w, a, b, c = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    A = np.empty((len(q), 3, 3))
    A[:, 0, 0] = 1 - 2 * (b * b + c * c); A[:, 0, 1] = 2 * (a * b - w * c); A[:, 0, 2] = 2 * (a * c + w * b)
    A[:, 1, 0] = 2 * (a * b + w * c); A[:, 1, 1] = 1 - 2 * (a * a + c * c); A[:, 1, 2] = 2 * (b * c - w * a)
    A[:, 2, 0] = 2 * (a * c - w * b); A[:, 2, 1] = 2 * (b * c + w * a); A[:, 2, 2] = 1 - 2 * (a * a + b * b)
    tb = desc.tmpl_sphere_begin.astype(np.int64)
    ct = desc.clump_template.astype(np.int64)
    cnt = tb[ct + 1] - tb[ct]
    owner = np.repeat(np.arange(len(ct)), cnt)
    local = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    ts = tb[ct][owner] + local
    o = desc.tmpl_offset[ts]
    xs = x[owner] + np.einsum("nij,nj->ni", A[owner], o)
    return xs, desc.tmpl_radius[ts]


def packing_fraction(xs, R, lo, hi, n_points=40000, seed=11):
    """Fraction of the box [lo, hi] covered by the union of spheres, by
    Monte-Carlo points from a fixed seed."""
    g = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    p = lo + (hi - lo) * g.random((n_points, 3))
    inside = np.zeros(n_points, bool)
    for k in range(0, len(xs), 256):  # chunks of spheres
        d2 = ((p[:, None, :] - xs[None, k:k + 256, :]) ** 2).sum(-1)
        inside |= (d2 < R[None, k:k + 256] ** 2).any(1)
    return float(inside.mean())


def bed_packing_fraction(xs, R, L, wall_gap):
    """Packing fraction of a settled bed in an L x L box: the sub-box
    `wall_gap` away from the side walls, from `wall_gap` above the floor up to
    the median height of the sphere centres."""
    ztop = float(np.median(xs[:, 2]))
    return packing_fraction(xs, R, (wall_gap, wall_gap, wall_gap), (L - wall_gap, L - wall_gap, ztop))


def slope_angle(xs, R, bin_width):
    """Angle (degrees) of the free surface of a deposit that descends along
    +x (a collapsed column against a wall at x = 0): the highest sphere top
    per x bin, and a least-squares line through the bins whose height lies
    between 10 % and 90 % of the tallest."""
    top = xs[:, 2] + R
    k = np.maximum((xs[:, 0] // bin_width).astype(int), 0)
    h = np.full(int(k.max()) + 1, -np.inf)
    np.maximum.at(h, k, top)
    xc = (np.arange(len(h)) + 0.5) * bin_width
    ok = np.isfinite(h)
    hmax = h[ok].max()
    sel = ok & (h >= 0.1 * hmax) & (h <= 0.9 * hmax)
    if sel.sum() < 3:
        return float("nan")
    slope = np.polyfit(xc[sel], h[sel], 1)[0]
    return float(np.degrees(np.arctan(-slope)))


def deposit_centroid(xs):
    """Mean distance of the sphere centres from the wall at x = 0: for a
    wedge-shaped deposit of fixed volume, a smaller centroid is a steeper
    slope (a lower-noise companion of the fitted angle)."""
    return float(xs[:, 0].mean())
