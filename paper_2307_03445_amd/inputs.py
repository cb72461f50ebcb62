"""Seeded synthetic scene generators for the clumped-sphere DEM timestep.

This module produces *inputs only*: clump templates (sphere offsets, radii,
mass and principal inertia), clump states, per-sphere materials, analytic
boundaries and prescribed-motion bodies.  It holds none of the timestep's
arithmetic (no contact detection, no force law, no integration), so that both
the FP64 CPU oracle and the HIP path can be driven from the same seeded inputs
without sharing any of the method's code.

The element model follows the paper's multi-sphere clump representation
(Sec. 2.1, "clump" paragraph and Fig. "force"): a clump is a rigid union of
possibly overlapping spheres; mass and moment of inertia belong to the clump,
while E, nu, mu and CoR belong to each sphere instance.

Conventions (shared by every consumer of a :class:`SceneDesc`):

* SI units, 0-based indices, structure-of-arrays.
* Template sphere offsets are expressed in the clump's principal body frame,
  relative to the clump centre of mass; ``tmpl_inertia`` holds the principal
  moments about the centre of mass.
* ``q`` is a unit quaternion (w, x, y, z) rotating body to world.
* ``w`` is the angular velocity in the *body* (principal) frame.
* Spheres are numbered clump by clump: clump ``c`` owns the consecutive sphere
  ids ``sphere_begin[c] .. sphere_begin[c+1]-1`` in template order.
* ``sphere_mat[s] = (E, nu, mu, CoR)`` for every sphere instance ``s``.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 230703445

# Boundary primitive types.  Parameters (12 doubles per boundary), at t = 0:
#   PLANE      : p0[3], n[3]                      (n: unit normal into the domain)
#   CYL_IN     : p0[3], a[3], R                   (domain inside the cylinder)
#   CONE_OUT   : apex[3], a[3], sin, cos, H       (solid cone + shaft, domain outside;
#                                                  a points from the apex into the solid)
#   FRUSTUM_IN : apex[3], a[3], sin, cos, t0, t1  (funnel wall, domain inside,
#                                                  active for axial distance t0..t1)
BND_PLANE, BND_CYL_IN, BND_CONE_OUT, BND_FRUSTUM_IN = 0, 1, 2, 3
BND_NPARAM = 12

# Prescribed-motion parameters (12 doubles per prescribed clump):
#   v_fixed[3], free[3] (1.0 = component integrated, 0.0 = held at v_fixed),
#   w_body[3] (angular velocity held fixed, body frame), f_extra[3] (world force
#   added to free components).
PRESC_NPARAM = 12

DENSITY = 2600.0


def rng(stream: int, replica: int = 0) -> np.random.Generator:
    """Generator of seed stream ``stream`` (one per workload: 1 walled box,
    2 bed templates, 4 funnels, 5 rover bed, 6 and 7 statistics scenes, 8 cone
    bed, 9 drum, 10 deposited funnels, 11 mesh bin) and replica."""
    return np.random.default_rng(np.random.SeedSequence(SEED_ROOT, spawn_key=(stream, replica)))


@dataclass
class SceneDesc:
    """Complete input of one (possibly batched) DEM simulation."""

    h: float
    tmpl_sphere_begin: np.ndarray
    tmpl_offset: np.ndarray
    tmpl_radius: np.ndarray
    tmpl_mass: np.ndarray
    tmpl_inertia: np.ndarray
    clump_template: np.ndarray
    clump_scene: np.ndarray
    x: np.ndarray
    q: np.ndarray
    v: np.ndarray
    w: np.ndarray
    sphere_mat: np.ndarray
    gravity: np.ndarray
    domain: np.ndarray
    bnd_type: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    bnd_param: np.ndarray = field(default_factory=lambda: np.zeros((0, BND_NPARAM)))
    bnd_mat: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    bnd_vel: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    bnd_omega: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    bnd_scene: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    presc_clump: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    presc_param: np.ndarray = field(default_factory=lambda: np.zeros((0, PRESC_NPARAM)))
    # triangle meshes: rigid boundaries with prescribed motion
    mesh_state: np.ndarray = field(default_factory=lambda: np.zeros((0, 13)))  # x[3], q[4], v[3], w[3] (world)
    mesh_mat: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    mesh_scene: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    tri_mesh: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    tri_vertex: np.ndarray = field(default_factory=lambda: np.zeros((0, 3, 3)))  # mesh frame
    # clump positions: 0 FP64, else fixed point with resolution 2^-pos_exp m
    pos_exp: int = 0
    name: str = "scene"

    # ---- derived sizes -------------------------------------------------
    @property
    def n_templates(self) -> int:
        return int(self.tmpl_mass.shape[0])

    @property
    def n_clumps(self) -> int:
        return int(self.clump_template.shape[0])

    @property
    def n_scenes(self) -> int:
        return int(self.gravity.shape[0])

    @property
    def n_bnd(self) -> int:
        return int(self.bnd_type.shape[0])

    @property
    def n_mesh(self) -> int:
        return int(np.asarray(self.mesh_scene).shape[0])

    @property
    def n_tri(self) -> int:
        return int(np.asarray(self.tri_mesh).shape[0])

    def clump_sphere_counts(self) -> np.ndarray:
        tsz = np.diff(self.tmpl_sphere_begin.astype(np.int64))
        return tsz[self.clump_template.astype(np.int64)]

    def sphere_begin(self) -> np.ndarray:
        cnt = self.clump_sphere_counts()
        out = np.zeros(self.n_clumps + 1, np.int64)
        np.cumsum(cnt, out=out[1:])
        return out

    @property
    def n_spheres(self) -> int:
        return int(self.clump_sphere_counts().sum())

    def canonical(self) -> "SceneDesc":
        """Return a copy with every array in the dtype/layout the bindings expect."""
        f = lambda a, s=None: np.ascontiguousarray(np.asarray(a, np.float64).reshape(s) if s else np.asarray(a, np.float64))
        nt, nc, nb, npr, ns = self.n_templates, self.n_clumps, len(self.bnd_type), len(self.presc_clump), self.gravity.size // 3
        return dataclasses.replace(
            self,
            h=float(self.h),
            tmpl_sphere_begin=np.ascontiguousarray(self.tmpl_sphere_begin, np.uint32),
            tmpl_offset=f(self.tmpl_offset, (-1, 3)),
            tmpl_radius=f(self.tmpl_radius),
            tmpl_mass=f(self.tmpl_mass),
            tmpl_inertia=f(self.tmpl_inertia, (nt, 3)),
            clump_template=np.ascontiguousarray(self.clump_template, np.uint32),
            clump_scene=np.ascontiguousarray(self.clump_scene, np.uint32),
            x=f(self.x, (nc, 3)), q=f(self.q, (nc, 4)), v=f(self.v, (nc, 3)), w=f(self.w, (nc, 3)),
            sphere_mat=f(self.sphere_mat, (-1, 4)),
            gravity=f(self.gravity, (ns, 3)), domain=f(self.domain, (ns, 6)),
            bnd_type=np.ascontiguousarray(self.bnd_type, np.int32),
            bnd_param=f(self.bnd_param, (nb, BND_NPARAM)), bnd_mat=f(self.bnd_mat, (nb, 4)),
            bnd_vel=f(self.bnd_vel, (nb, 3)), bnd_omega=f(self.bnd_omega, (nb, 3)),
            bnd_scene=np.ascontiguousarray(self.bnd_scene, np.int32),
            presc_clump=np.ascontiguousarray(self.presc_clump, np.int32),
            presc_param=f(self.presc_param, (npr, PRESC_NPARAM)),
            mesh_state=f(self.mesh_state, (self.n_mesh, 13)), mesh_mat=f(self.mesh_mat, (self.n_mesh, 4)),
            mesh_scene=np.ascontiguousarray(self.mesh_scene, np.int32),
            tri_mesh=np.ascontiguousarray(self.tri_mesh, np.int32),
            tri_vertex=f(self.tri_vertex, (self.n_tri, 3, 3)),
            pos_exp=int(self.pos_exp),
        )

    def validate(self) -> None:
        """Raise ValueError for inputs no consumer may accept."""
        d = self
        nt = d.n_templates
        if d.tmpl_sphere_begin.shape != (nt + 1,) or d.tmpl_sphere_begin[0] != 0:
            raise ValueError("tmpl_sphere_begin must be a CSR offset array starting at 0")
        if np.any(np.diff(d.tmpl_sphere_begin.astype(np.int64)) < 1):
            raise ValueError("every template needs at least one sphere")
        nts = int(d.tmpl_sphere_begin[-1])
        if d.tmpl_offset.shape != (nts, 3) or d.tmpl_radius.shape != (nts,):
            raise ValueError("template sphere arrays have the wrong shape")
        if np.any(d.tmpl_radius <= 0) or np.any(d.tmpl_mass <= 0) or np.any(d.tmpl_inertia <= 0):
            raise ValueError("radii, masses and inertias must be positive")
        if d.n_clumps and int(d.clump_template.max()) >= nt:
            raise ValueError("clump_template out of range")
        if d.n_clumps and int(d.clump_scene.max()) >= d.n_scenes:
            raise ValueError("clump_scene out of range")
        qn = np.linalg.norm(d.q, axis=1)
        if np.any(np.abs(qn - 1.0) > 1e-12):
            raise ValueError("quaternions must be unit")
        m = d.sphere_mat
        if m.shape != (d.n_spheres, 4):
            raise ValueError("sphere_mat must have one (E, nu, mu, CoR) row per sphere")
        for mm in (m, d.bnd_mat):
            if mm.size and (np.any(mm[:, 0] <= 0) or np.any(mm[:, 1] <= -1) or np.any(mm[:, 1] >= 0.5)
                            or np.any(mm[:, 2] < 0) or np.any(mm[:, 3] <= 0) or np.any(mm[:, 3] > 1)):
                raise ValueError("material out of range (E>0, -1<nu<0.5, mu>=0, 0<CoR<=1)")
        if not (d.h > 0):
            raise ValueError("time step must be positive")


# ---------------------------------------------------------------------------
# Rotations (input construction only)
# ---------------------------------------------------------------------------

def random_unit_quaternions(g: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed unit quaternions (Shoemake's subgroup method)."""
    u1, u2, u3 = g.random(n), g.random(n), g.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                  a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)], axis=1)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1.0
    return q


def random_unit_vectors(g: np.random.Generator, n: int) -> np.ndarray:
    z = g.normal(size=(n, 3))
    return z / np.linalg.norm(z, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# Template mass properties (voxel integration of the sphere union)
# ---------------------------------------------------------------------------

def union_mass_properties(offsets: np.ndarray, radii: np.ndarray, density: float = DENSITY, res: int = 48):
    """Mass, centre of mass and inertia tensor of a union of spheres.

    Midpoint-rule integration on a ``res``^3 grid over the union's bounding
    box.  Accuracy is that of the grid; both consumers receive the same numbers,
    so nothing downstream depends on it beyond physical plausibility.
    Returns (mass, com[3], inertia_about_com[3,3]).
    """
    offsets = np.asarray(offsets, np.float64).reshape(-1, 3)
    radii = np.asarray(radii, np.float64).reshape(-1)
    if offsets.shape[0] == 1:
        m = density * 4.0 / 3.0 * np.pi * radii[0] ** 3
        return m, offsets[0].copy(), np.eye(3) * (0.4 * m * radii[0] ** 2)
    lo = (offsets - radii[:, None]).min(0)
    hi = (offsets + radii[:, None]).max(0)
    step = (hi - lo) / res
    axes = [lo[k] + (np.arange(res) + 0.5) * step[k] for k in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    inside = np.zeros(P.shape[0], bool)
    for o, r in zip(offsets, radii):
        inside |= ((P - o) ** 2).sum(1) <= r * r
    P = P[inside]
    dV = float(np.prod(step))
    mass = density * dV * P.shape[0]
    com = P.mean(0)
    d = P - com
    dm = density * dV
    r2 = (d * d).sum(1)
    I = dm * (np.eye(3) * r2.sum() - d.T @ d)
    return mass, com, I


def principal_template(offsets: np.ndarray, radii: np.ndarray, density: float = DENSITY, res: int = 48):
    """Recentre a sphere set on its CoM and rotate it to principal axes.

    Returns (body_offsets[n,3], radii[n], mass, principal_moments[3]).
    """
    mass, com, I = union_mass_properties(offsets, radii, density, res)
    evals, evecs = np.linalg.eigh(I)
    if np.linalg.det(evecs) < 0:
        evecs[:, 2] *= -1.0
    body = (np.asarray(offsets, np.float64) - com) @ evecs
    return body, np.asarray(radii, np.float64).copy(), float(mass), evals.astype(np.float64)


def sphere_template(r: float, density: float = DENSITY):
    """A single-sphere clump: exact mass and moment of inertia."""
    m = density * 4.0 / 3.0 * math.pi * r ** 3
    return np.zeros((1, 3)), np.array([r]), m, np.full(3, 0.4 * m * r * r)


def bounding_radius(body_offsets: np.ndarray, radii: np.ndarray) -> float:
    return float((np.linalg.norm(body_offsets, axis=1) + radii).max())


# ---------------------------------------------------------------------------
# Assembly helpers
# ---------------------------------------------------------------------------

def assemble(templates, clump_template, x, q, v, w, sphere_mat, gravity, domain, h,
             clump_scene=None, bnd=None, presc=None, meshes=None, name="scene") -> SceneDesc:
    """Build a SceneDesc from a list of (offsets, radii, mass, moments) templates."""
    sizes = [t[0].shape[0] for t in templates]
    begin = np.zeros(len(templates) + 1, np.uint32)
    begin[1:] = np.cumsum(sizes)
    nc = len(clump_template)
    ng = np.asarray(gravity, np.float64).reshape(-1, 3).shape[0]
    d = SceneDesc(
        h=h,
        tmpl_sphere_begin=begin,
        tmpl_offset=np.concatenate([t[0] for t in templates]).reshape(-1, 3),
        tmpl_radius=np.concatenate([t[1] for t in templates]),
        tmpl_mass=np.array([t[2] for t in templates], np.float64),
        tmpl_inertia=np.array([t[3] for t in templates], np.float64).reshape(-1, 3),
        clump_template=np.asarray(clump_template, np.uint32),
        clump_scene=np.zeros(nc, np.uint32) if clump_scene is None else np.asarray(clump_scene, np.uint32),
        x=np.asarray(x, np.float64).reshape(nc, 3), q=np.asarray(q, np.float64).reshape(nc, 4),
        v=np.asarray(v, np.float64).reshape(nc, 3), w=np.asarray(w, np.float64).reshape(nc, 3),
        sphere_mat=np.asarray(sphere_mat, np.float64).reshape(-1, 4),
        gravity=np.asarray(gravity, np.float64).reshape(ng, 3),
        domain=np.asarray(domain, np.float64).reshape(ng, 6),
        name=name,
    )
    if bnd:
        d.bnd_type = np.array([b["type"] for b in bnd], np.int32)
        P = np.zeros((len(bnd), BND_NPARAM))
        for i, b in enumerate(bnd):
            P[i, :len(b["param"])] = b["param"]
        d.bnd_param = P
        d.bnd_mat = np.array([b["mat"] for b in bnd], np.float64).reshape(-1, 4)
        d.bnd_vel = np.array([b.get("vel", (0, 0, 0)) for b in bnd], np.float64).reshape(-1, 3)
        d.bnd_omega = np.array([b.get("omega", (0, 0, 0)) for b in bnd], np.float64).reshape(-1, 3)
        d.bnd_scene = np.array([b.get("scene", 0) for b in bnd], np.int32)
    if presc:
        d.presc_clump = np.array([p["clump"] for p in presc], np.int32)
        P = np.zeros((len(presc), PRESC_NPARAM))
        for i, p in enumerate(presc):
            P[i, 0:3] = p.get("v_fixed", (0, 0, 0))
            P[i, 3:6] = p.get("free", (0, 0, 0))
            P[i, 6:9] = p.get("w_body", (0, 0, 0))
            P[i, 9:12] = p.get("f_extra", (0, 0, 0))
        d.presc_param = P
    if meshes:
        # each: vertices [n][3][3] in the mesh frame, x, q, v, w (world angular velocity), mat, scene
        d.mesh_state = np.array([np.r_[m.get("x", (0, 0, 0)), m.get("q", (1, 0, 0, 0)), m.get("v", (0, 0, 0)),
                                       m.get("w", (0, 0, 0))] for m in meshes], np.float64).reshape(-1, 13)
        d.mesh_mat = np.array([m["mat"] for m in meshes], np.float64).reshape(-1, 4)
        d.mesh_scene = np.array([m.get("scene", 0) for m in meshes], np.int32)
        d.tri_vertex = np.concatenate([np.asarray(m["vertices"], np.float64).reshape(-1, 3, 3) for m in meshes])
        d.tri_mesh = np.concatenate([np.full(np.asarray(m["vertices"]).reshape(-1, 3, 3).shape[0], i, np.int32)
                                     for i, m in enumerate(meshes)])
    return d.canonical()


def box_walls(lo, hi, mat, floor=True, ceiling=False, scene=0):
    """Axis-aligned planes: floor (z=lo), the four sides, optionally a ceiling."""
    (x0, y0, z0), (x1, y1, z1) = lo, hi
    walls = []
    if floor:
        walls.append(dict(type=BND_PLANE, param=(0, 0, z0, 0, 0, 1), mat=mat, scene=scene))
    walls += [dict(type=BND_PLANE, param=(x0, 0, 0, 1, 0, 0), mat=mat, scene=scene),
              dict(type=BND_PLANE, param=(x1, 0, 0, -1, 0, 0), mat=mat, scene=scene),
              dict(type=BND_PLANE, param=(0, y0, 0, 0, 1, 0), mat=mat, scene=scene),
              dict(type=BND_PLANE, param=(0, y1, 0, 0, -1, 0), mat=mat, scene=scene)]
    if ceiling:
        walls.append(dict(type=BND_PLANE, param=(0, 0, z1, 0, 0, -1), mat=mat, scene=scene))
    return walls


def lattice_sites(nx, ny, nz, spacing, origin):
    """Simple-cubic lattice sites, x fastest, then y, then z."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(np.float64) * spacing
    return pts + np.asarray(origin, np.float64)


# ---------------------------------------------------------------------------
# Sequential deposition (contact-rich initial states)
# ---------------------------------------------------------------------------

def quat_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrices of unit quaternions (input construction only)."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def deposit(g: np.random.Generator, templates, clump_template, footprint, sink_max, floor_z=0.0, floor=None,
            edge=None, pre=None):
    """Drop clumps one by one onto a growing pile.

    Each clump gets a uniformly random orientation and a uniformly random
    (x, y) that keeps it inside ``footprint = (x0, y0, x1, y1)``; it falls
    vertically to the highest position at which one of its spheres first
    touches an already placed sphere or the floor, and is then lowered by a
    random sink ~ U[0, sink_max] so that it rests with a small overlap.
    ``floor(px, py, r)`` (arrays) may give the lowest centre height of a
    sphere of radius r at (px, py) for a floor other than the plane
    z = floor_z (a drum's curved bottom).  ``edge = (p, axes)`` places a
    clump, with probability p, flush against the low or high side of the
    footprint along one of ``axes`` ("x", "y" or "xy"), pressed into it by
    U[0, sink_max] (contacts with side walls and end caps).  ``pre`` lists
    poses (x[3], q[4]) of the first len(pre) clumps, placed as given before
    the others fall.  This is a geometric construction of a contact-rich
    initial state; no dynamics is simulated.  Returns (x[n,3], q[n,4]).
    """
    x0, y0, x1, y1 = footprint
    n = len(clump_template)
    q = random_unit_quaternions(g, n)
    rmax = max(float(t[1].max()) for t in templates)
    cell = 2.0 * rmax
    nx = max(1, int(math.ceil((x1 - x0) / cell)))
    ny = max(1, int(math.ceil((y1 - y0) / cell)))
    cols = [[] for _ in range(nx * ny)]
    P = []   # placed sphere centres
    Rr = []  # placed sphere radii
    xs = np.empty((n, 3))
    npre = 0 if pre is None else len(pre)
    for i in range(npre):
        q[i] = pre[i][1]
    R = quat_matrix(q)
    for i in range(n):
        off, rad = templates[clump_template[i]][0], templates[clump_template[i]][1]
        wo = off @ R[i].T
        if i < npre:
            cx, cy, zc = pre[i][0]
            xs[i] = (cx, cy, zc)
            for j in range(wo.shape[0]):
                p = (cx + wo[j, 0], cy + wo[j, 1], zc + wo[j, 2])
                k = len(P)
                P.append(p); Rr.append(float(rad[j]))
                jx = min(nx - 1, max(0, int((p[0] - x0) // cell))); jy = min(ny - 1, max(0, int((p[1] - y0) // cell)))
                cols[jy * nx + jx].append(k)
            continue
        lo_x = float((wo[:, 0] - rad).min()); hi_x = float((wo[:, 0] + rad).max())
        lo_y = float((wo[:, 1] - rad).min()); hi_y = float((wo[:, 1] + rad).max())
        cx = g.uniform(x0 - lo_x, x1 - hi_x)
        cy = g.uniform(y0 - lo_y, y1 - hi_y)
        if edge is not None and g.random() < edge[0]:
            ax = edge[1][int(g.integers(0, len(edge[1])))]
            hi_side = g.random() < 0.5
            sk = g.uniform(0.0, sink_max)
            if ax == "x":
                cx = (x1 - hi_x + sk) if hi_side else (x0 - lo_x - sk)
            else:
                cy = (y1 - hi_y + sk) if hi_side else (y0 - lo_y - sk)
        fl = floor_z + rad if floor is None else floor(cx + wo[:, 0], cy + wo[:, 1], rad)
        zc = float((fl - wo[:, 2]).max())  # resting on the floor
        ix0 = max(0, int((cx + lo_x - rmax - x0) // cell)); ix1 = min(nx - 1, int((cx + hi_x + rmax - x0) // cell))
        iy0 = max(0, int((cy + lo_y - rmax - y0) // cell)); iy1 = min(ny - 1, int((cy + hi_y + rmax - y0) // cell))
        cand = [k for jy in range(iy0, iy1 + 1) for jx in range(ix0, ix1 + 1) for k in cols[jy * nx + jx]]
        if cand:
            cand = np.asarray(cand)
            Pc = np.asarray(P)[cand] if isinstance(P, np.ndarray) else np.array([P[k] for k in cand])
            Rc = np.array([Rr[k] for k in cand])
            sx = cx + wo[:, 0]; sy = cy + wo[:, 1]
            dh2 = (sx[:, None] - Pc[None, :, 0]) ** 2 + (sy[:, None] - Pc[None, :, 1]) ** 2
            S2 = (rad[:, None] + Rc[None, :]) ** 2
            ok = dh2 < S2
            if ok.any():
                zt = np.where(ok, Pc[None, :, 2] + np.sqrt(np.where(ok, S2 - dh2, 0.0)) - wo[:, 2:3], -np.inf)
                zc = max(zc, float(zt.max()))
        zc -= g.uniform(0.0, sink_max)
        zc = max(zc, float((fl - wo[:, 2]).max()) - sink_max)
        xs[i] = (cx, cy, zc)
        for j in range(wo.shape[0]):
            p = (cx + wo[j, 0], cy + wo[j, 1], zc + wo[j, 2])
            k = len(P)
            P.append(p); Rr.append(float(rad[j]))
            jx = min(nx - 1, max(0, int((p[0] - x0) // cell))); jy = min(ny - 1, max(0, int((p[1] - y0) // cell)))
            cols[jy * nx + jx].append(k)
    return xs, q


# ---------------------------------------------------------------------------
# Configuration 1: 2,000 three-sphere clumps in a 5 cm box (CPU-checkable)
# ---------------------------------------------------------------------------

BOX_MAT = (1e7, 0.3, 0.5, 0.5)


def _unit_three_sphere_props(dirs: np.ndarray, res: int = 32):
    """Mass properties of unit-radius three-sphere unions (centres 0.6 along
    ``dirs[i, j]``), batched; returns (volume[n], com[n,3], inertia/density[n,3,3])."""
    n = dirs.shape[0]
    ext = 1.6
    step = 2 * ext / res
    ax = -ext + (np.arange(res) + 0.5) * step
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    dV = step ** 3
    PP = (P[:, :, None] * P[:, None, :]).reshape(-1, 9)
    vol = np.empty(n); com = np.empty((n, 3)); I = np.empty((n, 3, 3))
    for lo in range(0, n, 64):
        cen = 0.6 * dirs[lo:lo + 64]                              # [b,3,3]
        inside = np.zeros((cen.shape[0], P.shape[0]), bool)
        for j in range(3):
            c3 = cen[:, j, :]
            d2 = (P * P).sum(1)[None, :] - 2.0 * (c3 @ P.T) + (c3 * c3).sum(1)[:, None]
            inside |= d2 <= 1.0
        inside = inside.astype(np.float64)                        # [b,p]
        cnt = inside.sum(1)
        c = inside @ P / cnt[:, None]
        vol[lo:lo + 64] = cnt * dV
        com[lo:lo + 64] = c
        s1 = inside @ P                                           # [b,3]
        s2 = (inside @ PP).reshape(-1, 3, 3)                       # [b,3,3]
        cov = s2 - s1[:, :, None] * c[:, None, :] - c[:, :, None] * s1[:, None, :] \
            + cnt[:, None, None] * c[:, :, None] * c[:, None, :]
        tr = np.trace(cov, axis1=1, axis2=2)
        I[lo:lo + 64] = (tr[:, None, None] * np.eye(3) - cov) * dV
    return vol, com, I


def _box_templates(g: np.random.Generator, n: int, res: int = 32):
    """n three-sphere templates, radius r ~ U[1,2] mm shared by the three spheres,
    centres offset 0.6 r along independent random unit axes; recentred on the
    CoM and rotated to principal axes (mass properties by voxel integration)."""
    r = g.uniform(1e-3, 2e-3, n)
    dirs = random_unit_vectors(g, 3 * n).reshape(n, 3, 3)
    vol, com, I = _unit_three_sphere_props(dirs, res)
    out = []
    for i in range(n):
        evals, evecs = np.linalg.eigh(I[i])
        if np.linalg.det(evecs) < 0:
            evecs[:, 2] *= -1.0
        body = (0.6 * dirs[i] - com[i]) @ evecs * r[i]
        mass = DENSITY * vol[i] * r[i] ** 3
        out.append((body, np.full(3, r[i]), float(mass), DENSITY * evals * r[i] ** 5))
    return out


def walled_box(replica: int = 0, n_clumps: int = 2000, dense: bool = False, res: int = 32,
            vel_noise: float = 0.05) -> SceneDesc:
    """Configuration 1 (plain method, CPU-checkable).

    2,000 clumps of three spheres each, one template per clump, random
    orientation, simple-cubic lattice of spacing 2*max(bounding radius)+0.1 mm,
    7 x 7 sites per layer inside a 5 cm x 5 cm footprint with a floor and four
    side walls; the box height is raised to hold the lattice (the 5 cm cube of
    the configuration cannot hold 2,000 non-overlapping clumps).  Velocity per
    component ~ U[-0.05, 0.05] m/s, gravity -9.81 z, E=1e7 Pa, nu=0.3,
    mu=0.5, CoR=0.5 for spheres and walls, h = 1e-6 s.

    ``dense=True`` builds a contact-rich variant from the same clumps and
    materials: the clumps are deposited one by one (:func:`deposit`) into the
    5 cm x 5 cm footprint, each sinking up to 2 % of the smallest radius into
    the pile, with the same velocity noise.
    """
    g = rng(1, replica)
    tmpls = _box_templates(g, n_clumps, res)
    L = 0.05
    mat = np.tile(np.array(BOX_MAT), (3 * n_clumps, 1))
    if dense:
        x, q = deposit(g, tmpls, np.arange(n_clumps), (0.0, 0.0, L, L), 0.02 * 1e-3)
        top = float(x[:, 2].max()) + 0.02
    else:
        rb = max(bounding_radius(t[0], t[1]) for t in tmpls)
        spacing, nxy = 2.0 * rb + 1e-4, 7
        nz = -(-n_clumps // (nxy * nxy))
        origin = (L / 2 - spacing * (nxy - 1) / 2, L / 2 - spacing * (nxy - 1) / 2, spacing / 2 + 5e-5)
        sites = lattice_sites(nxy, nxy, nz, spacing, origin)
        perm = g.permutation(sites.shape[0])[:n_clumps]
        x = sites[perm]
        q = random_unit_quaternions(g, n_clumps)
        top = nz * spacing + 0.01
    v = g.uniform(-vel_noise, vel_noise, (n_clumps, 3))
    w = np.zeros((n_clumps, 3))
    walls = box_walls((0, 0, 0), (L, L, top), BOX_MAT)
    return assemble(tmpls, np.arange(n_clumps), x, q, v, w, mat, (0, 0, -9.81),
                    (0, 0, 0, L, L, top), 1e-6, bnd=walls,
                    name=f"box{'-dense' if dense else ''}-r{replica}")


# ---------------------------------------------------------------------------
# Shared templates of the bed, funnel and rover workloads
# ---------------------------------------------------------------------------

BED_SPHERE_COUNTS = (1, 2, 3, 3, 3, 3, 4, 6)


def lognormal_radii(g: np.random.Generator, n: int, median=2e-3, sigma=0.3):
    """Lognormal radii (median 2 mm, sigma 0.3) clipped to +-3 sigma."""
    z = np.clip(g.normal(size=n), -3.0, 3.0)
    return median * np.exp(sigma * z)


def multisphere_template(g: np.random.Generator, count: int, radii=None, res: int = 64):
    """A template of ``count`` spheres, each offset 0.6 r along a random axis."""
    r = lognormal_radii(g, count) if radii is None else np.asarray(radii, np.float64)
    if count == 1:
        return sphere_template(float(r[0]))
    dirs = random_unit_vectors(g, count)
    return principal_template(0.6 * r[:, None] * dirs, r, DENSITY, res)


def bed_templates(replica: int = 0, res: int = 64):
    g = rng(2, replica)
    return [multisphere_template(g, c, res=res) for c in BED_SPHERE_COUNTS]


# ---------------------------------------------------------------------------
# Small hand-built scenes used to pin the oracle against closed forms
# ---------------------------------------------------------------------------

def two_sphere_headon(r=1e-3, v0=0.05, mat=BOX_MAT, gap=1e-7, h=1e-6, r2=None):
    """Two single-sphere clumps approaching head-on along x, no gravity."""
    r2 = r if r2 is None else r2
    t1, t2 = sphere_template(r), sphere_template(r2)
    x = [(-(r + gap / 2), 0, 0), (r2 + gap / 2, 0, 0)]
    v = [(v0 / 2, 0, 0), (-v0 / 2, 0, 0)]
    q = [(1, 0, 0, 0)] * 2
    return assemble([t1, t2], [0, 1], x, q, v, np.zeros((2, 3)), [mat, mat], (0, 0, 0),
                    (-0.01, -0.01, -0.01, 0.01, 0.01, 0.01), h, name="headon")


# ---------------------------------------------------------------------------
# Configuration 5: rover-scale bed (~11M clumps, ~34M spheres) with a wheel
# ---------------------------------------------------------------------------

def morton_order(x: np.ndarray, cell: float) -> np.ndarray:
    """Permutation sorting points by the Morton (Z-order) code of their cell."""
    c = np.floor((x - x.min(0)) / cell).astype(np.int64)
    c = np.clip(c, 0, (1 << 20) - 1)

    def spread(v):
        v = v & 0x1FFFFF
        v = (v | (v << 32)) & 0x1F00000000FFFF
        v = (v | (v << 16)) & 0x1F0000FF0000FF
        v = (v | (v << 8)) & 0x100F00F00F00F00F
        v = (v | (v << 4)) & 0x10C30C30C30C30C3
        v = (v | (v << 2)) & 0x1249249249249249
        return v

    code = spread(c[:, 0]) | (spread(c[:, 1]) << 1) | (spread(c[:, 2]) << 2)
    return np.argsort(code, kind="stable")


def wheel_template(n_spheres=20000, R=0.25, width=0.2, r=4e-3, n_grouser=12, mass=10.0):
    """Rigid wheel made of spheres: a cylindrical rim (axle along body y) plus
    n_grouser grouser rows standing out of it; principal axes are x, y, z.
    Mass properties of a thin shell of the given mass."""
    n_g_layers = 2
    n_w = 50
    n_rim = n_spheres - n_grouser * n_g_layers * (n_spheres // 1000)
    n_gw = n_spheres // 1000                           # spheres across one grouser layer
    n_theta = n_rim // n_w
    n_rim = n_theta * n_w
    n_gw = (n_spheres - n_rim) // (n_grouser * n_g_layers)
    th = 2 * np.pi * np.arange(n_theta) / n_theta
    yy = np.linspace(-width / 2, width / 2, n_w)
    T, Y = np.meshgrid(th, yy, indexing="ij")
    rim = np.stack([R * np.cos(T).ravel(), Y.ravel(), R * np.sin(T).ravel()], 1)
    gth = 2 * np.pi * np.arange(n_grouser) / n_grouser
    gy = np.linspace(-width / 2, width / 2, n_gw)
    grs = []
    for L in range(1, n_g_layers + 1):
        rr = R + L * r
        G, Yg = np.meshgrid(gth, gy, indexing="ij")
        grs.append(np.stack([rr * np.cos(G).ravel(), Yg.ravel(), rr * np.sin(G).ravel()], 1))
    off = np.concatenate([rim] + grs)
    extra = n_spheres - off.shape[0]
    if extra > 0:  # pad the rim's middle ring so the count is exact
        ang = 2 * np.pi * (np.arange(extra) + 0.5) / extra
        off = np.concatenate([off, np.stack([R * np.cos(ang), np.zeros(extra), R * np.sin(ang)], 1)])
    off = off[:n_spheres]
    I_axle = mass * R * R
    I_other = mass * (R * R / 2 + width * width / 12)
    return off, np.full(off.shape[0], r), float(mass), np.array([I_other, I_axle, I_other])


def surface_points(tris: np.ndarray, spacing: float) -> np.ndarray:
    """Points covering every triangle at most `spacing` apart (a barycentric
    grid on each), for clearance checks of a mesh against a bed."""
    out = []
    for t in np.asarray(tris, np.float64):
        L = max(np.linalg.norm(t[1] - t[0]), np.linalg.norm(t[2] - t[1]), np.linalg.norm(t[0] - t[2]))
        n = max(1, int(np.ceil(L / spacing)))
        i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
        keep = i + j <= n
        u, v = i[keep] / n, j[keep] / n
        out.append(t[0] + u[:, None] * (t[1] - t[0]) + v[:, None] * (t[2] - t[0]))
    return np.concatenate(out)


def wheel_mesh(R=0.254, width=0.2, n_theta=120, n_grouser=12, gh=8e-3, gt=8e-3):
    """A rigid wheel as a triangle mesh in its body frame (axle along y,
    centre at the origin): a cylindrical rim of radius R (n_theta facets),
    two end discs, and n_grouser grousers, boxes gh tall and gt thick across
    the full width, standing on the rim.  Returns [n][3][3] vertices."""
    tris = []
    th = 2 * np.pi * np.arange(n_theta + 1) / n_theta
    y0, y1 = -width / 2, width / 2
    for i in range(n_theta):
        a = (R * np.cos(th[i]), R * np.sin(th[i]))
        b = (R * np.cos(th[i + 1]), R * np.sin(th[i + 1]))
        p00, p01 = (a[0], y0, a[1]), (a[0], y1, a[1])
        p10, p11 = (b[0], y0, b[1]), (b[0], y1, b[1])
        tris += [(p00, p10, p11), (p00, p11, p01)]
        tris += [((0.0, y0, 0.0), p10, p00), ((0.0, y1, 0.0), p01, p11)]
    for j in range(n_grouser):
        ph = 2 * np.pi * (j + 0.5) / n_grouser
        er, et = np.array([np.cos(ph), 0.0, np.sin(ph)]), np.array([-np.sin(ph), 0.0, np.cos(ph)])
        ey = np.array([0.0, 1.0, 0.0])
        c = [R * 0.99 * er + sr * gh * er + st * gt / 2 * et + sy * width / 2 * ey
             for sr in (0, 1) for st in (-1, 1) for sy in (-1, 1)]  # corners, index 4 sr + 2 st' + sy'
        P = lambda r, t, y: tuple(c[4 * r + 2 * t + y])
        faces = [((0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1)), ((1, 0, 0), (1, 0, 1), (1, 1, 1), (1, 1, 0)),
                 ((0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 0, 0)), ((0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1)),
                 ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)), ((0, 0, 1), (0, 1, 1), (1, 1, 1), (1, 0, 1))]
        for f in faces:
            q = [P(*v) for v in f]
            tris += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
    return np.asarray(tris, np.float64)


def layered_lattice(g: np.random.Generator, templates, clump_template, footprint, gap=2e-4, z0=0.0):
    """Spawn positions on a lattice of size-homogeneous layers.

    Clumps are sorted by bounding radius and cut into layers of equal count;
    each layer's spacing is 2 x its largest bounding radius + gap, so no two
    clumps overlap; layers are stacked in random order.  Returns (x, q) in the
    input order of ``clump_template``.
    """
    x0, y0, x1, y1 = footprint
    rb_t = np.array([bounding_radius(t[0], t[1]) for t in templates])
    rb = rb_t[clump_template]
    n = len(clump_template)
    order = np.argsort(rb, kind="stable")
    layers = []
    i = 0
    while i < n:
        # the layer size follows from the spacing its largest member needs
        s_guess = 2 * rb[order[i]] + gap
        per = max(1, int((x1 - x0) // s_guess)) * max(1, int((y1 - y0) // s_guess))
        j = min(n, i + per)
        s = 2 * rb[order[j - 1]] + gap
        nxl, nyl = max(1, int((x1 - x0) // s)), max(1, int((y1 - y0) // s))
        j = min(n, i + nxl * nyl)
        layers.append((order[i:j], s, nxl, nyl))
        i = j
    perm = g.permutation(len(layers))
    x = np.empty((n, 3))
    z = z0
    for li in perm:
        ids, s, nxl, nyl = layers[li]
        z += s / 2
        k = np.arange(len(ids))
        ox = x0 + ((x1 - x0) - nxl * s) / 2 + s / 2
        oy = y0 + ((y1 - y0) - nyl * s) / 2 + s / 2
        x[ids, 0] = ox + (k % nxl) * s
        x[ids, 1] = oy + (k // nxl) * s
        x[ids, 2] = z
        z += s / 2
    return x, random_unit_quaternions(g, n)


def rover_patch_scene(replica: int = 0, n_clumps: int = 6875, side: float = 0.05, h: float = 5e-6,
                     cor: float = 0.2) -> SceneDesc:
    """The preparation scene of the rover bed: one side x side patch
    of the bed templates spawned on a size-layered lattice inside
    a walled box, to be settled under gravity (with a larger step and a lower
    CoR than the measured run, which only speeds up the preparation)."""
    g = rng(5, replica)
    tmpls = bed_templates(replica)
    ct = g.integers(0, len(tmpls), n_clumps)
    x, q = layered_lattice(g, tmpls, ct, (0.0, 0.0, side, side))
    sizes = np.array([t[0].shape[0] for t in tmpls])
    ns = int(sizes[ct].sum())
    mat = np.empty((ns, 4))
    mat[:, 0] = g.uniform(1e7, 5e7, ns)
    mat[:, 1] = 0.3
    mat[:, 2] = g.uniform(0.3, 0.8, ns)
    mat[:, 3] = cor
    top = float(x[:, 2].max()) + 0.02
    walls = box_walls((0, 0, 0), (side, side, top), (5e7, 0.3, 0.5, cor))
    return assemble(tmpls, ct, x, q, np.zeros((n_clumps, 3)), np.zeros((n_clumps, 3)), mat, (0, 0, -9.81),
                    (0, 0, 0, side, side, top), h, bnd=walls, name=f"rover-patch-r{replica}")


def rover_deposited_patch(replica: int = 0, n_clumps: int = 6875, side: float = 0.05, sink_max: float = 2e-5):
    """A rover-bed patch built on the CPU alone: the clumps of
    :func:`rover_patch_scene` (same templates, same template draw) dropped one
    by one with :func:`deposit`.  Much looser than the settled patch, but every
    clump rests in contact; for checks whose input must not come from a
    simulation run.  Returns (x[n,3], q[n,4])."""
    g = rng(5, replica)
    tmpls = bed_templates(replica)
    ct = g.integers(0, len(tmpls), n_clumps)
    return deposit(g, tmpls, ct, (0.0, 0.0, side, side), sink_max)


def _bed_top_spheres(X, Q, CT, tmpls, cx, cy, half_x, half_y, depth=0.015):
    """Centres and radii of the bed spheres within `depth` of the top, under
    the rectangle |x - cx| < half_x, |y - cy| < half_y, sorted by x."""
    near = np.nonzero((np.abs(X[:, 0] - cx) < half_x) & (np.abs(X[:, 1] - cy) < half_y))[0]
    near = near[X[near, 2] > X[near, 2].max() - 2 * depth]
    Ps, Rs = [], []
    for t in np.unique(CT[near]):
        idx = near[CT[near] == t]
        Ps.append((X[idx][:, None, :] + np.einsum("kij,sj->ksi", quat_matrix(Q[idx]), tmpls[t][0])).reshape(-1, 3))
        Rs.append(np.tile(tmpls[t][1], len(idx)))
    Ps, Rs = np.concatenate(Ps), np.concatenate(Rs)
    keep = Ps[:, 2] + Rs > (Ps[:, 2] + Rs).max() - depth
    Ps, Rs = Ps[keep], Rs[keep]
    so = np.argsort(Ps[:, 0])
    return Ps[so], Rs[so]


def _resting_height(pts, r, cx, cy, Ps, Rs):
    """Lowest height of a body's reference point (at cx, cy) at which none of
    its points `pts` (offsets from the reference point, each a sphere of
    radius r; r = 0 for surface points) overlaps a sphere (Ps, Rs, sorted by
    x)."""
    pts = pts[np.argsort(pts[:, 0])]
    reach = float(Rs.max()) + r
    zc = -np.inf
    for k in range(0, pts.shape[0], 1024):  # points in x order against the spheres of their x strip
        q = pts[k:k + 1024]
        a = np.searchsorted(Ps[:, 0], cx + q[0, 0] - reach)
        b = np.searchsorted(Ps[:, 0], cx + q[-1, 0] + reach, side="right")
        if a >= b:
            continue
        P_, R_ = Ps[a:b], Rs[a:b] + r
        dx = (cx + q[:, None, 0]) - P_[None, :, 0]
        dy = (cy + q[:, None, 1]) - P_[None, :, 1]
        h2 = R_[None, :] ** 2 - dx * dx - dy * dy
        z = np.where(h2 > 0, P_[None, :, 2] + np.sqrt(np.where(h2 > 0, h2, 0.0)) - q[:, None, 2], -np.inf)
        zc = max(zc, float(z.max()))
    return zc


def rover_bed(patch_x: np.ndarray, patch_q: np.ndarray, replica: int = 0, n_clumps: int = 11_000_000,
            bed=(4.0, 1.0), side: float = 0.05, wheel_spheres: int = 20000, with_wheel: bool = True,
            wheel_x: float = 1.0, wheel: str = "clump") -> SceneDesc:
    """Configuration 5 (the metric's workload), tiled from a settled patch.

    ``patch_x``/``patch_q`` are the settled clump poses of
    :func:`rover_patch_scene` (same replica); the patch is Morton-sorted and
    copied over the 4 m x 1 m bed (the paper prepares large beds from copies of
    a settled base patch), truncated to ``n_clumps``.  Copies are spaced by the
    patch width plus the depth its spheres press into the patch walls, so no
    two copies overlap (the bed is that much wider than nominal).  Per-sphere-instance
    E ~ U[1e7, 5e7] Pa, mu ~ U[0.3, 0.8]; nu = 0.3; CoR = 0.5; h = 1e-6 s;
    clumps start at rest.  A rigid 20,000-sphere wheel (R = 0.25 m, width
    0.2 m, 12 grousers, 10 kg) rests on the surface, driven at slip 0.2
    (omega = 0.8 rad/s, v = (1 - 0.2) omega R) with a free vertical degree of
    freedom under a total load of 100 N; it starts pressed 20 um into the
    bed's top spheres beneath it and sinks in under its load.  With ``wheel="mesh"`` the wheel is
    the triangle mesh of :func:`wheel_mesh` instead (the rim's outer surface
    and grouser tips where the sphere wheel has them), moving at the same
    velocities, pressed the same 20 um into the bed; its vertical motion is
    then the caller's (co-simulation).
    """
    g = rng(5, 1000 + replica)
    tmpls = bed_templates(replica)
    ct_p = rng(5, replica).integers(0, len(tmpls), patch_x.shape[0])
    order = morton_order(patch_x, 0.01)
    xp, qp, ct_p = patch_x[order], patch_q[order], ct_p[order]
    # sphere centres of the patch: the settled spheres press into the patch's
    # walls, so copies are placed one wall-penetration apart (no overlap at seams)
    Rm = quat_matrix(qp)
    P = np.concatenate([xp[k] + tmpls[ct_p[k]][0] @ Rm[k].T for k in range(len(ct_p))])
    Rr = np.concatenate([tmpls[ct_p[k]][1] for k in range(len(ct_p))])
    lo = np.array([max(0.0, -(P[:, a] - Rr).min()) for a in range(2)])
    hi = np.array([max(0.0, (P[:, a] + Rr).max() - side) for a in range(2)])
    pitch = side + lo + hi + 1e-6
    ntx, nty = int(round(bed[0] / side)), int(round(bed[1] / side))
    tiles = [(i, j) for j in range(nty) for i in range(ntx)]
    tiles = [tiles[k] for k in morton_order(np.array([(i, j, 0) for i, j in tiles], float), 1.0)]
    X = np.concatenate([xp + np.array([lo[0] + i * pitch[0], lo[1] + j * pitch[1], 0.0]) for i, j in tiles])[:n_clumps]
    Q = np.tile(qp, (len(tiles), 1))[:n_clumps]
    CT = np.tile(ct_p, len(tiles))[:n_clumps]
    bed = (ntx * pitch[0], nty * pitch[1])
    nc = X.shape[0]
    sizes = np.array([t[0].shape[0] for t in tmpls])
    ns_bed = int(sizes[CT].sum())
    mat = np.empty((ns_bed, 4))
    mat[:, 0] = g.uniform(1e7, 5e7, ns_bed)
    mat[:, 1] = 0.3
    mat[:, 2] = g.uniform(0.3, 0.8, ns_bed)
    mat[:, 3] = 0.5
    V = np.zeros((nc, 3))
    W = np.zeros((nc, 3))
    templates = list(tmpls)
    presc = None
    top = float(X[:, 2].max())
    meshes = None
    if with_wheel and wheel == "mesh":
        R = 0.25
        tv = wheel_mesh(R=R + 4e-3, gh=8e-3)
        cx, cy = wheel_x, bed[1] / 2
        # points 2 mm apart over the wheel's lowest 15 mm, against the bed's
        # top spheres under it: the deepest point 20 um inside a sphere
        low = tv[tv[:, :, 2].min(1) < -0.5 * R]
        pts = surface_points(low, 2e-3)
        pts = pts[pts[:, 2] < pts[:, 2].min() + 0.015]
        Ps, Rs = _bed_top_spheres(X, Q, CT, tmpls, cx, cy, R + 0.03, 0.13)
        zc = _resting_height(pts, 0.0, cx, cy, Ps, Rs) - 2e-5
        om = 0.8
        vx = (1 - 0.2) * om * R
        meshes = [dict(vertices=tv, x=(cx, cy, zc), v=(vx, 0.0, 0.0), w=(0.0, om, 0.0), mat=(5e7, 0.3, 0.8, 0.5))]
        top = max(top, zc + R + 0.02)
    elif with_wheel:
        wt = wheel_template(wheel_spheres)
        templates.append(wt)
        R, wr = 0.25, float(wt[1][0])
        cx, cy = wheel_x, bed[1] / 2
        # its lowest spheres against the bed's top spheres under it: the
        # deepest overlap 20 um, so that it bears on the bed from the first step
        wo = wt[0]
        wlow = wo[wo[:, 2] < wo[:, 2].min() + 0.015]
        Ps, Rs = _bed_top_spheres(X, Q, CT, tmpls, cx, cy, R + 0.03, 0.13)
        zc = _resting_height(wlow, wr, cx, cy, Ps, Rs) - 2e-5
        X = np.vstack([X, [cx, cy, zc]])
        Q = np.vstack([Q, [1.0, 0.0, 0.0, 0.0]])
        CT = np.r_[CT, len(tmpls)]
        om = 0.8
        vx = (1 - 0.2) * om * R
        V = np.vstack([V, [vx, 0, 0]])
        W = np.vstack([W, [0, om, 0]])
        mat = np.vstack([mat, np.tile([5e7, 0.3, 0.8, 0.5], (wt[0].shape[0], 1))])
        presc = [dict(clump=nc, v_fixed=(vx, 0, 0), free=(0, 0, 1), w_body=(0, om, 0),
                      f_extra=(0, 0, -(100.0 - wt[2] * 9.81)))]
        top = max(top, zc + R + 0.02)
    walls = box_walls((0, 0, 0), (bed[0], bed[1], top + 0.05), (5e7, 0.3, 0.5, 0.5))
    return assemble(templates, CT, X, Q, V, W, mat, (0, 0, -9.81), (0, 0, 0, bed[0], bed[1], top + 0.05),
                    1e-6, bnd=walls, presc=presc, meshes=meshes, name=f"rover-r{replica}")


# ---------------------------------------------------------------------------
# Configuration 2: a bed penetrated by a descending cone; configuration 3: a
# rotating drum
# ---------------------------------------------------------------------------

CONE_SIN, CONE_COS = 0.5, math.sqrt(3.0) / 2.0   # half-angle 30 degrees (a 60-degree cone)
CONE_BASE_RADIUS = 10.14e-3                       # base area 323 mm^2
CONE_SPEED = 0.03                                 # descent [m/s]
WALL_MAT = (5e7, 0.3, 0.5, 0.5)


def bed_materials(g: np.random.Generator, ns: int, cor: float = 0.5) -> np.ndarray:
    """Per-sphere-instance materials of the bed workloads: E ~ U[1e7, 5e7] Pa,
    nu = 0.3, mu ~ U[0.3, 0.8], the given CoR."""
    mat = np.empty((ns, 4))
    mat[:, 0] = g.uniform(1e7, 5e7, ns)
    mat[:, 1] = 0.3
    mat[:, 2] = g.uniform(0.3, 0.8, ns)
    mat[:, 3] = cor
    return mat


def grid_mesh(half: float, n: int, jitter: float, g: np.random.Generator) -> np.ndarray:
    """A square surface of side 2*half about the origin in the plane z = 0,
    n x n cells, each split into two triangles along alternating diagonals,
    every vertex raised by U[-jitter, jitter] (so that spheres meet faces,
    edges and vertices).  Returns [2 n^2][3][3] vertices."""
    t = np.linspace(-half, half, n + 1)
    X, Y = np.meshgrid(t, t, indexing="ij")
    Z = g.uniform(-jitter, jitter, X.shape)
    V = np.stack([X, Y, Z], -1)
    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = V[i, j], V[i + 1, j], V[i + 1, j + 1], V[i, j + 1]
            if (i + j) % 2 == 0:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
    return np.asarray(tris, np.float64)


def mesh_bin(replica: int = 0, n_clumps: int = 600, n_grid: int = 24, jitter: float = 5e-6, spin: float = 20.0,
             push: float = 0.2, res: int = 32) -> SceneDesc:
    """Clumps on triangle meshes with prescribed motion (the paper's
    funnels and wheels are meshes).

    Three-sphere clumps (radius U[1, 2] mm, as in the walled box) deposited
    into a 5 cm x 5 cm bin with analytic side walls, onto a turntable: a
    triangulated floor (n_grid^2 cells, vertices jittered by +-jitter) that
    spins at ``spin`` rad/s about the vertical axis through the bin's centre
    and extends past the corners at any angle.  A vertical plate of two
    triangles, at the low-x side of the pile, moves into it at ``push`` m/s;
    a third of the clumps are pressed against the plate or the opposite
    wall.  Materials E = 1e7 Pa, nu = 0.3, mu = 0.5, CoR = 0.5; gravity
    -9.81 z; h = 1e-6 s."""
    g = rng(11, replica)
    tmpls = _box_templates(g, n_clumps, res)
    L = 0.05
    xp = 0.004  # the plate's plane
    x, q = deposit(g, tmpls, np.arange(n_clumps), (xp, 0.0, L, L), 2e-5, edge=(0.3, "x"))
    top = float(x[:, 2].max()) + 0.01
    v = g.uniform(-0.02, 0.02, (n_clumps, 3))
    w = np.zeros((n_clumps, 3))
    mat = np.tile(np.array(BOX_MAT), (3 * n_clumps, 1))
    floor = grid_mesh(0.75 * L, n_grid, jitter, g)
    hz = 0.5 * top
    plate = np.array([[(0.0, 0.0, -hz), (0.0, L, -hz), (0.0, L, hz)],
                      [(0.0, 0.0, -hz), (0.0, L, hz), (0.0, 0.0, hz)]])
    plate[:, :, 1] -= 0.5 * L
    meshes = [dict(vertices=floor, x=(0.5 * L, 0.5 * L, 0.0), w=(0.0, 0.0, spin), mat=BOX_MAT),
              dict(vertices=plate, x=(xp, 0.5 * L, hz), v=(push, 0.0, 0.0), mat=BOX_MAT)]
    walls = box_walls((0, 0, 0), (L, L, top), BOX_MAT, floor=False)
    return assemble(tmpls, np.arange(n_clumps), x, q, v, w, mat, (0, 0, -9.81), (0, 0, -0.005, L, L, top), 1e-6,
                    bnd=walls, meshes=meshes, name=f"mesh-bin-r{replica}")


def mesh_wheel_box(replica: int = 0, n_clumps: int = 600, res: int = 32) -> SceneDesc:
    """A small wheel mesh (R = 12 mm rim, 20 mm wide, 8 grousers 2 mm tall)
    pressed 20 um into a deposited pile of three-sphere clumps in a walled
    5 cm box, driven forward at 0.1 m/s while turning at 5 rad/s (its
    vertical motion is the co-simulation's)."""
    d = walled_box(replica=replica, n_clumps=n_clumps, dense=True, res=res)
    tv = wheel_mesh(R=0.012, width=0.02, n_theta=48, n_grouser=8, gh=2e-3, gt=2e-3)
    cx, cy = 0.018, 0.025
    sb = d.sphere_begin()
    P = np.concatenate([d.x[c] + (d.tmpl_offset[d.tmpl_sphere_begin[d.clump_template[c]]:
                                                 d.tmpl_sphere_begin[d.clump_template[c] + 1]]
                                  @ quat_matrix(d.q[c]).T) for c in range(d.n_clumps)])
    R = sphere_radii_of(d)
    assert P.shape[0] == sb[-1]
    # the lowest centre height at which no point of the surface (1 mm apart)
    # is inside a sphere, less 20 um
    V = surface_points(tv[tv[:, :, 2].min(1) < 0], 1e-3)
    zc = -np.inf
    for k in range(0, V.shape[0], 64):
        v = V[k:k + 64]
        dx = (cx + v[:, None, 0]) - P[None, :, 0]
        dy = (cy + v[:, None, 1]) - P[None, :, 1]
        h2 = R[None, :] ** 2 - dx ** 2 - dy ** 2
        z = np.where(h2 > 0, P[None, :, 2] + np.sqrt(np.where(h2 > 0, h2, 0.0)) - v[:, None, 2], -np.inf)
        zc = max(zc, float(z.max()))
    mesh = dict(vertices=tv, x=(cx, cy, zc - 2e-5), v=(0.1, 0.0, 0.0), w=(0.0, 5.0, 0.0), mat=WALL_MAT)
    return dataclasses.replace(d, mesh_state=np.r_[mesh["x"], (1, 0, 0, 0), mesh["v"], mesh["w"]][None, :],
                               mesh_mat=np.array([WALL_MAT], np.float64), mesh_scene=np.zeros(1, np.int32),
                               tri_mesh=np.zeros(tv.shape[0], np.int32), tri_vertex=tv,
                               name=f"mesh-wheel-box-r{replica}")


def sphere_radii_of(d: SceneDesc) -> np.ndarray:
    """Radius of every sphere instance of a description."""
    tb = np.asarray(d.tmpl_sphere_begin, np.int64)
    ct = np.asarray(d.clump_template, np.int64)
    return np.concatenate([d.tmpl_radius[tb[t]:tb[t + 1]] for t in ct])


def cone_bed(replica: int = 0, n_clumps: int = 600, side: float = 0.05, shaft: float = 12e-3,
             sink_max: float = 2e-5, h: float = 1e-6) -> SceneDesc:
    """Configuration 2 scaled down (the cone-penetration test, in the frame in
    which the cone rises into the bed from below): an analytic cone of
    half-angle 30 degrees and base radius 10.14 mm with a cylindrical shaft
    of that radius below its base stands on the floor of a side x side box
    (four walls), apex up, the shaft ``shaft`` long; it moves up at
    0.03 m/s.  Clumps of the eight bed templates (per-sphere-instance
    E ~ U[1e7, 5e7] Pa and mu ~ U[0.3, 0.8], nu = 0.3, CoR = 0.5) are
    deposited around and onto it, so that spheres rest on its tip, face and
    rim as well as on the floor and against the walls.  Clumps start at rest."""
    g = rng(8, replica)
    tmpls = bed_templates(replica)
    ct = g.integers(0, len(tmpls), n_clumps)
    ct[:3] = 0  # the one-sphere template: probes on the tip, the rim and the shaft
    rb = CONE_BASE_RADIUS
    H = rb * CONE_COS / CONE_SIN
    ax, ay, z_apex = side / 2, side / 2, shaft + H
    z_rim = z_apex - H
    cot = CONE_COS / CONE_SIN

    def floor(px, py, r):
        # lowest centre height of a sphere of radius r over (px, py): the
        # floor, or resting on the cone's tip, face or rim
        rho = np.hypot(px - ax, py - ay)
        foot = rho - r * CONE_COS
        on_face = z_apex - rho * cot + r / CONE_SIN
        on_tip = z_apex + np.sqrt(np.maximum(r * r - rho * rho, 0.0))
        on_rim = z_rim + np.sqrt(np.maximum(r * r - (rho - rb) ** 2, 0.0))
        z = np.where(foot < 0.0, on_tip, np.where(foot <= rb, on_face,
                     np.where(rho - rb < r, on_rim, -np.inf)))
        return np.maximum(r, z)

    # probes pressed 10 um into the cone: on the tip, at the rim edge (between
    # the face's and the shaft's normals) and against the shaft below the rim
    r0 = float(tmpls[0][1][0])
    dr = r0 - 1e-5
    c15, s15 = math.cos(math.radians(15.0)), math.sin(math.radians(15.0))
    one = (1.0, 0.0, 0.0, 0.0)
    pre = [((ax, ay, z_apex + dr), one),
           ((ax + rb + c15 * dr, ay, z_rim + s15 * dr), one),
           ((ax, ay - (rb + dr), z_rim - 0.5 * shaft), one)]
    x, q = deposit(g, tmpls, ct, (0.0, 0.0, side, side), sink_max, floor=floor, edge=(0.1, "xy"), pre=pre)
    sizes = np.array([t[0].shape[0] for t in tmpls])
    mat = bed_materials(g, int(sizes[ct].sum()))
    z_top = float(x[:, 2].max()) + 0.03
    walls = box_walls((0, 0, 0), (side, side, z_top), WALL_MAT)
    cone = dict(type=BND_CONE_OUT, param=(ax, ay, z_apex, 0, 0, -1, CONE_SIN, CONE_COS, H), mat=WALL_MAT,
                vel=(0, 0, CONE_SPEED))
    n = n_clumps
    return assemble(tmpls, ct, x, q, np.zeros((n, 3)), np.zeros((n, 3)), mat, (0, 0, -9.81),
                    (0, 0, 0, side, side, z_top), h, bnd=walls + [cone], name=f"cone-bed-r{replica}")


def drum_boundaries(center, R, L, omega, mat=WALL_MAT, scene=0):
    """A drum of radius R and length L with its axis along y through
    ``center`` (x, z) from y = 0 to y = L: the inner cylinder and two end
    caps, all spinning at ``omega`` rad/s about the axis (surface spin about
    reference points on the axis; the geometry is invariant under it)."""
    cx, cz = center
    w = (0.0, omega, 0.0)
    return [dict(type=BND_CYL_IN, param=(cx, 0.0, cz, 0, 1, 0, R), mat=mat, omega=w, scene=scene),
            dict(type=BND_PLANE, param=(cx, 0.0, cz, 0, 1, 0), mat=mat, omega=w, scene=scene),
            dict(type=BND_PLANE, param=(cx, L, cz, 0, -1, 0), mat=mat, omega=w, scene=scene)]


def drum(replica: int = 0, n_clumps: int = 700, R: float = 0.05, L: float = 0.1, omega: float = 2.0,
         sink_max: float = 2e-5, h: float = 1e-6) -> SceneDesc:
    """Configuration 3 scaled down (the rotating drum): clumps of the eight bed
    templates and bed materials deposited onto the curved bottom of a drum of
    radius R and length L (horizontal axis along y, through x = z = R), which
    spins at ``omega`` = 2 rad/s from the first step: the clumps start at rest
    and the wall drags them.  Deposit footprint: the middle 80 % of the
    drum's width; some clumps are placed against the end caps."""
    g = rng(9, replica)
    tmpls = bed_templates(replica)
    ct = g.integers(0, len(tmpls), n_clumps)
    cx = cz = R

    def floor(px, py, r):
        return cz - np.sqrt(np.maximum((R - r) ** 2 - (px - cx) ** 2, 0.0))

    x, q = deposit(g, tmpls, ct, (cx - 0.8 * R, 0.0, cx + 0.8 * R, L), sink_max, floor=floor, edge=(0.15, "y"))
    sizes = np.array([t[0].shape[0] for t in tmpls])
    mat = bed_materials(g, int(sizes[ct].sum()))
    n = n_clumps
    return assemble(tmpls, ct, x, q, np.zeros((n, 3)), np.zeros((n, 3)), mat, (0, 0, -9.81),
                    (0, 0, 0, 2 * R, L, 2 * R), h, bnd=drum_boundaries((cx, cz), R, L, omega),
                    name=f"drum-r{replica}")


def drum_bed(patch_x: np.ndarray, patch_q: np.ndarray, replica: int = 0, n_clumps: int = 4_000_000,
             R: float = 0.4, L: float = 3.0, omega: float = 2.0, side: float = 0.05) -> SceneDesc:
    """Configuration 3 at its size (the precision study): a drum of radius
    R = 0.4 m and length L = 3 m (horizontal axis along y through
    x = z = R), spinning at 2 rad/s from the first step, holding ``n_clumps``
    clumps of the eight bed templates with per-sphere-instance bed materials.
    The drum is filled from copies of a patch (``patch_x``/``patch_q``, the
    clump poses of a rover-bed patch of the same replica, as from
    :func:`rover_deposited_patch`), laid side by side over the drum's
    section and length with the same seam spacing as the rover bed; a clump
    is kept when its bounding sphere lies inside the drum, and the lowest
    ``n_clumps`` of those are the fill (about half the drum).  Clumps start
    at rest."""
    g = rng(9, 1000 + replica)
    tmpls = bed_templates(replica)
    ct_p = rng(5, replica).integers(0, len(tmpls), patch_x.shape[0])
    order = morton_order(patch_x, 0.01)
    xp, qp, ct_p = patch_x[order], patch_q[order], ct_p[order]
    Rm = quat_matrix(qp)
    P = np.concatenate([xp[k] + tmpls[ct_p[k]][0] @ Rm[k].T for k in range(len(ct_p))])
    Rr = np.concatenate([tmpls[ct_p[k]][1] for k in range(len(ct_p))])
    lo = np.array([max(0.0, -(P[:, a] - Rr).min()) for a in range(2)])
    hi = np.array([max(0.0, (P[:, a] + Rr).max() - side) for a in range(2)])
    pitch = side + lo + hi + 1e-6
    rb = np.array([bounding_radius(t[0], t[1]) for t in tmpls])[ct_p]
    ntx, nty = int(np.ceil(2 * R / pitch[0])), int(np.ceil(L / pitch[1]))
    cx = cz = R
    X, Q, CT = [], [], []
    for j in range(nty):
        for i in range(ntx):
            x = xp + np.array([lo[0] + i * pitch[0], lo[1] + j * pitch[1], 0.0])
            keep = (np.hypot(x[:, 0] - cx, x[:, 2] - cz) <= R - rb - 1e-4) & (x[:, 1] >= rb + 1e-4) & \
                   (x[:, 1] <= L - rb - 1e-4)
            X.append(x[keep]); Q.append(qp[keep]); CT.append(ct_p[keep])
    X, Q, CT = np.concatenate(X), np.concatenate(Q), np.concatenate(CT)
    low = np.argsort(X[:, 2], kind="stable")[:n_clumps]
    X, Q, CT = X[low], Q[low], CT[low]
    m = morton_order(X, 0.01)
    X, Q, CT = X[m], Q[m], CT[m]
    nc = X.shape[0]
    sizes = np.array([t[0].shape[0] for t in tmpls])
    mat = bed_materials(g, int(sizes[CT].sum()))
    return assemble(tmpls, CT, X, Q, np.zeros((nc, 3)), np.zeros((nc, 3)), mat, (0, 0, -9.81),
                    (0, 0, 0, 2 * R, L, 2 * R), 1e-6, bnd=drum_boundaries((cx, cz), R, L, omega),
                    name=f"drum-bed-r{replica}")


# ---------------------------------------------------------------------------
# Configuration 4: many independent funnel scenes of uneven size
# ---------------------------------------------------------------------------

def funnel_scene_parts(g: np.random.Generator, n_clumps: int, template, mu: float, scene: int):
    """One repose-angle scene: clumps of one template on a lattice inside an
    upward-opening funnel (half-angle 30 degrees from the vertical, outlet
    radius 6 bounding radii), a plate 0.2 m below the outlet.  Returns the
    clump poses, the boundaries and the scene's binning domain."""
    rb = bounding_radius(template[0], template[1])
    sp = 2.0 * rb + 2e-4
    tan30 = math.tan(math.radians(30.0))
    r_out = 6.0 * rb
    z_out = 0.0
    z_apex = z_out - r_out / tan30          # virtual apex of the funnel cone
    x = []
    z = z_out + rb + 1e-4
    while len(x) < n_clumps:
        r_in = (z - z_apex) * tan30 - rb - 1e-4   # sites keep clear of the wall
        m = int(r_in // sp)
        for i in range(-m, m + 1):
            for j in range(-m, m + 1):
                if (i * sp) ** 2 + (j * sp) ** 2 <= r_in ** 2 and len(x) < n_clumps:
                    x.append((i * sp, j * sp, z))
        z += sp
    x = np.array(x)
    q = random_unit_quaternions(g, n_clumps)
    top = float(x[:, 2].max()) + rb + 0.01
    s30, c30 = math.sin(math.radians(30.0)), math.cos(math.radians(30.0))
    mat = (1e7, 0.3, mu, 0.5)
    bnd = [dict(type=BND_FRUSTUM_IN, param=(0, 0, z_apex, 0, 0, 1, s30, c30, z_out - z_apex, top - z_apex),
                mat=mat, scene=scene),
           dict(type=BND_PLANE, param=(0, 0, z_out - 0.2, 0, 0, 1), mat=mat, scene=scene)]
    rmax = (top - z_apex) * tan30 + 0.1
    dom = (-rmax, -rmax, z_out - 0.2, rmax, rmax, top)
    return x, q, bnd, dom


def funnel_batch(replica: int = 0, n_scenes: int = 256, lo: int = 2000, hi: int = 60000, scale: float = 1.0,
            res: int = 32) -> SceneDesc:
    """Configuration 4: n_scenes independent funnel discharges batched in one
    simulation.  Clump counts log-uniform in [lo, hi] (times `scale`); per
    scene one template of 1-6 spheres (lognormal radii) and mu ~ U[0.2, 0.9];
    E = 1e7, nu = 0.3, CoR = 0.5; clumps start at rest; h = 1e-6 s.  Scenes
    share coordinates but never interact (each has its own bins)."""
    g = rng(4, replica)
    counts = np.exp(g.uniform(np.log(lo), np.log(hi), n_scenes)) * scale
    counts = np.maximum(1, counts.astype(np.int64))
    templates, X, Q, CT, CS, MAT, bnds, doms = [], [], [], [], [], [], [], []
    for k in range(n_scenes):
        nsph = int(g.integers(1, 7))
        t = multisphere_template(g, nsph, res=res)
        mu = float(g.uniform(0.2, 0.9))
        x, q, bnd, dom = funnel_scene_parts(g, int(counts[k]), t, mu, k)
        templates.append(t)
        X.append(x); Q.append(q)
        CT.append(np.full(len(x), k)); CS.append(np.full(len(x), k))
        MAT.append(np.tile([1e7, 0.3, mu, 0.5], (len(x) * nsph, 1)))
        bnds += bnd
        doms.append(dom)
    X = np.concatenate(X)
    n = X.shape[0]
    return assemble(templates, np.concatenate(CT), X, np.concatenate(Q), np.zeros((n, 3)), np.zeros((n, 3)),
                    np.concatenate(MAT), np.tile([0.0, 0.0, -9.81], (n_scenes, 1)), np.array(doms), 1e-6,
                    clump_scene=np.concatenate(CS), bnd=bnds, name=f"funnels-r{replica}")


def extract_scene(batch: SceneDesc, k: int) -> SceneDesc:
    """Scene k of a batched description as a stand-alone description (same
    templates, same per-sphere materials, its own boundaries)."""
    sel = np.nonzero(batch.clump_scene == k)[0]
    sb = batch.sphere_begin()
    sph = np.concatenate([np.arange(sb[c], sb[c + 1]) for c in sel]) if len(sel) else np.zeros(0, np.int64)
    bsel = np.nonzero(batch.bnd_scene == k)[0]
    d = dataclasses.replace(
        batch, clump_template=batch.clump_template[sel], clump_scene=np.zeros(len(sel), np.uint32),
        x=batch.x[sel], q=batch.q[sel], v=batch.v[sel], w=batch.w[sel], sphere_mat=batch.sphere_mat[sph],
        gravity=batch.gravity[k:k + 1], domain=batch.domain[k:k + 1], bnd_type=batch.bnd_type[bsel],
        bnd_param=batch.bnd_param[bsel], bnd_mat=batch.bnd_mat[bsel], bnd_vel=batch.bnd_vel[bsel],
        bnd_omega=batch.bnd_omega[bsel], bnd_scene=np.zeros(len(bsel), np.int32),
        presc_clump=np.zeros(0, np.int32), presc_param=np.zeros((0, PRESC_NPARAM)), name=f"{batch.name}-s{k}")
    return d.canonical()


def funnel_deposited(batch: SceneDesc, k: int, sink_max: float = 2e-5) -> SceneDesc:
    """Scene k of a funnel batch, stand-alone, with its clumps deposited into
    its funnel on the CPU (``deposit``) instead of spawned on a lattice: a
    clump whose spheres clear the outlet falls through it onto the plate, so
    a column of clumps stands on the plate under the outlet and the funnel
    is filled above it.  Same templates, materials and boundaries (the funnel
    wall is extended to the deposit's top); clumps start at rest.  A
    contact-rich state built without simulating anything."""
    e = extract_scene(batch, k)
    fi = int(np.nonzero(e.bnd_type == BND_FRUSTUM_IN)[0][0])
    pi = int(np.nonzero(e.bnd_type == BND_PLANE)[0][0])
    fr, pl = e.bnd_param[fi].copy(), e.bnd_param[pi]
    z_apex, sn, cs, t0 = fr[2], fr[6], fr[7], fr[8]
    z_out, z_plate = z_apex + t0, pl[2]
    tb = np.asarray(e.tmpl_sphere_begin, np.int64)
    tmpls = [(e.tmpl_offset[tb[t]:tb[t + 1]], e.tmpl_radius[tb[t]:tb[t + 1]]) for t in range(len(tb) - 1)]
    rb = max(bounding_radius(o, r) for o, r in tmpls)

    def floor(px, py, r):
        # resting on the funnel wall (the cone's surface at distance r along
        # its inward normal) where that height is above the outlet, else on
        # the plate below it
        rho = np.hypot(px, py)
        zw = z_apex + (r + rho * cs) / sn
        return np.where(zw >= z_out, zw, z_plate + r)

    # a square footprint inside the funnel's section at the top of the spawn lattice
    half = 0.7 * (fr[9] - rb) * (sn / cs) / math.sqrt(2.0)
    g = rng(10, k)
    x, q = deposit(g, tmpls, np.asarray(e.clump_template, np.int64), (-half, -half, half, half), sink_max,
                   floor=floor)
    top = float(x[:, 2].max()) + rb + 0.01
    fr[9] = max(fr[9], top - z_apex)
    P = e.bnd_param.copy()
    P[fi] = fr
    dom = e.domain.copy()
    rmax = fr[9] * (sn / cs) + 0.1
    dom[0] = (-rmax, -rmax, z_plate, rmax, rmax, z_apex + fr[9])
    n = e.n_clumps
    return dataclasses.replace(e, x=x, q=q, v=np.zeros((n, 3)), w=np.zeros((n, 3)), bnd_param=P, domain=dom,
                               name=f"{e.name}-deposited").canonical()


# ---------------------------------------------------------------------------
# Long-run statistics: a settled box (packing fraction) and a collapsed
# column (heap angle), in the materials and clumps of the walled box
# ---------------------------------------------------------------------------

STATS_H = 1e-5  # time step of the statistics runs (about 40 steps per contact at these stiffnesses)


def stats_scene(kind: str, replica: int = 0, n_clumps: int = 120, res: int = 16) -> SceneDesc:
    """One seeded scene of the long-run statistics.

    ``kind="box"``: clumps on a simple-cubic lattice in a 3 cm x 3 cm box
    (floor and four walls), velocity noise U[-0.05, 0.05] m/s per component;
    they fall and settle into a bed.  ``kind="heap"``: the same kind of clumps
    at rest in a column six sites wide against the back wall of a slot one
    site deep (a quasi-two-dimensional dam break); the column collapses onto
    the floor, open towards +x, and leaves a slope.  Configuration-1 clumps (three spheres of one
    radius in U[1, 2] mm, centres 0.6 r off the centre) and materials
    (E = 1e7 Pa, nu = 0.3, mu = 0.5, CoR = 0.5), gravity -9.81 z, h = 1e-5 s."""
    if kind not in ("box", "heap"):
        raise ValueError("kind is 'box' or 'heap'")
    g = rng(6 if kind == "box" else 7, replica)
    tmpls = _box_templates(g, n_clumps, res)
    rb = max(bounding_radius(t[0], t[1]) for t in tmpls)
    spacing = 2.0 * rb + 1e-4
    mat = np.tile(np.array(BOX_MAT), (3 * n_clumps, 1))
    if kind == "box":
        L = 0.03
        nxy = int(L // spacing)
        nz = -(-n_clumps // (nxy * nxy))
        origin = (L / 2 - spacing * (nxy - 1) / 2, L / 2 - spacing * (nxy - 1) / 2, spacing / 2 + 5e-5)
        sites = lattice_sites(nxy, nxy, nz, spacing, origin)
        x = sites[g.permutation(sites.shape[0])[:n_clumps]]
        v = g.uniform(-0.05, 0.05, (n_clumps, 3))
        top = nz * spacing + 0.01
        bnd = box_walls((0, 0, 0), (L, L, top), BOX_MAT)
        dom = (0, 0, 0, L, L, top)
    else:
        # a column against the back wall x = 0 of a slot one site deep
        # (walls y = 0 and y = W), open towards +x over the floor
        nx_ = 6
        nz = -(-n_clumps // nx_)
        W = spacing + 2e-4
        origin = (spacing / 2 + 5e-5, W / 2, spacing / 2 + 5e-5)
        x = lattice_sites(nx_, 1, nz, spacing, origin)[:n_clumps]
        v = np.zeros((n_clumps, 3))
        top = nz * spacing + 0.01
        Lx = 0.15
        bnd = [dict(type=BND_PLANE, param=(0, 0, 0, 0, 0, 1), mat=BOX_MAT, scene=0),
               dict(type=BND_PLANE, param=(0, 0, 0, 1, 0, 0), mat=BOX_MAT, scene=0),
               dict(type=BND_PLANE, param=(0, 0, 0, 0, 1, 0), mat=BOX_MAT, scene=0),
               dict(type=BND_PLANE, param=(0, W, 0, 0, -1, 0), mat=BOX_MAT, scene=0)]
        dom = (0, 0, 0, Lx, W, top)
    q = random_unit_quaternions(g, n_clumps)
    w = np.zeros((n_clumps, 3))
    return assemble(tmpls, np.arange(n_clumps), x, q, v, w, mat, (0, 0, -9.81), dom, STATS_H, bnd=bnd,
                    name=f"stats-{kind}-r{replica}")


def batch(descs) -> SceneDesc:
    """Independent scenes as one batched description (scene k = descs[k]);
    every input is copied, nothing is computed."""
    descs = [d.canonical() for d in descs]
    if len({d.h for d in descs}) != 1:
        raise ValueError("batched scenes share the time step")
    nts = np.cumsum([0] + [d.n_templates for d in descs])
    begin = [np.zeros(1, np.uint32)]
    off = 0
    for d in descs:
        begin.append(d.tmpl_sphere_begin[1:].astype(np.int64) + off)
        off += int(d.tmpl_sphere_begin[-1])
    cs, bs = [], []
    for k, d in enumerate(descs):
        if d.n_scenes != 1:
            raise ValueError("batch takes single-scene descriptions")
        cs.append(np.full(d.n_clumps, k, np.uint32))
        bs.append(np.full(d.n_bnd, k, np.int32))
    out = SceneDesc(
        h=descs[0].h,
        tmpl_sphere_begin=np.concatenate(begin).astype(np.uint32),
        tmpl_offset=np.concatenate([d.tmpl_offset for d in descs]),
        tmpl_radius=np.concatenate([d.tmpl_radius for d in descs]),
        tmpl_mass=np.concatenate([d.tmpl_mass for d in descs]),
        tmpl_inertia=np.concatenate([d.tmpl_inertia for d in descs]),
        clump_template=np.concatenate([d.clump_template.astype(np.int64) + nts[k] for k, d in enumerate(descs)]),
        clump_scene=np.concatenate(cs),
        x=np.concatenate([d.x for d in descs]), q=np.concatenate([d.q for d in descs]),
        v=np.concatenate([d.v for d in descs]), w=np.concatenate([d.w for d in descs]),
        sphere_mat=np.concatenate([d.sphere_mat for d in descs]),
        gravity=np.concatenate([d.gravity for d in descs]), domain=np.concatenate([d.domain for d in descs]),
        bnd_type=np.concatenate([d.bnd_type for d in descs]), bnd_param=np.concatenate([d.bnd_param for d in descs]),
        bnd_mat=np.concatenate([d.bnd_mat for d in descs]), bnd_vel=np.concatenate([d.bnd_vel for d in descs]),
        bnd_omega=np.concatenate([d.bnd_omega for d in descs]), bnd_scene=np.concatenate(bs),
        mesh_state=np.concatenate([d.mesh_state for d in descs]),
        mesh_mat=np.concatenate([d.mesh_mat for d in descs]),
        mesh_scene=np.concatenate([np.full(d.n_mesh, k, np.int32) for k, d in enumerate(descs)]),
        tri_mesh=np.concatenate([d.tri_mesh.astype(np.int64) + nm for d, nm in
                                 zip(descs, np.cumsum([0] + [d.n_mesh for d in descs]))]).astype(np.int32),
        tri_vertex=np.concatenate([d.tri_vertex for d in descs]),
        name="batch-" + "+".join(d.name for d in descs))
    if any(d.presc_clump.size for d in descs):
        raise ValueError("batch takes scenes without prescribed clumps")
    return out.canonical()
