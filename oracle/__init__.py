"""FP64 brute-force CPU oracle of the clumped-sphere DEM timestep (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The oracle shares no code with the HIP
implementation; see ``oracle.c`` for the step it computes and the readings of
the paper it takes (Sec. 2.1: Eqs. normal_tangential_force_model1/2,
kinematicsContactInfo, updateUt, cappingOfut, newton_law_1/2).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Desc(C.Structure):
    _fields_ = [
        ("h", C.c_double),
        ("n_templates", C.c_int32),
        ("tmpl_sphere_begin", C.c_void_p),
        ("tmpl_offset", C.c_void_p),
        ("tmpl_radius", C.c_void_p),
        ("tmpl_mass", C.c_void_p),
        ("tmpl_inertia", C.c_void_p),
        ("n_clumps", C.c_int64),
        ("clump_template", C.c_void_p),
        ("clump_scene", C.c_void_p),
        ("x", C.c_void_p), ("q", C.c_void_p), ("v", C.c_void_p), ("w", C.c_void_p),
        ("sphere_mat", C.c_void_p),
        ("n_scenes", C.c_int32),
        ("gravity", C.c_void_p),
        ("n_bnd", C.c_int32),
        ("bnd_type", C.c_void_p), ("bnd_param", C.c_void_p), ("bnd_mat", C.c_void_p),
        ("bnd_vel", C.c_void_p), ("bnd_omega", C.c_void_p), ("bnd_scene", C.c_void_p),
        ("n_presc", C.c_int32),
        ("presc_clump", C.c_void_p), ("presc_param", C.c_void_p),
        ("n_mesh", C.c_int32),
        ("mesh_state", C.c_void_p), ("mesh_mat", C.c_void_p), ("mesh_scene", C.c_void_p),
        ("n_tri", C.c_int64),
        ("tri_mesh", C.c_void_p), ("tri_vertex", C.c_void_p),
        ("pos_exp", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P, I64, V = C.c_void_p, C.c_int64, None
        sig = {
            "dem_oracle_create": (P, [P]), "dem_oracle_destroy": (V, [P]),
            "dem_oracle_last_error": (C.c_char_p, []), "dem_oracle_set_threads": (V, [C.c_int]),
            "dem_oracle_step": (V, [P, I64]), "dem_oracle_step_count": (I64, [P]),
            "dem_oracle_positions_ok": (C.c_int, [P]), "dem_oracle_read_fixed_positions": (V, [P, P]),
            "dem_oracle_eval": (I64, [P]),
            "dem_oracle_read_contacts": (V, [P, P, P, P, P, P]),
            "dem_oracle_read_contact_torques": (V, [P, P, P]),
            "dem_oracle_read_clump_forces": (V, [P, P, P]),
            "dem_oracle_read_sphere_forces": (V, [P, P, P]),
            "dem_oracle_read_boundary_forces": (V, [P, P, P]),
            "dem_oracle_read_mesh_forces": (V, [P, P, P]),
            "dem_oracle_read_mesh_state": (V, [P, P]),
            "dem_oracle_set_mesh_state": (C.c_int, [P, C.c_int32, P]),
            "dem_oracle_read_state": (V, [P, P, P, P, P]),
            "dem_oracle_read_sphere_pos": (V, [P, P]),
            "dem_oracle_n_spheres": (I64, [P]),
            "dem_oracle_candidates": (I64, [P, P, P, P, I64]),
            "dem_oracle_sample_spheres": (I64, [P, P, I64, P, P, I64, P, P, P, P, P]),
            "dem_oracle_sample_clumps": (C.c_int, [P, P, I64, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    lib().dem_oracle_set_threads(int(n))


class Oracle:
    """One oracle simulation created from a :class:`SceneDesc`."""

    def __init__(self, desc):
        d = desc.canonical()
        self._keep = d
        s = _Desc()
        s.h = d.h
        s.n_templates = d.n_templates
        s.tmpl_sphere_begin, s.tmpl_offset = _ptr(d.tmpl_sphere_begin), _ptr(d.tmpl_offset)
        s.tmpl_radius, s.tmpl_mass, s.tmpl_inertia = _ptr(d.tmpl_radius), _ptr(d.tmpl_mass), _ptr(d.tmpl_inertia)
        s.n_clumps = d.n_clumps
        s.clump_template, s.clump_scene = _ptr(d.clump_template), _ptr(d.clump_scene)
        s.x, s.q, s.v, s.w = _ptr(d.x), _ptr(d.q), _ptr(d.v), _ptr(d.w)
        s.sphere_mat = _ptr(d.sphere_mat)
        s.n_scenes = d.n_scenes
        s.gravity = _ptr(d.gravity)
        s.n_bnd = d.n_bnd
        s.bnd_type, s.bnd_param, s.bnd_mat = _ptr(d.bnd_type), _ptr(d.bnd_param), _ptr(d.bnd_mat)
        s.bnd_vel, s.bnd_omega, s.bnd_scene = _ptr(d.bnd_vel), _ptr(d.bnd_omega), _ptr(d.bnd_scene)
        s.n_presc = len(d.presc_clump)
        s.presc_clump, s.presc_param = _ptr(d.presc_clump), _ptr(d.presc_param)
        s.n_mesh, s.n_tri = d.n_mesh, d.n_tri
        s.mesh_state, s.mesh_mat, s.mesh_scene = _ptr(d.mesh_state), _ptr(d.mesh_mat), _ptr(d.mesh_scene)
        s.tri_mesh, s.tri_vertex = _ptr(d.tri_mesh), _ptr(d.tri_vertex)
        s.pos_exp = d.pos_exp
        self._h = lib().dem_oracle_create(C.byref(s))
        if not self._h:
            raise ValueError(lib().dem_oracle_last_error().decode())
        self.n_clumps = d.n_clumps
        self.n_spheres = int(lib().dem_oracle_n_spheres(self._h))
        self.n_bnd = d.n_bnd
        self.n_mesh = d.n_mesh
        self._ncont = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().dem_oracle_destroy(h)
            self._h = None

    def step(self, n: int = 1) -> None:
        lib().dem_oracle_step(self._h, int(n))
        self._ncont = -1
        if not lib().dem_oracle_positions_ok(self._h):
            raise OverflowError("a fixed-point position left its range")

    def fixed_positions(self) -> np.ndarray:
        """The fixed-point CoM integers [n_clumps][3] (fixed-point positions only)."""
        k = np.empty((self.n_clumps, 3), np.int64)
        lib().dem_oracle_read_fixed_positions(self._h, _ptr(k))
        return k

    @property
    def step_count(self) -> int:
        return int(lib().dem_oracle_step_count(self._h))

    def eval(self) -> int:
        """Evaluate contacts and forces at the current state (no advance)."""
        self._ncont = int(lib().dem_oracle_eval(self._h))
        return self._ncont

    def contacts(self) -> dict:
        """Contacts of the last evaluation (``eval`` or the last step's)."""
        if self._ncont < 0:
            raise RuntimeError("call eval() after step() to refresh contacts")
        n = self._ncont
        a = np.empty(n, np.uint32); b = np.empty(n, np.uint32); dl = np.empty(n)
        F = np.empty((n, 3)); u = np.empty((n, 3))
        Ta = np.empty((n, 3)); Tb = np.empty((n, 3))
        lib().dem_oracle_read_contacts(self._h, _ptr(a), _ptr(b), _ptr(dl), _ptr(F), _ptr(u))
        lib().dem_oracle_read_contact_torques(self._h, _ptr(Ta), _ptr(Tb))
        return dict(a=a, b=b, delta=dl, F=F, u=u, Ta=Ta, Tb=Tb)

    def mesh_forces(self):
        """Force the spheres exert on each mesh and its torque about the mesh's
        reference point, from the last evaluation: ([n_mesh, 3], [n_mesh, 3])."""
        F = np.empty((self.n_mesh, 3)); T = np.empty((self.n_mesh, 3))
        lib().dem_oracle_read_mesh_forces(self._h, _ptr(F), _ptr(T))
        return F, T

    def mesh_state(self):
        st = np.empty((self.n_mesh, 13))
        lib().dem_oracle_read_mesh_state(self._h, _ptr(st))
        return st

    def set_mesh_state(self, mesh: int, state):
        st = np.ascontiguousarray(state, np.float64).reshape(13)
        if lib().dem_oracle_set_mesh_state(self._h, int(mesh), _ptr(st)) != 0:
            raise ValueError("mesh index out of range")

    def clump_forces(self):
        F = np.empty((self.n_clumps, 3)); T = np.empty((self.n_clumps, 3))
        lib().dem_oracle_read_clump_forces(self._h, _ptr(F), _ptr(T))
        return F, T

    def sphere_forces(self):
        F = np.empty((self.n_spheres, 3)); T = np.empty((self.n_spheres, 3))
        lib().dem_oracle_read_sphere_forces(self._h, _ptr(F), _ptr(T))
        return F, T

    def boundary_forces(self):
        """Force on each boundary and torque about its reference point (last evaluation)."""
        F = np.empty((self.n_bnd, 3)); T = np.empty((self.n_bnd, 3))
        lib().dem_oracle_read_boundary_forces(self._h, _ptr(F), _ptr(T))
        return F, T

    def state(self) -> dict:
        n = self.n_clumps
        x = np.empty((n, 3)); q = np.empty((n, 4)); v = np.empty((n, 3)); w = np.empty((n, 3))
        lib().dem_oracle_read_state(self._h, _ptr(x), _ptr(q), _ptr(v), _ptr(w))
        return dict(x=x, q=q, v=v, w=w)

    def sphere_pos(self) -> np.ndarray:
        xs = np.empty((self.n_spheres, 3))
        lib().dem_oracle_read_sphere_pos(self._h, _ptr(xs))
        return xs

    def candidates(self, margin=None):
        m = None if margin is None else np.ascontiguousarray(margin, np.float64)
        n = int(lib().dem_oracle_candidates(self._h, _ptr(m), None, None, 0))
        a = np.empty(n, np.uint32); b = np.empty(n, np.uint32)
        lib().dem_oracle_candidates(self._h, _ptr(m), _ptr(a), _ptr(b), n)
        return a, b

    def sample_spheres(self, ids):
        """Forces, torques and contacts of the spheres `ids` at the current
        state, by brute force over every partner (for scenes too large for
        ``eval``).  Returns (F [n,3], T [n,3], contacts dict a, b, delta, F,
        beg), where sample k's contacts are rows beg[k]:beg[k+1]."""
        ids = np.ascontiguousarray(ids, np.int64)
        n = len(ids)
        F = np.empty((n, 3)); T = np.empty((n, 3))
        cap = 64 * max(n, 1)
        beg = np.empty(n + 1, np.int64)
        while True:
            a = np.empty(cap, np.uint32); b = np.empty(cap, np.uint32)
            dl = np.empty(cap); cF = np.empty((cap, 3))
            m = int(lib().dem_oracle_sample_spheres(self._h, _ptr(ids), n, _ptr(F), _ptr(T), cap, _ptr(beg),
                                                    _ptr(a), _ptr(b), _ptr(dl), _ptr(cF)))
            if m < 0:
                raise ValueError(lib().dem_oracle_last_error().decode())
            if m <= cap:
                return F, T, dict(a=a[:m], b=b[:m], delta=dl[:m], F=cF[:m], beg=beg)
            cap = m

    def sample_clumps(self, clumps):
        """Force (contacts + gravity) and torque of the clumps `clumps`."""
        c = np.ascontiguousarray(clumps, np.int64)
        F = np.empty((len(c), 3)); T = np.empty((len(c), 3))
        if lib().dem_oracle_sample_clumps(self._h, _ptr(c), len(c), _ptr(F), _ptr(T)) != 0:
            raise ValueError(lib().dem_oracle_last_error().decode())
        return F, T
