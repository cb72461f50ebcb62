"""ctypes binding of libcdem.so (the HIP library behind include/cdem.h).

Argument marshalling only: every step of the timestep runs in the library's
HIP kernels.  There is no CPU fallback; a missing or unloadable library raises.
PyTorch, when available, supplies device memory (its caching allocator) and
the stream; it is plumbing, not part of the computation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdem.so")

PREC_FP64, PREC_FP32_FORCE = 0, 1
DETECT_PLAIN, DETECT_FIXED, DETECT_LEARNED = 0, 1, 2
HOST, DEVICE = 0, 1
ERRORS = {0: "ok", -1: "CDEM_E_INVALID", -2: "CDEM_E_OOM", -3: "CDEM_E_HIP", -4: "CDEM_E_CAPACITY",
          -5: "CDEM_E_MISSED_CONTACT", -6: "CDEM_E_NAN", -7: "CDEM_E_STATE"}

P = C.c_void_p


class SceneDescC(C.Structure):
    _fields_ = [
        ("h", C.c_double), ("precision", C.c_int32), ("n_templates", C.c_int32),
        ("tmpl_sphere_begin", P), ("tmpl_offset", P), ("tmpl_radius", P), ("tmpl_mass", P), ("tmpl_inertia", P),
        ("n_clumps", C.c_int64), ("clump_template", P), ("clump_scene", P),
        ("x", P), ("q", P), ("v", P), ("w", P), ("sphere_mat", P),
        ("n_scenes", C.c_int32), ("gravity", P), ("domain", P),
        ("n_bnd", C.c_int32), ("bnd_type", P), ("bnd_param", P), ("bnd_mat", P), ("bnd_vel", P),
        ("bnd_omega", P), ("bnd_scene", P),
        ("n_presc", C.c_int32), ("presc_clump", P), ("presc_param", P),
        ("n_mesh", C.c_int32), ("mesh_state", P), ("mesh_mat", P), ("mesh_scene", P),
        ("n_tri", C.c_int64), ("tri_mesh", P), ("tri_vertex", P),
        ("pos_exp", C.c_int32),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class AllocatorC(C.Structure):
    _fields_ = [("ctx", P), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class DetectParamsC(C.Structure):
    _fields_ = [("mode", C.c_int32), ("k_max", C.c_int32), ("safety", C.c_double), ("v_max_user", C.c_double),
                ("margin_cap", C.c_double), ("audit_period", C.c_int32), ("overlap", C.c_int32)]


class CountsC(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("clumps", "spheres", "bins", "candidates", "steps", "detections",
                                          "guard_trips", "fallbacks", "audits", "missed", "capacity", "regrows",
                                          "pairs")] + \
               [("k_current", C.c_int32), ("reserved", C.c_int32), ("audit_contacts", C.c_int64)]


class StateViewC(C.Structure):
    _fields_ = [("x", P), ("q", P), ("v", P), ("w", P)]


class ContactsViewC(C.Structure):
    _fields_ = [("cap", C.c_int64), ("n", C.c_int64), ("a", P), ("b", P), ("delta", P), ("F", P), ("u", P),
                ("Ta", P), ("Tb", P)]


class KernelTimeC(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


class AuditResultC(C.Structure):
    _fields_ = [("true_contacts", C.c_int64), ("missed", C.c_int64), ("first_a", C.c_uint32), ("first_b", C.c_uint32)]


# every exported symbol of include/cdem.h with its ctypes signature
SIGNATURES = {
    "cdem_abi_version": (C.c_int, []),
    "cdem_strerror": (C.c_char_p, [C.c_int]),
    "cdem_last_error": (C.c_char_p, [P]),
    "cdem_create": (C.c_int, [P, P, P, C.POINTER(P)]),
    "cdem_destroy": (C.c_int, [P]),
    "cdem_step": (C.c_int, [P, C.c_int64, P]),
    "cdem_sync": (C.c_int, [P]),
    "cdem_set_detection": (C.c_int, [P, P]),
    "cdem_record_next_step": (C.c_int, [P, C.c_int]),
    "cdem_get_counts": (C.c_int, [P, P]),
    "cdem_read_state": (C.c_int, [P, P, C.c_int, P]),
    "cdem_write_state": (C.c_int, [P, P, C.c_int, P]),
    "cdem_read_contacts": (C.c_int, [P, P]),
    "cdem_read_clump_forces": (C.c_int, [P, P, P]),
    "cdem_read_sphere_pos": (C.c_int, [P, P]),
    "cdem_audit": (C.c_int, [P, P]),
    "cdem_profile": (C.c_int, [P, C.c_int]),
    "cdem_profile_kernels": (C.c_int, [P, C.c_char_p]),
    "cdem_profile_read": (C.c_int, [P, P, C.c_int, C.POINTER(C.c_int)]),
    "cdem_last_step_contacts": (C.c_int, [P, C.POINTER(C.c_int64)]),
    "cdem_mlp_param_count": (C.c_int, []),
    "cdem_set_mlp": (C.c_int, [P, P, C.c_int64]),
    "cdem_mlp_forward": (C.c_int, [P, P, P, C.c_int64, P]),
    "cdem_mlp_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "cdem_mlp_backward": (C.c_int, [P, P, P, C.c_int64, C.c_float, P, P, P, P]),
    "cdem_mlp_backward_static": (C.c_int, [P, P, P, C.c_int64, C.c_float, P, P, P]),
    "cdem_check_force_law": (C.c_int, [C.c_char_p, C.c_char_p, C.c_size_t]),
    "cdem_set_mesh_state": (C.c_int, [P, C.c_int32, P]),
    "cdem_read_mesh_state": (C.c_int, [P, P]),
    "cdem_read_mesh_forces": (C.c_int, [P, P, P]),
    "cdem_set_force_law": (C.c_int, [P, C.c_char_p, C.c_char_p, C.c_size_t]),
    "cdem_mlp_adam": (C.c_int, [P, P, P, P, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, P]),
    "cdem_collect_envelopes": (C.c_int, [P, C.c_int32, P, P, C.c_int64, C.POINTER(C.c_int64)]),
    "cdem_set_graph": (C.c_int, [P, C.c_int32]),
    "cdem_autotune": (C.c_int, [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "cdem_save": (C.c_int, [P, P, C.c_size_t, C.POINTER(C.c_size_t)]),
    "cdem_read_boundary_forces": (C.c_int, [P, P, P]),
    "cdem_load": (C.c_int, [P, P, C.c_size_t]),
}

_lib = None


def load():
    """Load libcdem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch bundles its own HIP runtime under the same soname as ROCm's;
        # loading torch first makes libcdem bind to that one runtime instead of
        # bringing a second, conflicting runtime into the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(the HIP library is required; there is no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


class CdemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(a):
    return None if a is None else a.ctypes.data_as(P)


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device

        def _alloc(ctx, nbytes, stream):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device))
            except Exception:
                return None

        def _free(ctx, p, stream):
            try:
                if p:
                    torch.cuda.caching_allocator_delete(int(p))
            except Exception:  # interpreter shutdown: the allocator is already gone
                pass

        self._a, self._f = ALLOC_FN(_alloc), FREE_FN(_free)
        self.struct = AllocatorC(None, self._a, self._f)


class Scene:
    """One simulation on the GPU, created from a :class:`inputs.SceneDesc`."""

    def __init__(self, desc, precision: str = "fp64", stream=None, torch_allocator: bool = True):
        L = load()
        d = desc.canonical()
        self._keep = d
        self.n_clumps, self.n_spheres, self.n_bnd = d.n_clumps, d.n_spheres, d.n_bnd
        s = SceneDescC()
        s.h = d.h
        s.precision = {"fp64": PREC_FP64, "fp32": PREC_FP32_FORCE}[precision]
        s.n_templates = d.n_templates
        s.tmpl_sphere_begin, s.tmpl_offset, s.tmpl_radius = _ptr(d.tmpl_sphere_begin), _ptr(d.tmpl_offset), _ptr(d.tmpl_radius)
        s.tmpl_mass, s.tmpl_inertia = _ptr(d.tmpl_mass), _ptr(d.tmpl_inertia)
        s.n_clumps = d.n_clumps
        s.clump_template, s.clump_scene = _ptr(d.clump_template), _ptr(d.clump_scene)
        s.x, s.q, s.v, s.w = _ptr(d.x), _ptr(d.q), _ptr(d.v), _ptr(d.w)
        s.sphere_mat = _ptr(d.sphere_mat)
        s.n_scenes, s.gravity, s.domain = d.n_scenes, _ptr(d.gravity), _ptr(d.domain)
        s.n_bnd = d.n_bnd
        s.bnd_type, s.bnd_param, s.bnd_mat = _ptr(d.bnd_type), _ptr(d.bnd_param), _ptr(d.bnd_mat)
        s.bnd_vel, s.bnd_omega, s.bnd_scene = _ptr(d.bnd_vel), _ptr(d.bnd_omega), _ptr(d.bnd_scene)
        s.n_presc, s.presc_clump, s.presc_param = len(d.presc_clump), _ptr(d.presc_clump), _ptr(d.presc_param)
        s.n_mesh, s.mesh_state, s.mesh_mat = d.n_mesh, _ptr(d.mesh_state), _ptr(d.mesh_mat)
        s.mesh_scene, s.n_tri = _ptr(d.mesh_scene), d.n_tri
        s.tri_mesh, s.tri_vertex = _ptr(d.tri_mesh), _ptr(d.tri_vertex)
        s.pos_exp = d.pos_exp
        self.n_mesh = d.n_mesh
        self._alloc = None
        self._stream = stream
        try:
            import torch
            if torch.cuda.is_available():
                if torch_allocator:
                    self._alloc = _TorchAllocator(torch.cuda.current_device())
                if self._stream is None:
                    self._stream = torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        h = P()
        rc = L.cdem_create(C.byref(s), C.byref(self._alloc.struct) if self._alloc else None,
                           P(self._stream) if self._stream else None, C.byref(h))
        if rc != 0:
            raise CdemError(rc, L.cdem_last_error(None).decode())
        self._h = h
        self._L = L

    # ---------------------------------------------------------------- helpers
    def _check(self, rc):
        if rc != 0:
            raise CdemError(rc, self._L.cdem_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.cdem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sp(self):
        return P(self._stream) if self._stream else None

    # ---------------------------------------------------------------- API
    def step(self, n: int = 1):
        self._check(self._L.cdem_step(self._h, int(n), P(self._stream) if self._stream else None))

    def sync(self):
        self._check(self._L.cdem_sync(self._h))

    def set_detection(self, mode="plain", k_max=1, safety=1.5, v_max_user=0.0, margin_cap=0.0, audit_period=0,
                      overlap=False):
        m = {"plain": DETECT_PLAIN, "fixed": DETECT_FIXED, "learned": DETECT_LEARNED}[mode]
        p = DetectParamsC(m, int(k_max), float(safety), float(v_max_user), float(margin_cap), int(audit_period),
                          1 if overlap else 0)
        self._check(self._L.cdem_set_detection(self._h, C.byref(p)))

    def record_next_step(self, on: bool = True, walls_only: bool = False):
        """Record the next step's contacts (all of them, or with walls_only
        those with boundaries and mesh triangles)."""
        self._check(self._L.cdem_record_next_step(self._h, (2 if walls_only else 1) if on else 0))

    def counts(self) -> dict:
        c = CountsC()
        self._check(self._L.cdem_get_counts(self._h, C.byref(c)))
        return {n: getattr(c, n) for n, _ in CountsC._fields_ if n != "reserved"}

    def state(self) -> dict:
        n = self.n_clumps
        out = dict(x=np.empty((n, 3)), q=np.empty((n, 4)), v=np.empty((n, 3)), w=np.empty((n, 3)))
        v = StateViewC(_ptr(out["x"]), _ptr(out["q"]), _ptr(out["v"]), _ptr(out["w"]))
        self._check(self._L.cdem_read_state(self._h, C.byref(v), HOST, self._sp()))
        return out

    def state_device(self) -> dict:
        """The clump state copied into fresh torch device tensors (on the scene's stream)."""
        import torch
        n = self.n_clumps
        out = {k: torch.empty((n, w), dtype=torch.float64, device="cuda") for k, w in
               (("x", 3), ("q", 4), ("v", 3), ("w", 3))}
        v = StateViewC(*[P(out[k].data_ptr()) for k in ("x", "q", "v", "w")])
        self._check(self._L.cdem_read_state(self._h, C.byref(v), DEVICE, self._sp()))
        return out

    def write_state_device(self, x=None, q=None, v=None, w=None):
        """Overwrite the clump state from contiguous float64 torch device tensors (None = keep)."""
        for t in (x, q, v, w):
            if t is not None and not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float64"):
                raise ValueError("device state must be contiguous float64 cuda tensors")
        sv = StateViewC(*[None if t is None else P(t.data_ptr()) for t in (x, q, v, w)])
        self._check(self._L.cdem_write_state(self._h, C.byref(sv), DEVICE, self._sp()))

    def write_state(self, x=None, q=None, v=None, w=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (x, q, v, w)]
        sv = StateViewC(*[_ptr(a) for a in arrs])
        self._check(self._L.cdem_write_state(self._h, C.byref(sv), HOST, self._sp()))

    def contacts(self) -> dict:
        v = ContactsViewC(0, 0, None, None, None, None, None, None, None)
        self._check(self._L.cdem_read_contacts(self._h, C.byref(v)))
        n = v.n
        out = dict(a=np.empty(n, np.uint32), b=np.empty(n, np.uint32), delta=np.empty(n),
                   F=np.empty((n, 3)), u=np.empty((n, 3)), Ta=np.empty((n, 3)), Tb=np.empty((n, 3)))
        v = ContactsViewC(n, 0, _ptr(out["a"]), _ptr(out["b"]), _ptr(out["delta"]), _ptr(out["F"]), _ptr(out["u"]),
                          _ptr(out["Ta"]), _ptr(out["Tb"]))
        self._check(self._L.cdem_read_contacts(self._h, C.byref(v)))
        return out

    def boundary_forces(self):
        """Force on each boundary and torque about its reference point at the recorded step."""
        n = self.n_bnd
        F = np.zeros((n, 3)); T = np.zeros((n, 3))
        self._check(self._L.cdem_read_boundary_forces(self._h, _ptr(F), _ptr(T)))
        return F, T

    def clump_forces(self):
        F, T = np.empty((self.n_clumps, 3)), np.empty((self.n_clumps, 3))
        self._check(self._L.cdem_read_clump_forces(self._h, _ptr(F), _ptr(T)))
        return F, T

    def sphere_pos(self) -> np.ndarray:
        xs = np.empty((self.n_spheres, 3))
        self._check(self._L.cdem_read_sphere_pos(self._h, _ptr(xs)))
        return xs

    def audit(self) -> dict:
        r = AuditResultC()
        rc = self._L.cdem_audit(self._h, C.byref(r))
        if rc not in (0, -5):
            self._check(rc)
        return dict(true_contacts=r.true_contacts, missed=r.missed, first=(r.first_a, r.first_b))

    # ---------------------------------------------------------------- measurement
    def profile(self, on: bool = True, only=None):
        """Per-kernel event timing on/off; `only`: names of the kernels to time."""
        if on and only:
            self._check(self._L.cdem_profile_kernels(self._h, ",".join(only).encode()))
        else:
            self._check(self._L.cdem_profile(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        n = C.c_int(0)
        self._check(self._L.cdem_profile_read(self._h, None, 0, C.byref(n)))
        arr = (KernelTimeC * max(n.value, 1))()
        self._check(self._L.cdem_profile_read(self._h, arr, n.value, C.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}

    def last_step_contacts(self) -> int:
        v = C.c_int64(0)
        self._check(self._L.cdem_last_step_contacts(self._h, C.byref(v)))
        return v.value

    def set_graph(self, steps_per_graph: int):
        self._check(self._L.cdem_set_graph(self._h, int(steps_per_graph)))

    def autotune(self, steps: int = 5):
        f, c = C.c_double(0), C.c_int32(0)
        self._check(self._L.cdem_autotune(self._h, int(steps), C.byref(f), C.byref(c)))
        return dict(bin_factor=f.value, stride_cap=c.value)

    # ---------------------------------------------------------------- learned envelopes
    def save(self) -> bytes:
        """Checkpoint of the scene's dynamic state (see cdem_save)."""
        n = C.c_size_t(0)
        self._check(self._L.cdem_save(self._h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self._L.cdem_save(self._h, buf, n.value, C.byref(n)))
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        """Restore a checkpoint written by :meth:`save` of a scene with the same description."""
        self._check(self._L.cdem_load(self._h, blob, len(blob)))

    def set_mesh_state(self, mesh: int, state):
        """Prescribe a mesh's state: x[3], q[4], v[3], w[3] (world angular velocity)."""
        st = np.ascontiguousarray(state, np.float64).reshape(13)
        self._check(self._L.cdem_set_mesh_state(self._h, int(mesh), _ptr(st)))

    def mesh_state(self) -> np.ndarray:
        st = np.empty((self.n_mesh, 13))
        self._check(self._L.cdem_read_mesh_state(self._h, _ptr(st)))
        return st

    def mesh_forces(self):
        """Force on each mesh and torque about its reference point at the recorded step."""
        F, T = np.empty((self.n_mesh, 3)), np.empty((self.n_mesh, 3))
        self._check(self._L.cdem_read_mesh_forces(self._h, _ptr(F), _ptr(T)))
        return F, T

    def set_force_law(self, source):
        """Compile a user force law (the source of `cdem_user_law`, see
        include/cdem.h) into the pair kernel; None restores the built-in law.
        Raises CdemError with the compiler's messages when it does not compile."""
        log = C.create_string_buffer(1 << 16)
        rc = self._L.cdem_set_force_law(self._h, source.encode() if source else None, log, len(log))
        if rc:
            raise CdemError(rc, f"{self._L.cdem_last_error(self._h).decode()}\n{log.value.decode()}")
        return log.value.decode()

    def set_mlp(self, params):
        p = np.ascontiguousarray(params, np.float32)
        self._check(self._L.cdem_set_mlp(self._h, _ptr(p), p.size))

    def collect_envelopes(self, horizon: int = 20):
        """Per-bin features of the current state and the envelopes the bins'
        spheres show over the next `horizon` steps (which this call runs)."""
        n = C.c_int64(0)
        cap = max(1, self.counts()["bins"])
        f = np.empty((cap, 3), np.float32)
        y = np.empty((cap, 2), np.float32)
        self._check(self._L.cdem_collect_envelopes(self._h, int(horizon), _ptr(f), _ptr(y), cap, C.byref(n)))
        return f[:n.value].copy(), y[:n.value].copy()


def _dev(t):
    return P(t.data_ptr())


def _stream():
    import torch
    s = torch.cuda.current_stream().cuda_stream
    return P(s) if s else None


def mlp_param_count() -> int:
    return load().cdem_mlp_param_count()


def mlp_forward(params, features):
    """params: device float32 tensor; features [n, 3] device float32 -> [n, 2]."""
    import torch
    L = load()
    out = torch.empty((features.shape[0], 2), dtype=torch.float32, device=features.device)
    rc = L.cdem_mlp_forward(_dev(params), _dev(features), _dev(out), features.shape[0], _stream())
    if rc:
        raise CdemError(rc, "cdem_mlp_forward")
    return out


def mlp_backward(params, features, target, tau):
    """Gradient and loss of the mean pinball loss (device tensors)."""
    import torch
    L = load()
    n = features.shape[0]
    ws = torch.empty(int(L.cdem_mlp_workspace_bytes(n)) // 4 + 1, dtype=torch.float32, device=features.device)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=features.device)
    rc = L.cdem_mlp_backward(_dev(params), _dev(features), _dev(target), n, float(tau), _dev(grad), _dev(loss),
                             _dev(ws), _stream())
    if rc:
        raise CdemError(rc, "cdem_mlp_backward")
    return grad, loss


def check_force_law(source: str):
    """Compile a user force law without a device: (ok, compiler messages)."""
    log = C.create_string_buffer(1 << 16)
    rc = load().cdem_check_force_law(source.encode(), log, len(log))
    return rc == 0, log.value.decode()


MLP_STATIC_MAX_SAMPLES = 16384  # CDEM_MLP_STATIC_MAX_SAMPLES of include/cdem.h


def mlp_backward_static(params, features, target, tau, grad, loss):
    """cdem_mlp_backward_static: the gradient and loss into caller-owned
    device tensors `grad` and `loss`, with no workspace (the library's static
    device array holds the partials).  Raises CdemError on a failed call."""
    L = load()
    rc = L.cdem_mlp_backward_static(_dev(params), _dev(features), _dev(target), features.shape[0], float(tau),
                                    _dev(grad), _dev(loss), _stream())
    if rc:
        raise CdemError(rc, "cdem_mlp_backward_static")


def mlp_adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    rc = load().cdem_mlp_adam(_dev(params), _dev(grad), _dev(m), _dev(v), int(t), float(lr), float(beta1),
                              float(beta2), float(eps), _stream())
    if rc:
        raise CdemError(rc, "cdem_mlp_adam")
