"""Thin ctypes binding of libdect.so (C-ABI in include/dect.h).

Only argument marshalling lives here: torch CUDA tensors provide device
memory and the current HIP stream; every step of the computation runs in the
library's HIP kernels.  Importing this module fails loudly when the library
is not built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field, fields
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdect.so")

DECT_OK = 0


class DectError(RuntimeError):
    pass


class _Geometry(C.Structure):
    _fields_ = [("n_x", C.c_int32), ("n_y", C.c_int32), ("pixel_mm", C.c_double),
                ("n_views", C.c_int32), ("angle0_rad", C.c_double), ("arc_rad", C.c_double),
                ("n_det", C.c_int32), ("det_pitch_mm", C.c_double), ("det_offset_mm", C.c_double),
                ("sid_mm", C.c_double), ("sdd_mm", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("E_lo_keV", C.c_double), ("E_hi_keV", C.c_double), ("E1_keV", C.c_double),
                ("E2_keV", C.c_double), ("m", C.c_double), ("n", C.c_double), ("Cp", C.c_double),
                ("Z_w", C.c_double), ("basis_Z", C.c_double * 2), ("basis_rho", C.c_double * 2),
                ("lambda_", C.c_double), ("beta0", C.c_double), ("beta_max", C.c_double),
                ("kappa", C.c_double), ("eta", C.c_double), ("xi", C.c_double),
                ("n_iter", C.c_int32), ("f_inner", C.c_int32), ("t_tol", C.c_double),
                ("t_maxit", C.c_int32), ("rho_min", C.c_double), ("t_min", C.c_double),
                ("t_precond", C.c_int32), ("storage", C.c_int32)]


class _Schedule(C.Structure):
    _fields_ = [("fp_rays_per_lane", C.c_int32), ("bp_cu_percent", C.c_int32),
                ("rho_stream", C.c_int32), ("graphs", C.c_int32), ("pcg_chunk_extra", C.c_int32),
                ("pcg_chunk_first", C.c_int32)]


SCHEDULE_KEYS = [f[0] for f in _Schedule._fields_]


EXPORTS = [
    "dect_default_params", "dect_resolve_geometry", "dect_attenuation", "dect_project",
    "dect_backproject", "dect_fbp", "dect_l0_step_workspace_bytes", "dect_l0_step",
    "dect_l0_step_static_max_values", "dect_l0_step_static",
    "dect_solve_workspace_bytes", "dect_solver_create", "dect_solver_destroy", "dect_solver_init",
    "dect_solver_set_state", "dect_solver_iterate", "dect_solver_get_state", "dect_solver_finish",
    "dect_solver_stats", "dect_solver_get_schedule", "dect_solver_set_schedule",
    "dect_solver_autotune", "dect_solver_set_graphs", "dect_solver_enable_timing",
    "dect_solver_timing", "dect_solver_timeline", "dect_solve",
    "dect_solve_workspace_bytes_multi", "dect_solver_create_multi", "dect_solve_multi",
    "dect_engine_workspace_bytes", "dect_engine_create", "dect_engine_destroy", "dect_engine_admit",
    "dect_engine_step", "dect_engine_step_n", "dect_engine_status", "dect_engine_completed",
    "dect_engine_cancel",
    "dect_uneven_create", "dect_uneven_destroy", "dect_uneven_groups", "dect_uneven_init",
    "dect_uneven_iterate", "dect_uneven_finish", "dect_uneven_autotune", "dect_uneven_get_schedule",
    "dect_solve_uneven",
    "dect_image_workspace_bytes", "dect_image_solver_create", "dect_image_solver_init",
    "dect_image_solver_set_state", "dect_solve_image",
    "dect_last_error",
]

DECT_EBUSY = -6
DECT_STORAGE_FP32 = 0
DECT_STORAGE_BF16 = 1
DECT_STORAGE_BF16_STATE = 2


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libdect.so is not built ({path}); run __graft_entry__.build() "
                          "or python paper_2308_01290_amd/build.py")
    # torch brings its own HIP runtime; loading it first makes libdect.so bind
    # to that same runtime (one device context, shared streams and memory)
    # instead of pulling a second copy from /opt/rocm into the process.
    import torch  # noqa: F401
    L = C.CDLL(path)
    P, vp = C.POINTER, C.c_void_p
    G, Pp = P(_Geometry), P(_Params)
    L.dect_default_params.argtypes = [Pp]
    L.dect_default_params.restype = None
    L.dect_resolve_geometry.argtypes = [G]
    L.dect_attenuation.argtypes = [Pp, P(C.c_double), P(C.c_double), C.c_int64, P(C.c_double), P(C.c_double)]
    for name in ("dect_project", "dect_backproject", "dect_fbp"):
        getattr(L, name).argtypes = [G, vp, vp, C.c_int32, vp]
    L.dect_l0_step_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int]
    L.dect_l0_step_workspace_bytes.restype = C.c_size_t
    L.dect_l0_step.argtypes = [vp, vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                               C.c_double, C.c_double, C.c_int32, vp, C.c_size_t, vp]
    L.dect_l0_step_static_max_values.argtypes = []
    L.dect_l0_step_static_max_values.restype = C.c_size_t
    L.dect_l0_step_static.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                      C.c_double, vp]
    L.dect_solve_workspace_bytes.argtypes = [G, Pp, C.c_int32]
    L.dect_solve_workspace_bytes.restype = C.c_size_t
    L.dect_solver_create.argtypes = [G, Pp, C.c_int32, vp, C.c_size_t, vp, P(vp)]
    L.dect_solver_destroy.argtypes = [vp]
    L.dect_solver_init.argtypes = [vp, vp, vp]
    L.dect_solver_set_state.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_int32]
    L.dect_solver_iterate.argtypes = [vp, C.c_int32]
    L.dect_solver_get_state.argtypes = [vp, vp, vp, vp, vp]
    L.dect_solver_finish.argtypes = [vp, vp, vp]
    L.dect_solver_stats.argtypes = [vp, P(C.c_int32), P(C.c_int32)]
    L.dect_solver_get_schedule.argtypes = [vp, P(_Schedule)]
    L.dect_solver_set_schedule.argtypes = [vp, P(_Schedule)]
    L.dect_solver_autotune.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, P(_Schedule), P(C.c_double)]
    L.dect_solver_set_graphs.argtypes = [vp, C.c_int]
    L.dect_solver_enable_timing.argtypes = [vp, C.c_int]
    L.dect_solver_timing.argtypes = [vp, P(C.c_double), P(C.c_int32), P(C.c_double), P(C.c_int32)]
    L.dect_solver_timeline.argtypes = [vp, vp, C.c_int32, P(C.c_int32)]
    L.dect_solve.argtypes = [vp, vp, G, Pp, vp, vp, C.c_int32, vp, C.c_size_t, vp]
    L.dect_solve_workspace_bytes_multi.argtypes = [G, Pp, C.c_int32]
    L.dect_solve_workspace_bytes_multi.restype = C.c_size_t
    L.dect_solver_create_multi.argtypes = [G, Pp, C.c_int32, vp, C.c_size_t, vp, P(vp)]
    L.dect_solve_multi.argtypes = [vp, vp, G, Pp, vp, vp, C.c_int32, vp, C.c_size_t, vp]
    i32 = C.c_int32
    L.dect_engine_workspace_bytes.argtypes = [i32, i32, C.c_double, i32, i32, i32, Pp]
    L.dect_engine_workspace_bytes.restype = C.c_size_t
    L.dect_engine_create.argtypes = [i32, i32, C.c_double, i32, i32, i32, Pp, vp, C.c_size_t, vp, P(vp)]
    L.dect_engine_destroy.argtypes = [vp]
    L.dect_engine_admit.argtypes = [vp, G, vp, vp, i32, vp, vp, P(i32)]
    L.dect_engine_step.argtypes = [vp]
    L.dect_engine_step_n.argtypes = [vp, i32, P(i32)]
    L.dect_engine_status.argtypes = [vp, P(i32), P(i32)]
    L.dect_engine_cancel.argtypes = [vp, i32]
    L.dect_uneven_create.argtypes = [G, i32, Pp, vp, P(vp)]
    L.dect_uneven_destroy.argtypes = [vp]
    L.dect_uneven_groups.argtypes = [vp, P(i32)]
    L.dect_uneven_init.argtypes = [vp, vp, vp]
    L.dect_uneven_iterate.argtypes = [vp, i32]
    L.dect_uneven_finish.argtypes = [vp, vp, vp]
    L.dect_uneven_autotune.argtypes = [vp, vp, vp, i32, i32]
    L.dect_uneven_get_schedule.argtypes = [vp, i32, P(_Schedule)]
    L.dect_solve_uneven.argtypes = [vp, vp, G, Pp, vp, vp, i32, vp]
    L.dect_engine_completed.argtypes = [vp, P(i32), i32, P(i32)]
    L.dect_image_workspace_bytes.argtypes = [i32, i32, Pp, i32]
    L.dect_image_workspace_bytes.restype = C.c_size_t
    L.dect_image_solver_create.argtypes = [i32, i32, Pp, i32, vp, C.c_size_t, vp, P(vp)]
    L.dect_image_solver_init.argtypes = [vp, vp, vp]
    L.dect_image_solver_set_state.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32]
    L.dect_solve_image.argtypes = [vp, vp, i32, i32, Pp, vp, vp, i32, vp, C.c_size_t, vp]
    L.dect_last_error.argtypes = []
    L.dect_last_error.restype = C.c_char_p
    return L


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(rc: int, what: str):
    if rc != DECT_OK:
        msg = lib().dect_last_error().decode(errors="replace")
        raise DectError(f"{what} failed ({rc}): {msg}")


# ---------------------------------------------------------------------------
# configuration objects
# ---------------------------------------------------------------------------
@dataclass
class Geometry:
    n_x: int
    n_y: int
    pixel_mm: float
    n_views: int
    n_det: int
    sid_mm: float
    sdd_mm: float
    det_pitch_mm: float = 0.0
    det_offset_mm: float = 0.0
    angle0_rad: float = 0.0
    arc_rad: float = 2.0 * math.pi

    @staticmethod
    def of(obj) -> "Geometry":
        return Geometry(**{f.name: getattr(obj, f.name) for f in fields(Geometry)})

    def c(self) -> _Geometry:
        return _Geometry(self.n_x, self.n_y, self.pixel_mm, self.n_views, self.angle0_rad,
                         self.arc_rad, self.n_det, self.det_pitch_mm, self.det_offset_mm,
                         self.sid_mm, self.sdd_mm)


_PARAM_NAMES = [f[0] for f in _Params._fields_]


def default_params(**overrides) -> _Params:
    p = _Params()
    lib().dect_default_params(C.byref(p))
    for k, v in overrides.items():
        key = "lambda_" if k in ("lambda", "lam") else k
        if key not in _PARAM_NAMES:
            raise KeyError(k)
        if key in ("basis_Z", "basis_rho"):
            getattr(p, key)[0], getattr(p, key)[1] = v
        else:
            setattr(p, key, v)
    return p


def resolve_geometry(geom) -> Geometry:
    g = Geometry.of(geom).c()
    _check(lib().dect_resolve_geometry(C.byref(g)), "dect_resolve_geometry")
    return Geometry(g.n_x, g.n_y, g.pixel_mm, g.n_views, g.n_det, g.sid_mm, g.sdd_mm,
                    g.det_pitch_mm, g.det_offset_mm, g.angle0_rad, g.arc_rad)


def attenuation(params: _Params, Z, rho_e):
    """Host FP64 model: (mu_lo, mu_hi) in 1/mm for arrays of (Z, rho_e)."""
    import numpy as np
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    R = np.ascontiguousarray(rho_e, dtype=np.float64)
    shape = np.broadcast(Z, R).shape
    Z = np.ascontiguousarray(np.broadcast_to(Z, shape))
    R = np.ascontiguousarray(np.broadcast_to(R, shape))
    lo = np.empty(shape)
    hi = np.empty(shape)
    dp = C.POINTER(C.c_double)
    _check(lib().dect_attenuation(C.byref(params), Z.ctypes.data_as(dp), R.ctypes.data_as(dp),
                                  Z.size, lo.ctypes.data_as(dp), hi.ctypes.data_as(dp)),
           "dect_attenuation")
    return lo, hi


# ---------------------------------------------------------------------------
# tensor helpers
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_f32(t, shape_tail, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [..., {shape_tail}]")
    return t


def _batch(t, ndim_tail=2):
    n = 1
    for s in t.shape[:-ndim_tail]:
        n *= int(s)
    return n


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------
def project(geom, img, out=None, stream=None):
    """sino = A img, img [..., n_y, n_x] -> [..., n_views, n_det] (float32)."""
    torch = _torch()
    g = Geometry.of(geom)
    _dev_f32(img, (g.n_y, g.n_x), "img")
    if out is None:
        out = torch.empty(img.shape[:-2] + (g.n_views, g.n_det), device=img.device, dtype=torch.float32)
    _dev_f32(out, (g.n_views, g.n_det), "out")
    gc = g.c()
    _check(lib().dect_project(C.byref(gc), _ptr(img), _ptr(out), _batch(img), C.c_void_p(_stream(stream))),
           "dect_project")
    return out


def backproject(geom, sino, out=None, stream=None):
    """img = A^T sino, [..., n_views, n_det] -> [..., n_y, n_x] (float32)."""
    torch = _torch()
    g = Geometry.of(geom)
    _dev_f32(sino, (g.n_views, g.n_det), "sino")
    if out is None:
        out = torch.empty(sino.shape[:-2] + (g.n_y, g.n_x), device=sino.device, dtype=torch.float32)
    _dev_f32(out, (g.n_y, g.n_x), "out")
    gc = g.c()
    _check(lib().dect_backproject(C.byref(gc), _ptr(sino), _ptr(out), _batch(sino),
                                  C.c_void_p(_stream(stream))), "dect_backproject")
    return out


def fbp(geom, sino, out=None, stream=None):
    """Fan-beam FBP, [..., n_views, n_det] -> attenuation image [..., n_y, n_x]."""
    torch = _torch()
    g = Geometry.of(geom)
    _dev_f32(sino, (g.n_views, g.n_det), "sino")
    if out is None:
        out = torch.empty(sino.shape[:-2] + (g.n_y, g.n_x), device=sino.device, dtype=torch.float32)
    gc = g.c()
    _check(lib().dect_fbp(C.byref(gc), _ptr(sino), _ptr(out), _batch(sino), C.c_void_p(_stream(stream))),
           "dect_fbp")
    return out


def l0_step(g_tilde, g, lam, beta, weight=None, tol=1e-6, max_iter=200, return_hv=False,
            stream=None):
    """One HQS step of the gradient-L0 model (in place on g); see include/dect.h."""
    torch = _torch()
    ny, nx = g.shape[-2:]
    _dev_f32(g, (ny, nx), "g")
    _dev_f32(g_tilde, (ny, nx), "g_tilde")
    if weight is not None:
        _dev_f32(weight, (ny, nx), "weight")
    for t, name in ((g_tilde, "g_tilde"), (weight, "weight")):
        if t is not None and tuple(t.shape) != tuple(g.shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, g has {tuple(g.shape)}")
    h = v = None
    if return_hv:
        h = torch.empty_like(g)
        v = torch.empty_like(g)
    _check(lib().dect_l0_step(_ptr(g_tilde), _ptr(weight), _ptr(g), _ptr(h), _ptr(v), ny, nx,
                               _batch(g), float(lam), float(beta), float(tol), int(max_iter), None, 0,
                               C.c_void_p(_stream(stream))), "dect_l0_step")
    return (g, h, v) if return_hv else g


def l0_step_static(g_tilde, g, lam, beta, h=None, v=None, stream=None):
    """The allocation-free unit-weight HQS step (in place on g; h, v are
    optional caller-allocated outputs); see include/dect.h."""
    ny, nx = g.shape[-2:]
    _dev_f32(g, (ny, nx), "g")
    _dev_f32(g_tilde, (ny, nx), "g_tilde")
    for t, name in ((g_tilde, "g_tilde"), (h, "h"), (v, "v")):
        if t is not None:
            _dev_f32(t, (ny, nx), name)
            if tuple(t.shape) != tuple(g.shape):
                raise ValueError(f"{name} has shape {tuple(t.shape)}, g has {tuple(g.shape)}")
    _check(lib().dect_l0_step_static(_ptr(g_tilde), _ptr(g), _ptr(h), _ptr(v), ny, nx, _batch(g),
                                      float(lam), float(beta), C.c_void_p(_stream(stream))),
           "dect_l0_step_static")
    return g


def _geometry_array(geoms):
    gs = [Geometry.of(g) for g in geoms]
    arr = (_Geometry * len(gs))(*[g.c() for g in gs])
    return gs, arr


def sinogram_elements(geoms) -> int:
    """Length of the back-to-back sinograms of a batch of uneven slices."""
    return sum(int(g.n_views) * int(g.n_det) for g in geoms)


def concat_sinograms(sinos):
    """Slices' [n_views, n_det] sinograms back to back (the layout of the
    uneven-batch entry points)."""
    torch = _torch()
    return torch.cat([t.reshape(-1) for t in sinos]).contiguous()


class Solver:
    """A batch of slices with shared parameters and image grid, state on device.

    `geom` is one geometry (with `batch` slices of it) or a sequence of
    per-slice geometries (uneven batch; sinograms then go back to back, see
    concat_sinograms)."""

    def __init__(self, geom, params=None, batch: int = 1, device="cuda", stream=None):
        self.params = params if params is not None else default_params()
        self.device = device
        self._stream = stream
        h = C.c_void_p()
        if isinstance(geom, (list, tuple)):
            self.geoms, arr = _geometry_array(geom)
            self.geom = self.geoms[0]
            self.batch = len(self.geoms)
            self.uneven = True
            _check(lib().dect_solver_create_multi(arr, C.byref(self.params), self.batch, None, 0,
                                                  C.c_void_p(_stream(stream)), C.byref(h)),
                   "dect_solver_create_multi")
        else:
            self.geom = Geometry.of(geom)
            self.batch = int(batch)
            self.geoms = [self.geom] * self.batch
            self.uneven = False
            gc = self.geom.c()
            _check(lib().dect_solver_create(C.byref(gc), C.byref(self.params), self.batch, None, 0,
                                            C.c_void_p(_stream(stream)), C.byref(h)),
                   "dect_solver_create")
        self._h = h

    def _check_sinos(self, lo, hi):
        if self.uneven:
            n = sinogram_elements(self.geoms)
            for name, t in (("sino_lo", lo), ("sino_hi", hi)):
                _dev_f32(t, (t.shape[-1],), name)
                if t.numel() != n:
                    raise ValueError(f"{name} has {t.numel()} elements, the batch needs {n}")
        else:
            _dev_f32(lo, (self.geom.n_views, self.geom.n_det), "sino_lo")
            _dev_f32(hi, (self.geom.n_views, self.geom.n_det), "sino_hi")

    def close(self):
        if getattr(self, "_h", None):
            lib().dect_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _img(self, n=1):
        torch = _torch()
        return torch.empty((self.batch, self.geom.n_y, self.geom.n_x), device=self.device,
                           dtype=torch.float32)

    def _check_inputs(self, lo, hi):
        self._check_sinos(lo, hi)

    def init(self, sino_lo, sino_hi):
        self._check_sinos(sino_lo, sino_hi)
        _check(lib().dect_solver_init(self._h, _ptr(sino_lo), _ptr(sino_hi)), "dect_solver_init")
        self._keep = (sino_lo, sino_hi)
        return self

    def set_state(self, sino_lo, sino_hi, f1, f2, rho, t, k=0):
        self._check_sinos(sino_lo, sino_hi)
        for name, a in (("f1", f1), ("f2", f2), ("rho", rho), ("t", t)):
            _dev_f32(a, (self.geom.n_y, self.geom.n_x), name)
        _check(lib().dect_solver_set_state(self._h, _ptr(sino_lo), _ptr(sino_hi), _ptr(f1), _ptr(f2),
                                           _ptr(rho), _ptr(t), int(k)), "dect_solver_set_state")
        self._keep = (sino_lo, sino_hi, f1, f2, rho, t)
        return self

    def iterate(self, n: int = 1):
        _check(lib().dect_solver_iterate(self._h, int(n)), "dect_solver_iterate")
        return self

    def state(self):
        f1, f2, rho, t = self._img(), self._img(), self._img(), self._img()
        _check(lib().dect_solver_get_state(self._h, _ptr(f1), _ptr(f2), _ptr(rho), _ptr(t)),
               "dect_solver_get_state")
        return f1, f2, rho, t

    def finish(self):
        Z, rho = self._img(), self._img()
        _check(lib().dect_solver_finish(self._h, _ptr(Z), _ptr(rho)), "dect_solver_finish")
        return Z, rho

    def schedule(self):
        """The launch schedule as a dict (see dect_schedule)."""
        sc = _Schedule()
        _check(lib().dect_solver_get_schedule(self._h, C.byref(sc)), "dect_solver_get_schedule")
        return {k: int(getattr(sc, k)) for k in SCHEDULE_KEYS}

    def set_schedule(self, **kw):
        """Change schedule fields by name; results do not depend on them."""
        cur = self.schedule()
        for k, v in kw.items():
            if k not in cur:
                raise KeyError(k)
            cur[k] = int(v)
        sc = _Schedule(**cur)
        _check(lib().dect_solver_set_schedule(self._h, C.byref(sc)), "dect_solver_set_schedule")
        return self

    def autotune(self, lo, hi, iters: int = 8, reps: int = 3):
        """Time candidate schedules on these inputs, keep the fastest; returns
        (schedule dict, ms per outer iteration).  The iterate is left at the
        last trial's: init before solving."""
        self._check_inputs(lo, hi)
        sc, ms = _Schedule(), C.c_double()
        _check(lib().dect_solver_autotune(self._h, _ptr(lo), _ptr(hi), int(iters), int(reps),
                                          C.byref(sc), C.byref(ms)), "dect_solver_autotune")
        return {k: int(getattr(sc, k)) for k in SCHEDULE_KEYS}, float(ms.value)

    def set_graphs(self, on: bool = True):
        """Replay each outer iteration's first chunk of PCG iterations from a
        captured HIP graph (bit-identical to launching them one by one)."""
        _check(lib().dect_solver_set_graphs(self._h, 1 if on else 0), "dect_solver_set_graphs")
        return self

    def enable_timing(self, on: bool = True, timeline: bool = False, bp_only: bool = False):
        """Kernel timing (timing()) and, with `timeline`, the iteration
        timeline (timeline()); both off with on=False.  With `bp_only` the
        forward projections are not timed (half the events per iteration)."""
        flags = (1 if on else 0) | (2 if on and timeline else 0) | (4 if on and bp_only else 0)
        _check(lib().dect_solver_enable_timing(self._h, flags), "dect_solver_enable_timing")
        return self

    def timing(self):
        """(backproject_ms, n_bp, project_ms, n_fp) since the last call (synchronises)."""
        bms, fms = C.c_double(), C.c_double()
        bn, fn = C.c_int32(), C.c_int32()
        _check(lib().dect_solver_timing(self._h, C.byref(bms), C.byref(bn), C.byref(fms), C.byref(fn)),
               "dect_solver_timing")
        return bms.value, bn.value, fms.value, fn.value

    def timeline(self, max_rows: int = 4096):
        """Iteration timeline since the last call (dect_solver_timeline): an
        array of rows (gradient reached, forward projection done, update done,
        PCG set-up done, PCG done), microseconds after the previous update."""
        import numpy as np
        out = np.zeros((max_rows, 5), np.float32)
        n = C.c_int32()
        _check(lib().dect_solver_timeline(self._h, out.ctypes.data, max_rows, C.byref(n)),
               "dect_solver_timeline")
        return out[: n.value].astype(np.float64)

    def stats(self):
        k = C.c_int32()
        it = C.c_int32()
        _check(lib().dect_solver_stats(self._h, C.byref(k), C.byref(it)), "dect_solver_stats")
        return int(k.value), int(it.value)


class ImageSolver(Solver):
    """The image-domain form of Algorithm 1: a batch of [n_y, n_x] attenuation
    image pairs, state on device.  iterate / state / finish / stats as Solver."""

    def __init__(self, n_x: int, n_y: int, params=None, batch: int = 1, device="cuda", stream=None):
        self.params = params if params is not None else default_params()
        self.device = device
        self._stream = stream
        self.batch = int(batch)
        self.n_x, self.n_y = int(n_x), int(n_y)
        self.geom = _ImageGrid(self.n_x, self.n_y)
        self.uneven = False
        h = C.c_void_p()
        _check(lib().dect_image_solver_create(self.n_x, self.n_y, C.byref(self.params), self.batch,
                                              None, 0, C.c_void_p(_stream(stream)), C.byref(h)),
               "dect_image_solver_create")
        self._h = h

    def _check_mu(self, mu_lo, mu_hi):
        for name, a in (("mu_lo", mu_lo), ("mu_hi", mu_hi)):
            _dev_f32(a, (self.n_y, self.n_x), name)
            if _batch(a) != self.batch:
                raise ValueError(f"{name} holds {_batch(a)} images, the solver {self.batch}")

    def _check_inputs(self, lo, hi):
        self._check_mu(lo, hi)

    def init(self, mu_lo, mu_hi):
        self._check_mu(mu_lo, mu_hi)
        _check(lib().dect_image_solver_init(self._h, _ptr(mu_lo), _ptr(mu_hi)), "dect_image_solver_init")
        self._keep = (mu_lo, mu_hi)
        return self

    def set_state(self, mu_lo, mu_hi, f1, f2, rho, t, k=0):
        self._check_mu(mu_lo, mu_hi)
        for name, a in (("f1", f1), ("f2", f2), ("rho", rho), ("t", t)):
            _dev_f32(a, (self.n_y, self.n_x), name)
            if _batch(a) != self.batch:
                raise ValueError(f"{name} holds {_batch(a)} images, the solver {self.batch}")
        _check(lib().dect_image_solver_set_state(self._h, _ptr(mu_lo), _ptr(mu_hi), _ptr(f1), _ptr(f2),
                                                 _ptr(rho), _ptr(t), int(k)),
               "dect_image_solver_set_state")
        self._keep = (mu_lo, mu_hi, f1, f2, rho, t)
        return self


@dataclass
class _ImageGrid:
    n_x: int
    n_y: int


def solve_image(mu_lo, mu_hi, params=None, stream=None):
    """Whole image-domain solve of [batch,] n_y x n_x attenuation image pairs
    -> (Z, rho_e), each [batch, n_y, n_x]."""
    torch = _torch()
    if mu_lo.dim() < 2:
        raise ValueError("mu_lo must be [batch,] n_y x n_x")
    n_y, n_x = int(mu_lo.shape[-2]), int(mu_lo.shape[-1])
    _dev_f32(mu_lo, (n_y, n_x), "mu_lo")
    _dev_f32(mu_hi, (n_y, n_x), "mu_hi")
    b = _batch(mu_lo)
    if _batch(mu_hi) != b:
        raise ValueError("mu_lo and mu_hi hold different numbers of images")
    p = params if params is not None else default_params()
    Z = torch.empty((b, n_y, n_x), device=mu_lo.device, dtype=torch.float32)
    R = torch.empty_like(Z)
    _check(lib().dect_solve_image(_ptr(mu_lo), _ptr(mu_hi), n_x, n_y, C.byref(p), _ptr(Z), _ptr(R), b,
                                  None, 0, C.c_void_p(_stream(stream))), "dect_solve_image")
    return Z, R


def solve(sino_lo, sino_hi, geom, params=None, stream=None):
    """Whole solve -> (Z, rho_e), each [batch, n_y, n_x]."""
    torch = _torch()
    g = Geometry.of(geom)
    p = params if params is not None else default_params()
    _dev_f32(sino_lo, (g.n_views, g.n_det), "sino_lo")
    _dev_f32(sino_hi, (g.n_views, g.n_det), "sino_hi")
    b = _batch(sino_lo)
    Z = torch.empty((b, g.n_y, g.n_x), device=sino_lo.device, dtype=torch.float32)
    R = torch.empty_like(Z)
    gc = g.c()
    _check(lib().dect_solve(_ptr(sino_lo), _ptr(sino_hi), C.byref(gc), C.byref(p), _ptr(Z), _ptr(R), b,
                            None, 0, C.c_void_p(_stream(stream))), "dect_solve")
    return Z, R


def solve_multi(sino_lo, sino_hi, geoms, params=None, stream=None):
    """Whole solve of a batch of uneven slices (sinograms back to back, see
    concat_sinograms) -> (Z, rho_e), each [batch, n_y, n_x]."""
    torch = _torch()
    gs, arr = _geometry_array(geoms)
    p = params if params is not None else default_params()
    n = sinogram_elements(gs)
    for name, t in (("sino_lo", sino_lo), ("sino_hi", sino_hi)):
        _dev_f32(t, (t.shape[-1],), name)
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} elements, the batch needs {n}")
    b = len(gs)
    Z = torch.empty((b, gs[0].n_y, gs[0].n_x), device=sino_lo.device, dtype=torch.float32)
    R = torch.empty_like(Z)
    _check(lib().dect_solve_multi(_ptr(sino_lo), _ptr(sino_hi), arr, C.byref(p), _ptr(Z), _ptr(R), b,
                                  None, 0, C.c_void_p(_stream(stream))), "dect_solve_multi")
    return Z, R


def image_elements(geoms) -> int:
    """Length of the back-to-back images of a batch of mixed image sizes."""
    return sum(int(Geometry.of(g).n_x) * int(Geometry.of(g).n_y) for g in geoms)


def split_images(flat, geoms):
    """[n_y, n_x] views of the slices' back-to-back images."""
    out, o = [], 0
    for g in geoms:
        g = Geometry.of(g)
        n = int(g.n_x) * int(g.n_y)
        out.append(flat[o:o + n].view(int(g.n_y), int(g.n_x)))
        o += n
    return out


class UnevenSolver:
    """A batch of slices of mixed image sizes (and views, bins, detectors): one
    uneven-batch solver per image grid, iterated together (see include/dect.h).
    Sinograms and images go back to back in slice order."""

    def __init__(self, geoms, params=None, device="cuda", stream=None):
        self.params = params if params is not None else default_params()
        self.geoms, arr = _geometry_array(geoms)
        self.batch = len(self.geoms)
        self.device = device
        h = C.c_void_p()
        _check(lib().dect_uneven_create(arr, self.batch, C.byref(self.params),
                                        C.c_void_p(_stream(stream)), C.byref(h)), "dect_uneven_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().dect_uneven_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def groups(self) -> int:
        n = C.c_int32()
        _check(lib().dect_uneven_groups(self._h, C.byref(n)), "dect_uneven_groups")
        return int(n.value)

    def _check_sinos(self, lo, hi):
        n = sinogram_elements(self.geoms)
        for name, t in (("sino_lo", lo), ("sino_hi", hi)):
            _dev_f32(t, (t.shape[-1],), name)
            if t.numel() != n:
                raise ValueError(f"{name} has {t.numel()} elements, the batch needs {n}")

    def init(self, lo, hi):
        self._check_sinos(lo, hi)
        _check(lib().dect_uneven_init(self._h, _ptr(lo), _ptr(hi)), "dect_uneven_init")
        return self

    def iterate(self, n: int = 1):
        _check(lib().dect_uneven_iterate(self._h, int(n)), "dect_uneven_iterate")
        return self

    def finish(self):
        """(Z, rho_e): back-to-back images (see split_images)."""
        torch = _torch()
        n = image_elements(self.geoms)
        Z = torch.empty(n, device=self.device, dtype=torch.float32)
        R = torch.empty_like(Z)
        _check(lib().dect_uneven_finish(self._h, _ptr(Z), _ptr(R)), "dect_uneven_finish")
        return Z, R

    def autotune(self, lo, hi, iters: int = 4, reps: int = 3):
        self._check_sinos(lo, hi)
        _check(lib().dect_uneven_autotune(self._h, _ptr(lo), _ptr(hi), int(iters), int(reps)),
               "dect_uneven_autotune")
        return [self.schedule(q) for q in range(self.groups())]

    def schedule(self, group: int):
        sc = _Schedule()
        _check(lib().dect_uneven_get_schedule(self._h, int(group), C.byref(sc)), "dect_uneven_get_schedule")
        return {k: getattr(sc, k) for k in SCHEDULE_KEYS}


def solve_uneven(sino_lo, sino_hi, geoms, params=None, stream=None):
    """Whole solve of a batch of mixed image sizes -> (Z, rho_e) back to back."""
    torch = _torch()
    gs, arr = _geometry_array(geoms)
    p = params if params is not None else default_params()
    n = sinogram_elements(gs)
    for name, t in (("sino_lo", sino_lo), ("sino_hi", sino_hi)):
        _dev_f32(t, (t.shape[-1],), name)
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} elements, the batch needs {n}")
    m = image_elements(gs)
    Z = torch.empty(m, device=sino_lo.device, dtype=torch.float32)
    R = torch.empty_like(Z)
    _check(lib().dect_solve_uneven(_ptr(sino_lo), _ptr(sino_hi), arr, C.byref(p), _ptr(Z), _ptr(R),
                                   len(gs), C.c_void_p(_stream(stream))), "dect_solve_uneven")
    return Z, R


class Engine:
    """Continuous batching: a pool of slots on one image grid, each holding one
    request at its own outer iteration (see include/dect.h)."""

    def __init__(self, n_x, n_y, pixel_mm, slots, max_views, max_det, params=None, device="cuda",
                 stream=None):
        self.params = params if params is not None else default_params()
        self.n_x, self.n_y, self.slots = int(n_x), int(n_y), int(slots)
        self.device = device
        h = C.c_void_p()
        _check(lib().dect_engine_create(self.n_x, self.n_y, float(pixel_mm), self.slots, int(max_views),
                                        int(max_det), C.byref(self.params), None, 0,
                                        C.c_void_p(_stream(stream)), C.byref(h)), "dect_engine_create")
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().dect_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, geom, sino_lo, sino_hi, n_iter, Z=None, rho=None):
        """Slot of the admitted request, or None when every slot is busy.
        Z / rho: [n_y, n_x] float32 device outputs (allocated when omitted)."""
        torch = _torch()
        g = Geometry.of(geom)
        _dev_f32(sino_lo, (g.n_views, g.n_det), "sino_lo")
        _dev_f32(sino_hi, (g.n_views, g.n_det), "sino_hi")
        if Z is None:
            Z = torch.empty((self.n_y, self.n_x), device=self.device, dtype=torch.float32)
        if rho is None:
            rho = torch.empty((self.n_y, self.n_x), device=self.device, dtype=torch.float32)
        slot = C.c_int32(-1)
        gc = g.c()
        rc = lib().dect_engine_admit(self._h, C.byref(gc), _ptr(sino_lo), _ptr(sino_hi), int(n_iter),
                                     _ptr(Z), _ptr(rho), C.byref(slot))
        if rc == DECT_EBUSY:
            return None
        _check(rc, "dect_engine_admit")
        self._keep[slot.value] = (sino_lo, sino_hi, Z, rho)
        return slot.value

    def step(self, n: int = 1) -> int:
        """Up to n outer iterations of every occupied slot (pipelined), no more
        than the first slot to complete needs; returns the number run."""
        done = C.c_int32()
        _check(lib().dect_engine_step_n(self._h, int(n), C.byref(done)), "dect_engine_step_n")
        return int(done.value)

    def cancel(self, slot: int):
        """Free an occupied slot between steps; its outputs are never written."""
        _check(lib().dect_engine_cancel(self._h, int(slot)), "dect_engine_cancel")
        self._keep.pop(int(slot), None)

    def status(self):
        a, f = C.c_int32(), C.c_int32()
        _check(lib().dect_engine_status(self._h, C.byref(a), C.byref(f)), "dect_engine_status")
        return a.value, f.value

    def completed(self):
        """[(slot, Z, rho)] of requests completed since the last call (their maps
        are enqueued on the stream)."""
        buf = (C.c_int32 * max(self.slots, 1))()
        n = C.c_int32()
        _check(lib().dect_engine_completed(self._h, buf, self.slots, C.byref(n)), "dect_engine_completed")
        out = []
        for i in range(n.value):
            lo, hi, Z, rho = self._keep.pop(buf[i])
            out.append((buf[i], Z, rho))
        return out
