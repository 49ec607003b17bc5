"""ctypes front end of the FP64 C oracle (dect_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dect_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("dx", C.c_double),
                ("nv", C.c_int), ("angle0", C.c_double), ("arc", C.c_double),
                ("nd", C.c_int), ("pitch", C.c_double), ("offset", C.c_double),
                ("sid", C.c_double), ("sdd", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp = P(C.c_double)
        L.ora_project.argtypes = [P(_Geom), dp, dp, C.c_int, C.c_int]
        L.ora_backproject.argtypes = [P(_Geom), dp, dp, C.c_int, C.c_int]
        L.ora_fbp.argtypes = [P(_Geom), dp, dp, C.c_int, C.c_int]
        L.ora_ray_chords.argtypes = [P(_Geom), C.c_int, C.c_int, P(C.c_int), dp]
        L.ora_ray_chords.restype = C.c_int
        L.ora_clip_chord.argtypes = [P(_Geom), C.c_int, C.c_int, C.c_int, C.c_int]
        L.ora_clip_chord.restype = C.c_double
        _lib = L
    return _lib


@dataclass
class Geometry:
    """Fan-beam geometry (mm, rad); pitch 0 selects the corner-covering pitch."""
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
    arc_rad: float = 2.0 * np.pi

    @staticmethod
    def of(obj) -> "Geometry":
        names = Geometry.__dataclass_fields__.keys()
        return Geometry(**{k: getattr(obj, k) for k in names})

    def pitch(self) -> float:
        if self.det_pitch_mm > 0:
            return float(self.det_pitch_mm)
        r = 0.5 * self.pixel_mm * np.hypot(self.n_x, self.n_y)
        return float(2.0 * self.sdd_mm * np.tan(np.arcsin(r / self.sid_mm)) / self.n_det)

    def c(self) -> _Geom:
        return _Geom(self.n_x, self.n_y, self.pixel_mm, self.n_views, self.angle0_rad,
                     self.arc_rad, self.n_det, self.pitch(), self.det_offset_mm,
                     self.sid_mm, self.sdd_mm)


def _threads(nthreads):
    return int(nthreads) if nthreads else 0


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def project(geom, img, nthreads=None) -> np.ndarray:
    """A applied to img [.., n_y, n_x] -> sinogram [.., n_views, n_det] (FP64)."""
    g = Geometry.of(geom)
    a = np.ascontiguousarray(img, dtype=np.float64)
    lead = a.shape[:-2]
    b = int(np.prod(lead)) if lead else 1
    out = np.empty(lead + (g.n_views, g.n_det))
    gc = g.c()
    lib().ora_project(C.byref(gc), _dptr(a), _dptr(out), b, _threads(nthreads))
    return out


def backproject(geom, sino, nthreads=None) -> np.ndarray:
    """A^T applied to sino [.., n_views, n_det] -> image [.., n_y, n_x] (FP64)."""
    g = Geometry.of(geom)
    a = np.ascontiguousarray(sino, dtype=np.float64)
    lead = a.shape[:-2]
    b = int(np.prod(lead)) if lead else 1
    out = np.empty(lead + (g.n_y, g.n_x))
    gc = g.c()
    lib().ora_backproject(C.byref(gc), _dptr(a), _dptr(out), b, _threads(nthreads))
    return out


def fbp(geom, sino, nthreads=None) -> np.ndarray:
    """Flat-detector fan-beam FBP (Ram-Lak, linear interpolation) -> mu image."""
    g = Geometry.of(geom)
    a = np.ascontiguousarray(sino, dtype=np.float64)
    lead = a.shape[:-2]
    b = int(np.prod(lead)) if lead else 1
    out = np.empty(lead + (g.n_y, g.n_x))
    gc = g.c()
    lib().ora_fbp(C.byref(gc), _dptr(a), _dptr(out), b, _threads(nthreads))
    return out


def ray_chords(geom, v: int, j: int):
    """Nonzeros of row (v, j) of A: (pixel index i*n_x + k, chord mm)."""
    g = Geometry.of(geom)
    cap = g.n_x + g.n_y + 4
    pix = (C.c_int * cap)()
    ln = (C.c_double * cap)()
    gc = g.c()
    n = lib().ora_ray_chords(C.byref(gc), v, j, pix, ln)
    return np.array(pix[:n], dtype=np.int64), np.array(ln[:n])


def clip_chord(geom, v: int, j: int, i: int, k: int) -> float:
    """Brute-force chord of ray (v, j) through pixel (row i, column k)."""
    g = Geometry.of(geom)
    gc = g.c()
    return float(lib().ora_clip_chord(C.byref(gc), v, j, i, k))
