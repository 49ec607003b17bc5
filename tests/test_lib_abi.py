"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-only paths (defaults, geometry validation,
attenuation model, argument checks) behave.  No GPU compute is issued."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2308_01290_amd import dect
from paper_2308_01290_amd import phantoms as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dect.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dect_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("dect_project", "dect_backproject", "dect_l0_step", "dect_solve", "dect_last_error"):
        assert must in names
    assert sorted(names) == sorted(dect.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = dect.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_default_params():
    p = dect.default_params()
    assert (p.E_lo_keV, p.E_hi_keV, p.E1_keV, p.E2_keV) == (60.0, 90.0, 50.0, 200.0)
    assert (p.m, p.n, p.Cp, p.Z_w) == (3.94, 3.2, 9.8e-24, 7.42)
    assert tuple(p.basis_Z) == (14.14, 7.42) and tuple(p.basis_rho) == (1.69, 1.0)
    assert p.lambda_ == 0.01 and p.beta_max == 1e5 and p.f_inner == 1
    assert p.t_tol == 1e-7 and p.t_maxit == 200 and p.rho_min == 0.1
    assert p.t_precond == 0   # DECT_PRECOND_AUTO
    assert p.storage == dect.DECT_STORAGE_FP32


def test_geometry_resolution_matches_corner_pitch():
    for g in (P.geometry_small(), P.geometry_slice512()):
        r = dect.resolve_geometry(P.FanGeometry(**{**g.__dict__, "det_pitch_mm": 0.0}))
        R = 0.5 * g.pixel_mm * math.hypot(g.n_x, g.n_y)
        want = 2 * g.sdd_mm * math.tan(math.asin(R / g.sid_mm)) / g.n_det
        assert abs(r.det_pitch_mm - want) < 1e-12


@pytest.mark.parametrize("bad", [
    dict(sdd_mm=900.0),              # detector inside the source circle
    dict(n_x=0),
    dict(pixel_mm=-1.0),
    dict(n_x=4096, n_y=4096),        # image reaches the source
])
def test_invalid_geometry_rejected(bad):
    g = P.FanGeometry(**{**P.geometry_small().__dict__, **bad})
    with pytest.raises(dect.DectError):
        dect.resolve_geometry(g)


def test_attenuation_matches_oracle_model():
    from oracle.physics import Physics
    p = dect.default_params()
    rng = np.random.default_rng(0)
    Z = rng.uniform(5.5, 20.0, 64)
    R = rng.uniform(0.2, 1.9, 64)
    lo, hi = dect.attenuation(p, Z, R)
    olo, ohi = Physics().mu_pair(Z, R)
    assert np.allclose(lo, olo, rtol=1e-13, atol=0)
    assert np.allclose(hi, ohi, rtol=1e-13, atol=0)


def test_entry_points_reject_bad_arguments_before_enqueueing():
    L = dect.lib()
    g = dect.Geometry.of(P.geometry_small()).c()
    # NULL arrays: validated on the host, nothing reaches the device
    assert L.dect_project(C.byref(g), None, None, 1, None) == -1
    assert L.dect_backproject(C.byref(g), None, None, 1, None) == -1
    assert b"NULL" in L.dect_last_error()
    assert L.dect_project(C.byref(g), None, None, -1, None) == -1
    p = dect.default_params(f_inner=2)
    h = C.c_void_p()
    assert L.dect_solver_create(C.byref(g), C.byref(p), 1, None, 0, None, C.byref(h)) == -5
    p = dect.default_params(n_iter=0)
    assert L.dect_solver_create(C.byref(g), C.byref(p), 1, None, 0, None, C.byref(h)) == -1
    bad = dect.Geometry.of(P.FanGeometry(**{**P.geometry_small().__dict__, "n_x": 100})).c()
    p = dect.default_params()
    assert L.dect_solver_create(C.byref(bad), C.byref(p), 1, None, 0, None, C.byref(h)) == -1
    assert b"2^a*3^b" in L.dect_last_error()
    # preconditioner selector: out of range; multigrid on sizes it cannot coarsen
    p = dect.default_params(t_precond=7)
    assert L.dect_solver_create(C.byref(g), C.byref(p), 1, None, 0, None, C.byref(h)) == -1
    odd = dect.Geometry.of(P.FanGeometry(**{**P.geometry_small().__dict__, "n_x": 96, "n_y": 24})).c()
    p = dect.default_params(t_precond=3)
    assert L.dect_solver_create(C.byref(odd), C.byref(p), 1, None, 0, None, C.byref(h)) == -5
    assert b"multigrid" in L.dect_last_error()
    # uneven batch: the image grid must agree across slices
    ga = dect.Geometry.of(P.geometry_small())
    gb = dect.Geometry.of(P.FanGeometry(**{**P.geometry_small().__dict__, "n_x": 96}))
    arr = (dect._Geometry * 2)(ga.c(), gb.c())
    p = dect.default_params()
    assert L.dect_solver_create_multi(arr, C.byref(p), 2, None, 0, None, C.byref(h)) == -1
    assert b"differs from slice 0" in L.dect_last_error()
    assert L.dect_solve_workspace_bytes_multi(arr, C.byref(p), 2) == 0
    # engine: kappa follows each request's budget; sizes checked on the host
    eh = C.c_void_p()
    p = dect.default_params(kappa=1.5)
    assert L.dect_engine_create(128, 128, 1.0, 4, 180, 256, C.byref(p), None, 0, None, C.byref(eh)) == -1
    p = dect.default_params()
    assert L.dect_engine_create(128, 128, 1.0, 0, 180, 256, C.byref(p), None, 0, None, C.byref(eh)) == -1
    assert L.dect_engine_workspace_bytes(128, 128, 1.0, 4, 180, 256, C.byref(p)) > \
        L.dect_engine_workspace_bytes(128, 128, 1.0, 2, 180, 256, C.byref(p)) > 0
    # storage selector: out of range; BF16 needs the projector (sinogram form)
    p = dect.default_params(storage=3)
    assert L.dect_solver_create(C.byref(g), C.byref(p), 1, None, 0, None, C.byref(h)) == -1
    assert b"storage" in L.dect_last_error()
    p = dect.default_params(storage=dect.DECT_STORAGE_BF16)
    assert L.dect_image_solver_create(128, 128, C.byref(p), 1, None, 0, None, C.byref(h)) == -5
    # image-domain form: sizes, params and NULL arrays are checked on the host
    p = dect.default_params()
    assert L.dect_image_solver_create(100, 128, C.byref(p), 1, None, 0, None, C.byref(h)) == -1
    assert b"2^a*3^b" in L.dect_last_error()
    assert L.dect_image_solver_create(128, 128, C.byref(p), 0, None, 0, None, C.byref(h)) == -1
    p = dect.default_params(t_precond=3)
    assert L.dect_image_solver_create(96, 24, C.byref(p), 1, None, 0, None, C.byref(h)) == -5
    p = dect.default_params()
    assert L.dect_solve_image(None, None, 128, 128, C.byref(p), None, None, 1, None, 0, None) == -1
    assert L.dect_image_solver_init(None, None, None) == -1
    assert L.dect_image_workspace_bytes(100, 128, C.byref(p), 1) == 0
    # l0 step: unsupported FFT size, NULL input
    assert L.dect_l0_step(None, None, None, None, None, 16, 16, 1, 0.1, 1.0, 1e-6, 10, None, 0, None) == -1
    assert L.dect_l0_step(C.c_void_p(1), None, C.c_void_p(1), None, None, 10, 16, 1, 0.1, 1.0, 1e-6,
                          10, None, 0, None) == -1


def test_bf16_storage_workspace():
    """BF16 storage adds the direction's BF16 pair blocks: about 4 bytes per
    padded entry, a small fraction of the FP32 workspace."""
    L = dect.lib()
    g = dect.Geometry.of(P.geometry_slice512()).c()
    a = L.dect_solve_workspace_bytes(C.byref(g), C.byref(dect.default_params()), 2)
    b = L.dect_solve_workspace_bytes(C.byref(g), C.byref(dect.default_params(storage=1)), 2)
    # four padded layouts per image: rows, columns and both reversed (the
    # 720-view 512^2 slice is quarter-turn symmetric)
    pad = 4 * 512 * (512 + 4)
    assert 2 * pad * 4 <= b - a <= 2 * pad * 4 + 512


def test_image_workspace_sizes():
    L = dect.lib()
    p = dect.default_params()
    one = L.dect_image_workspace_bytes(512, 512, C.byref(p), 1)
    two = L.dect_image_workspace_bytes(512, 512, C.byref(p), 2)
    # f, f^(k+1), FFT scratch (2 floats each), rho, t', mu_L, mu_H, PCG vectors
    assert 512 * 512 * 4 * 10 < one < two <= 2 * one + 4096 * 64


def test_workspace_sizes_are_consistent():
    L = dect.lib()
    g = dect.Geometry.of(P.geometry_slice512()).c()
    p = dect.default_params()
    one = L.dect_solve_workspace_bytes(C.byref(g), C.byref(p), 1)
    four = L.dect_solve_workspace_bytes(C.byref(g), C.byref(p), 4)
    assert 0 < one < four <= 4 * one + 4096 * 64
    # 512^2 slice, 720 x 736 sinogram: a few tens of MB per slice
    assert 20e6 < one < 120e6
    assert L.dect_l0_step_workspace_bytes(512, 512, 1, 0) >= 512 * 512 * 8
    # uneven batch of one geometry repeated == the plain batch
    arr = (dect._Geometry * 4)(*([g] * 4))
    assert L.dect_solve_workspace_bytes_multi(arr, C.byref(p), 4) == four
    # a second geometry with more views and bins needs more
    g2 = dect.Geometry.of(P.FanGeometry(**{**P.geometry_slice512().__dict__, "n_views": 984,
                                           "n_det": 888, "det_pitch_mm": 0.0})).c()
    arr = (dect._Geometry * 2)(g, g2)
    assert L.dect_solve_workspace_bytes_multi(arr, C.byref(p), 2) > L.dect_solve_workspace_bytes(
        C.byref(g), C.byref(p), 2)
    assert L.dect_l0_step_workspace_bytes(512, 512, 1, 1) > L.dect_l0_step_workspace_bytes(512, 512, 1, 0)
