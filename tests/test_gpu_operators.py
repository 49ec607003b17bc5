"""GPU parity of the fan-beam operators against the FP64 oracle: forward
projection, matched back-projection, adjointness, FBP.  Inputs are identical
FP32 arrays on both sides (the oracle promotes them to FP64)."""
import numpy as np
import pytest

from oracle import operators as ops
from paper_2308_01290_amd import dect
from paper_2308_01290_amd import phantoms as P
from tests.gpu_util import cuda, host, ragged_geometry, rel_inf, workload

pytestmark = pytest.mark.gpu

# per-projection tolerance: sup-norm error relative to the sup-norm of the
# oracle's projection
PROJ_TOL = 1e-5


def geoms():
    return {
        "gridline_offset": gridline_offset(),
        "small": P.geometry_small(),
        "ragged": ragged_geometry(),
        # square grid, side a multiple of 32, views a multiple of 4: the
        # quarter-turn symmetric projector; the detector offset and the first
        # view away from 0 break the transpose symmetry (four-fold kernels)
        "quarter": P.FanGeometry(n_x=64, n_y=64, pixel_mm=1.0, n_views=64, n_det=96, sid_mm=500.0,
                                 sdd_mm=800.0, det_offset_mm=0.25, angle0_rad=0.1).resolved(),
        # transpose-symmetric (eight-fold back-projector): three tiles of 32
        # per side (an odd count, one work unit with a single diagonal orbit)
        # and nv/4 = 18 even (view 9 is its own transpose)
        "octo_odd": P.FanGeometry(n_x=96, n_y=96, pixel_mm=1.0, n_views=72, n_det=160, sid_mm=600.0,
                                  sdd_mm=900.0).resolved(),
        # one tile orbit, four views (nv/4 = 1: view 0 only)
        "octo_tiny": P.FanGeometry(n_x=32, n_y=32, pixel_mm=1.0, n_views=4, n_det=48, sid_mm=300.0,
                                   sdd_mm=450.0).resolved(),
        # rays exactly on a grid line: an odd bin count on a centred detector
        # puts the central ray of the views at 0, 90, 180, 270 degrees on the
        # line through the centre (the half-open rule decides its pixel); and a
        # half-bin detector offset with an even count does the same off the
        # transpose symmetry
        "gridline_odd": P.FanGeometry(n_x=64, n_y=64, pixel_mm=1.0, n_views=32, n_det=95, sid_mm=500.0,
                                      sdd_mm=800.0).resolved(),
    }


def gridline_offset():
    g = P.FanGeometry(n_x=64, n_y=64, pixel_mm=1.0, n_views=32, n_det=96, sid_mm=500.0,
                      sdd_mm=800.0).resolved()
    return P.FanGeometry(n_x=64, n_y=64, pixel_mm=1.0, n_views=32, n_det=96, sid_mm=500.0,
                         sdd_mm=800.0, det_pitch_mm=g.det_pitch_mm,
                         det_offset_mm=-0.5 * g.det_pitch_mm).resolved()


SYM = ["quarter", "octo_odd", "octo_tiny", "gridline_odd", "gridline_offset"]


@pytest.mark.parametrize("name", ["small", "ragged"] + SYM)
@pytest.mark.parametrize("batch", [1, 3])
def test_project_matches_oracle_random(name, batch):
    g = geoms()[name]
    rng = np.random.default_rng(100 + batch)
    img = rng.uniform(0.0, 1.0, (batch, g.n_y, g.n_x)).astype(np.float32)
    got = host(dect.project(g, cuda(img)))
    ref = ops.project(g, img.astype(np.float64))
    assert got.shape == ref.shape
    for b in range(batch):
        assert rel_inf(got[b], ref[b]) <= PROJ_TOL, (name, b)


def test_project_matches_oracle_per_ray_on_phantom():
    g, ph, _, _ = workload("small")
    from oracle.physics import Physics
    muL, _ = P.mu_maps(ph, g, Physics().mu_pair, supersample=2)
    img = muL.astype(np.float32)
    got = host(dect.project(g, cuda(img)))
    ref = ops.project(g, img.astype(np.float64))
    assert rel_inf(got, ref) <= PROJ_TOL
    big = ref >= 1e-3 * ref.max()
    assert np.max(np.abs(got - ref)[big] / ref[big]) <= PROJ_TOL


@pytest.mark.parametrize("name", ["small", "ragged"] + SYM)
@pytest.mark.parametrize("batch", [1, 2, 3])
def test_backproject_matches_oracle(name, batch):
    g = geoms()[name]
    rng = np.random.default_rng(7 + batch)
    s = rng.standard_normal((batch, g.n_views, g.n_det)).astype(np.float32)
    got = host(dect.backproject(g, cuda(s)))
    ref = ops.backproject(g, s.astype(np.float64))
    for b in range(batch):
        assert rel_inf(got[b], ref[b]) <= PROJ_TOL, (name, b)


@pytest.mark.parametrize("name", ["small", "ragged"] + SYM)
def test_adjointness_on_gpu(name):
    g = geoms()[name]
    rng = np.random.default_rng(21)
    x = rng.standard_normal((g.n_y, g.n_x)).astype(np.float32)
    y = rng.standard_normal((g.n_views, g.n_det)).astype(np.float32)
    Ax = host(dect.project(g, cuda(x)))
    Aty = host(dect.backproject(g, cuda(y)))
    lhs = float(np.sum(Ax * y.astype(np.float64)))
    rhs = float(np.sum(x.astype(np.float64) * Aty))
    assert abs(lhs - rhs) <= 1e-6 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_operators_are_deterministic():
    g = P.geometry_small()
    rng = np.random.default_rng(5)
    x = cuda(rng.uniform(0, 1, (2, g.n_y, g.n_x)))
    y = cuda(rng.standard_normal((2, g.n_views, g.n_det)))
    assert np.array_equal(host(dect.project(g, x)), host(dect.project(g, x)))
    assert np.array_equal(host(dect.backproject(g, y)), host(dect.backproject(g, y)))


def test_empty_batch_is_a_no_op():
    import torch
    g = P.geometry_small()
    img = torch.empty((0, g.n_y, g.n_x), device="cuda")
    out = dect.project(g, img)
    assert out.shape == (0, g.n_views, g.n_det)


@pytest.mark.parametrize("name", ["small", "ragged"])
def test_fbp_matches_oracle(name):
    g = geoms()[name]
    if name == "small":
        _, _, pL, pH = workload("small")
        s = np.stack([pL, pH])
    else:
        rng = np.random.default_rng(9)
        s = rng.uniform(0, 2, (2, g.n_views, g.n_det)).astype(np.float32)
    got = host(dect.fbp(g, cuda(s)))
    ref = ops.fbp(g, s.astype(np.float64))
    for b in range(2):
        assert rel_inf(got[b], ref[b]) <= PROJ_TOL, (name, b)


# ---- the 512^2 / 720-view / 736-bin slice, at full size ----------------------

def test_slice512_project_and_backproject():
    g, ph, pL, _ = workload("slice512")
    from oracle.physics import Physics
    muL, muH = P.mu_maps(ph, g, Physics().mu_pair)
    img = np.stack([muL, muH]).astype(np.float32)
    got = host(dect.project(g, cuda(img)))
    ref = ops.project(g, img.astype(np.float64))
    for b in range(2):
        assert rel_inf(got[b], ref[b]) <= PROJ_TOL
    got_bp = host(dect.backproject(g, cuda(pL[None])))
    ref_bp = ops.backproject(g, pL[None].astype(np.float64))
    assert rel_inf(got_bp, ref_bp) <= PROJ_TOL


def test_slice512_fbp():
    g, _, pL, _ = workload("slice512")
    got = host(dect.fbp(g, cuda(pL[None])))
    ref = ops.fbp(g, pL[None].astype(np.float64))
    assert rel_inf(got, ref) <= PROJ_TOL
