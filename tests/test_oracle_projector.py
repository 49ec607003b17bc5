"""Pins of the oracle's fan-beam operators: Siddon projector A, scatter adjoint
A^T, FBP, and the input generator's ellipse chords.  CPU only."""
import math

import numpy as np
import pytest

from oracle import operators as ops
from paper_2308_01290_amd import phantoms as P


def tiny(nx=4, ny=4, nv=12, nd=7, offset=0.0, sid=10.0, sdd=15.0, dx=1.0, angle0=0.0):
    return P.FanGeometry(n_x=nx, n_y=ny, pixel_mm=dx, n_views=nv, n_det=nd, sid_mm=sid,
                         sdd_mm=sdd, det_offset_mm=offset, angle0_rad=angle0).resolved()


@pytest.mark.parametrize("geom", [tiny(), tiny(nd=8, offset=0.3), tiny(nx=4, ny=3, nv=9, nd=5),
                                  tiny(nx=5, ny=4, nv=16, nd=9, angle0=0.1)])
def test_siddon_equals_bruteforce_clipping(geom):
    """Every entry of A on a small image equals an independent Liang-Barsky clip."""
    g = geom
    worst = 0.0
    for v in range(g.n_views):
        for j in range(g.n_det):
            pix, ln = ops.ray_chords(g, v, j)
            dense = np.zeros(g.n_x * g.n_y)
            np.add.at(dense, pix, ln)
            bf = np.array([ops.clip_chord(g, v, j, i, k) for i in range(g.n_y) for k in range(g.n_x)])
            worst = max(worst, float(np.abs(dense - bf).max()))
    assert worst < 1e-12


def test_rays_along_grid_lines_follow_half_open_rule():
    """An odd detector puts the central ray of the views at 0, 90, 180 and 270
    degrees exactly on the line through the centre (y = 0 or x = 0), the
    boundary between rows (columns) n/2-1 and n/2.  A pixel is the half-open
    square [x, x + dx) x [y, y + dx), so the whole chord belongs to row n_y/2
    (views 0 and 2) or column n_x/2 (views 1 and 3), one pixel length in each
    of the four pixels along it."""
    g = tiny(nx=4, ny=4, nv=4, nd=5)
    for v in range(4):
        pix, ln = ops.ray_chords(g, v, 2)
        rows = sorted(set((pix // g.n_x).tolist()))
        cols = sorted(set((pix % g.n_x).tolist()))
        if v % 2 == 0:
            assert rows == [2] and cols == [0, 1, 2, 3], v
        else:
            assert cols == [2] and rows == [0, 1, 2, 3], v
        assert np.allclose(ln, 1.0, atol=1e-12), v
    # a half-bin detector offset with an even count does the same
    g2 = tiny(nx=4, ny=4, nv=4, nd=6)
    g2 = tiny(nx=4, ny=4, nv=4, nd=6, offset=-0.5 * g2.det_pitch_mm)
    for v in range(4):
        pix, ln = ops.ray_chords(g2, v, 3)
        sel = (pix // g2.n_x) if v % 2 == 0 else (pix % g2.n_x)
        assert set(sel.tolist()) == {2} and np.allclose(ln, 1.0, atol=1e-12), v
    assert ops.clip_chord(g, 0, 2, 1, 0) == 0.0
    assert abs(ops.clip_chord(g, 0, 2, 2, 0) - 1.0) < 1e-12


def test_adjointness_fp64():
    g = P.geometry_small()
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, g.n_y, g.n_x))
    y = rng.standard_normal((2, g.n_views, g.n_det))
    Ax = ops.project(g, x)
    Aty = ops.backproject(g, y)
    lhs = float(np.sum(Ax * y))
    rhs = float(np.sum(x * Aty))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_uniform_image_ray_sum_is_chord_of_box():
    """Uniform image: each ray sum is mu times the length of the ray inside the
    image box (closed-form slab clipping of the whole box)."""
    g = tiny(nx=6, ny=4, nv=10, nd=9, offset=0.17)
    mu = 0.37
    img = np.full((g.n_y, g.n_x), mu)
    s = ops.project(g, img)
    src, dst = P.ray_endpoints(g)
    for v in range(g.n_views):
        for j in range(g.n_det):
            S, Q = src[v], dst[v, j]
            d = Q - S
            t0, t1 = -np.inf, np.inf
            for a, half in ((0, g.n_x * g.pixel_mm / 2), (1, g.n_y * g.pixel_mm / 2)):
                ta, tb = (-half - S[a]) / d[a], (half - S[a]) / d[a]
                t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
            L = max(0.0, t1 - t0) * np.linalg.norm(d)
            assert abs(s[v, j] - mu * L) < 1e-12


def test_ellipse_chord_closed_form_vs_dense_sampling():
    e = P.Ellipse(3.0, -2.0, 7.0, 4.0, 0.6, 10.0, 1.0)
    src = np.array([[100.0, 5.0], [-80.0, 60.0], [10.0, -90.0]])
    dst = np.array([[-100.0, -7.0], [90.0, -50.0], [-6.0, 95.0]])
    ch = P.ellipse_chords(e, src, dst)
    for q in range(3):
        t = np.linspace(0.0, 1.0, 2_000_001)
        pts = src[q][None, :] + t[:, None] * (dst[q] - src[q])[None, :]
        inside = P._inside(e, pts[:, 0], pts[:, 1])
        L = inside.mean() * np.linalg.norm(dst[q] - src[q])
        assert abs(L - ch[q]) < 2e-4 * np.linalg.norm(dst[q] - src[q]) / 1000 + 1e-3


def test_siddon_of_rasterised_ellipse_converges_to_analytic():
    """Siddon of a supersampled rasterised ellipse approaches the analytic
    line integral as the pixel shrinks (first order in the pixel size)."""
    e = P.Ellipse(4.0, -3.0, 20.0, 11.0, 0.4, 7.42, 1.0)
    ph = P.Phantom(e, [])
    errs = []
    for n, dx in ((32, 2.0), (64, 1.0), (128, 0.5)):
        g = P.FanGeometry(n_x=n, n_y=n, pixel_mm=dx, n_views=24, n_det=96, sid_mm=500.0,
                          sdd_mm=800.0).resolved()
        lab = P.label_map(ph, g, supersample=8)
        img = lab[1]
        s = ops.project(g, img)
        src, dst = P.ray_endpoints(g)
        ref = P.ellipse_chords(e, np.broadcast_to(src[:, None, :], dst.shape), dst)
        errs.append(float(np.abs(s - ref).mean()))
    assert errs[1] < 0.7 * errs[0] and errs[2] < 0.7 * errs[1]
    assert errs[2] < 0.05


def test_centred_disk_projection_is_view_independent():
    g = P.geometry_small()
    ph = P.phantom_water_disk(40.0)
    pL, _ = P.analytic_sinograms(ph, g, lambda Z, R: (np.full(np.shape(Z), 0.02), np.full(np.shape(Z), 0.017)))
    assert np.abs(pL - pL[0][None, :]).max() < 1e-11 * pL.max()
    # symmetric bins about the centre (zero offset)
    assert np.abs(pL - pL[:, ::-1]).max() < 1e-11 * pL.max()


def test_fbp_uniform_disk_interior_mean():
    g = P.geometry_small()
    mu = 0.0196
    ph = P.phantom_water_disk(50.0)
    pL, _ = P.analytic_sinograms(ph, g, lambda Z, R: (np.full(np.shape(Z), mu), np.full(np.shape(Z), mu)))
    rec = ops.fbp(g, pL)
    X, Y = P.pixel_centres(g)
    roi = np.hypot(X, Y) < 35.0
    assert abs(rec[roi].mean() / mu - 1.0) < 1e-2
    assert rec[roi].std() / mu < 2e-2
    out = np.hypot(X, Y) > 60.0
    assert np.abs(rec[out]).mean() < 0.05 * mu


def test_fbp_is_linear():
    g = tiny(nx=16, ny=16, nv=24, nd=20, sid=40.0, sdd=60.0)
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((2, g.n_views, g.n_det))
    assert np.allclose(ops.fbp(g, 2.0 * a - 3.0 * b), 2.0 * ops.fbp(g, a) - 3.0 * ops.fbp(g, b),
                       atol=1e-12)
