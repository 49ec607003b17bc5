"""Pins of the oracle's gradient-L0 pieces (Section II-C, eq. (5)-(9)). CPU only."""
import numpy as np
import pytest

from oracle import l0


def explicit_D(ny, nx):
    """Forward-difference matrices built entry by entry from the definition
    (periodic): (Dx g)(i,j) = g(i,j+1) - g(i,j), (Dy g)(i,j) = g(i+1,j) - g(i,j)."""
    n = ny * nx
    Dx = np.zeros((n, n))
    Dy = np.zeros((n, n))
    for i in range(ny):
        for j in range(nx):
            r = i * nx + j
            Dx[r, r] -= 1.0
            Dx[r, i * nx + (j + 1) % nx] += 1.0
            Dy[r, r] -= 1.0
            Dy[r, ((i + 1) % ny) * nx + j] += 1.0
    return Dx, Dy


@pytest.mark.parametrize("shape", [(8, 8), (6, 10), (5, 7)])
def test_difference_operators_match_explicit_matrices(shape):
    ny, nx = shape
    Dx, Dy = explicit_D(ny, nx)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(shape)
    h, v = rng.standard_normal((2,) + shape)
    assert np.allclose(l0.dx(g).ravel(), Dx @ g.ravel(), atol=1e-14)
    assert np.allclose(l0.dy(g).ravel(), Dy @ g.ravel(), atol=1e-14)
    assert np.allclose(l0.dT(h, v).ravel(), Dx.T @ h.ravel() + Dy.T @ v.ravel(), atol=1e-14)


def test_hard_threshold_rule_and_tie():
    lam, beta = 0.25, 1.0      # threshold 0.25 is exact in binary
    gx = np.array([0.3, 0.5, 0.0, 0.4, -0.6])
    gy = np.array([0.4, 0.0, 0.5, 0.3, 0.0])
    # squared norms: 0.25 (tie), 0.25 (tie), 0.25 (tie), 0.25 (tie), 0.36 (> thr)
    h, v = l0.hard_threshold(gx, gy, lam, beta)
    assert np.all(h[:4] == 0) and np.all(v[:4] == 0)
    assert h[4] == -0.6 and v[4] == 0.0
    h, v = l0.hard_threshold(np.array([0.51]), np.array([0.0]), lam, beta)
    assert h[0] == 0.51


def test_hard_threshold_minimises_pixel_energy():
    """eq. (9) is the exact minimiser of E(r) = (h-gx)^2 + (v-gy)^2 + (lambda/beta) H(|h|+|v|):
    compare against brute-force over the two candidate minimisers."""
    rng = np.random.default_rng(7)
    gx, gy = rng.standard_normal((2, 1000)) * 0.5
    lam, beta = 0.1, 0.7
    h, v = l0.hard_threshold(gx, gy, lam, beta)
    e_zero = gx ** 2 + gy ** 2
    e_keep = np.full_like(gx, lam / beta)
    e_got = (h - gx) ** 2 + (v - gy) ** 2 + (lam / beta) * ((np.abs(h) + np.abs(v)) > 0)
    assert np.all(e_got <= np.minimum(e_zero, e_keep) + 1e-15)


def test_hard_threshold_lambda_zero_and_idempotent():
    rng = np.random.default_rng(2)
    gx, gy = rng.standard_normal((2, 50))
    gx[:5] = 0.0
    gy[:5] = 0.0
    h, v = l0.hard_threshold(gx, gy, 0.0, 1.0)
    assert np.array_equal(h, gx) and np.array_equal(v, gy)
    h1, v1 = l0.hard_threshold(gx, gy, 0.3, 1.0)
    h2, v2 = l0.hard_threshold(h1, v1, 0.3, 1.0)
    assert np.array_equal(h1, h2) and np.array_equal(v1, v2)


@pytest.mark.parametrize("shape,beta", [((8, 8), 0.7), ((6, 10), 3.0), ((9, 5), 1e3)])
def test_fft_closed_form_equals_dense_solve(shape, beta):
    """Section II-C closed form == dense solve of (I + beta D^T D) g = g~ + beta D^T (h, v)."""
    ny, nx = shape
    Dx, Dy = explicit_D(ny, nx)
    rng = np.random.default_rng(4)
    gt = rng.standard_normal(shape)
    h, v = rng.standard_normal((2,) + shape)
    A = np.eye(ny * nx) + beta * (Dx.T @ Dx + Dy.T @ Dy)
    b = gt.ravel() + beta * (Dx.T @ h.ravel() + Dy.T @ v.ravel())
    ref = np.linalg.solve(A, b).reshape(shape)
    assert np.allclose(l0.fft_solve(gt, h, v, beta), ref, rtol=0, atol=1e-11 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("beta", [0.02, 1.0, 1e4])
def test_weighted_solve_equals_dense_solve(beta):
    ny, nx = 8, 7
    Dx, Dy = explicit_D(ny, nx)
    rng = np.random.default_rng(9)
    w = rng.uniform(0.0, 2.0, (ny, nx))
    w[0, :3] = 0.0                       # air-like pixels with zero data weight
    gt = rng.standard_normal((ny, nx))
    h, v = rng.standard_normal((2, ny, nx))
    A = np.diag(w.ravel() ** 2) + beta * (Dx.T @ Dx + Dy.T @ Dy)
    b = (w * gt).ravel() + beta * (Dx.T @ h.ravel() + Dy.T @ v.ravel())
    ref = np.linalg.solve(A, b).reshape(ny, nx)
    got, it, res = l0.weighted_solve(w, gt, h, v, beta, rtol=1e-13)
    assert res <= 1e-13
    assert np.allclose(got, ref, atol=1e-9 * max(1.0, np.abs(ref).max()))


def test_weighted_solve_unit_weight_equals_fft():
    rng = np.random.default_rng(12)
    gt, h, v = rng.standard_normal((3, 16, 16))
    a = l0.fft_solve(gt, h, v, 2.5)
    b, _, _ = l0.weighted_solve(np.ones((16, 16)), gt, h, v, 2.5, rtol=1e-13)
    assert np.allclose(a, b, atol=1e-10)


def test_l0_step_smooths_noise_and_keeps_edges():
    """Qualitative property of model (5): a noisy step edge is flattened on
    both sides while the jump survives (gradient sparsity)."""
    rng = np.random.default_rng(0)
    clean = np.zeros((32, 32))
    clean[:, 16:] = 1.0
    noisy = clean + 0.02 * rng.standard_normal(clean.shape)
    g = noisy.copy()
    beta = 0.02
    while beta < 1e5:
        g, _, _ = l0.l0_step(noisy, g, 0.02, beta)
        beta *= 2.0
    assert np.abs(g - clean)[:, 2:14].std() < 0.5 * 0.02
    assert g[:, 20].mean() - g[:, 10].mean() > 0.9
