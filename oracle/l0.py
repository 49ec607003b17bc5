"""FP64 gradient-L0 pieces by half-quadratic splitting (Section II-C).

TEST INFRASTRUCTURE ONLY (oracle).

  * forward differences d_x g, d_y g with periodic boundaries: the paper's FFT
    closed form diagonalises them, which fixes the boundary as periodic
    (the paper states no stencil; reading: d_x g(i,j) = g(i,j+1) - g(i,j),
    d_y g(i,j) = g(i+1,j) - g(i,j), indices mod N);
  * hard threshold, eq. (9): (h, v) = (0, 0) where (d_x g)^2 + (d_y g)^2 <= lambda/beta,
    else (d_x g, d_y g).  Equality maps to zero, as printed.  The comparison
    is the real-valued one of eq. (9), evaluated in FP64 like every other
    step here;
  * the g-subproblem closed form of Section II-C (FFT), with F(1) read as 1;
  * the weighted quadratic of subproblem (13c) as an SPD linear solve.
"""
from __future__ import annotations

import numpy as np


def dx(g):
    return np.roll(g, -1, axis=-1) - g


def dy(g):
    return np.roll(g, -1, axis=-2) - g


def dT(h, v):
    """Adjoint of (d_x, d_y): D^T(h, v)(i,j) = h(i,j-1) - h(i,j) + v(i-1,j) - v(i,j)."""
    return (np.roll(h, 1, axis=-1) - h) + (np.roll(v, 1, axis=-2) - v)


def ht_keep(gx, gy, lam, beta):
    """Boolean map of pixels that keep their gradient under eq. (9):
    (d_x g)^2 + (d_y g)^2 > lambda / beta."""
    x = np.asarray(gx, dtype=np.float64)
    y = np.asarray(gy, dtype=np.float64)
    return x * x + y * y > lam / beta


def hard_threshold(gx, gy, lam, beta):
    """eq. (9): auxiliary (h, v) for given gradients."""
    keep = ht_keep(gx, gy, lam, beta)
    return np.where(keep, gx, 0.0), np.where(keep, gy, 0.0)


def ht_of(g, lam, beta):
    return hard_threshold(dx(g), dy(g), lam, beta)


def _otf(shape, axis):
    """F of the forward-difference kernel along axis (-1: x, -2: y)."""
    k = np.zeros(shape[-2:])
    k[0, 0] = -1.0
    if axis == -1:
        k[0, -1] = 1.0
    else:
        k[-1, 0] = 1.0
    return np.fft.fft2(k)


def fft_solve(g_tilde, h, v, beta):
    """Section II-C closed form:
    g = F^-1[(F(g~) + beta (F*(dx) F(h) + F*(dy) F(v))) / (1 + beta (F*(dx)F(dx) + F*(dy)F(dy)))].
    """
    shp = np.shape(g_tilde)
    ox, oy = _otf(shp, -1), _otf(shp, -2)
    num = np.fft.fft2(g_tilde) + beta * (np.conj(ox) * np.fft.fft2(h) + np.conj(oy) * np.fft.fft2(v))
    den = 1.0 + beta * (np.abs(ox) ** 2 + np.abs(oy) ** 2)
    return np.real(np.fft.ifft2(num / den))


def weighted_apply(x, w2, beta):
    """(diag(w^2) + beta D^T D) x."""
    return w2 * x + beta * dT(dx(x), dy(x))


def weighted_solve(w, g_tilde, h, v, beta, x0=None, rtol=1e-12, maxit=20000):
    """Minimiser of ||w*g - g~||^2 + beta ||D g - (h, v)||^2, i.e. the SPD system
    (diag(w^2) + beta D^T D) g = w*g~ + beta D^T(h, v)  (subproblem (13c), in the
    normalised t' variable).  Conjugate gradients preconditioned with the FFT
    inverse of (c + beta D^T D), c = mean(w^2); stops at relative residual rtol.
    Returns (g, iterations, relative residual)."""
    w2 = w * w
    b = w * g_tilde + beta * dT(h, v)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    c = max(float(np.mean(w2)), 1e-12)
    shp = b.shape
    ox, oy = _otf(shp, -1), _otf(shp, -2)
    den = c + beta * (np.abs(ox) ** 2 + np.abs(oy) ** 2)

    def prec(r):
        return np.real(np.fft.ifft2(np.fft.fft2(r) / den))

    r = b - weighted_apply(x, w2, beta)
    bn = float(np.linalg.norm(b)) or 1.0
    z = prec(r)
    p = z.copy()
    rz = float(np.vdot(r, z))
    it = 0
    res = float(np.linalg.norm(r)) / bn
    while res > rtol and it < maxit:
        q = weighted_apply(p, w2, beta)
        a = rz / float(np.vdot(p, q))
        x += a * p
        r -= a * q
        it += 1
        res = float(np.linalg.norm(r)) / bn
        if res <= rtol:
            break
        z = prec(r)
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, res


def l0_step(g_tilde, g, lam, beta, weight=None, rtol=1e-12):
    """One HQS step of the gradient-L0 model (5): (h, v) = eq. (9) on g, then the
    g-subproblem (8a) — FFT closed form for unit weight, SPD solve otherwise."""
    h, v = ht_of(g, lam, beta)
    if weight is None:
        return fft_solve(g_tilde, h, v, beta), h, v
    x, _, _ = weighted_solve(weight, g_tilde, h, v, beta, x0=g, rtol=rtol)
    return x, h, v
