"""Hard-threshold decisions of eq. (9) that floating point may take either way,
and what one such decision can move.

Eq. (9) keeps the gradient of pixel p when (d_x g)^2 + (d_y g)^2 > lambda/beta.
The oracle evaluates it in FP64.  An FP32 evaluation from the same FP32
image rounds d_x g and d_y g once each (relative error <= u = 2^-24), the
squares and their sum once more each, and lambda/beta once: at most about
8u = 4.8e-7 relative in all.  A pixel whose FP64 sum lies within REL_TIE of
the threshold is a near-tie: there, and only there, the two evaluations may
disagree.  Everywhere else they must agree.

A decision that flips changes (h, v) at one pixel by that pixel's gradient
(|dh| + |dv| <= 2 sqrt(lambda/beta) at a near-tie).  The allowances below
bound what that moves in each step of one outer iteration, from the step's
own operator:
  * f-step (one steepest-descent step): the gradient changes by
    2 beta D^T(dh, dv) on the pixel and its two upper/left neighbours, so
    f moves by at most alpha * 2 beta (|dh| + |dv|) there (plus a relative
    change of alpha far below the FP32 tolerance);
  * rho_e step, FFT closed form: rho moves by beta (1 + beta L)^-1 D^T(dh, dv),
    bounded by |dh| sup|r_h| + |dv| sup|r_v| with r the response to a unit
    impulse in h (v);
  * t' step, weighted SPD solve: the same with (W^2 + beta L)^-1, whose
    response depends on the pixel (it is computed there).
Allowances add over the flips (the steps are linear in (h, v)).
"""
from __future__ import annotations

import numpy as np

from oracle import l0

REL_TIE = 1e-6


def grad_sq(g):
    g = np.asarray(g, np.float64)
    return l0.dx(g) ** 2 + l0.dy(g) ** 2


def near_ties(g, lam, beta, rel=REL_TIE):
    """Pixels whose eq. (9) decision is within `rel` of the threshold."""
    thr = lam / beta
    return np.abs(grad_sq(g) - thr) <= rel * thr


def decisions(h, v):
    return (np.asarray(h) != 0) | (np.asarray(v) != 0)


def flipped_gradients(g, mask):
    """|d_x g| + |d_y g| at the masked pixels (what a flip there moves in (h, v))."""
    g = np.asarray(g, np.float64)
    return (np.abs(l0.dx(g)) + np.abs(l0.dy(g)))[mask]


def _impulse(shape, beta, comp):
    e = np.zeros(shape)
    e[shape[0] // 2, shape[1] // 2] = 1.0
    z = np.zeros(shape)
    return l0.fft_solve(z, e, z, beta) if comp == 0 else l0.fft_solve(z, z, e, beta)


def fft_step_allowance(g, mask, beta):
    """Bound on |delta| of the unit-weight FFT step (rho_e step, L0 step) from
    flipping the decisions at `mask` (g = the thresholded image)."""
    if not np.any(mask):
        return 0.0
    shape = np.shape(g)
    sup = max(float(np.abs(_impulse(shape, beta, 0)).max()),
              float(np.abs(_impulse(shape, beta, 1)).max()))
    return float(flipped_gradients(g, mask).sum()) * sup


def weighted_step_allowance(g, mask, w, beta):
    """Bound on |delta| of the weighted solve (t' step) from flipping the
    decisions at `mask`: the response of (W^2 + beta L)^-1 beta D^T at each
    flipped pixel, times that pixel's gradient."""
    if not np.any(mask):
        return 0.0
    g = np.asarray(g, np.float64)
    shape = g.shape
    z = np.zeros(shape)
    total = 0.0
    gx, gy = np.abs(l0.dx(g)), np.abs(l0.dy(g))
    for iy, ix in zip(*np.nonzero(mask)):
        e = np.zeros(shape)
        e[iy, ix] = 1.0
        rh, _, _ = l0.weighted_solve(w, z, e, z, beta, rtol=1e-10)
        rv, _, _ = l0.weighted_solve(w, z, z, e, beta, rtol=1e-10)
        total += gx[iy, ix] * float(np.abs(rh).max()) + gy[iy, ix] * float(np.abs(rv).max())
    return total


def f_step_allowance(g1, g2, m1, m2, alpha, beta):
    """Bound on |delta f| of one steepest-descent f-step from flipping the
    decisions at m1 (in f1) and m2 (in f2)."""
    s = float(flipped_gradients(g1, m1).sum()) + float(flipped_gradients(g2, m2).sum())
    return abs(alpha) * 2.0 * beta * s


def image_f_allowance(g1, g2, m1, m2, H, beta):
    """Bound on |delta f| of the image-domain f-step (the joint 2x2 FFT solve
    of (13a), matrix H of its data and coupling terms) from flipping the
    decisions at m1 (in f1) and m2 (in f2)."""
    s = float(flipped_gradients(g1, m1).sum()) + float(flipped_gradients(g2, m2).sum())
    if s == 0.0:
        return 0.0
    shape = np.shape(g1)
    ox, oy = l0._otf(shape, -1), l0._otf(shape, -2)
    lap = np.abs(ox) ** 2 + np.abs(oy) ** 2
    a11, a22, a12 = H[0, 0] + beta * lap, H[1, 1] + beta * lap, H[0, 1]
    det = a11 * a22 - a12 * a12
    e = np.zeros(shape)
    e[shape[0] // 2, shape[1] // 2] = 1.0
    E = np.fft.fft2(e)
    sup = 0.0
    for o in (ox, oy):
        r = beta * np.conj(o) * E
        for r1, r2 in ((r, 0.0 * r), (0.0 * r, r)):
            x1 = np.real(np.fft.ifft2((a22 * r1 - a12 * r2) / det))
            x2 = np.real(np.fft.ifft2((a11 * r2 - a12 * r1) / det))
            sup = max(sup, float(np.abs(x1).max()), float(np.abs(x2).max()))
    return s * sup


def iteration_allowances(st, phys, params, f_alpha=None, image_H=None):
    """Near-tie counts of the four domains of state `st` and the allowances
    they give one outer iteration (keys f, rho, t).  `f_alpha()` returns the
    sinogram form's line-search step (called only when f has near-ties);
    `image_H` is the image form's 2x2 f matrix (then the f-step is the joint
    FFT solve)."""
    lam, beta = params.lam, st.beta
    m = {k: near_ties(getattr(st, k), lam, beta) for k in ("f1", "f2", "rho", "t")}
    counts = {k: int(v.sum()) for k, v in m.items()}
    allow = {"f": 0.0, "rho": 0.0, "t": 0.0}
    if counts["f1"] or counts["f2"]:
        if image_H is not None:
            allow["f"] = image_f_allowance(st.f1, st.f2, m["f1"], m["f2"], image_H, beta)
        else:
            allow["f"] = f_step_allowance(st.f1, st.f2, m["f1"], m["f2"], f_alpha(), beta)
    if counts["rho"]:
        allow["rho"] = fft_step_allowance(st.rho, m["rho"], beta)
    if counts["t"]:
        M1, M2 = phys.synth(st.f1, st.f2)
        w = phys.W(M1, M2) / phys.W_water()
        allow["t"] = weighted_step_allowance(st.t, m["t"], w, beta)
    return counts, allow


def sino_alpha(st, pL, pH, g, phys, params):
    """The oracle's line-search step of the sinogram f-step from state `st`."""
    from oracle import solve as S
    hv = (l0.ht_of(st.f1, params.lam, st.beta), l0.ht_of(st.f2, params.lam, st.beta))
    G1, G2 = S.f_gradient(st.f1, st.f2, pL, pH, hv, S.coupling_target(st, phys), g, phys, params, st.beta)
    q = S.f_curvature(-G1, -G2, g, phys, params, st.beta)
    return float(np.sum(G1 * G1) + np.sum(G2 * G2)) / q


def assert_iteration_close(got, ref, st, counts, allow, t_mask, tag, f_tol=1e-5, rho_tol=1e-5,
                           t_tol=5e-4):
    """One outer iteration's GPU result (f1, f2, rho, t) against the oracle's:
    FP32 tolerance relative to the sup-norm plus the near-tie allowances."""
    f1, f2, rho, t = got
    print(f"{tag}: near-ties {counts}, allowances {allow}")
    for a, r in ((f1, ref.f1), (f2, ref.f2)):
        assert np.abs(a - r).max() <= f_tol * np.abs(r).max() + allow["f"], tag
    assert np.abs(rho - ref.rho).max() <= rho_tol * np.abs(ref.rho).max() + allow["rho"], tag
    if t_mask.any():
        assert (np.abs(t - ref.t)[t_mask].max()
                <= t_tol * max(1.0, np.abs(ref.t[t_mask]).max()) + allow["t"]), tag
