"""FP64 oracle of the one-step iterative (Z, rho_e) estimation, Algorithm 1,
with the image-domain data terms of objective (10) moved to the projection
domain (the sinogram form of the method).

TEST INFRASTRUCTURE ONLY (oracle).

Objective per outer iteration k, f-subproblem (13a) in sinogram form:
  Phi(f) = eta  sum_k || A(C_k1 f1 + C_k2 f2) - p_k ||^2                (data, k = L, H)
         + xi   sum_j || m_j1 f1 + m_j2 f2 - rho (a'_j Zw^m t' + psi_j) ||^2   (coupling, j = 1, 2)
         + beta sum_i || D f_i - (h_i, v_i) ||^2                          (relaxation)
Because A^T A is not diagonalised by the FFT, the closed forms printed for f1, f2
no longer apply; the f-subproblem is minimised by f_inner conjugate-gradient
steps with exact line search (one steepest-descent step for f_inner = 1),
restarted every outer iteration.  All right-hand sides read iterate k
(Jacobi, as Algorithm 1 updates f1 from f2^(k) and f2 from f1^(k)).

Readings, where the paper is silent or garbled:
  * input images mu(E_L), mu(E_H) are fan-beam FBP reconstructions of the
    sinograms (Algorithm 1 requires reconstructed images);
  * (mu/rho)^(k) = synthesis of f^(k) for the rho_e and Z^m subproblems
    (the printed indices lag by one step);
  * tilde-beta = tau beta is read as a per-domain rescaling to unit data weight
    for water: the rho_e subproblem becomes ||rho - rho_hat||^2 + beta||D rho - h||^2
    and the Z^m subproblem uses t' = Z^m / Zw^m with weights W/W_w;
  * beta^(k+1) = kappa beta^(k), beta^(0) = 2 lambda, beta_max = 1e5 and
    kappa = (beta_max / beta^(0))^(1/K), so "until beta >= beta_max" stops after K
    iterations;
  * t' starts at 1 where the closed form (4b) is undefined or meaningless:
    |W| < 1e-6 |W_w|, or rho_e^(0) < rho_min (air, where Z is not defined);
  * output Z = Zw max(t', t_min)^(1/m), and Z = 0 where rho_e < rho_min.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from . import l0
from . import operators as ops
from .physics import Physics


@dataclass
class Params:
    lam: float = 0.01
    beta0: float = 0.0          # 0 -> 2*lambda
    beta_max: float = 1e5
    kappa: float = 0.0          # 0 -> (beta_max/beta0)^(1/n_iter)
    eta: float = 0.0            # 0 -> default projection-data weight
    xi: float = 0.0             # 0 -> default coupling weight
    n_iter: int = 10
    f_inner: int = 1
    t_rtol: float = 1e-12
    rho_min: float = 0.1
    t_min: float = 1e-6

    def resolved(self, phys: Physics, geom) -> "Params":
        p = replace(self)
        if p.beta0 <= 0:
            p.beta0 = 2.0 * p.lam
        if p.kappa <= 0:
            p.kappa = (p.beta_max / p.beta0) ** (1.0 / max(p.n_iter, 1))
        if p.eta <= 0:
            p.eta = phys.eta(ops.Geometry.of(geom))
        if p.xi <= 0:
            p.xi = phys.xi()
        return p


@dataclass
class State:
    f1: np.ndarray
    f2: np.ndarray
    rho: np.ndarray
    t: np.ndarray
    beta: float
    k: int = 0


def init_from_mu(muL, muH, phys: Physics, params: Params) -> State:
    """Algorithm 1 initialisation from the two attenuation images."""
    f1, f2 = phys.decompose(muL, muH)
    M1, M2 = phys.synth(f1, f2)
    rho = phys.rho_closed(M1, M2)
    W = phys.W(M1, M2)
    Ww = phys.W_water()
    small = (np.abs(W) < 1e-6 * abs(Ww)) | (rho < params.rho_min)
    t = np.where(small, 1.0, phys.d_t(M1, M2) / np.where(small, 1.0, W))
    return State(f1, f2, rho, t, params.beta0, 0)


def init_state(pL, pH, geom, phys: Physics, params: Params, nthreads=None) -> State:
    muL = ops.fbp(geom, pL, nthreads)
    muH = ops.fbp(geom, pH, nthreads)
    return init_from_mu(muL, muH, phys, params)


def coupling_target(st: State, phys: Physics):
    """T_j = rho (Cp' Zw^m t' / E_j^n + psi_j): the model side of the coupling terms."""
    a = phys.cp_barn() * phys.Zw ** phys.m
    psi = phys.psi()
    return (st.rho * (a * st.t / phys.E1 ** phys.n + psi[0]),
            st.rho * (a * st.t / phys.E2 ** phys.n + psi[1]))


def f_gradient(f1, f2, pL, pH, hv, T, geom, phys, params, beta, nthreads=None):
    """Gradient of Phi at (f1, f2)."""
    C = phys.C()
    m = phys.Msyn()
    rL = ops.project(geom, C[0, 0] * f1 + C[0, 1] * f2, nthreads) - pL
    rH = ops.project(geom, C[1, 0] * f1 + C[1, 1] * f2, nthreads) - pH
    bL = ops.backproject(geom, rL, nthreads)
    bH = ops.backproject(geom, rH, nthreads)
    c1 = m[0, 0] * f1 + m[0, 1] * f2 - T[0]
    c2 = m[1, 0] * f1 + m[1, 1] * f2 - T[1]
    (h1, v1), (h2, v2) = hv
    g1 = (2 * params.eta * (C[0, 0] * bL + C[1, 0] * bH)
          + 2 * params.xi * (m[0, 0] * c1 + m[1, 0] * c2)
          + 2 * beta * l0.dT(l0.dx(f1) - h1, l0.dy(f1) - v1))
    g2 = (2 * params.eta * (C[0, 1] * bL + C[1, 1] * bH)
          + 2 * params.xi * (m[0, 1] * c1 + m[1, 1] * c2)
          + 2 * beta * l0.dT(l0.dx(f2) - h2, l0.dy(f2) - v2))
    return g1, g2


def f_curvature(d1, d2, geom, phys, params, beta, nthreads=None):
    """d^T H d of Phi along (d1, d2)."""
    C = phys.C()
    m = phys.Msyn()
    YL = ops.project(geom, C[0, 0] * d1 + C[0, 1] * d2, nthreads)
    YH = ops.project(geom, C[1, 0] * d1 + C[1, 1] * d2, nthreads)
    e1 = m[0, 0] * d1 + m[0, 1] * d2
    e2 = m[1, 0] * d1 + m[1, 1] * d2
    q = 2 * params.eta * (np.sum(YL ** 2) + np.sum(YH ** 2))
    q += 2 * params.xi * (np.sum(e1 ** 2) + np.sum(e2 ** 2))
    q += 2 * beta * sum(np.sum(l0.dx(d) ** 2) + np.sum(l0.dy(d) ** 2) for d in (d1, d2))
    return float(q)


def f_step(st: State, pL, pH, geom, phys, params, nthreads=None):
    """f-subproblem (13a), sinogram form: f_inner CG steps, exact line search."""
    beta = st.beta
    hv = (l0.ht_of(st.f1, params.lam, beta), l0.ht_of(st.f2, params.lam, beta))
    T = coupling_target(st, phys)
    f1, f2 = st.f1.copy(), st.f2.copy()
    d1 = d2 = None
    gg_prev = None
    for it in range(params.f_inner):
        g1, g2 = f_gradient(f1, f2, pL, pH, hv, T, geom, phys, params, beta, nthreads)
        gg = float(np.sum(g1 * g1) + np.sum(g2 * g2))
        if it == 0:
            d1, d2 = -g1, -g2
        else:
            cg = gg / gg_prev
            d1, d2 = -g1 + cg * d1, -g2 + cg * d2
        q = f_curvature(d1, d2, geom, phys, params, beta, nthreads)
        if q <= 0.0:
            break
        alpha = -float(np.sum(g1 * d1) + np.sum(g2 * d2)) / q
        f1 = f1 + alpha * d1
        f2 = f2 + alpha * d2
        gg_prev = gg
    return f1, f2


def rho_step(st: State, phys, params):
    """rho_e subproblem (13b), normalised, by the FFT closed form."""
    M1, M2 = phys.synth(st.f1, st.f2)
    rho_hat = phys.rho_closed(M1, M2)
    h, v = l0.ht_of(st.rho, params.lam, st.beta)
    return l0.fft_solve(rho_hat, h, v, st.beta)


def t_step(st: State, phys, params):
    """Z^m subproblem (13c) in t' = Z^m/Zw^m with weights W/W_w: SPD solve."""
    M1, M2 = phys.synth(st.f1, st.f2)
    Ww = phys.W_water()
    w = phys.W(M1, M2) / Ww
    gt = phys.d_t(M1, M2) / Ww
    h, v = l0.ht_of(st.t, params.lam, st.beta)
    t, _, _ = l0.weighted_solve(w, gt, h, v, st.beta, x0=st.t, rtol=params.t_rtol)
    return t


def iterate(st: State, pL, pH, geom, phys, params, nthreads=None) -> State:
    """One outer iteration of Algorithm 1 (sinogram form)."""
    f1, f2 = f_step(st, pL, pH, geom, phys, params, nthreads)
    rho = rho_step(st, phys, params)
    t = t_step(st, phys, params)
    return State(f1, f2, rho, t, st.beta * params.kappa, st.k + 1)


def finalize(st: State, phys, params):
    """Z = Zw max(t', t_min)^(1/m); Z = 0 where rho_e < rho_min."""
    Z = phys.Zw * np.maximum(st.t, params.t_min) ** (1.0 / phys.m)
    Z = np.where(st.rho < params.rho_min, 0.0, Z)
    return Z, st.rho.copy()


def solve(pL, pH, geom, phys: Optional[Physics] = None, params: Optional[Params] = None,
          nthreads=None, return_state=False):
    phys = phys or Physics()
    params = (params or Params()).resolved(phys, geom)
    st = init_state(np.asarray(pL, np.float64), np.asarray(pH, np.float64), geom, phys, params, nthreads)
    for _ in range(params.n_iter):
        st = iterate(st, pL, pH, geom, phys, params, nthreads)
    Z, rho = finalize(st, phys, params)
    if return_state:
        return Z, rho, st
    return Z, rho
