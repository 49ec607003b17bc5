"""FP64 oracle of Algorithm 1 as the paper prints it: the image-domain form,
whose inputs are the two attenuation images mu(E_L), mu(E_H) (1/mm).

TEST INFRASTRUCTURE ONLY (oracle).

Objective (10) per outer iteration k, relaxed as in (12):
  Phi = eta_i sum_k || C_k1 f1 + C_k2 f2 - mu_k ||^2              (data, k = L, H)
      + xi    sum_j || m_j1 f1 + m_j2 f2 - T_j ||^2                (coupling, j = 1, 2)
      + beta  sum_g || D g - (h_g, v_g) ||^2                       (relaxation)
f-subproblem (13a): its minimiser over (f1, f2) jointly.  The two closed
forms printed after (13a) are the two stationarity conditions of (13a), one
per basis:
  (c_i + beta D^T D) f_i + o f_other = b_i + beta D^T (h_i, v_i)
  c_i = eta_i sum_k C_ki^2 + xi sum_j m_ji^2,   o = eta_i sum_k C_k1 C_k2 + xi sum_j m_j1 m_j2
  b_i = eta_i sum_k C_ki mu_k + xi sum_j m_ji T_j
Every coupling between f1 and f2 is a scalar times the identity and D^T D is
diagonalised by the FFT (periodic differences), so the joint minimiser is a
2x2 solve per frequency.  The rho_e and Z^m subproblems (13b, 13c), the hard
threshold (13d), the schedule and the output are those of the sinogram form
(oracle.solve), with the same readings.

Readings specific to this form:
  * the data weight is eta_i = 1 / sum_k mu_w(E_k)^2, the unit water curvature
    in f2 (the image-domain counterpart of the projection weight eta of the
    sinogram form); the paper prints the data terms unweighted next to terms
    of other units;
  * Algorithm 1 prints each f_i update with the other basis at iterate k (a
    Jacobi pair).  Taken literally, with the coupling target built from
    rho_e^(k), Z^(k), that pair is unstable at low frequencies: linearised about
    a fixed point, its zero-frequency iteration matrix has spectral radius 1.63
    with the default physics, so slowly varying errors grow every outer
    iteration (a noisy 512^2 solve of 50 iterations diverges).  Subproblem (13a)
    itself asks for the minimiser over (f1, f2) together; that minimiser
    satisfies both printed stationarity conditions at once, and its iteration
    contracts (radius 0.94 at zero frequency, less above).  `f_step` takes that
    reading; `f_step_jacobi` keeps the printed pair for the tests that show
    the difference.
"""
from __future__ import annotations

from dataclasses import replace
from typing import Optional

import numpy as np

from . import l0
from .physics import Physics
from .solve import Params, State, coupling_target, finalize, init_from_mu, rho_step, t_step


def eta_image(phys: Physics) -> float:
    """Image-domain data weight: 1 / (mu_w(E_L)^2 + mu_w(E_H)^2)."""
    mw = phys.mu(phys.Zw, 1.0, np.array([phys.E_lo, phys.E_hi]))
    return 1.0 / float(np.sum(mw ** 2))


def resolved(params: Params, phys: Physics) -> Params:
    p = replace(params)
    if p.beta0 <= 0:
        p.beta0 = 2.0 * p.lam
    if p.kappa <= 0:
        p.kappa = (p.beta_max / p.beta0) ** (1.0 / max(p.n_iter, 1))
    if p.eta <= 0:
        p.eta = eta_image(phys)
    if p.xi <= 0:
        p.xi = phys.xi()
    return p


def fft_solve_c(b, c, h, v, beta):
    """(c + beta D^T D) x = b + beta D^T (h, v), periodic, by the FFT (the
    closed form printed for (13a) divided through by nothing: c is the
    constant diagonal of the data and coupling terms)."""
    shp = np.shape(b)
    ox, oy = l0._otf(shp, -1), l0._otf(shp, -2)
    num = np.fft.fft2(b) + beta * (np.conj(ox) * np.fft.fft2(h) + np.conj(oy) * np.fft.fft2(v))
    den = c + beta * (np.abs(ox) ** 2 + np.abs(oy) ** 2)
    return np.real(np.fft.ifft2(num / den))


def f_rhs(st: State, muL, muH, phys: Physics, params: Params, i: int):
    """(b_i, c_i) of the f_i closed form, the other basis at iterate k."""
    C, m = phys.C(), phys.Msyn()
    T = coupling_target(st, phys)
    o = 1 - i
    fo = (st.f1, st.f2)[o]
    mu = (muL, muH)
    b = sum(params.eta * C[k, i] * (mu[k] - C[k, o] * fo) for k in range(2))
    b = b + sum(params.xi * m[j, i] * (T[j] - m[j, o] * fo) for j in range(2))
    c = params.eta * float(np.sum(C[:, i] ** 2)) + params.xi * float(np.sum(m[:, i] ** 2))
    return b, c


def f_step_jacobi(st: State, muL, muH, phys: Physics, params: Params):
    """The printed pair of closed forms taken literally: f1 with f2 at iterate
    k and f2 with f1 at iterate k (a Jacobi sweep over the two bases)."""
    out = []
    for i, g in enumerate((st.f1, st.f2)):
        b, c = f_rhs(st, muL, muH, phys, params, i)
        h, v = l0.ht_of(g, params.lam, st.beta)
        out.append(fft_solve_c(b, c, h, v, st.beta))
    return out[0], out[1]


def f_system(st: State, muL, muH, phys: Physics, params: Params):
    """Right sides b_1, b_2 and the constant 2x2 matrix [[c1, o], [o, c2]] of
    the data and coupling terms of (13a), from objective (12) term by term."""
    C, m = phys.C(), phys.Msyn()
    T = coupling_target(st, phys)
    mu = (muL, muH)
    b = [sum(params.eta * C[k, i] * mu[k] for k in range(2))
         + sum(params.xi * m[j, i] * T[j] for j in range(2)) for i in range(2)]
    H = params.eta * (C.T @ C) + params.xi * (m.T @ m)
    return b, H


def f_step(st: State, muL, muH, phys: Physics, params: Params):
    """f-subproblem (13a): joint minimiser over (f1, f2), one 2x2 solve per
    frequency of  (H + beta |F D|^2 I) F(f) = F(b) + beta F(D^T (h, v))."""
    b, H = f_system(st, muL, muH, phys, params)
    beta = st.beta
    shp = np.shape(st.f1)
    ox, oy = l0._otf(shp, -1), l0._otf(shp, -2)
    lap = np.abs(ox) ** 2 + np.abs(oy) ** 2
    rhs = []
    for i, g in enumerate((st.f1, st.f2)):
        h, v = l0.ht_of(g, params.lam, beta)
        rhs.append(np.fft.fft2(b[i]) + beta * (np.conj(ox) * np.fft.fft2(h) + np.conj(oy) * np.fft.fft2(v)))
    a11 = H[0, 0] + beta * lap
    a22 = H[1, 1] + beta * lap
    a12 = H[0, 1]
    det = a11 * a22 - a12 * a12
    x1 = (a22 * rhs[0] - a12 * rhs[1]) / det
    x2 = (a11 * rhs[1] - a12 * rhs[0]) / det
    return np.real(np.fft.ifft2(x1)), np.real(np.fft.ifft2(x2))


def iterate(st: State, muL, muH, phys: Physics, params: Params) -> State:
    """One outer iteration of Algorithm 1 (image domain); all updates read iterate k."""
    f1, f2 = f_step(st, muL, muH, phys, params)
    rho = rho_step(st, phys, params)
    t = t_step(st, phys, params)
    return State(f1, f2, rho, t, st.beta * params.kappa, st.k + 1)


def solve(muL, muH, phys: Optional[Physics] = None, params: Optional[Params] = None,
          return_state=False):
    phys = phys or Physics()
    params = resolved(params or Params(), phys)
    muL = np.asarray(muL, np.float64)
    muH = np.asarray(muH, np.float64)
    st = init_from_mu(muL, muH, phys, params)
    for _ in range(params.n_iter):
        st = iterate(st, muL, muH, phys, params)
    Z, R = finalize(st, phys, params)
    return (Z, R, st) if return_state else (Z, R)
