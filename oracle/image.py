"""FP64 oracle of Algorithm 1 as the paper prints it: the image-domain form,
whose inputs are the two attenuation images mu(E_L), mu(E_H) (1/mm).

TEST INFRASTRUCTURE ONLY (oracle).

Objective (10) per outer iteration k, relaxed as in (12):
  Phi = eta_i sum_k || C_k1 f1 + C_k2 f2 - mu_k ||^2              (data, k = L, H)
      + xi    sum_j || m_j1 f1 + m_j2 f2 - T_j ||^2                (coupling, j = 1, 2)
      + beta  sum_g || D g - (h_g, v_g) ||^2                       (relaxation)
f-subproblem (13a) by the closed forms printed with Algorithm 1: f1 is solved
with f2 held at iterate k and f2 with f1 at iterate k, each from
  (c_i + beta D^T D) f_i = b_i + beta D^T (h_i, v_i)
  c_i = eta_i sum_k C_ki^2 + xi sum_j m_ji^2
  b_i = eta_i sum_k C_ki (mu_k - C_ko f_o) + xi sum_j m_ji (T_j - m_jo f_o),   o = the other basis
which the FFT diagonalises (periodic differences).  The rho_e and Z^m
subproblems (13b, 13c), the hard threshold (13d), the schedule and the
output are those of the sinogram form (oracle.solve), with the same readings.

Reading specific to this form: the data weight is eta_i = 1 / sum_k mu_w(E_k)^2,
the unit water curvature in f2 (the image-domain counterpart of the projection
weight eta of the sinogram form); the paper prints the data terms unweighted
next to terms of other units.
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


def f_step(st: State, muL, muH, phys: Physics, params: Params):
    """f-subproblem (13a): the printed FFT closed forms (Jacobi in f1, f2)."""
    out = []
    for i, g in enumerate((st.f1, st.f2)):
        b, c = f_rhs(st, muL, muH, phys, params, i)
        h, v = l0.ht_of(g, params.lam, st.beta)
        out.append(fft_solve_c(b, c, h, v, st.beta))
    return out[0], out[1]


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
