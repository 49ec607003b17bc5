"""Pins of the oracle's attenuation model and per-pixel closed forms
(Section II-A, II-B; eq. (1)-(4)).  CPU only."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import physics as ph
from oracle.physics import Physics

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_printed_constants_match_paper():
    assert ph.CP == GOLD["Cp"]["value"]
    assert ph.R0_CM == GOLD["r0_cm"]["value"]
    assert ph.ME_KEV == GOLD["gamma_denominator_keV"]["value"]
    p = Physics()
    assert p.n == GOLD["n"]["value"]
    assert (p.E1, p.E2) == (GOLD["E1_keV"]["value"], GOLD["E2_keV"]["value"])
    assert p.Zw == GOLD["true_water"]["Z"]
    assert p.basis_Z == (GOLD["sb3_cortical_bone"]["Z"], GOLD["true_water"]["Z"])
    assert p.basis_rho == (GOLD["sb3_cortical_bone"]["rho_e"], GOLD["true_water"]["rho_e"])


def test_klein_nishina_thomson_limit():
    """gamma -> 0: the total KN cross section tends to 8 pi r0^2 / 3."""
    thomson = 8.0 * math.pi * ph.R0_CM ** 2 / 3.0
    # the closed form cancels catastrophically at tiny gamma; 0.5 keV is far enough
    kn = float(ph.klein_nishina(0.5))
    assert abs(kn / thomson - 1.0) < 3e-3
    # the leading correction is -2 gamma: check the slope as well
    g = 0.5 / ph.ME_KEV
    assert abs((kn / thomson - 1.0) / (-2.0 * g) - 1.0) < 0.05


@pytest.mark.parametrize("E", [30.0, 50.0, 60.0, 90.0, 200.0, 510.975, 1000.0])
def test_klein_nishina_equals_integrated_differential(E):
    """The printed closed form equals the angular integral of the KN
    differential cross section (an independent route to the same number)."""
    k = E / ph.ME_KEV
    r0 = ph.R0_CM

    def dsig(theta):
        P = 1.0 / (1.0 + k * (1.0 - math.cos(theta)))
        return 0.5 * r0 ** 2 * P ** 2 * (P + 1.0 / P - math.sin(theta) ** 2) * 2 * math.pi * math.sin(theta)

    val, _ = integrate.quad(dsig, 0.0, math.pi, epsabs=0, epsrel=1e-13, limit=200)
    assert abs(float(ph.klein_nishina(E)) / val - 1.0) < 1e-10


def test_water_normalisation_of_photoelectric_term():
    """At Z = Zw the normalised photoelectric term equals the printed m = 3.8 term."""
    for m in (3.8, 3.94):
        p = Physics(m=m)
        for E in (50.0, 60.0, 90.0):
            lhs = p.a_coef(E) * p.Zw ** m
            rhs = ph.CP * p.Zw ** 3.8 / E ** 3.2
            assert abs(lhs / rhs - 1.0) < 1e-13


@pytest.mark.parametrize("m", [3.94, 3.8])
def test_closed_forms_invert_the_model(m):
    """Any (Z, rho_e) is an exact mixture of two basis materials in this model,
    so decomposition (1), synthesis (2) and the closed forms (4a,b) must return
    the material's own (Z, rho_e) to rounding."""
    p = Physics(m=m)
    rng = np.random.default_rng(5)
    Z = rng.uniform(5.5, 20.0, 200)
    R = rng.uniform(0.2, 1.9, 200)
    muL, muH = p.mu_pair(Z, R)
    f1, f2 = p.decompose(muL, muH)
    M1, M2 = p.synth(f1, f2)
    assert np.allclose(p.rho_closed(M1, M2), R, rtol=1e-11, atol=0)
    t = p.t_closed(M1, M2)
    assert np.allclose(p.Zw * t ** (1.0 / m), Z, rtol=1e-10, atol=0)


def test_basis_materials_decompose_to_unit_vectors():
    p = Physics()
    muL, muH = p.mu_pair(np.array(p.basis_Z), np.array(p.basis_rho))
    f1, f2 = p.decompose(muL, muH)
    assert np.allclose(f1, [1.0, 0.0], atol=1e-13)
    assert np.allclose(f2, [0.0, 1.0], atol=1e-13)


def test_water_is_one_and_742():
    p = Physics()
    muL, muH = p.mu_pair(p.Zw, 1.0)
    M1, M2 = p.synth(*p.decompose(muL, muH))
    assert abs(p.rho_closed(M1, M2) - 1.0) < 1e-12
    assert abs(p.t_closed(M1, M2) - 1.0) < 1e-12
    assert abs(p.W(M1, M2) / p.W_water() - 1.0) < 1e-12


def test_water_attenuation_in_physical_range():
    """Sanity: water mu at 60 keV is ~0.0206/mm in NIST tables (incl. coherent);
    the two-process model without Rayleigh must land a little below."""
    p = Physics()
    mu60 = float(p.mu(p.Zw, 1.0, 60.0))
    assert 0.0185 < mu60 < 0.0206


def test_normalised_weights_positive_and_order_one():
    from paper_2308_01290_amd import phantoms as P
    p = Physics()
    g = P.geometry_small()
    from oracle import operators as ops
    eta = p.eta(ops.Geometry.of(g))
    assert eta > 0 and p.xi() > 0
    # per-pixel data curvature of a unit water-fraction change ~ 1 at the centre
    e = np.zeros((g.n_y, g.n_x))
    e[g.n_y // 2, g.n_x // 2] = 1.0
    Ae = ops.project(g, e)
    C = p.C()
    curv = eta * float(np.sum(Ae ** 2)) * float(C[0, 1] ** 2 + C[1, 1] ** 2)
    assert 0.5 < curv < 1.5
