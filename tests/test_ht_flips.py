"""The flip allowances used by the parity tests, checked on the oracle: a
hard-threshold decision of eq. (9) is flipped on purpose inside the FP64
oracle (CPU only) and the step's output must move by no more than the
allowance says, in the flipped domain, and not at all in the others."""
import numpy as np
import pytest

from oracle import l0, solve as S
from oracle.physics import Physics
from tests import ht_flips as HF
from tests.gpu_util import workload


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def closest_to_tie(g, lam, beta, skip=0):
    """Pixel whose eq. (9) sum is nearest the threshold (a plausible flip)."""
    d = np.abs(HF.grad_sq(g) - lam / beta)
    order = np.argsort(d, axis=None)
    return np.unravel_index(order[skip], d.shape)


def iterate_with_flip(st, target, pixel, pL, pH, g, phys, params):
    """The oracle's iteration with the decision of `pixel` in the domain whose
    image is `target` flipped (planted in the oracle, test only)."""
    orig = l0.ht_keep
    tx, ty = l0.dx(target), l0.dy(target)

    def patched(gx, gy, lam, beta):
        keep = orig(gx, gy, lam, beta)
        if np.shape(gx) == tx.shape and np.array_equal(gx, tx) and np.array_equal(gy, ty):
            keep = keep.copy()
            keep[pixel] = ~keep[pixel]
        return keep

    l0.ht_keep = patched
    try:
        return S.iterate(st, pL, pH, g, phys, params)
    finally:
        l0.ht_keep = orig


@pytest.fixture(scope="module")
def small_state():
    g, ph, pL, pH = workload("small")
    phys = Physics()
    params = S.Params(n_iter=10).resolved(phys, g)
    st = S.init_state(f32(pL), f32(pH), g, phys, params)
    for _ in range(3):
        st = S.iterate(st, f32(pL), f32(pH), g, phys, params)
    st = S.State(f32(st.f1), f32(st.f2), f32(st.rho), f32(st.t), st.beta, st.k)
    ref = S.iterate(st, f32(pL), f32(pH), g, phys, params)
    return g, f32(pL), f32(pH), phys, params, st, ref


def test_near_tie_bound_covers_fp32_evaluation():
    """Decisions taken in FP32 (gradients, squares and sum rounded, threshold
    rounded) differ from the FP64 ones only at near-ties."""
    rng = np.random.default_rng(11)
    lam = 0.01
    for beta in (0.02, 3.0, 4e4):
        thr = lam / beta
        g = (np.sqrt(thr) * rng.standard_normal((256, 256))).astype(np.float32)
        gx = (np.roll(g, -1, 1) - g).astype(np.float32)
        gy = (np.roll(g, -1, 0) - g).astype(np.float32)
        s32 = (gx * gx).astype(np.float32) + (gy * gy).astype(np.float32)
        keep32 = s32 > np.float32(thr)
        keep64 = l0.ht_keep(l0.dx(f32(g)), l0.dy(f32(g)), lam, beta)
        diff = keep32 != keep64
        assert not np.any(diff & ~HF.near_ties(f32(g), lam, beta))


@pytest.mark.parametrize("domain", ["f1", "f2", "rho", "t"])
def test_flip_allowance_bounds_a_planted_flip(small_state, domain):
    g, pL, pH, phys, params, st, ref = small_state
    target = getattr(st, domain)
    pix = closest_to_tie(target, params.lam, st.beta)
    got = iterate_with_flip(st, target, pix, pL, pH, g, phys, params)
    mask = np.zeros(target.shape, bool)
    mask[pix] = True
    moved = {k: float(np.abs(getattr(got, k) - getattr(ref, k)).max()) for k in ("f1", "f2", "rho", "t")}
    if domain in ("f1", "f2"):
        alpha = HF.sino_alpha(st, pL, pH, g, phys, params)
        m1 = mask if domain == "f1" else np.zeros_like(mask)
        m2 = mask if domain == "f2" else np.zeros_like(mask)
        allow = HF.f_step_allowance(st.f1, st.f2, m1, m2, alpha, st.beta)
        # the line-search step alpha also moves slightly: allow its relative
        # change on the whole step
        allow += 1e-6 * max(float(np.abs(ref.f1 - st.f1).max()), float(np.abs(ref.f2 - st.f2).max()))
        assert moved["f1"] <= allow and moved["f2"] <= allow, (moved, allow)
        assert moved["f1"] + moved["f2"] > 0.0
        assert moved["rho"] == 0.0 and moved["t"] == 0.0
    elif domain == "rho":
        allow = HF.fft_step_allowance(st.rho, mask, st.beta)
        assert 0.0 < moved["rho"] <= allow * (1 + 1e-9), (moved, allow)
        assert moved["f1"] == 0.0 and moved["t"] == 0.0
    else:
        M1, M2 = phys.synth(st.f1, st.f2)
        w = phys.W(M1, M2) / phys.W_water()
        allow = HF.weighted_step_allowance(st.t, mask, w, st.beta)
        # both t' solves stop at relative residual 1e-12: add that slack
        assert 0.0 < moved["t"] <= allow * (1 + 1e-6) + 1e-9, (moved, allow)
        assert moved["f1"] == 0.0 and moved["rho"] == 0.0


@pytest.mark.parametrize("domain", ["f1", "f2"])
def test_image_f_allowance_bounds_a_planted_flip(domain):
    from oracle import image as I
    from paper_2308_01290_amd import phantoms as P
    phys = Physics()
    g, ph, L, H = P.workload_image_small(phys.mu_pair)
    L, H = f32(L), f32(H)
    params = I.resolved(S.Params(n_iter=10), phys)
    st = I.init_from_mu(L, H, phys, params)
    st = S.State(st.f1, st.f2, st.rho, st.t, params.beta0 * params.kappa ** 3, 3)
    ref = I.f_step(st, L, H, phys, params)
    target = getattr(st, domain)
    pix = closest_to_tie(target, params.lam, st.beta)
    orig = l0.ht_keep
    tx = l0.dx(target)

    def patched(gx, gy, lam, beta):
        keep = orig(gx, gy, lam, beta)
        if np.array_equal(gx, tx):
            keep = keep.copy()
            keep[pix] = ~keep[pix]
        return keep

    l0.ht_keep = patched
    try:
        got = I.f_step(st, L, H, phys, params)
    finally:
        l0.ht_keep = orig
    mask = np.zeros(target.shape, bool)
    mask[pix] = True
    _, Hm = I.f_system(st, L, H, phys, params)
    m1 = mask if domain == "f1" else np.zeros_like(mask)
    m2 = mask if domain == "f2" else np.zeros_like(mask)
    allow = HF.image_f_allowance(st.f1, st.f2, m1, m2, Hm, st.beta)
    moved = max(float(np.abs(got[0] - ref[0]).max()), float(np.abs(got[1] - ref[1]).max()))
    assert 0.0 < moved <= allow * (1 + 1e-9), (moved, allow)
