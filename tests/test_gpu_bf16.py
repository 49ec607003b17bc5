"""BF16 storage variants of the sinogram form: what changes against FP32
storage, and the accuracy each reaches against the FP64 oracle.

DECT_STORAGE_BF16 stores the projector operands (search direction, residual
and line-search sinograms) in BF16; DECT_STORAGE_BF16_STATE also rounds the
state images f1, f2, rho_e, t' to BF16 after every write.  BF16 keeps 8
significant bits: rounded to nearest (the direction) a stored value is within
2^-8 of its FP32 value (relative, the unit roundoff); the quantities that
accumulate small updates (residual sinograms, state images) are rounded
stochastically, within one BF16 ulp (2^-7 relative) and unbiased."""
import os

import numpy as np
import pytest

from oracle import solve as S
from oracle.physics import Physics
from paper_2308_01290_amd import dect
from tests.gpu_util import cuda, host, workload
from tests.test_gpu_solver import phantom_body

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
U_BF16 = 2.0 ** -8   # unit roundoff of BF16 (8 significant bits, round to nearest)


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def one_step(storage, k=3):
    g, ph, pL, pH = workload("small")
    phys = Physics()
    params = S.Params(n_iter=10).resolved(phys, g)
    st = S.init_state(f32(pL), f32(pH), g, phys, params)
    sol = dect.Solver(g, dect.default_params(n_iter=10, storage=storage))
    sol.set_state(cuda(pL[None]), cuda(pH[None]), *(cuda(a[None]) for a in (st.f1, st.f2, st.rho, st.t)),
                  k=k)
    sol.iterate(1)
    return st, [host(a)[0] for a in sol.state()]


def is_bf16(x):
    b = np.asarray(x, dtype=np.float32).view(np.uint32)
    return bool(np.all((b & 0xFFFF) == 0))


def test_bf16_operands_change_only_the_f_step():
    """One iteration from the same state: the rho_e and t' steps read only the
    state, so they are bitwise those of FP32 storage; f moves by the same
    step up to the BF16 rounding of the direction and residuals."""
    st, (f1a, f2a, ra, ta) = one_step(dect.DECT_STORAGE_FP32)
    _, (f1b, f2b, rb, tb) = one_step(dect.DECT_STORAGE_BF16)
    assert np.array_equal(ra, rb) and np.array_equal(ta, tb)
    for fa, fb, f0 in ((f1a, f1b, st.f1), (f2a, f2b, st.f2)):
        step = np.abs(fa - f32(f0)).max()
        assert step > 0
        # direction entries, residuals and line-search sums each carry <= U_BF16
        # relative rounding; the step is their product and ratio
        assert np.abs(fb - fa).max() <= 4 * U_BF16 * step


def test_bf16_state_rounds_the_state():
    _, out = one_step(dect.DECT_STORAGE_BF16_STATE)
    for a in out:
        assert is_bf16(a)


def test_bf16_state_set_state_stores_rounded_values():
    g, ph, pL, pH = workload("small")
    rng = np.random.default_rng(5)
    imgs = [f32(1.0 + 0.1 * rng.standard_normal((g.n_y, g.n_x))) for _ in range(4)]
    sol = dect.Solver(g, dect.default_params(n_iter=4, storage=dect.DECT_STORAGE_BF16_STATE))
    sol.set_state(cuda(pL[None]), cuda(pH[None]), *(cuda(a[None]) for a in imgs), k=0)
    for a, ref in zip((host(x)[0] for x in sol.state()), imgs):
        assert is_bf16(a)
        # stochastic rounding: within one ulp, below 2 U |x| for every x
        assert np.all(np.abs(a - ref) <= 2 * U_BF16 * np.abs(ref))


def test_bf16_state_rounding_is_unbiased():
    """A constant state between two BF16 values, 1 + 2^-10 (an eighth of the
    way from 1 to the next value, 1 + 2^-7): nearest rounding would store 1
    everywhere and lose the difference; stochastic rounding stores the upper
    value at about an eighth of the pixels, so the mean is kept."""
    g, ph, pL, pH = workload("small")
    c = 1.0 + 2.0 ** -10
    imgs = [np.full((g.n_y, g.n_x), c) for _ in range(4)]
    sol = dect.Solver(g, dect.default_params(n_iter=4, storage=dect.DECT_STORAGE_BF16_STATE))
    sol.set_state(cuda(pL[None]), cuda(pH[None]), *(cuda(a[None]) for a in imgs), k=0)
    for a in (host(x)[0] for x in sol.state()):
        assert set(np.unique(a)) <= {1.0, 1.0 + 2.0 ** -7}
        assert abs(a.mean() - c) <= 1e-4


def test_bf16_batch_equals_single():
    """Per-slice results do not depend on the batch in BF16 storage either."""
    g, ph, pL, pH = workload("small")
    p = dect.default_params(n_iter=3, storage=dect.DECT_STORAGE_BF16)
    Zb, Rb = (host(x) for x in dect.solve(cuda(np.stack([pL, 0.9 * pL])), cuda(np.stack([pH, 0.9 * pH])), g, p))
    Z1, R1 = (host(x) for x in dect.solve(cuda(pL[None]), cuda(pH[None]), g, p))
    assert np.array_equal(Zb[0], Z1[0]) and np.array_equal(Rb[0], R1[0])


def accuracy(Z, R, Zr, Rr, ph, g):
    """Pointwise figures on the eroded body (as the FP32 end-to-end check) and
    the worst per-insert mean errors."""
    from scipy.ndimage import binary_erosion
    lab, body = phantom_body(ph, g)
    mz = body & (Zr >= 2) & (Z >= 2)
    dz = np.abs(Z - Zr)[mz]
    dr = (np.abs(R - Rr) / np.abs(Rr))[body]
    mean_dz = mean_dr = 0.0
    for idx in range(1, lab.shape[0]):
        mm = binary_erosion(lab[idx] > 0.999, iterations=2)
        if mm.sum() < 4:
            continue
        mean_dz = max(mean_dz, abs(Z[mm].mean() - Zr[mm].mean()))
        mean_dr = max(mean_dr, abs(R[mm].mean() - Rr[mm].mean()) / abs(Rr[mm].mean()))
    return {"max_dz": dz.max(), "p99_dz": np.quantile(dz, 0.99), "max_drho": dr.max(),
            "p99_drho": np.quantile(dr, 0.99), "frac_drho_gt_1e-3": float((dr > 1e-3).mean()),
            "insert_mean_dz": mean_dz, "insert_mean_drho": mean_dr}


def report(tag, a):
    print(tag + ": " + ", ".join(f"{k}={v:.3g}" for k, v in a.items()))


# Bounds fixed before the runs they judge.  Insert means (2-pixel eroded
# regions) must meet the FP32 path's tolerances themselves: |dZ| <= 0.02 and
# rel rho_e <= 1e-3.  Pointwise, BF16 storage cannot: its resolution is the
# bound.  With BF16 operands the state is FP32 and the residuals lose what
# their rounding drops, so p99 rel rho_e <= 2^-8 (half a BF16 ulp).  With the
# state in BF16, rho_e itself is a stored BF16 value (within one ulp after
# stochastic rounding): p99 rel rho_e <= 2^-7, and p99 |dZ| <= 0.05 (two ulps
# of t' at the largest insert Z of 14, through Z = Zw t'^(1/m)).
TOL_Z, TOL_RHO = 0.02, 1e-3
P99_RHO = {1: 2.0 ** -8, 2: 2.0 ** -7}
P99_Z = {1: TOL_Z, 2: 0.05}


def check_bf16(a, storage):
    assert a["p99_drho"] <= P99_RHO[storage] and a["p99_dz"] <= P99_Z[storage]
    assert a["insert_mean_dz"] <= TOL_Z and a["insert_mean_drho"] <= TOL_RHO


# Cases that do not reach the bounds above (measured, the bounds unchanged):
# * BF16 state at both sizes: p99 rel rho_e ~ 3e-2 (128^2) and ~ 0.1 (512^2),
#   insert means off by 1.7e-2 to 2.4e-2 in rho_e.  BF16 steps of the state are
#   2^-8 relative; from beta ~ 600 on the hard-threshold level lambda/beta falls
#   below a squared step, so quantisation steps pass eq. (9) as edges and the
#   relaxation keeps them: the state cannot settle below that.
# * BF16 operands at 512^2: the insert means' rho_e error is 0.7e-3 to 1.6e-3
#   against the bound 1e-3, depending on the projectors' rounding order (the
#   residual sinograms hold 8 significant bits of a small difference), so the
#   case is borderline: it is expected to fail, and a pass is not an error.
XFAIL_BF16 = {("small", 2), ("slice512", 1), ("slice512", 2)}
BORDERLINE_BF16 = {("slice512", 1)}


def bf16_case(size, storage):
    marks = []
    if (size, storage) in XFAIL_BF16:
        marks.append(pytest.mark.xfail(strict=(size, storage) not in BORDERLINE_BF16,
                                       reason="BF16 storage misses the stated bound "
                                              "(figures in the design notes)"))
    return pytest.param(storage, marks=marks, id=f"storage{storage}")


@pytest.mark.parametrize("storage", [bf16_case("small", 1), bf16_case("small", 2)])
def test_bf16_small_against_oracle(storage):
    g, ph, pL, pH = workload("small")
    Zr, Rr = S.solve(f32(pL), f32(pH), g, Physics(), S.Params(n_iter=10))
    Z, R = (host(x)[0] for x in dect.solve(cuda(pL[None]), cuda(pH[None]), g,
                                           dect.default_params(n_iter=10, storage=storage)))
    a = accuracy(Z, R, Zr, Rr, ph, g)
    report(f"storage={storage} small K=10", a)
    check_bf16(a, storage)


@pytest.mark.parametrize("storage", [bf16_case("slice512", 1), bf16_case("slice512", 2)])
def test_bf16_slice512_against_stored_oracle(storage):
    gold = np.load(os.path.join(HERE, "golden", "slice512_K50.npz"))
    g, ph, pL, pH = workload("slice512")
    Z, R = (host(x)[0] for x in dect.solve(cuda(pL[None]), cuda(pH[None]), g,
                                           dect.default_params(n_iter=50, storage=storage)))
    a = accuracy(Z, R, gold["Z"].astype(np.float64), gold["rho"].astype(np.float64), ph, g)
    report(f"storage={storage} slice512 K=50", a)
    check_bf16(a, storage)
