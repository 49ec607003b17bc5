"""GPU parity of the image-domain form of Algorithm 1 (the FFT closed forms of
the f-subproblem on attenuation images) against the FP64 oracle."""
import os

import numpy as np
import pytest

from oracle import image as I
from oracle.physics import Physics
from oracle.solve import Params, State
from paper_2308_01290_amd import dect
from paper_2308_01290_amd import phantoms as P
from tests import ht_flips as HF
from tests.gpu_util import cuda, host, rel_inf
from tests.test_gpu_solver import check_end_to_end, phantom_body

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def small():
    phys = Physics()
    g, ph, L, H = P.workload_image_small(phys.mu_pair)
    return phys, g, ph, f32(L), f32(H)


def grid_case(ny, nx, seed):
    """Noisy attenuation images of a disk phantom on an ny x nx / 1 mm grid."""
    phys = Physics()
    g = P.FanGeometry(n_x=nx, n_y=ny, pixel_mm=1.0, n_views=8, n_det=8, sid_mm=1000.0,
                      sdd_mm=1500.0)
    r = 0.42 * min(nx, ny)
    n_ins = 3 if min(nx, ny) >= 24 else 1
    ph = P.phantom_disk_inserts(seed=seed, radius=r, n_inserts=n_ins, semi=(0.08 * r, 0.18 * r))
    L, H = P.noisy_mu_pair(ph, g, phys.mu_pair, seed + 1)
    return phys, f32(L), f32(H)


def lib_params(n_iter, **kw):
    return dect.default_params(n_iter=n_iter, **kw)


def body_mask(rho_ref, rho_got, rho_min=0.1, margin=0.02):
    return (rho_ref >= rho_min + margin) & (rho_got >= rho_min + margin)


def run_one(phys, L, H, st0, k, precond=0):
    sol = dect.ImageSolver(L.shape[1], L.shape[0], lib_params(10, t_precond=precond))
    sol.set_state(cuda(L[None]), cuda(H[None]), *(cuda(a[None]) for a in (st0.f1, st0.f2, st0.rho, st0.t)),
                  k=k)
    sol.iterate(1)
    return [host(a)[0] for a in sol.state()]


def f32_state(st, beta, k):
    return State(f32(st.f1), f32(st.f2), f32(st.rho), f32(st.t), beta, k)


def check_iteration(got, ref, st0, L, H, phys, params, t_mask, tag, t_tol):
    """One iteration against the oracle's, with the near-tie allowances of
    eq. (9) (the f allowance from the joint 2x2 solve of (13a))."""
    _, Hm = I.f_system(st0, L, H, phys, params)
    counts, allow = HF.iteration_allowances(st0, phys, params, image_H=Hm)
    HF.assert_iteration_close(got, ref, st0, counts, allow, t_mask, tag, t_tol=t_tol)


def test_init_matches_oracle():
    phys, g, ph, L, H = small()
    params = I.resolved(Params(n_iter=10), phys)
    st = I.init_from_mu(L, H, phys, params)
    sol = dect.ImageSolver(g.n_x, g.n_y, lib_params(10)).init(cuda(L[None]), cuda(H[None]))
    f1, f2, rho, t = (host(a)[0] for a in sol.state())
    assert rel_inf(f1, st.f1) <= 1e-5 and rel_inf(f2, st.f2) <= 1e-5
    assert rel_inf(rho, st.rho) <= 1e-5
    m = body_mask(st.rho, rho) & (np.abs(phys.W(*phys.synth(st.f1, st.f2)) / phys.W_water()) > 0.3)
    assert np.abs(t - st.t)[m].max() <= 1e-3 * max(1.0, np.abs(st.t[m]).max())


@pytest.mark.parametrize("precond", [0, 1, 2, 3])
@pytest.mark.parametrize("k", [0, 7])
def test_one_iteration_matches_oracle(k, precond):
    """From an identical FP32 state, one outer iteration (both f closed forms,
    rho step, t' step, beta update) equals the oracle's."""
    phys, g, ph, L, H = small()
    params = I.resolved(Params(n_iter=10), phys)
    st0 = I.init_from_mu(L, H, phys, params)
    beta = params.beta0 * params.kappa ** k
    st0 = f32_state(st0, beta, k)
    ref = I.iterate(st0, L, H, phys, params)
    got = run_one(phys, L, H, st0, k, precond)
    check_iteration(got, ref, st0, L, H, phys, params, body_mask(ref.rho, got[2]),
                    f"image k={k} precond={precond}", 2e-3)


# non-square grids, several FFT tiles and radix-3 sides; (48, 24): the
# multigrid V-cycle cannot coarsen 24, the automatic choice falls back
@pytest.mark.parametrize("shape", [(96, 64), (64, 192), (48, 24), (8, 16)])
def test_one_iteration_ragged_matches_oracle(shape):
    ny, nx = shape
    phys, L, H = grid_case(ny, nx, seed=ny + nx)
    params = I.resolved(Params(n_iter=10), phys)
    st0 = f32_state(I.init_from_mu(L, H, phys, params), params.beta0 * params.kappa ** 3, 3)
    ref = I.iterate(st0, L, H, phys, params)
    got = run_one(phys, L, H, st0, 3)
    check_iteration(got, ref, st0, L, H, phys, params, body_mask(ref.rho, got[2]), f"image {shape}", 2e-3)


def test_lockstep_small_all_iterations():
    """Every outer iteration of the oracle's own trajectory, replayed on the GPU
    from the oracle's FP32-rounded state."""
    phys, g, ph, L, H = small()
    params = I.resolved(Params(n_iter=10), phys)
    _, body = phantom_body(ph, g)
    st = I.init_from_mu(L, H, phys, params)
    for k in range(params.n_iter):
        s32 = f32_state(st, st.beta, k)
        ref = I.iterate(s32, L, H, phys, params)
        got = run_one(phys, L, H, s32, k)
        check_iteration(got, ref, s32, L, H, phys, params, body, f"image lockstep k={k}", 5e-4)
        st = ref


def test_full_solve_small_matches_oracle():
    phys, g, ph, L, H = small()
    Zr, Rr = I.solve(L, H, phys, Params(n_iter=10))
    Z, R = dect.solve_image(cuda(L[None]), cuda(H[None]), lib_params(10))
    check_end_to_end(host(Z)[0], host(R)[0], Zr, Rr, ph, g, "image small K=10")


def test_batch_equals_single_and_solver_matches_solve():
    """A slice alone equals the same slice inside a batch (bitwise), and the
    stepwise solver equals the whole-solve entry point (bitwise)."""
    phys, g, ph, L, H = small()
    lo = np.stack([L, 0.9 * L, L])
    hi = np.stack([H, 0.9 * H, H])
    Zb, Rb = (host(x) for x in dect.solve_image(cuda(lo), cuda(hi), lib_params(4)))
    Z1, R1 = (host(x) for x in dect.solve_image(cuda(L[None]), cuda(H[None]), lib_params(4)))
    assert np.array_equal(Zb[0], Z1[0]) and np.array_equal(Rb[0], R1[0])
    assert np.array_equal(Zb[2], Z1[0]) and not np.array_equal(Zb[1], Z1[0])
    sol = dect.ImageSolver(g.n_x, g.n_y, lib_params(4)).init(cuda(L[None]), cuda(H[None])).iterate(4)
    Zs, Rs = (host(x) for x in sol.finish())
    assert np.array_equal(Zs, Z1) and np.array_equal(Rs, R1)
    assert sol.stats()[0] == 4


def test_wrong_form_entry_points_rejected():
    phys, g, ph, L, H = small()
    sol = dect.ImageSolver(g.n_x, g.n_y, lib_params(2))
    with pytest.raises(dect.DectError, match="image-domain"):
        dect._check(dect.lib().dect_solver_init(sol._h, dect._ptr(cuda(L[None])), dect._ptr(cuda(H[None]))),
                    "dect_solver_init")
    sino = dect.Solver(g, lib_params(2))
    with pytest.raises(dect.DectError, match="not an image-domain solver"):
        dect._check(dect.lib().dect_image_solver_init(sino._h, dect._ptr(cuda(L[None])),
                                                      dect._ptr(cuda(H[None]))), "dect_image_solver_init")


def test_full_solve_image512_matches_stored_oracle():
    """512^2 attenuation image pair, 50 iterations, against the stored oracle
    result written by tests/golden/make_golden.py image512 (oracle only)."""
    path = os.path.join(HERE, "golden", "image512_K50.npz")
    gold = np.load(path)
    phys = Physics()
    g, ph, L, H = P.workload_image512(phys.mu_pair)
    Z, R = dect.solve_image(cuda(L[None]), cuda(H[None]), lib_params(50))
    check_end_to_end(host(Z)[0], host(R)[0], gold["Z"].astype(np.float64), gold["rho"].astype(np.float64),
                     ph, g, "image512 K=50")
