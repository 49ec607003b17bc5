"""Oracle parity of the batched and served forms on the geometries they run:
four slices of the uneven batch (image 256, 384, 384, 512; 984, 360, 720,
984 views; 882, 535, 864, 829 bins) and two served requests (768^2 with 1152
views, 256^2 with 360 views).

Per geometry, one outer iteration from the oracle's own FP32-rounded start
is compared step by step (near-tie allowances of eq. (9)).  End to end, the
slices are solved as the batched and served paths run them (slices of one
image size in one uneven batch; requests through the server's engines) and
compared with the stored oracle results (tests/golden/make_golden.py uneven
served, oracle only) by the whole-body rule of tests/e2e.py."""
import os

import numpy as np
import pytest

from oracle import solve as S
from oracle.physics import Physics
from paper_2308_01290_amd import dect
from paper_2308_01290_amd import phantoms as P
from tests import ht_flips as HF
from tests.golden.make_golden import SERVED, SERVED_K, UNEVEN_SEEDS
from tests.gpu_util import cuda, host
from tests.test_gpu_solver import check_end_to_end

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def gold(name):
    d = np.load(os.path.join(HERE, "golden", name))
    return d["Z"].astype(np.float64), d["rho"].astype(np.float64), int(d["n_iter"])


def uneven_case(seed):
    phys = Physics()
    g, ph, pL, pH = P.slice_uneven(seed, phys.mu_pair)
    return phys, g, ph, pL.astype(np.float32), pH.astype(np.float32)


def served_case(n, seed, views):
    phys = Physics()
    g, ph, pL, pH = P.slice_served(n, seed, phys.mu_pair, n_views=views)
    return phys, g, ph, pL.astype(np.float32), pH.astype(np.float32)


def lockstep_first(phys, g, ph, pL, pH, n_iter, tag):
    from tests.e2e import body_mask
    params = S.Params(n_iter=n_iter).resolved(phys, g)
    st = S.init_state(f32(pL), f32(pH), g, phys, params)
    s32 = S.State(f32(st.f1), f32(st.f2), f32(st.rho), f32(st.t), st.beta, 0)
    ref = S.iterate(s32, f32(pL), f32(pH), g, phys, params)
    sol = dect.Solver(g, dect.default_params(n_iter=n_iter)).set_state(
        cuda(pL[None]), cuda(pH[None]), *(cuda(a[None]) for a in (s32.f1, s32.f2, s32.rho, s32.t)), k=0)
    sol.iterate(1)
    got = [host(a)[0] for a in sol.state()]
    _, body = body_mask(ph, g)
    counts, allow = HF.iteration_allowances(
        s32, phys, params, f_alpha=lambda: HF.sino_alpha(s32, f32(pL), f32(pH), g, phys, params))
    HF.assert_iteration_close(got, ref, s32, counts, allow, body, tag)


@pytest.mark.parametrize("seed", UNEVEN_SEEDS)
def test_uneven_slice_first_iteration_matches_oracle(seed):
    phys, g, ph, pL, pH = uneven_case(seed)
    lockstep_first(phys, g, ph, pL, pH, 50, f"uneven {seed} ({g.n_x}^2, {g.n_views}x{g.n_det}) k=0")


@pytest.mark.parametrize("n,seed,views", SERVED)
def test_served_geometry_first_iteration_matches_oracle(n, seed, views):
    phys, g, ph, pL, pH = served_case(n, seed, views)
    lockstep_first(phys, g, ph, pL, pH, SERVED_K, f"served {n}^2 {views}x{g.n_det} k=0")


def test_uneven_batch_matches_stored_oracle():
    """The four slices solved as the uneven-batch path runs them: one handle
    for the mixed image sizes (both 384^2 slices in one launch per kernel and
    iteration, the three image-size groups iterated together), 50 iterations."""
    cases = [uneven_case(seed) for seed in UNEVEN_SEEDS]
    geoms = [c[1] for c in cases]
    lo = dect.concat_sinograms([cuda(c[3]) for c in cases])
    hi = dect.concat_sinograms([cuda(c[4]) for c in cases])
    sol = dect.UnevenSolver(geoms, dect.default_params(n_iter=50))
    assert sol.groups() == 3
    Z, R = sol.init(lo, hi).iterate(50).finish()
    Zs, Rs = dect.split_images(Z, geoms), dect.split_images(R, geoms)
    for i, (seed, (phys, g, ph, _, _)) in enumerate(zip(UNEVEN_SEEDS, cases)):
        Zr, Rr, K = gold(f"uneven_{seed}_K50.npz")
        assert K == 50
        check_end_to_end(host(Zs[i]), host(Rs[i]), Zr, Rr, ph, g,
                         f"uneven {seed} ({g.n_x}^2, {g.n_views}x{g.n_det})")


def test_served_requests_match_stored_oracle():
    """The two requests through the server (one engine per image size, the
    requests admitted mid-stream as the serving path runs them)."""
    from paper_2308_01290_amd.serve import DONE, EngineSpec, Request, Server
    cases = [served_case(n, seed, views) for n, seed, views in SERVED]
    specs = [EngineSpec(n, 0.8, 4, 1152, 1024) for n, _, _ in SERVED]
    server = Server(specs, iters_per_step=4)
    reqs = [Request(g, cuda(pL), cuda(pH), SERVED_K, arrival=0.0, tag=i)
            for i, (phys, g, ph, pL, pH) in enumerate(cases)]
    server.run(reqs)
    for r, (n, seed, views), (phys, g, ph, _, _) in zip(reqs, SERVED, cases):
        assert r.status == DONE
        Zr, Rr, K = gold(f"served_{n}_{views}_K{SERVED_K}.npz")
        assert K == SERVED_K
        check_end_to_end(host(r.Z), host(r.rho), Zr, Rr, ph, g, f"served {n}^2 {views} views K={K}")
    server.close()
