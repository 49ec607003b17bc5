"""Launch schedules and the autotuner: every schedule maps the same
operations onto the device differently, so every one of them must give the
default schedule's results bit for bit, and a solve after autotuning must
equal a solve without it."""
import numpy as np
import pytest

from paper_2308_01290_amd import dect
from tests.gpu_util import cuda, host, workload
from tests.test_gpu_batch import uneven_inputs

pytestmark = pytest.mark.gpu

DEFAULT = {"fp_rays_per_lane": 4, "bp_cu_percent": 0, "rho_stream": 1, "graphs": 0,
           "pcg_chunk_extra": 0, "pcg_chunk_first": 1}

VARIANTS = [
    {"fp_rays_per_lane": 1},
    {"bp_cu_percent": 25},
    {"bp_cu_percent": 100},
    {"bp_cu_percent": 400},
    {"rho_stream": 0},
    {"graphs": 1},
    {"pcg_chunk_extra": 3},
    {"pcg_chunk_first": 0},
    {"fp_rays_per_lane": 1, "bp_cu_percent": 10, "rho_stream": 0, "graphs": 1, "pcg_chunk_extra": 8,
     "pcg_chunk_first": 0},
]


def solve(sol, lo, hi, k):
    sol.init(lo, hi).iterate(k)
    Z, R = (host(x) for x in sol.finish())
    return Z, R, sol.stats()


def small_case():
    g, _, pL, pH = workload("small")
    return g, cuda(pL[None]), cuda(pH[None])


def uneven_case():
    data = uneven_inputs()
    geoms = [d[0] for d in data]
    lo = dect.concat_sinograms([cuda(d[1]) for d in data])
    hi = dect.concat_sinograms([cuda(d[2]) for d in data])
    return geoms, lo, hi


def test_new_solver_has_the_default_schedule():
    g, _, _ = small_case()
    assert dect.Solver(g, dect.default_params(n_iter=2)).schedule() == DEFAULT


@pytest.mark.parametrize("case", ["small", "uneven"])
def test_every_schedule_gives_identical_results(case):
    g, lo, hi = small_case() if case == "small" else uneven_case()
    params = dect.default_params(n_iter=6)
    ref = solve(dect.Solver(g, params), lo, hi, 6)
    sol = dect.Solver(g, params)
    for v in VARIANTS:
        sol.set_schedule(**{**DEFAULT, **v})
        got = solve(sol, lo, hi, 6)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), v
        assert got[2] == ref[2], v


def test_slice512_schedules_identical():
    g, _, pL, pH = workload("slice512")
    lo, hi = cuda(pL[None]), cuda(pH[None])
    params = dect.default_params(n_iter=5)
    ref = solve(dect.Solver(g, params), lo, hi, 5)
    sol = dect.Solver(g, params)
    for v in ({"fp_rays_per_lane": 1}, {"bp_cu_percent": 100, "rho_stream": 0, "graphs": 1}):
        sol.set_schedule(**{**DEFAULT, **v})
        got = solve(sol, lo, hi, 5)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), v


@pytest.mark.parametrize("case", ["small", "uneven"])
def test_autotune_keeps_results(case):
    g, lo, hi = small_case() if case == "small" else uneven_case()
    params = dect.default_params(n_iter=6)
    ref = solve(dect.Solver(g, params), lo, hi, 6)
    sol = dect.Solver(g, params)
    chosen, ms = sol.autotune(lo, hi, iters=3, reps=2)
    assert sol.schedule() == chosen and ms > 0.0
    got = solve(sol, lo, hi, 6)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), chosen


def test_autotune_image_form():
    from oracle.physics import Physics
    from paper_2308_01290_amd import phantoms as P
    g, _, L, H = P.workload_image_small(Physics().mu_pair)
    lo, hi = (cuda(np.asarray(a, np.float32)[None]) for a in (L, H))
    params = dect.default_params(n_iter=6)
    ref = solve(dect.ImageSolver(g.n_x, g.n_y, params), lo, hi, 6)
    sol = dect.ImageSolver(g.n_x, g.n_y, params)
    chosen, _ = sol.autotune(lo, hi, iters=3, reps=2)
    got = solve(sol, lo, hi, 6)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), chosen


@pytest.mark.parametrize("bad", [{"fp_rays_per_lane": 2}, {"bp_cu_percent": 5},
                                 {"bp_cu_percent": 401}, {"rho_stream": 2}, {"graphs": -1},
                                 {"pcg_chunk_extra": 9}, {"pcg_chunk_first": 2}])
def test_schedule_values_out_of_range_rejected(bad):
    g, lo, hi = small_case()
    sol = dect.Solver(g, dect.default_params(n_iter=2))
    with pytest.raises(dect.DectError):
        sol.set_schedule(**bad)
    assert sol.schedule() == DEFAULT
    with pytest.raises(dect.DectError):
        sol.autotune(lo, hi, iters=0)


def test_iteration_timeline():
    """The timeline has one row per outer iteration after a solve's first,
    its points in stream order, and recording it changes no result bit."""
    g, lo, hi = small_case()
    params = dect.default_params(n_iter=6)
    ref = solve(dect.Solver(g, params), lo, hi, 6)
    sol = dect.Solver(g, params).enable_timing(True, timeline=True)
    got = solve(sol, lo, hi, 6)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    tl = sol.timeline()
    assert tl.shape == (5, 5) and np.isfinite(tl).all()
    grad, fp, upd, setup, done = tl.T
    assert (grad > 0).all() and (grad < fp).all() and (fp < upd).all()
    assert (setup > 0).all() and (setup < done).all()
    assert sol.timeline().shape == (0, 5)   # cleared by the read
    solve(sol, lo, hi, 3)
    solve(sol, lo, hi, 3)
    assert sol.timeline().shape == (4, 5)   # two rows per solve: none across solves


def test_kernel_timing_back_projections_only():
    """Timing the back-projections only records no forward-projection
    intervals and as many back-projection ones; no result bit changes."""
    g, lo, hi = small_case()
    params = dect.default_params(n_iter=6)
    ref = solve(dect.Solver(g, params), lo, hi, 6)
    sol = dect.Solver(g, params).enable_timing(True)
    full = solve(sol, lo, hi, 6)
    bp_ms, bp_n, fp_ms, fp_n = sol.timing()
    sol.enable_timing(True, bp_only=True)
    only = solve(sol, lo, hi, 6)
    bp_ms2, bp_n2, fp_ms2, fp_n2 = sol.timing()
    assert bp_n > 0 and fp_n > 0 and bp_ms > 0.0 and fp_ms > 0.0
    assert bp_n2 == bp_n and bp_ms2 > 0.0 and fp_n2 == 0 and fp_ms2 == 0.0
    for got in (full, only):
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
