"""Graph replay of the t' PCG's first chunk in every outer iteration: a solver
with graphs enabled must give exactly the results of the same solver launching
every kernel itself, on every replay of its graphs, with other GPU work and
synchronisations in between."""
import numpy as np
import pytest
import torch

from oracle.physics import Physics
from paper_2308_01290_amd import dect
from paper_2308_01290_amd import phantoms as P
from tests.gpu_util import cuda, host, workload
from tests.test_gpu_batch import uneven_inputs

pytestmark = pytest.mark.gpu


def run(sol, lo, hi, k):
    sol.init(lo, hi).iterate(k)
    Z, R = (host(x) for x in sol.finish())
    return Z, R, sol.stats()


def eager_work_between(g):
    x = cuda(np.ones((1, g.n_y, g.n_x), np.float32))
    dect.project(g, x)
    torch.cuda.synchronize()


@pytest.mark.parametrize("name,k", [("small", 10), ("slice512", 50)])
def test_graph_replays_equal_eager_solve(name, k):
    g, _, pL, pH = workload(name)
    params = dect.default_params(n_iter=k)
    lo, hi = cuda(pL[None]), cuda(pH[None])
    Ze, Re, se = run(dect.Solver(g, params), lo, hi, k)
    sol = dect.Solver(g, params).set_graphs(True)
    for rep in range(3):
        Zg, Rg, sg = run(sol, lo, hi, k)
        assert np.array_equal(Zg, Ze) and np.array_equal(Rg, Re), (name, rep)
        assert sg == se, (name, rep)
        eager_work_between(g)


def test_graphs_across_iterate_calls_and_toggling():
    g, _, pL, pH = workload("small")
    params = dect.default_params(n_iter=10)
    lo, hi = cuda(pL[None]), cuda(pH[None])
    Ze, Re, _ = run(dect.Solver(g, params), lo, hi, 10)
    sol = dect.Solver(g, params).set_graphs(True)
    sol.init(lo, hi).iterate(3)
    sol.set_graphs(False).iterate(2)
    sol.set_graphs(True).iterate(5)
    Z, R = (host(x) for x in sol.finish())
    assert np.array_equal(Z, Ze) and np.array_equal(R, Re)


def test_graphs_uneven_batch():
    data = uneven_inputs()
    geoms = [d[0] for d in data]
    params = dect.default_params(n_iter=4)
    lo = dect.concat_sinograms([cuda(d[1]) for d in data])
    hi = dect.concat_sinograms([cuda(d[2]) for d in data])
    Ze, Re, se = run(dect.Solver(geoms, params), lo, hi, 4)
    sol = dect.Solver(geoms, params).set_graphs(True)
    for rep in range(2):
        Zg, Rg, sg = run(sol, lo, hi, 4)
        assert np.array_equal(Zg, Ze) and np.array_equal(Rg, Re), rep
        assert sg == se, rep
        eager_work_between(geoms[0])


def test_graphs_image_form():
    phys = Physics()
    g, _, L, H = P.workload_image_small(phys.mu_pair)
    lo, hi = (cuda(np.asarray(a, np.float32)[None]) for a in (L, H))
    params = dect.default_params(n_iter=10)
    Ze, Re, se = run(dect.ImageSolver(g.n_x, g.n_y, params), lo, hi, 10)
    sol = dect.ImageSolver(g.n_x, g.n_y, params).set_graphs(True)
    for rep in range(2):
        Zg, Rg, sg = run(sol, lo, hi, 10)
        assert np.array_equal(Zg, Ze) and np.array_equal(Rg, Re), rep
        assert sg == se, rep
        eager_work_between(g)


@pytest.mark.parametrize("storage", [dect.DECT_STORAGE_BF16, dect.DECT_STORAGE_BF16_STATE])
def test_graphs_with_bf16_storage(storage):
    g, _, pL, pH = workload("small")
    params = dect.default_params(n_iter=6, storage=storage)
    lo, hi = cuda(pL[None]), cuda(pH[None])
    Ze, Re, se = run(dect.Solver(g, params), lo, hi, 6)
    sol = dect.Solver(g, params).set_graphs(True)
    for rep in range(2):
        Zg, Rg, sg = run(sol, lo, hi, 6)
        assert np.array_equal(Zg, Ze) and np.array_equal(Rg, Re), (storage, rep)
        assert sg == se
        eager_work_between(g)
