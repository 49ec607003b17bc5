"""Continuous batching: requests of different geometry and iteration budget
enter and leave a slot pool while others are mid-solve; each result must equal
the same slice solved alone."""
import numpy as np
import pytest

from oracle.physics import Physics
from paper_2308_01290_amd import dect
from paper_2308_01290_amd import phantoms as P
from tests.gpu_util import cuda, host

pytestmark = pytest.mark.gpu


def requests():
    phys = Physics()
    specs = [(120, 200, 0.0, 3), (180, 256, 0.3, 5), (150, 300, -0.2, 4), (240, 220, 0.1, 2),
             (200, 280, 0.0, 6)]
    out = []
    for i, (v, d, off, K) in enumerate(specs):
        g = P.FanGeometry(n_x=128, n_y=128, pixel_mm=1.0, n_views=v, n_det=d, sid_mm=1000.0,
                          sdd_mm=1500.0, det_offset_mm=off, angle0_rad=0.1 * i).resolved()
        ph = P.phantom_disk_inserts(seed=40 + i)
        pL, pH = P.analytic_sinograms(ph, g, phys.mu_pair)
        out.append((g, P.poisson_log(pL, 1e5, 50 + i).astype(np.float32),
                    P.poisson_log(pH, 1e5, 60 + i).astype(np.float32), K))
    return out


def test_requests_in_the_mix_equal_each_alone():
    reqs = requests()
    eng = dect.Engine(128, 128, 1.0, slots=3, max_views=240, max_det=300)
    pending = list(range(len(reqs)))
    slot_of, results = {}, {}
    steps = 0
    while len(results) < len(reqs):
        # admit while slots are free (later requests join slots mid-solve of others)
        while pending and (steps > 0 or len(slot_of) < 2):
            i = pending[0]
            g, pL, pH, K = reqs[i]
            s = eng.admit(g, cuda(pL), cuda(pH), K)
            if s is None:
                break
            slot_of[s] = i
            pending.pop(0)
        eng.step()
        steps += 1
        for s, Z, R in eng.completed():
            results[slot_of.pop(s)] = (host(Z), host(R))
        assert steps < 100
    for i, (g, pL, pH, K) in enumerate(reqs):
        Z1, R1 = (host(x)[0] for x in dect.solve(cuda(pL[None]), cuda(pH[None]), g,
                                                  dect.default_params(n_iter=K)))
        assert np.array_equal(results[i][0], Z1) and np.array_equal(results[i][1], R1), i


def test_engine_rejects_what_it_cannot_hold():
    eng = dect.Engine(128, 128, 1.0, slots=1, max_views=100, max_det=128)
    g, pL, pH, K = requests()[0]            # 120 views > 100
    with pytest.raises(dect.DectError):
        eng.admit(g, cuda(pL), cuda(pH), K)
    small = P.FanGeometry(n_x=128, n_y=128, pixel_mm=1.0, n_views=90, n_det=128, sid_mm=1000.0,
                          sdd_mm=1500.0).resolved()
    z = np.zeros((90, 128), np.float32)
    assert eng.admit(small, cuda(z), cuda(z), 2) == 0
    assert eng.admit(small, cuda(z), cuda(z), 2) is None   # the only slot is busy
    assert eng.status() == (1, 0)


def test_multi_iteration_steps_stop_at_a_completion_and_equal_each_alone():
    reqs = requests()
    eng = dect.Engine(128, 128, 1.0, slots=3, max_views=240, max_det=300)
    pending = list(range(len(reqs)))
    slot_of, results, runs = {}, {}, []
    while len(results) < len(reqs):
        while pending:
            i = pending[0]
            g, pL, pH, K = reqs[i]
            s = eng.admit(g, cuda(pL), cuda(pH), K)
            if s is None:
                break
            slot_of[s] = i
            pending.pop(0)
        n = eng.step(4)
        runs.append(n)
        assert 1 <= n <= 4
        done = eng.completed()
        for s, Z, R in done:
            results[slot_of.pop(s)] = (host(Z), host(R))
        # a step shorter than asked ends with a completion
        assert n == 4 or done
        assert len(runs) < 60
    # budgets 3, 5, 4, 2, 6 in 3 slots: the first step stops at the first completion (3)
    assert runs[0] == 3
    for i, (g, pL, pH, K) in enumerate(reqs):
        Z1, R1 = (host(x)[0] for x in dect.solve(cuda(pL[None]), cuda(pH[None]), g,
                                                  dect.default_params(n_iter=K)))
        assert np.array_equal(results[i][0], Z1) and np.array_equal(results[i][1], R1), i
    assert eng.step(4) == 0
    with pytest.raises(dect.DectError):
        eng.step(0)


def test_server_with_two_sizes_threads_equal_each_alone():
    """The server steps its per-size engines from one host thread each; every
    result must still equal the slice solved alone."""
    from paper_2308_01290_amd.serve import EngineSpec, Request, Server
    phys = Physics()
    reqs = []
    for i, (n, v, d, K) in enumerate([(64, 96, 120, 3), (96, 120, 160, 4), (64, 80, 100, 5),
                                      (96, 100, 150, 2), (64, 96, 110, 4)]):
        g = P.FanGeometry(n_x=n, n_y=n, pixel_mm=1.0, n_views=v, n_det=d, sid_mm=800.0,
                          sdd_mm=1200.0, det_offset_mm=0.2 * (i % 2)).resolved()
        ph = P.phantom_disk_inserts(seed=70 + i, radius=0.35 * n, n_inserts=3,
                                    semi=(0.04 * n, 0.08 * n))
        pL, pH = P.analytic_sinograms(ph, g, phys.mu_pair)
        reqs.append(Request(g, cuda(P.poisson_log(pL, 1e5, 80 + i).astype(np.float32)),
                            cuda(P.poisson_log(pH, 1e5, 90 + i).astype(np.float32)), K,
                            arrival=0.001 * i, tag=i))
    server = Server([EngineSpec(64, 1.0, 2, 128, 128), EngineSpec(96, 1.0, 2, 128, 192)],
                    iters_per_step=3)
    done = server.run(reqs)
    assert len(done) == len(reqs)
    for r in done:
        Z1, R1 = (host(x)[0] for x in dect.solve(r.sino_lo[None], r.sino_hi[None], r.geom,
                                                  dect.default_params(n_iter=r.n_iter)))
        assert np.array_equal(host(r.Z), Z1) and np.array_equal(host(r.rho), R1), r.tag


def test_server_budget_admission_and_cancel_equal_each_alone():
    """An HBM budget that holds one engine at a time: the two sizes take turns
    (the idle engine is retired to make room), a request cancelled mid-solve
    never writes its maps, a queued one is dropped, and every completed
    result equals the slice solved alone."""
    from paper_2308_01290_amd.serve import CANCELLED, DONE, EngineSpec, Request, Server
    phys = Physics()
    specs = [EngineSpec(64, 1.0, 2, 128, 128), EngineSpec(96, 1.0, 2, 128, 192)]
    lib = dect.lib()
    params = dect.default_params()
    nbytes = [lib.dect_engine_workspace_bytes(s.n, s.n, s.pixel_mm, s.slots, s.max_views, s.max_det,
                                              params) for s in specs]
    budget = max(nbytes) + min(nbytes) // 2
    reqs = []
    for i, (n, v, d, K) in enumerate([(64, 96, 120, 6), (96, 120, 160, 3), (64, 80, 100, 2),
                                      (96, 100, 150, 2), (64, 96, 110, 3)]):
        g = P.FanGeometry(n_x=n, n_y=n, pixel_mm=1.0, n_views=v, n_det=d, sid_mm=800.0,
                          sdd_mm=1200.0).resolved()
        ph = P.phantom_disk_inserts(seed=170 + i, radius=0.35 * n, n_inserts=3,
                                    semi=(0.04 * n, 0.08 * n))
        pL, pH = P.analytic_sinograms(ph, g, phys.mu_pair)
        reqs.append(Request(g, cuda(P.poisson_log(pL, 1e5, 180 + i).astype(np.float32)),
                            cuda(P.poisson_log(pH, 1e5, 190 + i).astype(np.float32)), K, tag=i))
    server = Server(specs, hbm_budget_bytes=budget, iters_per_step=2)
    for r in reqs:
        assert server.submit(r)
    t = [0.0]
    clock = lambda: t[0]  # noqa: E731
    server.step(clock)                       # 64^2 engine: requests 0 and 2 running
    assert reqs[0].status == "running" and reqs[1].status == "queued"
    assert server.cancel(reqs[0])            # mid-solve (2 of its 6 iterations done)
    assert server.cancel(reqs[4])            # still queued
    while server.pending():
        t[0] += 1.0
        server.step(clock)
        assert server.hbm_bytes <= budget
    assert server.hbm_peak <= budget and server.engines_retired >= 1
    assert reqs[0].status == CANCELLED and reqs[0].Z is None
    assert reqs[4].status == CANCELLED and reqs[4].Z is None
    for r in (reqs[1], reqs[2], reqs[3]):
        assert r.status == DONE
        Z1, R1 = (host(x)[0] for x in dect.solve(r.sino_lo[None], r.sino_hi[None], r.geom,
                                                  dect.default_params(n_iter=r.n_iter)))
        assert np.array_equal(host(r.Z), Z1) and np.array_equal(host(r.rho), R1), r.tag
    server.close()
