"""Scheduling of the serving loop on the CPU: HBM-budget admission, engines
created and retired against the budget, rejection of requests that can never
run, and cancellation of queued and running requests.  A stand-in engine
counts outer iterations the way dect_engine_step_n does (a step of n
iterations stops at the first slot to complete); the numerics are the
library's and are tested on the GPU."""
from types import SimpleNamespace

import pytest

from paper_2308_01290_amd.serve import (CANCELLED, DONE, REJECTED, EngineSpec, Request,
                                        Server)


class FakeEngine:
    live = 0

    def __init__(self, spec):
        self.spec = spec
        self.k = {}            # slot -> [iterations done, budget]
        self.done = []
        self.closed = False
        FakeEngine.live += 1

    def admit(self, geom, lo, hi, n_iter):
        free = [s for s in range(self.spec.slots) if s not in self.k]
        if not free:
            return None
        self.k[free[0]] = [0, int(n_iter)]
        return free[0]

    def step(self, n):
        if not self.k:
            return 0
        m = min(n, min(K - k for k, K in self.k.values()))
        for s in list(self.k):
            self.k[s][0] += m
            if self.k[s][0] >= self.k[s][1]:
                del self.k[s]
                self.done.append(s)
        return m

    def completed(self):
        out = [(s, ("Z", s), ("rho", s)) for s in self.done]
        self.done = []
        return out

    def cancel(self, slot):
        if slot not in self.k:
            raise ValueError("slot holds no request")
        del self.k[slot]

    def close(self):
        assert not self.closed
        self.closed = True
        FakeEngine.live -= 1


BYTES = {64: 100, 96: 150}


def server(budget, slots=2, iters=3):
    FakeEngine.live = 0
    specs = [EngineSpec(64, 1.0, slots, 128, 128), EngineSpec(96, 1.0, slots, 128, 192)]
    return Server(specs, params=object(), hbm_budget_bytes=budget, iters_per_step=iters,
                  engine_factory=FakeEngine, engine_bytes=lambda sp: BYTES[sp.n], sync=lambda: None)


def req(n, K, views=100, det=100, arrival=0.0, tag=None):
    g = SimpleNamespace(n_x=n, n_y=n, n_views=views, n_det=det)
    return Request(g, None, None, K, arrival=arrival, tag=tag)


def drive(srv, reqs, max_steps=200):
    for r in reqs:
        srv.submit(r)
    steps = 0
    held = []
    while srv.pending():
        srv.step(lambda: float(steps))
        held.append(srv.hbm_bytes)
        steps += 1
        assert steps < max_steps
    return held


def test_budget_zero_rejects_every_request():
    srv = server(0)
    reqs = [req(64, 3), req(96, 2)]
    out = srv.run(reqs)
    assert all(r.status == REJECTED and "budget" in r.reason for r in out)
    assert srv.engines_created == 0 and srv.hbm_bytes == 0


def test_requests_beyond_slot_capacity_or_without_engine_are_rejected():
    srv = server(1000)
    a, b, c = req(64, 3, views=129), req(96, 3, det=193), req(128, 3)
    for r in (a, b, c):
        assert srv.submit(r) is False and r.status == REJECTED
    assert "slot capacity" in a.reason and "slot capacity" in b.reason and "no engine" in c.reason
    assert srv.pending() == 0


def test_budget_for_one_engine_serialises_sizes_and_never_exceeds_it():
    """Budget 160: one engine of either size fits, never both.  The 96^2
    requests wait until the 64^2 engine is idle and retired."""
    srv = server(160)
    reqs = [req(64, 4, tag=0), req(64, 2, tag=1), req(96, 3, tag=2), req(64, 5, tag=3), req(96, 1, tag=4)]
    held = drive(srv, reqs)
    assert max(held) <= 160 and srv.hbm_peak <= 160
    assert all(r.status == DONE for r in reqs)
    assert srv.engines_created >= 2 and srv.engines_retired >= 1
    # while a 64^2 request runs no 96^2 engine can exist: sizes never overlap
    for a in reqs:
        for b in reqs:
            if a.geom.n_x != b.geom.n_x:
                assert a.finished <= b.admitted or b.finished <= a.admitted, (a.tag, b.tag)


def test_budget_for_both_sizes_runs_them_together():
    srv = server(250)
    reqs = [req(64, 4), req(96, 4), req(64, 3), req(96, 2)]
    drive(srv, reqs)
    assert srv.hbm_peak == 250 and srv.engines_retired == 0
    assert all(r.status == DONE for r in reqs)
    assert max(r.admitted for r in reqs) == 0.0     # all four admitted at once (two slots each)


def test_more_engines_of_one_size_when_the_budget_allows():
    srv = server(1000, slots=1)
    reqs = [req(64, 3) for _ in range(5)]
    drive(srv, reqs)
    assert srv.engines_created == 5 and srv.hbm_peak == 500
    assert all(r.status == DONE for r in reqs)


def test_cancel_queued_and_running_requests():
    srv = server(100, slots=1)          # one 64^2 engine with one slot
    a, b, c = req(64, 6, tag="a"), req(64, 2, tag="b"), req(64, 2, tag="c")
    for r in (a, b, c):
        srv.submit(r)
    srv.step(lambda: 0.0)               # a admitted, 3 of its 6 iterations run
    assert a.status == "running" and b.status == "queued"
    assert srv.cancel(b) and b.status == CANCELLED       # queued
    assert srv.cancel(a) and a.status == CANCELLED       # mid-solve
    assert not srv.cancel(a)
    t = 1
    while srv.pending():
        srv.step(lambda: float(t))
        t += 1
    assert c.status == DONE and c.Z == ("Z", 0)          # the freed slot served c
    assert a.Z is None and b.Z is None and a.finished is None
    assert [r.tag for r in srv.done if r.status == CANCELLED] == ["b", "a"]


def test_run_cancels_at_the_given_time():
    srv = server(1000, slots=2, iters=1)
    reqs = [req(64, 50, arrival=0.0), req(64, 2, arrival=0.0)]
    out = srv.run(reqs, cancel_at={0: 0.0})
    assert out[0].status == CANCELLED and out[1].status == DONE


@pytest.mark.parametrize("budget", [99, 100])
def test_engine_exactly_at_the_budget(budget):
    srv = server(budget)
    r = req(64, 1)
    ok = srv.submit(r)
    assert ok == (budget >= 100)
