"""Serving loop: single-slice solves arriving over time, continuously batched.

Requests of one image size share engines (dect_engine_*): pools of slots on
the device in which each request runs at its own outer iteration.  A request
waits in its size's FIFO queue until a slot is free; it is admitted between
two steps while the other slots are mid-solve, and leaves when its iteration
budget is done (or when it is cancelled).

Device memory is admitted against an HBM budget.  Every engine's workspace
(its slots at their capacity: state images, residual sinograms, ray tables)
is charged to the budget while the engine exists.  Engines are created on
demand, when a request finds no free slot and the new engine's workspace
fits what the budget has left; an engine with no running request is retired
when another size is waiting for budget, which returns its bytes.  A request
that could never fit (its size has no engine specification, its views or
bins exceed the slot capacity, or one engine of its size exceeds the whole
budget) is rejected at submission instead of waiting forever.

The numerics of every request are those of solving it alone; this module
only schedules (argument marshalling and bookkeeping; the work runs in the
library).  The engine constructor, the engine byte count and the device
synchronisation are injectable, so the scheduling can be exercised without a
GPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import Callable, Deque, Dict, List, Optional

QUEUED, RUNNING, DONE, REJECTED, CANCELLED = "queued", "running", "done", "rejected", "cancelled"


@dataclass(eq=False)
class Request:
    geom: object            # FanGeometry / dect.Geometry
    sino_lo: object         # [n_views, n_det] float32 device tensor
    sino_hi: object
    n_iter: int
    arrival: float = 0.0    # seconds on the server's clock
    tag: object = None
    # filled in by the server
    status: Optional[str] = None
    reason: Optional[str] = None
    admitted: Optional[float] = None
    finished: Optional[float] = None
    Z: object = None
    rho: object = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


@dataclass
class EngineSpec:
    n: int                  # image side (pixels)
    pixel_mm: float
    slots: int              # slots per engine of this size
    max_views: int
    max_det: int


class _Pool:
    """One engine and the requests in its slots."""

    def __init__(self, spec: EngineSpec, engine, nbytes: int):
        self.spec, self.engine, self.nbytes = spec, engine, int(nbytes)
        self.running: Dict[int, Request] = {}

    @property
    def free(self) -> int:
        return self.spec.slots - len(self.running)


def _library_engine(spec: EngineSpec, params, device):
    from . import dect
    return dect.Engine(spec.n, spec.n, spec.pixel_mm, spec.slots, spec.max_views, spec.max_det,
                       params, device=device)


def _library_engine_bytes(spec: EngineSpec, params) -> int:
    from . import dect
    need = int(dect.lib().dect_engine_workspace_bytes(spec.n, spec.n, spec.pixel_mm, spec.slots,
                                                      spec.max_views, spec.max_det, params))
    if need == 0:
        raise ValueError(f"engine {spec} is not valid")
    return need


def _cuda_sync():
    import torch
    torch.cuda.synchronize()


class Server:
    """Routes requests to per-size engines, admits them against the HBM
    budget and steps the engines."""

    def __init__(self, specs: List[EngineSpec], params=None, hbm_budget_bytes: float = 200e9,
                 device="cuda", iters_per_step: int = 4,
                 engine_factory: Optional[Callable] = None,
                 engine_bytes: Optional[Callable] = None,
                 sync: Optional[Callable] = None):
        # outer iterations per step: pipelined within the step, and a step ends
        # early when a slot completes, so a freed slot waits for no more than
        # this many iterations of the others before it is refilled
        self.iters_per_step = int(iters_per_step)
        if params is None:
            from . import dect
            params = dect.default_params()
        self.params = params
        self.device = device
        self.budget = float(hbm_budget_bytes)
        self._make = engine_factory or (lambda sp: _library_engine(sp, self.params, self.device))
        self._bytes_of = engine_bytes or (lambda sp: _library_engine_bytes(sp, self.params))
        self._sync = sync or _cuda_sync
        self.specs: Dict[int, EngineSpec] = {sp.n: sp for sp in specs}
        self.spec_bytes: Dict[int, int] = {n: int(self._bytes_of(sp)) for n, sp in self.specs.items()}
        self.pools: Dict[int, List[_Pool]] = {n: [] for n in self.specs}
        self.queues: Dict[int, Deque[Request]] = {n: collections.deque() for n in self.specs}
        self.hbm_bytes = 0          # engine workspaces held now
        self.hbm_peak = 0
        self.engines_created = 0
        self.engines_retired = 0
        self._thread_pool = None
        self.done: List[Request] = []

    # ---- requests ----------------------------------------------------------
    def _reject(self, req: Request, why: str):
        req.status, req.reason = REJECTED, why
        self.done.append(req)

    def submit(self, req: Request) -> bool:
        """Queue a request; False (and status 'rejected') if it can never run."""
        n = int(req.geom.n_x)
        sp = self.specs.get(n)
        if sp is None:
            self._reject(req, f"no engine for {n}^2 images")
            return False
        if int(req.geom.n_views) > sp.max_views or int(req.geom.n_det) > sp.max_det:
            self._reject(req, f"{req.geom.n_views} views x {req.geom.n_det} bins exceed the "
                              f"{sp.max_views} x {sp.max_det} slot capacity")
            return False
        if self.spec_bytes[n] > self.budget:
            self._reject(req, f"an engine for {n}^2 needs {self.spec_bytes[n] / 1e9:.3g} GB, above "
                              f"the {self.budget / 1e9:.3g} GB budget")
            return False
        req.status = QUEUED
        self.queues[n].append(req)
        return True

    def cancel(self, req: Request) -> bool:
        """Cancel a queued or running request (between steps); its maps are
        never written.  False if it had already finished or was rejected."""
        if req.status == QUEUED:
            self.queues[int(req.geom.n_x)].remove(req)
        elif req.status == RUNNING:
            for pool in self.pools[int(req.geom.n_x)]:
                slot = next((s for s, r in pool.running.items() if r is req), None)
                if slot is not None:
                    pool.engine.cancel(slot)
                    del pool.running[slot]
                    break
        else:
            return False
        req.status = CANCELLED
        self.done.append(req)
        return True

    def pending(self) -> int:
        return (sum(len(q) for q in self.queues.values())
                + sum(len(p.running) for ps in self.pools.values() for p in ps))

    # ---- engines and budget ------------------------------------------------
    def _retire_idle(self, keep: int, need: int) -> None:
        """Retire idle engines (no running request) of sizes other than `keep`
        whose queues are empty, until `need` bytes fit the budget."""
        for n, ps in self.pools.items():
            if n == keep or self.queues[n]:
                continue
            for pool in [p for p in ps if not p.running]:
                if self.hbm_bytes + need <= self.budget:
                    return
                ps.remove(pool)
                pool.engine.close()
                self.hbm_bytes -= pool.nbytes
                self.engines_retired += 1

    def _new_pool(self, n: int) -> Optional[_Pool]:
        need = self.spec_bytes[n]
        if self.hbm_bytes + need > self.budget:
            self._retire_idle(n, need)
        if self.hbm_bytes + need > self.budget:
            return None
        pool = _Pool(self.specs[n], self._make(self.specs[n]), need)
        self.pools[n].append(pool)
        self.hbm_bytes += need
        self.hbm_peak = max(self.hbm_peak, self.hbm_bytes)
        self.engines_created += 1
        return pool

    def _admit(self, now: float):
        for n, q in self.queues.items():
            while q:
                pool = next((p for p in self.pools[n] if p.free > 0), None) or self._new_pool(n)
                if pool is None:
                    break               # over budget: wait for memory to free up
                r = q[0]
                slot = pool.engine.admit(r.geom, r.sino_lo, r.sino_hi, r.n_iter)
                if slot is None:
                    raise RuntimeError("engine reported no free slot where the server counted one")
                q.popleft()
                r.admitted, r.status = now, RUNNING
                pool.running[slot] = r

    # ---- stepping ----------------------------------------------------------
    def step(self, clock) -> List[Request]:
        """Admit what fits, advance every engine with work by up to
        `iters_per_step` outer iterations (fewer when a slot completes
        sooner), and return the requests that completed (their maps are
        synchronised)."""
        self._admit(clock())
        active = [p for ps in self.pools.values() for p in ps if p.running]
        if not active:
            return []
        if len(active) == 1:
            active[0].engine.step(self.iters_per_step)
        else:
            # one host thread per engine: each engine's PCG waits on the host
            # once per iteration, and the engines' streams overlap on the
            # device only if those waits do (the library calls release the GIL)
            if self._thread_pool is None:
                from concurrent.futures import ThreadPoolExecutor
                self._thread_pool = ThreadPoolExecutor(max_workers=16)
            list(self._thread_pool.map(lambda p: p.engine.step(self.iters_per_step), active))
        self._sync()
        now = clock()
        out = []
        for p in active:
            for slot, Z, rho in p.engine.completed():
                r = p.running.pop(slot)
                r.finished, r.Z, r.rho, r.status = now, Z, rho, DONE
                out.append(r)
        self.done.extend(out)
        return out

    def run(self, arrivals: List[Request], idle_sleep: float = 2e-4,
            cancel_at: Optional[Dict[int, float]] = None):
        """Replay an arrival stream (each request's `arrival` in seconds from
        now) until every request has completed, been cancelled or been
        rejected; returns the requests.  cancel_at maps a request's index in
        `arrivals` to the time at which it is cancelled."""
        stream = sorted(arrivals, key=lambda r: r.arrival)
        cancels = sorted(((t, arrivals[i]) for i, t in (cancel_at or {}).items()), key=lambda x: x[0])
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        i = 0
        while i < len(stream) or self.pending():
            now = clock()
            while i < len(stream) and stream[i].arrival <= now:
                self.submit(stream[i])
                i += 1
            while cancels and cancels[0][0] <= now:
                self.cancel(cancels.pop(0)[1])
            if not self.step(clock) and not self.pending() and i < len(stream):
                time.sleep(min(idle_sleep, max(0.0, stream[i].arrival - clock())))
        return stream

    def close(self):
        for ps in self.pools.values():
            for p in ps:
                p.engine.close()
            ps.clear()
        self.hbm_bytes = 0
        if self._thread_pool is not None:
            self._thread_pool.shutdown()
            self._thread_pool = None
