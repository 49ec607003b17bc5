"""Serving loop: single-slice solves arriving over time, continuously batched.

One engine (dect_engine_*) per image size holds a pool of slots on the device;
a request waits in its size's FIFO queue until a slot is free, is admitted
between two steps while the other slots are mid-solve, and leaves when its
iteration budget is done.  Engines are created up to an HBM budget.  The
numerics of every request are those of solving it alone; this module only
schedules (argument marshalling and bookkeeping; the work runs in the
library).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Deque, Dict, List, Optional

from . import dect


@dataclass
class Request:
    geom: object            # FanGeometry / dect.Geometry
    sino_lo: object         # [n_views, n_det] float32 device tensor
    sino_hi: object
    n_iter: int
    arrival: float = 0.0    # seconds on the server's clock
    tag: object = None
    # filled in by the server
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
    slots: int
    max_views: int
    max_det: int


class Server:
    """Routes requests to per-size engines and steps them."""

    def __init__(self, specs: List[EngineSpec], params=None, hbm_budget_bytes: float = 200e9,
                 device="cuda", iters_per_step: int = 4):
        # outer iterations per step: pipelined within the step, and a step ends
        # early when a slot completes, so a freed slot waits for no more than
        # this many iterations of the others before it is refilled
        self.iters_per_step = int(iters_per_step)
        self._pool = None
        self.params = params if params is not None else dect.default_params()
        self.engines: Dict[int, dect.Engine] = {}
        self.queues: Dict[int, Deque[Request]] = {}
        self.running: Dict[int, Dict[int, Request]] = {}
        self.hbm_bytes = 0
        lib = dect.lib()
        for sp in specs:
            need = lib.dect_engine_workspace_bytes(sp.n, sp.n, sp.pixel_mm, sp.slots, sp.max_views,
                                                   sp.max_det, self.params)
            if need == 0:
                raise ValueError(f"engine {sp} is not valid")
            if self.hbm_bytes + need > hbm_budget_bytes:
                raise MemoryError(f"engine for {sp.n}^2 needs {need / 1e9:.1f} GB beyond the "
                                  f"{hbm_budget_bytes / 1e9:.0f} GB budget")
            self.hbm_bytes += need
            self.engines[sp.n] = dect.Engine(sp.n, sp.n, sp.pixel_mm, sp.slots, sp.max_views,
                                             sp.max_det, self.params, device=device)
            self.queues[sp.n] = collections.deque()
            self.running[sp.n] = {}
        self.done: List[Request] = []

    def submit(self, req: Request):
        n = req.geom.n_x
        if n not in self.engines:
            raise ValueError(f"no engine for {n}^2 images")
        self.queues[n].append(req)

    def pending(self) -> int:
        return sum(len(q) for q in self.queues.values()) + sum(len(r) for r in self.running.values())

    def _admit(self, now: float):
        for n, q in self.queues.items():
            eng = self.engines[n]
            while q:
                r = q[0]
                slot = eng.admit(r.geom, r.sino_lo, r.sino_hi, r.n_iter)
                if slot is None:
                    break
                q.popleft()
                r.admitted = now
                self.running[n][slot] = r

    def step(self, clock) -> List[Request]:
        """Admit what fits, advance every engine with work by up to
        `iters_per_step` outer iterations (fewer when a slot completes
        sooner), and return the requests that completed (their maps are
        synchronised)."""
        import torch
        self._admit(clock())
        active = [eng for n, eng in self.engines.items() if self.running[n]]
        if not active:
            return []
        if len(active) == 1:
            active[0].step(self.iters_per_step)
        else:
            # one host thread per engine: each engine's PCG waits on the host
            # once per iteration, and the engines' streams overlap on the
            # device only if those waits do (the library calls release the GIL)
            if self._pool is None:
                from concurrent.futures import ThreadPoolExecutor
                self._pool = ThreadPoolExecutor(max_workers=len(self.engines))
            list(self._pool.map(lambda e: e.step(self.iters_per_step), active))
        torch.cuda.synchronize()
        now = clock()
        out = []
        for n, eng in self.engines.items():
            for slot, Z, rho in eng.completed():
                r = self.running[n].pop(slot)
                r.finished, r.Z, r.rho = now, Z, rho
                out.append(r)
        self.done.extend(out)
        return out

    def run(self, arrivals: List[Request], idle_sleep: float = 2e-4):
        """Replay an arrival stream (each request's `arrival` in seconds from
        now) until every request has completed; returns the requests."""
        stream = sorted(arrivals, key=lambda r: r.arrival)
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        i = 0
        while i < len(stream) or self.pending():
            now = clock()
            while i < len(stream) and stream[i].arrival <= now:
                self.submit(stream[i])
                i += 1
            if not self.step(clock) and not self.pending() and i < len(stream):
                time.sleep(min(idle_sleep, max(0.0, stream[i].arrival - clock())))
        return stream
