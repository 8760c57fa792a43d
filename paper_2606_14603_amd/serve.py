"""Serving loop: independent simulation requests arriving over time.

Each request is a model (species, rules, volume, initial counts, seed) and a
horizon in steps.  The server keeps every admitted request's state resident
in HBM (its own arena of ``mabm_arena_bytes``), admits queued requests in
arrival order while the admitted arenas fit the HBM budget, and advances
every admitted simulation in chunks of steps, each simulation on a stream of
its own, so that small simulations (whose steps are short and launch-bound)
overlap on the GPU's hardware queues instead of waiting behind large ones.
Steps are replayed from captured multi-step graphs, so the host issues one
launch per 16 steps.  A request completes when its last chunk has run; its
result is its per-species counts.

This is the multiple-runs use of the simulator (the paper's concurrent seeds
on one GPU, Sec. 3.2), organised as a request stream.  ``max_active=1``
gives the FIFO baseline that serves one request at a time.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import Sim, arena_bytes


@dataclass
class Result:
    name: str
    arrival_s: float       # offset from the start of serving
    admitted_s: float
    completed_s: float
    steps: int
    agents: int
    counts: np.ndarray = field(repr=False)
    digest: int = 0        # order-independent digest of the final id-keyed state
    grid: int = 0          # cells per axis the simulation ran on
    state: Optional[dict] = field(default=None, repr=False)  # final export (keep_state)

    @property
    def latency_s(self) -> float:
        return self.completed_s - self.arrival_s


class _Active:
    __slots__ = ("model", "arrival", "admitted", "sim", "left", "event", "bytes")


class Server:
    """``budget_bytes``: HBM the admitted arenas may hold together;
    ``chunk``: steps enqueued per simulation per turn; ``max_active``:
    simulations admitted at once (1 = FIFO, one request at a time);
    ``fill_agents``: admission stops while the admitted simulations hold at
    least this many agents, enough to fill the GPU (a large request then
    runs nearly alone, as under FIFO, while small ones overlap).  Every
    result carries the digest of its final state (``mabm_digest``);
    ``keep_state`` also exports the state itself, id-keyed (with the last
    step's cell ids, events and partners when ``record``)."""

    def __init__(self, budget_bytes: int, chunk: int = 256, max_active: int = 64,
                 device: str = "cuda", progress=None, fill_agents: int = 1 << 62,
                 record: bool = False, keep_state: bool = False):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.max_active = int(max_active)
        self.device = device
        self.progress = progress  # called with each Result as it completes
        self.fill_agents = int(fill_agents)
        self.record = bool(record)
        self.keep_state = bool(keep_state)
        self._streams: List = []

    def _stream(self):
        if self._streams:
            return self._streams.pop()
        return self.torch.cuda.Stream(self.device)

    def run(self, models, arrivals_s) -> List[Result]:
        """Serve ``models`` (horizon = ``model.steps``) arriving at the given
        offsets (seconds from now); returns one Result per request, in
        completion order."""
        torch = self.torch
        order = np.argsort(np.asarray(arrivals_s, dtype=np.float64), kind="stable")
        pending = collections.deque((float(arrivals_s[i]), models[i]) for i in order)
        queue: collections.deque = collections.deque()
        active: List[_Active] = []
        done: List[Result] = []
        used = 0
        t0 = time.perf_counter()
        while pending or queue or active:
            now = time.perf_counter() - t0
            while pending and pending[0][0] <= now:
                queue.append(pending.popleft())
            # admission: arrival order, while the arenas fit the budget
            while queue and len(active) < self.max_active:
                arr, m = queue[0]
                need = arena_bytes(m)
                if active and (used + need > self.budget or
                               sum(x.model.n_agents for x in active) >= self.fill_agents):
                    break
                queue.popleft()
                a = _Active()
                a.model, a.arrival, a.admitted = m, arr, time.perf_counter() - t0
                a.sim = Sim(m, stream=self._stream(), graphs=True, record=self.record)
                a.left, a.event, a.bytes = int(m.steps), None, need
                used += need
                active.append(a)
            busy = False
            for a in list(active):
                if a.event is not None and not a.event.query():
                    continue
                busy = True
                if a.left == 0:
                    counts, _ = a.sim.counts()
                    r = Result(a.model.name, a.arrival, a.admitted, time.perf_counter() - t0,
                               int(a.model.steps), int(a.model.n_agents), counts,
                               digest=int(a.sim.digest()[0]))
                    if self.keep_state:
                        r.grid = a.sim.grid()[0]
                        r.state = a.sim.export()
                    done.append(r)
                    if self.progress:
                        self.progress(done[-1])
                    self._streams.append(a.sim.stream)
                    a.sim.close()
                    used -= a.bytes
                    active.remove(a)
                    continue
                n = min(self.chunk, a.left)
                a.sim.step(n)
                a.left -= n
                a.event = torch.cuda.Event()
                a.event.record(a.sim.stream)
            if not busy:
                if active:
                    time.sleep(20e-6)
                elif pending:
                    time.sleep(max(0.0, min(1e-3, pending[0][0] - (time.perf_counter() - t0))))
        return done


def summarize(results: List[Result]) -> dict:
    lat = np.array([r.latency_s for r in results])
    span = max(r.completed_s for r in results) - min(r.arrival_s for r in results)
    return {"requests": len(results), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "sims_per_s": len(results) / span, "makespan_s": span,
            "agent_updates": int(sum(r.agents * r.steps for r in results))}
