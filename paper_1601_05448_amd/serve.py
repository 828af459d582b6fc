"""Serving driver: replays a stream of solve requests against the C server.

The scheduling itself (admission by footprint, batching per grid size,
retirement) is in the library (``poisson_server_*`` in include/poisson.h);
this module only submits requests when their arrival time has come, calls the
tick, and collects per-request latencies from arrival to completion.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

from . import poisson as P


class Server:
    """Owning wrapper of a poisson_server_t."""

    def __init__(self, budget_bytes: int, max_slots: int, precision: int = P.POISSON_FP64,
                 coef: int = P.POISSON_COEF_RHO_FACE_MEAN, weight: int = P.POISSON_W_RHO,
                 max_iter: int = 0, stream=None, use_graphs: bool = False):
        self.h = P.poisson_server_create(budget_bytes, max_slots, precision, coef, weight, max_iter, stream)
        if use_graphs:
            P.poisson_server_use_graphs(self.h, True)

    def submit(self, shape, lengths, rho, b, p, tol: float, bc_x: int = P.POISSON_BC_PERIODIC) -> int:
        return P.poisson_server_submit(self.h, shape, lengths, rho, b, p, tol, bc_x)

    def tick(self) -> int:
        return P.poisson_server_tick(self.h)

    def poll(self, rid: int) -> Optional[dict]:
        return P.poisson_server_poll(self.h, rid)

    def close(self) -> None:
        if getattr(self, "h", None):
            P.poisson_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Job:
    """One request of a replayed stream: arrival time (s, from the start of the
    replay), grid, box and device fields."""
    arrival_s: float
    shape: Sequence[int]
    lengths: Sequence[float]
    rho: object
    b: object
    p: object
    tol: float = 1e-10
    tag: object = None
    bc_x: int = P.POISSON_BC_PERIODIC


@dataclass
class Outcome:
    job: Job
    stats: dict
    latency_ms: float  # arrival to completion


@dataclass
class ReplayResult:
    outcomes: List[Outcome] = field(default_factory=list)
    wall_s: float = 0.0
    ticks: int = 0

    def latencies(self) -> List[float]:
        return [o.latency_ms for o in self.outcomes]


def replay(server: Server, jobs: Sequence[Job], realtime: bool = True,
           on_done: Optional[Callable[[Outcome], None]] = None) -> ReplayResult:
    """Submit each job at its arrival time (or all at once if not realtime),
    tick until every job is done.  Latency = completion - arrival."""
    order = sorted(range(len(jobs)), key=lambda k: jobs[k].arrival_s)
    res = ReplayResult()
    t0 = time.perf_counter()
    nxt = 0
    inflight: Dict[int, tuple] = {}
    while nxt < len(order) or inflight:
        now = time.perf_counter() - t0
        while nxt < len(order) and (not realtime or jobs[order[nxt]].arrival_s <= now):
            j = jobs[order[nxt]]
            rid = server.submit(j.shape, j.lengths, j.rho, j.b, j.p, j.tol, j.bc_x)
            inflight[rid] = (j, time.perf_counter() - t0)
            nxt += 1
        if not inflight:
            wait = jobs[order[nxt]].arrival_s - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
            continue
        server.tick()
        res.ticks += 1
        for rid in list(inflight):
            st = server.poll(rid)
            if st is None:
                continue
            j, t_sub = inflight.pop(rid)
            arrival = j.arrival_s if realtime else 0.0
            lat = (t_sub - arrival) * 1e3 + st["ms"]
            out = Outcome(j, st, lat)
            res.outcomes.append(out)
            if on_done:
                on_done(out)
    res.wall_s = time.perf_counter() - t0
    return res


@dataclass
class Chain:
    """A time series of dependent solves on one grid: step t+1 starts from the
    solution of step t (p is one device field, updated in place by each step;
    warm=False zeroes it before every step instead)."""
    shape: Sequence[int]
    lengths: Sequence[float]
    steps: Sequence[tuple]  # (rho_t, b_t) device fields
    p: object
    tol: float = 1e-10
    warm: bool = True
    bc_x: int = P.POISSON_BC_PERIODIC


@dataclass
class ChainResult:
    stats: List[List[dict]] = field(default_factory=list)  # per chain, per step
    wall_s: float = 0.0
    ticks: int = 0

    def solves(self) -> int:
        return sum(len(s) for s in self.stats)


def run_chains(server: Server, chains: Sequence[Chain]) -> ChainResult:
    """Serve several chains at once: every chain has at most one request in
    flight, and its next step is submitted as soon as the previous one is done
    (with the same p, so the server starts it from the previous solution)."""
    res = ChainResult(stats=[[] for _ in chains])
    nxt = [0] * len(chains)
    inflight: Dict[int, int] = {}

    def submit(c: int) -> None:
        ch = chains[c]
        rho, b = ch.steps[nxt[c]]
        if not ch.warm:
            import torch

            ch.p.zero_()
            torch.cuda.current_stream().synchronize()  # the server reads p on its own streams
        rid = server.submit(ch.shape, ch.lengths, rho, b, ch.p, ch.tol, ch.bc_x)
        inflight[rid] = c
        nxt[c] += 1

    t0 = time.perf_counter()
    for c in range(len(chains)):
        if chains[c].steps:
            submit(c)
    while inflight:
        server.tick()
        res.ticks += 1
        for rid in list(inflight):
            st = server.poll(rid)
            if st is None:
                continue
            c = inflight.pop(rid)
            res.stats[c].append(st)
            if nxt[c] < len(chains[c].steps):
                submit(c)
    res.wall_s = time.perf_counter() - t0
    return res
