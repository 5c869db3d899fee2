"""Continuous-batching solve server for the USApHMP GA on one GPU.

Requests (an instance, p, population, generations, GA seed) arrive over time.
The server keeps every admitted request's instance, population and GA state
resident on the GPU (one context each, in a workspace sized by
ga_workspace_bytes).  Admission is FIFO: a waiting request is admitted while
a slot is free and its workspace fits into the HBM budget next to the
resident ones.  Every tick advances all resident requests by one generation
in one replayed batch graph (ga_batch_*), with one grouped matrix-core launch
for their populations.  Requests join and leave at generation boundaries;
each result is exactly what the request would give alone.  Latency is
measured from the scheduled arrival to the result on the host.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import hubga


@dataclasses.dataclass
class SolveRequest:
    rid: int
    arrival: float                 # seconds after the start of the run
    C: np.ndarray
    W: np.ndarray
    p: int
    chi: float
    alpha: float
    delta: float
    population: int
    generations: int
    seed: int
    island_size: int = 64
    n1: int = 10
    precision: str = "split_bf16"


@dataclasses.dataclass
class SolveResult:
    rid: int
    hubs: np.ndarray
    cost: float
    generations: int
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class _Job:
    req: SolveRequest
    solver: object
    nbytes: int
    admitted: float
    gens: int = 0


def workspace_bytes(req: SolveRequest) -> int:
    n = req.C.shape[0]
    q = hubga.make_params(n, req.p, chi=req.chi, alpha=req.alpha, delta=req.delta, seed=req.seed,
                          population=req.population, island_size=min(req.island_size, req.population), n1=req.n1,
                          precision=req.precision, c_symmetric=bool(np.array_equal(req.C, req.C.T)))
    cdt = hubga.GA_DT_F32 if req.C.dtype == np.float32 else hubga.GA_DT_F64
    wdt = hubga.GA_DT_F32 if req.W.dtype == np.float32 else hubga.GA_DT_F64
    return hubga.ga_workspace_bytes(q, cdt, wdt)


class Server:
    def __init__(self, hbm_budget: int = 16 << 30, max_slots: int = 32, tile_config: int = 7, device: int = 0):
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.batch = hubga.Batch(device=device, tile_config=tile_config)
        self.device = device
        self.resident: list[_Job] = []
        self.used = 0
        self.ticks = 0
        self.evaluations = 0
        self.max_resident = 0

    def _admit(self, req: SolveRequest, now: float) -> _Job:
        solver = hubga.Solver(req.C, req.W, req.p, chi=req.chi, alpha=req.alpha, delta=req.delta, seed=req.seed,
                              population=req.population, island_size=min(req.island_size, req.population),
                              n1=req.n1, precision=req.precision, stream=self.batch.stream, device=self.device)
        return _Job(req, solver, solver.workspace_bytes, now)

    def run(self, requests, realtime: bool = True, clock=time.perf_counter):
        """Serve ``requests`` (sorted by arrival).  With ``realtime`` arrivals
        are released at their scheduled times; otherwise all are available at
        once (closed loop).  Returns the results in completion order."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        results: list[SolveResult] = []
        t0 = clock()
        while pending or waiting or self.resident:
            now = clock() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            changed = False
            while waiting and len(self.resident) < self.max_slots:
                need = workspace_bytes(waiting[0])
                if self.used + need > self.budget:
                    if not self.resident:
                        raise MemoryError(f"request {waiting[0].rid} needs {need} bytes > budget {self.budget}")
                    break
                req = waiting.popleft()
                job = self._admit(req, clock() - t0)
                self.resident.append(job)
                self.used += job.nbytes
                changed = True
            if changed:
                self.batch.set([j.solver for j in self.resident])
                self.max_resident = max(self.max_resident, len(self.resident))
            if not self.resident:
                if pending:
                    delay = pending[0].arrival - (clock() - t0)
                    if delay > 0:
                        time.sleep(min(delay, 0.01))
                continue
            self.batch.step(1)
            self.ticks += 1
            for j in self.resident:
                j.gens += 1
                self.evaluations += j.req.population
            done = [j for j in self.resident if j.gens >= j.req.generations]
            if done:
                for j in done:
                    b = j.solver.best()          # waits for this request's generations
                    results.append(SolveResult(j.req.rid, b["hubs"], b["cost"], b["generation"], j.req.arrival,
                                               j.admitted, clock() - t0))
                self.resident = [j for j in self.resident if j.gens < j.req.generations]
                self.batch.set([j.solver for j in self.resident])
                for j in done:                   # out of the batch before it is freed
                    j.solver.close()
                    self.used -= j.nbytes
        self.batch.synchronize()
        return results

    def close(self):
        for j in self.resident:
            j.solver.close()
        self.resident = []
        self.batch.close()


def solve_alone(req: SolveRequest, device: int = 0):
    """The same request on its own context, stepped generation by generation."""
    with hubga.Solver(req.C, req.W, req.p, chi=req.chi, alpha=req.alpha, delta=req.delta, seed=req.seed,
                      population=req.population, island_size=min(req.island_size, req.population), n1=req.n1,
                      precision=req.precision, device=device) as s:
        s.step(req.generations)
        return s.best()


def latency_stats(results, skip: int = 0):
    lat = np.array([r.latency for r in sorted(results, key=lambda r: r.rid)[skip:]])
    if lat.size == 0:
        return {}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "count": int(lat.size)}
