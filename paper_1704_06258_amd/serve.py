"""Continuous-batching solve server for the USApHMP GA on one GPU.

Requests (an instance, p, population, generations, GA seed) arrive over time.
The server keeps every admitted request's instance, population and GA state
resident on the GPU (one context each, in a workspace sized by
ga_workspace_bytes).  Admission is FIFO: a waiting request is admitted while
a slot is free and its workspace fits into the HBM budget next to the
resident and in-flight ones.  Every tick advances all resident requests by
one generation (ga_batch_step): one launch per GA step over all their
populations.  Requests join and leave at generation boundaries; each result
is exactly what the request would give alone.  Latency is measured from the
scheduled arrival to the result on the host.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import threading
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
    error: str | None = None       # set when building or reading back the request failed


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


def c_symmetric(req: SolveRequest) -> bool:
    """Whether the request's C is symmetric (computed once per request)."""
    sym = getattr(req, "_c_symmetric", None)
    if sym is None:
        sym = bool(np.array_equal(req.C, req.C.T))
        req._c_symmetric = sym
    return sym


def workspace_bytes(req: SolveRequest) -> int:
    n = req.C.shape[0]
    q = hubga.make_params(n, req.p, chi=req.chi, alpha=req.alpha, delta=req.delta, seed=req.seed,
                          population=req.population, island_size=min(req.island_size, req.population), n1=req.n1,
                          precision=req.precision, c_symmetric=c_symmetric(req))
    cdt = hubga.GA_DT_F32 if req.C.dtype == np.float32 else hubga.GA_DT_F64
    wdt = hubga.GA_DT_F32 if req.W.dtype == np.float32 else hubga.GA_DT_F64
    return hubga.ga_workspace_bytes(q, cdt, wdt)


class Server:
    """Continuous batching on one GPU.

    The tick loop (this thread) only launches work: every tick is one batched
    generation of all resident requests.  Building a request's context (copy
    of C and W, preparation, evaluation of P0) runs on worker threads, each
    with a stream of its own, and a finished request is read back and freed
    on a worker too; contexts move between those streams and the batch stream
    with ga_set_stream, which orders them by an event instead of a host wait.
    So admissions and completions overlap the generations of the others."""

    # Tile configuration 16 (128 x 256, K tiles of 64) multiplies the folded W
    # of symmetric instances and groups every context with p >= 3; on the
    # serving mix it kept up with 200 requests/s where the unfolded
    # configuration 7 fell behind (p99 0.27 s against 1.83 s).
    def __init__(self, hbm_budget: int = 16 << 30, max_slots: int = 64, tile_config: int = 16, device: int = 0,
                 workers: int = 8):
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.batch = hubga.Batch(device=device, tile_config=tile_config)
        self.device = device
        self.resident: list[_Job] = []
        self.used = 0
        self.ticks = 0
        self.evaluations = 0
        self.max_resident = 0
        self.workers = int(workers)
        self._pool = concurrent.futures.ThreadPoolExecutor(self.workers) if self.workers > 0 else None
        self._local = threading.local()
        self._harvest = None

    def _stream(self):
        """This thread's side stream (None with a backend that has no streams)."""
        if self.batch.stream is None:
            return None
        st = getattr(self._local, "stream", None)
        if st is None:
            import torch
            st = self._local.stream = torch.cuda.Stream(torch.device("cuda", self.device))
        return st

    def _admit(self, req: SolveRequest, now: float) -> _Job:
        solver = hubga.Solver(req.C, req.W, req.p, chi=req.chi, alpha=req.alpha, delta=req.delta, seed=req.seed,
                              population=req.population, island_size=min(req.island_size, req.population),
                              n1=req.n1, precision=req.precision, stream=self._stream(), device=self.device,
                              c_symmetric=c_symmetric(req))
        return _Job(req, solver, solver.workspace_bytes, now)

    def _finish(self, job: _Job, t0: float, clock) -> SolveResult:
        b = job.solver.best()                  # waits for this request's last generation only
        res = SolveResult(job.req.rid, b["hubs"], b["cost"], b["generation"], job.req.arrival, job.admitted,
                          clock() - t0)
        job.solver.close()
        return res

    @staticmethod
    def _failed(req: SolveRequest, now: float, exc: BaseException) -> SolveResult:
        return SolveResult(req.rid, None, float("nan"), 0, req.arrival, now, now, error=f"{type(exc).__name__}: {exc}")

    def _submit(self, fn, *args):
        if self._pool is None:
            f = concurrent.futures.Future()
            try:
                f.set_result(fn(*args))
            except Exception as exc:
                f.set_exception(exc)
            return f
        return self._pool.submit(fn, *args)

    def run(self, requests, realtime: bool = True, clock=time.perf_counter):
        """Serve ``requests`` (sorted by arrival).  With ``realtime`` arrivals
        are released at their scheduled times; otherwise all are available at
        once (closed loop).  Returns the results in completion order."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        building: list = []                    # (future, bytes reserved, request)
        finishing: list = []                   # (future, bytes held, request)
        results: list[SolveResult] = []
        if self.batch.stream is not None and self._harvest is None:
            import torch
            self._harvest = torch.cuda.Stream(torch.device("cuda", self.device))
        t0 = clock()
        while pending or waiting or building or self.resident or finishing:
            now = clock() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            # FIFO admission by slots and HBM budget (building contexts hold both)
            while waiting and len(self.resident) + len(building) < self.max_slots:
                need = workspace_bytes(waiting[0])
                if self.used + need > self.budget:
                    if not (self.resident or building or finishing):
                        raise MemoryError(f"request {waiting[0].rid} needs {need} bytes > budget {self.budget}")
                    break
                req = waiting.popleft()
                self.used += need
                building.append((self._submit(self._admit, req, clock() - t0), need, req))
            # contexts built since the last tick join at this generation boundary
            changed = False
            still = []
            for fut, need, req in building:
                if not fut.done():
                    still.append((fut, need, req))
                    continue
                try:
                    job = fut.result()
                except Exception as exc:       # this request failed to build: release it, keep serving
                    self.used -= need
                    results.append(self._failed(req, clock() - t0, exc))
                    continue
                job.nbytes = need
                if job.req.generations <= 0:   # nothing to run: read back P0 as it stands
                    finishing.append((self._submit(self._finish, job, t0, clock), need, job.req))
                    continue
                if self.batch.stream is not None:
                    job.solver.set_stream(self.batch.stream)
                self.resident.append(job)
                changed = True
            building = still
            if changed:
                self.batch.set([j.solver for j in self.resident])
                self.max_resident = max(self.max_resident, len(self.resident))
            if self.resident:
                self.batch.step(1)
                self.ticks += 1
                for j in self.resident:
                    j.gens += 1
                    self.evaluations += j.req.population
                done = [j for j in self.resident if j.gens >= j.req.generations]
                if done:
                    self.resident = [j for j in self.resident if j.gens < j.req.generations]
                    self.batch.set([j.solver for j in self.resident])
                    for j in done:             # out of the batch: read back and freed on a worker
                        if self._harvest is not None:
                            j.solver.set_stream(self._harvest)
                        finishing.append((self._submit(self._finish, j, t0, clock), j.nbytes, j.req))
            else:
                delay = 0.0005 if (building or finishing) else (
                    pending[0].arrival - (clock() - t0) if pending and realtime else 0.0)
                if delay > 0:
                    time.sleep(min(delay, 0.01))
            still = []
            for fut, nb, req in finishing:
                if not fut.done():
                    still.append((fut, nb, req))
                    continue
                self.used -= nb
                try:
                    results.append(fut.result())
                except Exception as exc:       # reading back failed: report it, keep serving
                    results.append(self._failed(req, clock() - t0, exc))
            finishing = still
        self.batch.synchronize()
        return results

    def close(self):
        for j in self.resident:
            j.solver.close()
        self.resident = []
        if self._pool is not None:
            self._pool.shutdown(wait=True)
            self._pool = None
        self.batch.close()


def solve_alone(req: SolveRequest, device: int = 0):
    """The same request on its own context, stepped generation by generation."""
    with hubga.Solver(req.C, req.W, req.p, chi=req.chi, alpha=req.alpha, delta=req.delta, seed=req.seed,
                      population=req.population, island_size=min(req.island_size, req.population), n1=req.n1,
                      precision=req.precision, device=device) as s:
        s.step(req.generations)
        return s.best()


def latency_stats(results, skip: int = 0):
    """Latency percentiles of the served requests after the first ``skip``
    (by request id); failed requests are counted, not timed."""
    kept = sorted(results, key=lambda r: r.rid)[skip:]
    lat = np.array([r.latency for r in kept if r.error is None])
    if lat.size == 0:
        return {}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "count": int(lat.size),
            "failed": int(sum(r.error is not None for r in kept))}
