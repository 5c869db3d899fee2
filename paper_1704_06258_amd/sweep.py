"""Sensitivity of the solution's hub network to the cost factors (the study
behind Fig. 3 of Sec. 6.2): on one instance, the GA is solved for every
combination of hub count p, collection/distribution factor chi = delta and
inter-hub discount alpha, and each solution's average inter-hub distance is
reported.  The paper runs this on the CAB data (n = 25); the CAB-sized
synthetic instance stands in for it.

All solves of a sweep go through the continuous-batching server at once (one
context per cell, grouped generations); each result is exactly the GA's
result for that cell alone.  Optionally every cell's exhaustive optimum over
the nearest-hub space (ga_enumerate) is computed too, which tells whether the
GA reached it.
"""
from __future__ import annotations

import dataclasses
import itertools
import time

import numpy as np

from . import hubga, serve


@dataclasses.dataclass
class SweepCell:
    p: int
    chi: float
    alpha: float
    delta: float
    hubs: np.ndarray
    cost: float
    interhub: float                    # average inter-hub distance of the solution
    optimum: float | None = None       # exhaustive optimum over the nearest-hub space
    optimum_hubs: np.ndarray | None = None

    @property
    def optimal(self) -> bool | None:
        return None if self.optimum is None else self.cost == self.optimum


def average_interhub_distance(C: np.ndarray, hubs) -> float:
    """Mean of C[h_k][h_l] over ordered pairs of distinct open hubs (0 for
    fewer than two hubs)."""
    h = np.asarray(hubs, dtype=np.int64)
    k = len(h)
    if k < 2:
        return 0.0
    sub = np.asarray(C, dtype=np.float64)[np.ix_(h, h)]
    return float((sub.sum() - np.trace(sub)) / (k * (k - 1)))


def sweep_grid(ps, factors, alphas):
    """Cells (p, chi, alpha, delta) with chi = delta = each factor."""
    return [(p, f, a, f) for p, f, a in itertools.product(ps, factors, alphas)]


def run_sweep(C, W, cells, *, generations=100, population=256, island_size=64, n1=10, seed=1,
              precision="split_bf16", exhaustive=False, server=None, device=0):
    """Solve every cell (p, chi, alpha, delta) of the sweep on instance (C, W)
    through one server run.  Returns (cells in input order, seconds)."""
    reqs = [serve.SolveRequest(r, 0.0, C, W, p, chi, alpha, delta, population, generations, seed,
                               island_size=island_size, n1=n1, precision=precision)
            for r, (p, chi, alpha, delta) in enumerate(cells)]
    own = server is None
    srv = server or serve.Server(hbm_budget=8 << 30, max_slots=max(1, len(reqs)), device=device)
    t0 = time.perf_counter()
    try:
        res = srv.run(reqs, realtime=False)
    finally:
        if own:
            srv.close()
    wall = time.perf_counter() - t0
    by_rid = {r.rid: r for r in res}
    out = []
    for r, (p, chi, alpha, delta) in enumerate(cells):
        got = by_rid[r]
        if got.error is not None:
            raise RuntimeError(f"sweep cell {cells[r]} failed: {got.error}")
        cell = SweepCell(p, chi, alpha, delta, got.hubs, got.cost, average_interhub_distance(C, got.hubs))
        if exhaustive:
            with hubga.Solver(C, W, p, chi=chi, alpha=alpha, delta=delta, population=population,
                              island_size=min(island_size, population), precision="fp64", device=device) as s:
                e = s.enumerate()
            cell.optimum, cell.optimum_hubs = e["cost"], e["hubs"]
        out.append(cell)
    return out, wall


def summary(cells):
    """Average inter-hub distance per (p, chi = delta, alpha), as rows."""
    return [{"p": c.p, "chi": c.chi, "delta": c.delta, "alpha": c.alpha, "interhub": c.interhub, "cost": c.cost,
             "hubs": [int(h) for h in c.hubs], "optimal": c.optimal} for c in cells]
