"""Tile autotuner for the batched split-bf16 evaluation kernel.

For a live context it searches the tile configurations of the batched kernel
(ga_tile_config_count / ga_set_tile_config: workgroup rows x columns, K tile,
pipeline depth, each a compiled kernel) on the context's own current
population, with HIP events around each launch, by successive halving: every
configuration is timed briefly, the fastest third again with more launches,
the best few once more, and the fastest of the last round wins.  The choice
is cached in a JSON file keyed by (architecture, n bucket, p, population),
with every configuration's (rows, cols, K tile) and time.  Timing
re-evaluates the population through ga_evaluate_dev, so the GA state
(ancestors, best, generation) is left untouched.
"""
from __future__ import annotations

import json
import os
import time

from . import hubga

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hubga", "tiles.json")


def cache_key(n, p, S, arch="gfx950"):
    bucket = 1 << max(0, (int(n) - 1).bit_length())   # next power of two
    return f"{arch}|n{bucket}|p{p}|S{S}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_config(solver, cfg, d_hubs, reps=5):
    """Mean milliseconds of one batched-kernel launch over the population."""
    import torch
    solver.set_tile_config(cfg)
    solver.evaluate_dev(d_hubs)              # warm-up (code object load, caches)
    torch.cuda.synchronize()
    solver.profile_enable(True)
    for _ in range(reps):
        solver.evaluate_dev(d_hubs)
    ms, k = solver.profile_read()
    solver.profile_enable(False)
    return ms / max(k, 1)


def successive_halving(candidates, time_fn, reps=(1, 3, 10), keep=(1 / 3, 3)):
    """Fastest of `candidates` under `time_fn(c, r)` (mean ms over r launches):
    round t times the survivors with reps[t] launches; after round t the best
    keep[t] survive (a fraction of those timed, or a count; at least one).
    Returns (best, {c: ms of its last round}, [survivors after each round])."""
    alive = list(candidates)
    times, rounds = {}, []
    for t, r in enumerate(reps):
        for c in alive:
            times[c] = time_fn(c, r)
        alive = sorted(alive, key=lambda c: (times[c], c))
        if t < len(keep):
            k = keep[t]
            alive = alive[:max(1, int(round(k * len(alive))) if isinstance(k, float) else k)]
        else:
            alive = alive[:1]
        rounds.append(list(alive))
    return alive[0], times, rounds


def autotune(solver, cache_path=DEFAULT_CACHE, force=False, reps=5):
    """Pick (and apply) the fastest tile configuration for this context.
    Returns {"config": c, "ms": {c: ms}, "cached": bool}."""
    import numpy as np
    import torch
    if solver.params.precision not in (hubga.GA_PREC_SPLIT_BF16, hubga.GA_PREC_SPLIT3_BF16):
        return {"config": None, "ms": {}, "cached": False}
    # the three-part split runs in the register-staged configurations 0, 2, 3, 5
    candidates = ([0, 2, 3, 5] if solver.params.precision == hubga.GA_PREC_SPLIT3_BF16
                  else list(range(len(hubga.tile_configs()))))
    key = cache_key(solver.n, solver.p, solver.S) + ("|split3" if solver.params.precision == hubga.GA_PREC_SPLIT3_BF16
                                                     else "")
    cache = _load(cache_path)
    if not force and key in cache:
        solver.set_tile_config(int(cache[key]["config"]))
        return {"config": int(cache[key]["config"]), "ms": cache[key].get("ms", {}), "cached": True}
    hubs, _ = solver.population()
    if not np.all(np.diff(hubs, axis=1) > 0):     # before the first generation: use the ancestors
        anc, _ = solver.ancestors()
        hubs = np.repeat(anc, solver.S // anc.shape[0], axis=0)
    d_hubs = torch.from_numpy(np.ascontiguousarray(hubs)).to(solver.device)
    best, times, rounds = successive_halving(candidates, lambda c, r: time_config(solver, c, d_hubs, r),
                                             reps=(1, 3, max(1, reps)))
    solver.set_tile_config(best)
    shapes = hubga.tile_configs()
    cache[key] = {"config": best, "ms": times, "rounds": rounds, "shapes": {c: list(shapes[c]) for c in times},
                  "time": time.time()}
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    except OSError:
        pass
    return {"config": best, "ms": times, "rounds": rounds, "cached": False}
