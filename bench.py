"""Throughput benchmark: fitness evaluations per second of the USApHMP GA on one GPU.

One step = one GA generation over the whole hot path on the GPU: genetic
operators, nearest-hub allocation, batched split-bf16 evaluation on matrix
cores (the dominant kernel), cost assembly, certified selection with exact
re-evaluation of candidates, and the outer-loop global step.  Workload: the
clustered instance n=1000, p=20 (20 Gaussian clusters, sigma=300, lognormal
flows normalised to 1e6, chi=3, alpha=0.75, delta=2), population 4096 in 64
islands of 64, inputs resident in HBM before the timed region.

Prints one JSON line.  The dominant kernel's roofline uses its own average
launch time, measured with HIP events on the stream it runs on.  The CPU
baseline is the FP64 oracle timed on the host cores over a bounded sample, at
one thread and at all threads (median of 5 after a warm-up).  Further legs,
each in its own JSON object: the plain per-individual kernels over the same
generations (the comparators of the batched path), the steady-state
generation time after the early candidate bursts, the exhaustive search of
n=100, p=3 (161,700 hub sets), the chi/delta/alpha sweep of Sec. 6.2 on the
CAB-sized instance, and the serving stream (200 warm-up + 2000 measured
requests, each with its own instance).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0        # MI355X dense bf16 matrix peak
PEAK_HBM_GBS = 8000.0
WORKLOADS = {
    # name: (instance factory, n, p, population, island size, n1, description)
    "clustered": ("clustered", 1000, 20, 4096, 64, 10,
                  "clustered n=1000 p=20 population=4096 (64 islands x 64), one GA generation per step, split-bf16 "
                  "batched matrix-core evaluation"),
    "large": ("large", 6000, 50, 2048, 64, 10,
              "large n=6000 p=50 population=2048 (32 islands x 64), FP32 instance, one GA generation per step, "
              "split-bf16 batched matrix-core evaluation"),
}
MFMA_SRC = os.path.join(ROOT, "paper_1704_06258_amd", "csrc", "eval_mfma.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "eval_mfma_clustered_n1000_p20_traffic.md")


def flops_per_eval(n, p, folded=False):
    """Matrix-core flops per individual: two passes (hi, lo) of an n x n by n x p
    product, or, folded (C symmetric), of its upper triangle with the diagonal."""
    return 2 * p * n * (n + 1) if folded else 2 * 2 * n * n * p


def traffic_from_profile():
    """HBM bytes per launch of the batched kernel from the committed counter
    summary, or None when that summary is missing or predates the kernel source."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    text = open(TRAFFIC_SUMMARY).read()
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b:
        return None
    cur = hashlib.sha256(open(MFMA_SRC, "rb").read()).hexdigest()
    return float(m_b.group(1)) if cur == m_sha.group(1) else None


def time_steps(solver, steps, warmup, kernel_steps=20):
    """Wall time of `steps` generations (after `warmup`), then the summed HIP
    event time and launch count of the dominant kernel over `kernel_steps`
    further generations (events recorded on the solver's stream)."""
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solver.profile_enable(True)
    solver.step(kernel_steps)
    kms, launches = solver.profile_read()
    solver.profile_enable(False)
    return dt, kms, launches


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inst, gpu_hubs, gpu_cost, label="n=1000, p=20", one_thread_sample=128, all_sample=2048,
                 reps=5):
    """The FP64 oracle (OpenMP over individuals) on the GPU's last population:
    median evaluations per second of `reps` runs after one warm-up, at one
    thread on the first `one_thread_sample` children and at all host threads
    on the first `all_sample`; plus the measured error of the GPU's split-bf16
    costs on the larger sample."""
    import oracle
    C, W = inst.C64(), inst.W64()
    all_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def rate(k, threads):
        used = oracle.set_threads(threads)
        h = gpu_hubs[:k]
        ref, _ = oracle.evaluate(C, W, h, inst.chi, inst.alpha, inst.delta, inst.scale)   # warm-up
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.evaluate(C, W, h, inst.chi, inst.alpha, inst.delta, inst.scale)
            ts.append(time.perf_counter() - t0)
        return k / float(np.median(ts)), used, ref, float(np.sum(ts))

    one, _, _, t1 = rate(min(one_thread_sample, len(gpu_hubs)), 1)
    k = min(all_sample, len(gpu_hubs))
    many, used, ref, tm = rate(k, all_threads)
    err = float(np.max(np.abs(gpu_cost[:k] - ref) / ref))
    return dict(value=many, unit="evals/s", cores=used, kind="oracle", single_thread=one,
                cpu_model=cpu_model(),
                sample=f"the first {k} children of the last GPU generation ({label}) at {used} threads and "
                       f"the first {min(one_thread_sample, len(gpu_hubs))} at 1 thread, FP64 oracle, median of "
                       f"{reps} runs after a warm-up ({t1 + tm * used:.1f} s of CPU work)"), err


def serving_leg(count, warmup, rate=200.0, budget=16 << 30, slots=64, threads=16):
    """Continuous-batching serving of a Poisson request stream: p50/p99
    latency from scheduled arrival to result over the requests after the
    first `warmup`, completed solves/s and evaluations/s.  Request r carries
    its own instance (seed 5e6 + r) and GA seed r; the instances are drawn
    before the run on a thread pool (the client's data, not service time)."""
    from paper_1704_06258_amd import instances as I
    from paper_1704_06258_amd import serve
    stream = I.serving_requests(count, rate=rate, seed=5, generations=100)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max(1, min(threads, os.cpu_count() or 1))) as ex:
        insts = list(ex.map(lambda q: q.instance(), stream))
    gen_s = time.perf_counter() - t0
    log(f"serving: {count} instances drawn in {gen_s:.1f} s")
    reqs = [serve.SolveRequest(q.rid, q.arrival, inst.C, inst.W, q.p, inst.chi, inst.alpha, inst.delta, q.S,
                               q.generations, q.ga_seed) for q, inst in zip(stream, insts)]
    del insts
    srv = serve.Server(hbm_budget=budget, max_slots=slots)
    t0 = time.perf_counter()
    res = srv.run(reqs, realtime=True)
    wall = time.perf_counter() - t0
    srv.close()
    measured = [r for r in res if r.rid >= warmup]
    st = serve.latency_stats(measured)
    evals = sum(reqs[r.rid].population * reqs[r.rid].generations for r in res if r.error is None)
    offered = rate * sum(q.population * q.generations for q in reqs) / len(reqs)
    return {"requests": count, "warmup": warmup, "measured": len(measured), "rate_per_s": rate,
            "generations": 100, "instances": "one per request, seed 5000000 + r",
            "offered_evals_per_s": offered,
            "p50_latency_s": st.get("p50_s"), "p99_latency_s": st.get("p99_s"), "mean_latency_s": st.get("mean_s"),
            "failed": st.get("failed", 0),
            "completed_per_s": len(res) / wall, "evals_per_s": evals / wall, "max_resident": srv.max_resident,
            "ticks": srv.ticks, "budget_bytes": budget, "slots": slots, "instance_draw_s": gen_s}


def enumeration_leg(n=100, p=3, population=4096):
    """Exhaustive search of every hub set of an n-node instance (ga_enumerate)
    in split-bf16 through the batched kernel, and in FP64 through the plain
    one: sets per second, and whether both found the same optimum."""
    import math
    import torch
    from paper_1704_06258_amd import hubga
    from paper_1704_06258_amd import instances as I
    inst = I.uniform(seed=83, n=n, p=p)
    out = {"workload": f"uniform n={n} p={p}, all {math.comb(n, p)} hub sets", "sets": math.comb(n, p)}
    best = {}
    for prec in ("split_bf16", "fp64"):
        with hubga.Solver(inst.C, inst.W, p, chi=inst.chi, alpha=inst.alpha, delta=inst.delta,
                          population=population, island_size=64, precision=prec) as s:
            s.enumerate(first=0, count=population)           # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.enumerate()
            dt = time.perf_counter() - t0
        out[prec] = {"sets_per_s": out["sets"] / dt, "seconds": dt, "rechecks": r["rechecks"]}
        best[prec] = (r["rank"], r["cost"])
    out["same_optimum"] = best["split_bf16"] == best["fp64"]
    out["best_rank"], out["best_cost"] = best["fp64"]
    return out


def sweep_leg(generations=100, population=256):
    """The chi = delta / alpha / p sweep of Sec. 6.2 (Fig. 3) on the CAB-sized
    instance through the server: solves per second and each cell's average
    inter-hub distance and whether the GA reached the exhaustive optimum."""
    from paper_1704_06258_amd import instances as I
    from paper_1704_06258_amd import sweep
    inst = I.small()
    cells = sweep.sweep_grid([2, 3, 4], [1.0, 2.0, 3.0], [0.2, 0.4, 0.6, 0.8, 1.0])
    got, wall = sweep.run_sweep(inst.C64(), inst.W64(), cells, generations=generations, population=population,
                                island_size=64, n1=10, seed=1, exhaustive=True)
    return {"workload": f"small n=25 (CAB-sized), p in 2..4, chi = delta in 1..3, alpha in 0.2..1.0, "
                        f"{generations} generations, population {population}",
            "cells": len(cells), "solves_per_s": len(cells) / wall, "seconds": wall,
            "optimal_cells": int(sum(bool(c.optimal) for c in got)),
            "rows": [[c.p, c.chi, c.alpha, round(c.interhub, 3), bool(c.optimal)] for c in got],
            "row_fields": ["p", "chi=delta", "alpha", "average inter-hub distance", "GA reached the optimum"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison")
    ap.add_argument("--workload", default="clustered", choices=sorted(WORKLOADS))
    ap.add_argument("--tile-config", default="auto",
                    help="tile configuration of the batched kernel: an index, or 'auto' to run the autotuner "
                         "(outside the timed region)")
    ap.add_argument("--serve-requests", type=int, default=2200,
                    help="requests of the serving leg (Poisson arrivals at 200/s, size mix n in "
                         "{50..2000}, p in {3,5,10,20}, population in {256..2048}, 100 generations, one "
                         "instance per request); 0 skips it")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-only", action="store_true", help="only the serving leg")
    ap.add_argument("--no-enumerate", action="store_true", help="skip the exhaustive-search leg")
    ap.add_argument("--no-sweep", action="store_true", help="skip the factor-sweep leg")
    ap.add_argument("--steady-steps", type=int, default=200,
                    help="generations timed after the headline window and 200 more generations (0 skips)")
    ap.add_argument("--prewarm-ms", type=float, default=0.0,
                    help="before the timed generations, re-evaluate the population with the batched kernel for "
                         "this long (GA state untouched), so the device runs at its sustained clock")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run an elementwise copy of 256 MiB (reads 256 MiB, writes 256 MiB) five times, "
                         "to scale HBM byte counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(64 * 2**20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "elementwise copy", "bytes_read": a.numel() * 4,
                          "bytes_written": b.numel() * 4, "launches": 5}))
        return
    if args.serve_only:
        print(json.dumps({"serving": serving_leg(args.serve_requests, args.serve_warmup)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_06258_amd import hubga
    from paper_1704_06258_amd import instances as I

    hubga.lib()
    factory, N, P, S, M, N1, wdesc = WORKLOADS[args.workload]
    inst = getattr(I, factory)()
    kw = dict(chi=inst.chi, alpha=inst.alpha, delta=inst.delta, scale=inst.scale, seed=1, population=S,
              island_size=M, n1=N1)
    solver = hubga.Solver(inst.C, inst.W, inst.p, precision="split_bf16", **kw)
    log(f"headline: {wdesc}")
    if args.tile_config == "auto":
        from paper_1704_06258_amd import autotune
        solver.step(1)
        tune = autotune.autotune(solver, force=True)
        tile_cfg = tune["config"]
    else:
        tile_cfg = int(args.tile_config)
        tune = None
        solver.set_tile_config(tile_cfg)
    torch.cuda.synchronize()
    prewarm = None
    if args.prewarm_ms > 0:
        hubs, _ = solver.population()
        if not np.all(np.diff(hubs, axis=1) > 0):   # before the first generation: the ancestors
            anc, _ = solver.ancestors()
            hubs = np.repeat(anc, S // anc.shape[0], axis=0)
        d_hubs = torch.from_numpy(np.ascontiguousarray(hubs)).to(solver.device)
        t0, k = time.perf_counter(), 0
        while time.perf_counter() - t0 < args.prewarm_ms / 1e3:
            for _ in range(8):
                solver.evaluate_dev(d_hubs)
            torch.cuda.synchronize()
            k += 8
        prewarm = {"ms": round(1e3 * (time.perf_counter() - t0), 1), "evaluations_of_the_population": k}
    pre = 1 if args.tile_config == "auto" else 0   # the generation the autotuner's population came from
    dt, kms, launches = time_steps(solver, args.steps, args.warmup)
    ms_per_step = 1e3 * dt / args.steps
    window = [pre + args.warmup, pre + args.warmup + args.steps - 1]   # generations timed (0-based)
    steady = None
    if args.steady_steps > 0:
        solver.step(200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.step(args.steady_steps)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t0
        g0 = window[1] + 1 + 20 + 200     # after the kernel-profiled generations and 200 more
        steady = {"generations": [g0, g0 + args.steady_steps - 1], "ms_per_step": 1e3 * dts / args.steady_steps,
                  "evals_per_s": S * args.steady_steps / dts}
    log(f"headline: {ms_per_step:.3f} ms per generation over generations {window[0]}-{window[1]}")
    value = S * args.steps / dt
    k_avg_ms = kms / max(launches, 1)
    folded = solver.folded()
    flop_launch = flops_per_eval(N, P, folded) * S
    achieved = flop_launch / (k_avg_ms * 1e-3) / 1e12
    stats = solver.stats()
    out = {
        "metric": "fitness evals/sec at n=1000,p=20 (batched MFMA vs plain) + p99 solve latency",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": wdesc,
                   "n": N, "p": P, "population": S, "islands": S // M, "n1": N1,
                   "precision": "W = bf16 hi + lo, FP32 accumulate, FP64 epilogue and selection",
                   "instance_sha256": inst.sha256()},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS,
                     # the committed counter summary covers the clustered workload only
                     "traffic": traffic_from_profile() if args.workload == "clustered" else None,
                     "kernel": "k_eval_mfma", "avg_launch_ms": k_avg_ms, "launches": launches,
                     "flop_per_launch": flop_launch, "folded": folded,
                     "unfolded_flop_per_launch": flops_per_eval(N, P) * S, "tile_config": tile_cfg,
                     "tile": hubga.tile_configs()[tile_cfg],
                     "autotune_ms": tune["ms"] if tune else None},
        "recheck_per_generation": stats["rechecks"] / max(stats["generations"], 1),
        "timed_generations": window,
        "steady": steady,
        "prewarm": prewarm,
    }
    gpu_hubs, gpu_cost = solver.population()
    solver.close()

    if not args.no_plain:
        # the same generations as the batched leg's timed window
        plain = {}
        steps = args.steps if N <= 2000 else min(args.steps, 3)
        # plain per-individual kernels (FP64, FP32) and the batched FP32 vector kernel
        for name, prec, kern in (("fp64", "fp64", "plain"), ("fp32", "fp32", "plain"),
                                 ("fp32_vector_batched", "fp32", "batched"),
                                 ("split3_bf16_batched", "split3_bf16", "batched")):
            s2 = hubga.Solver(inst.C, inst.W, inst.p, precision=prec, kernel=kern, **kw)
            if prec == "split3_bf16":
                from paper_1704_06258_amd import autotune
                s2.step(1)
                autotune.autotune(s2, force=True)
            dt2, kms2, l2 = time_steps(s2, steps, pre + args.warmup, kernel_steps=3)
            s2.close()
            plain[name] = {"evals_per_s": S * steps / dt2, "ms_per_step": 1e3 * dt2 / steps,
                           "kernel_avg_ms": kms2 / max(l2, 1),
                           "timed_generations": [pre + args.warmup, pre + args.warmup + steps - 1]}
            log(f"{name}: {1e3 * dt2 / steps:.3f} ms per generation, kernel {kms2 / max(l2, 1):.3f} ms")
        out["plain"] = plain
        out["speedup_vs_plain_fp64"] = value / plain["fp64"]["evals_per_s"]
        out["speedup_vs_plain_fp32"] = value / plain["fp32"]["evals_per_s"]
        out["speedup_vs_fp32_vector_batched"] = value / plain["fp32_vector_batched"]["evals_per_s"]

    if not args.no_enumerate and args.workload == "clustered":
        out["enumeration"] = enumeration_leg()
        log(f"enumeration: {out['enumeration']['split_bf16']['sets_per_s']:.3g} sets/s")
    if not args.no_sweep and args.workload == "clustered":
        out["sweep"] = sweep_leg()
        log(f"sweep: {out['sweep']['cells']} cells in {out['sweep']['seconds']:.2f} s")
    if args.serve_requests > 0 and args.workload == "clustered":
        out["serving"] = serving_leg(args.serve_requests, min(args.serve_warmup, args.serve_requests // 2))
        log(f"serving: p50 {out['serving']['p50_latency_s']} s, p99 {out['serving']['p99_latency_s']} s")

    if not args.no_cpu:
        cb, err = cpu_baseline(inst, gpu_hubs, gpu_cost, label=f"n={N}, p={P}")
        out["cpu_baseline"] = cb
        out["max_rel_err_vs_oracle"] = err
        log(f"cpu baseline: {cb['value']:.0f} evals/s at {cb['cores']} threads")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
