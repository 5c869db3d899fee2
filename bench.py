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
baseline is the FP64 oracle timed on the host cores over a bounded sample.
"""
from __future__ import annotations

import argparse
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


def cpu_baseline(inst, gpu_hubs, gpu_cost, budget_s=12.0, label="n=1000, p=20"):
    """The FP64 oracle (OpenMP over individuals) on the GPU's last population:
    evaluations per second over a bounded sample, plus the measured error of
    the GPU's split-bf16 costs on that sample."""
    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    C, W = inst.C64(), inst.W64()
    done, t_used, k = 0, 0.0, 16
    errs = []
    pos = 0
    while t_used < budget_s:
        idx = np.arange(pos, pos + k) % len(gpu_hubs)
        t0 = time.perf_counter()
        ref, _ = oracle.evaluate(C, W, gpu_hubs[idx], inst.chi, inst.alpha, inst.delta, inst.scale)
        t_used += time.perf_counter() - t0
        errs.append(np.abs(gpu_cost[idx] - ref) / ref)
        done += k
        pos += k
        k = min(k * 2, 1024)
    err = np.concatenate(errs)
    return dict(value=done / t_used, unit="evals/s", cores=cores, kind="oracle",
                sample=f"{done} children of the last GPU generation ({label}), FP64 oracle, "
                       f"{t_used:.1f} s of CPU work"), float(err.max())


def serving_leg(count, warmup, rate=200.0, budget=16 << 30, slots=64):
    """Continuous-batching serving of a Poisson request stream: p50/p99
    latency from scheduled arrival to result, completed solves/s and
    evaluations/s.  Instances come from a pool of 4 seeded instances per size
    (generated before the run); every request has its own GA seed."""
    from paper_1704_06258_amd import instances as I
    from paper_1704_06258_amd import serve
    stream = I.serving_requests(count, rate=rate, seed=5, generations=100)
    pool = {}
    reqs = []
    for q in stream:
        key = (q.n, q.rid % 4)
        if key not in pool:
            pool[key] = I.uniform(seed=5_000_000 + 7 * q.n + key[1], n=q.n, p=3)
        inst = pool[key]
        reqs.append(serve.SolveRequest(q.rid, q.arrival, inst.C, inst.W, q.p, 3.0, 0.75, 2.0, q.S, q.generations,
                                       q.ga_seed))
    srv = serve.Server(hbm_budget=budget, max_slots=slots)
    t0 = time.perf_counter()
    res = srv.run(reqs, realtime=True)
    wall = time.perf_counter() - t0
    srv.close()
    measured = [r for r in res if r.rid >= warmup]
    st = serve.latency_stats(measured)
    evals = sum(reqs[r.rid].population * reqs[r.rid].generations for r in res)
    offered = rate * sum(q.population * q.generations for q in reqs) / len(reqs)
    return {"requests": count, "warmup": warmup, "rate_per_s": rate, "generations": 100,
            "offered_evals_per_s": offered,
            "p50_latency_s": st.get("p50_s"), "p99_latency_s": st.get("p99_s"), "mean_latency_s": st.get("mean_s"),
            "completed_per_s": len(res) / wall, "evals_per_s": evals / wall, "max_resident": srv.max_resident,
            "ticks": srv.ticks, "budget_bytes": budget, "slots": slots}


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
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests of the serving leg (Poisson arrivals at 200/s, size mix n in "
                         "{50..2000}, p in {3,5,10,20}, population in {256..2048}, 100 generations); 0 skips it")
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-full", action="store_true",
                    help="only the serving workload at full size: 200 warm-up + 2000 measured requests")
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
    if args.serve_full:
        print(json.dumps({"serving": serving_leg(2200, 200)}), flush=True)
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
    dt, kms, launches = time_steps(solver, args.steps, args.warmup)
    ms_per_step = 1e3 * dt / args.steps
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
    }
    gpu_hubs, gpu_cost = solver.population()
    solver.close()

    if not args.no_plain:
        plain = {}
        for prec in ("fp64", "fp32"):
            s2 = hubga.Solver(inst.C, inst.W, inst.p, precision=prec, **kw)
            steps = 10 if N <= 2000 else 2
            dt2, kms2, l2 = time_steps(s2, steps, 2, kernel_steps=3)
            s2.close()
            plain[prec] = {"evals_per_s": S * steps / dt2, "ms_per_step": 1e3 * dt2 / steps,
                           "kernel_avg_ms": kms2 / max(l2, 1)}
        out["plain"] = plain
        out["speedup_vs_plain_fp64"] = value / plain["fp64"]["evals_per_s"]
        out["speedup_vs_plain_fp32"] = value / plain["fp32"]["evals_per_s"]

    if args.serve_requests > 0 and args.workload == "clustered":
        out["serving"] = serving_leg(args.serve_requests, args.serve_warmup)

    if not args.no_cpu:
        cb, err = cpu_baseline(inst, gpu_hubs, gpu_cost, label=f"n={N}, p={P}")
        out["cpu_baseline"] = cb
        out["max_rel_err_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
