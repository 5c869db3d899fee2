"""GPU: the long and large workloads against the FP64 oracle, element by element.

* medium (n=200, p=10, population 1024 in 16 islands), FP32 evaluation with
  certified selection: the 500-generation trajectory equals the oracle's
  (ancestors, their exact costs and parts, best so far) at every 100th
  generation;
* large (n=6000, p=50, population 2048 in 32 islands, FP32 instance), split
  bf16 in the folded tile configuration the benchmark selects: three
  generations equal the oracle's trajectory bit for bit, the last
  generation's children are the oracle's, and every one of their 2048 costs
  lies within its error bound of the oracle's exact cost;
* serving mix: 32 requests drawn from the Poisson serving stream (its own
  per-request instance and GA seeds), among them n = 1000 and n = 2000 with
  p = 20 resident in one grouped batch, each served result bit-identical to
  the request solved alone.
"""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1704_06258_amd import hubga, serve
from paper_1704_06258_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hubga.lib()
    yield


def make(inst, **kw):
    return hubga.Solver(inst.C, inst.W, inst.p, chi=inst.chi, alpha=inst.alpha, delta=inst.delta,
                        scale=inst.scale, **kw)


def same_state(s, st):
    anc, anc_cost = s.ancestors()
    best = s.best()
    assert np.array_equal(anc, st.anc)
    assert np.array_equal(anc_cost, st.anc_cost)
    assert np.array_equal(best["hubs"], st.best) and best["cost"] == st.best_cost[0]
    assert np.array_equal(best["parts"], st.best_parts)
    assert best["generation"] == st.gen[0]


def test_medium_fp32_500_generations():
    inst = I.medium()
    C, W = inst.C64(), inst.W64()
    kw = dict(S=1024, m=64, n1=10, seed=1, chi=inst.chi, alpha=inst.alpha, delta=inst.delta)
    st = oracle.ga_init(C, W, inst.p, 1024, 64, inst.chi, inst.alpha, inst.delta)
    with make(inst, population=1024, island_size=64, n1=10, seed=1, precision="fp32") as s:
        for block in range(5):
            oracle.ga_run(C, W, st, 100, **kw)
            s.step(100)
            same_state(s, st)
            print(f"medium fp32: generation {st.gen[0]} equal", flush=True)
        stats = s.stats()
    assert stats["generations"] == 500 and stats["evaluations"] == 500 * 1024


def test_large_split_three_generations_and_full_population():
    inst = I.large()
    C, W = inst.C64(), inst.W64()
    S, m, seed = 2048, 64, 1
    kw = dict(S=S, m=m, n1=10, seed=seed, chi=inst.chi, alpha=inst.alpha, delta=inst.delta)
    t0 = time.time()
    st = oracle.ga_init(C, W, inst.p, S, m, inst.chi, inst.alpha, inst.delta)
    oracle.ga_run(C, W, st, 2, **kw)
    children = oracle.ga_children(inst.n, inst.p, S, m, seed, 2, st.anc)
    ref_cost, _ = oracle.evaluate(C, W, children, inst.chi, inst.alpha, inst.delta)
    oracle.ga_run(C, W, st, 1, **kw)
    print(f"large: oracle trajectory and population in {time.time() - t0:.1f} s", flush=True)
    with make(inst, population=S, island_size=m, n1=10, seed=seed, precision="split_bf16") as s:
        s.set_tile_config(16)
        assert s.folded()
        s.step(3)
        same_state(s, st)
        hubs, cost = s.population()
        out = s.evaluate(hubs)
    assert np.array_equal(hubs, children)
    assert np.array_equal(out["cost"], cost)          # the same kernel on the same sets
    err = np.abs(cost - ref_cost) / ref_cost
    assert np.all(err <= out["eps"]), (err.max(), out["eps"].min())
    print(f"large: max relative error {err.max():.3g}, smallest bound {out['eps'].min():.3g}", flush=True)


def serving_sample(k=32, pool=400):
    """k requests of the serving stream (Poisson arrivals, per-request
    instance seed 5e6 + r and GA seed r): every n = 1000 and n = 2000 request
    with p = 20 among the first ``pool``, the first two of each, then the
    earliest others."""
    reqs = I.serving_requests(pool, rate=200.0, seed=5, generations=100)
    big = [r for n in (1000, 2000) for r in [q for q in reqs if q.p == 20 and q.n == n][:2]]
    assert {r.n for r in big} == {1000, 2000}, "the stream prefix lacks a large p=20 request"
    rest = [r for r in reqs if r not in big][: k - len(big)]
    return big, rest


def test_serving_mix_sample_equals_alone():
    big, rest = serving_sample()
    reqs = []
    for q in big + rest:     # closed loop: the large requests are admitted first
        inst = q.instance()
        reqs.append(serve.SolveRequest(q.rid, 0.0, inst.C, inst.W, q.p, inst.chi, inst.alpha, inst.delta, q.S,
                                       q.generations, q.ga_seed))
    srv = serve.Server(hbm_budget=64 << 30, max_slots=len(reqs), workers=8)
    compositions = []
    orig_set, orig_admit = srv.batch.set, srv._admit
    big_ids = {q.rid for q in big}
    together = threading.Barrier(len(big_ids), timeout=120)

    def record(solvers):
        compositions.append([(s.n, s.p) for s in solvers])
        return orig_set(solvers)

    def admit(req, now):     # the large requests finish building together, so they join one tick
        job = orig_admit(req, now)
        if req.rid in big_ids:
            job.solver.stream.synchronize()
            together.wait()
        return job

    srv.batch.set = record
    srv._admit = admit
    res = srv.run(reqs, realtime=False)
    srv.close()
    print(f"serving sample: {len(res)} served, at most {srv.max_resident} resident", flush=True)
    assert sorted(r.rid for r in res) == sorted(q.rid for q in big + rest)
    assert any((1000, 20) in c and (2000, 20) in c for c in compositions), "large requests never shared a batch"
    by_rid = {r.rid: r for r in reqs}
    for r in res:
        assert r.error is None, r.error
        alone = serve.solve_alone(by_rid[r.rid])
        assert np.array_equal(r.hubs, alone["hubs"]), r.rid
        assert r.cost == alone["cost"], r.rid
        assert r.generations == 100
