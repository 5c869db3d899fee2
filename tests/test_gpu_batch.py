"""GPU: graph-replayed generations and multi-context batches.

Bar: every context's GA state (ancestors, exact costs, best so far,
generation) after batched generations is bit-identical to stepping it alone and
to the oracle's trajectory, whatever else shares the batch.
"""
import numpy as np
import pytest

import oracle
from paper_1704_06258_amd import hubga
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


def state_of(s):
    anc, cost = s.ancestors()
    b = s.best()
    return anc, cost, b["hubs"], b["cost"], b["generation"], s.get_state()


def same(a, b):
    return all(np.array_equal(x, y) if isinstance(x, np.ndarray) else x == y for x, y in zip(a, b))


def test_graph_replay_equals_direct_launches():
    inst = I.medium()
    kw = dict(population=512, island_size=64, n1=4, seed=3, precision="split_bf16")
    with make(inst, **kw) as a, make(inst, **kw) as b:
        a.step(9)                      # graph replay
        b.profile_enable(True)         # profiling launches kernels directly
        b.step(9)
        b.profile_enable(False)
        sa = state_of(a)
        assert same(sa, state_of(b))
    st = oracle.ga_init(inst.C64(), inst.W64(), inst.p, 512, 64, inst.chi, inst.alpha, inst.delta)
    oracle.ga_run(inst.C64(), inst.W64(), st, 9, S=512, m=64, n1=4, seed=3, chi=inst.chi, alpha=inst.alpha,
                  delta=inst.delta)
    assert np.array_equal(sa[0], st.anc) and sa[3] == st.best_cost[0]


MIX = [  # (instance, population, island, precision)
    (lambda: I.uniform(seed=1, n=200, p=10), 512, 64, "split_bf16"),
    (lambda: I.uniform(seed=2, n=500, p=5), 256, 64, "split_bf16"),
    (lambda: I.uniform(seed=3, n=100, p=3), 1024, 64, "split_bf16"),
    (lambda: I.uniform(seed=4, n=150, p=2), 256, 32, "split_bf16"),   # p < 3: own matrix-core launch
    (lambda: I.small(seed=5), 64, 16, "fp64"),
    (lambda: I.uniform(seed=6, n=120, p=7), 256, 64, "fp32"),
]


@pytest.mark.parametrize("cfg", [7, 6, 10, 14, 16, 17, 18])
def test_batch_equals_alone(cfg):
    import torch
    insts = [(mk(), S, m, prec) for mk, S, m, prec in MIX]
    alone = []
    for k, (inst, S, m, prec) in enumerate(insts):
        with make(inst, population=S, island_size=m, n1=3, seed=10 + k, precision=prec) as s:
            s.step(7)
            alone.append(state_of(s))
    batch = hubga.Batch(tile_config=cfg)
    members = [make(inst, population=S, island_size=m, n1=3, seed=10 + k, precision=prec, stream=batch.stream)
               for k, (inst, S, m, prec) in enumerate(insts)]
    batch.set(members)
    batch.step(7)
    batch.synchronize()
    for k, s in enumerate(members):
        assert same(state_of(s), alone[k]), k
    for s in members:
        s.close()
    batch.close()
    torch.cuda.synchronize()


def test_batch_recomposition_and_oracle():
    insts = [I.uniform(seed=20 + k, n=150 + 50 * k, p=4 + k) for k in range(3)]
    batch = hubga.Batch(tile_config=7)
    sol = [make(inst, population=256, island_size=32, n1=2, seed=k, precision="split_bf16", stream=batch.stream)
           for k, inst in enumerate(insts)]
    batch.set(sol[:2])
    batch.step(3)
    batch.set(sol[1:])
    batch.step(2)
    batch.set([sol[0]])
    batch.step(4)
    batch.synchronize()
    gens = {0: 7, 1: 5, 2: 2}
    for k, inst in enumerate(insts):
        st = oracle.ga_init(inst.C64(), inst.W64(), inst.p, 256, 32, inst.chi, inst.alpha, inst.delta)
        oracle.ga_run(inst.C64(), inst.W64(), st, gens[k], S=256, m=32, n1=2, seed=k, chi=inst.chi,
                      alpha=inst.alpha, delta=inst.delta)
        anc, cost, hubs, bc, g, _ = state_of(sol[k])
        assert g == gens[k]
        assert np.array_equal(anc, st.anc) and np.array_equal(cost, st.anc_cost)
        assert np.array_equal(hubs, st.best) and bc == st.best_cost[0]
    for s in sol:
        s.close()
    batch.close()


def test_batch_rejects_foreign_stream_and_empty_is_noop():
    inst = I.small()
    batch = hubga.Batch(tile_config=7)
    with make(inst, population=64, island_size=32, precision="split_bf16") as s:
        with pytest.raises(hubga.HubGAError):
            batch.set([s])
    batch.set([])
    batch.step(3)
    with pytest.raises(hubga.HubGAError):
        hubga.Batch(tile_config=0)    # not a pipelined configuration
    batch.close()


def test_set_stream_keeps_order_and_trajectory():
    import torch
    inst = I.medium()
    kw = dict(population=512, island_size=64, n1=4, seed=8, precision="split_bf16")
    with make(inst, **kw) as a:
        a.step(7)
        ref = state_of(a)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with make(inst, stream=s1, **kw) as b:
        b.step(3)                      # queued on s1, not waited for
        b.set_stream(s2)
        b.step(4)
        assert same(state_of(b), ref)


def test_many_contexts_share_the_reevaluation_pool():
    """Two dozen split-bf16 contexts of different sizes in one batch: early
    generations give them very different numbers of exactly re-evaluated
    candidates, all drawn from one pool; each state must equal stepping alone."""
    import torch
    specs = [(60 + 37 * (k % 7), 3 + (k % 5), 128 * (1 + k % 3), 32) for k in range(24)]
    insts = [I.uniform(seed=200 + k, n=n, p=p) for k, (n, p, S, m) in enumerate(specs)]
    alone = []
    for k, (inst, (n, p, S, m)) in enumerate(zip(insts, specs)):
        with make(inst, population=S, island_size=m, n1=3, seed=40 + k, precision="split_bf16") as s:
            s.step(5)
            alone.append(state_of(s))
    batch = hubga.Batch(tile_config=16)
    members = [make(inst, population=S, island_size=m, n1=3, seed=40 + k, precision="split_bf16",
                    stream=batch.stream) for k, (inst, (n, p, S, m)) in enumerate(zip(insts, specs))]
    batch.set(members)
    batch.step(5)
    batch.synchronize()
    assert sum(s.stats()["rechecks"] for s in members) > 0
    for k, s in enumerate(members):
        assert same(state_of(s), alone[k]), k
    for s in members:
        s.close()
    batch.close()
    torch.cuda.synchronize()


def test_member_evaluated_alone_between_batch_steps():
    """A grouped member evaluated on its own tile configuration between
    batched generations (its W split rewritten to that configuration's layout
    and back) keeps the trajectory of stepping alone."""
    inst = I.uniform(seed=7, n=300, p=8)
    kw = dict(population=512, island_size=64, n1=3, seed=4, precision="split_bf16")
    hubs = I.random_hub_sets(9, inst.n, inst.p, 32)
    with make(inst, **kw) as a:
        a.step(6)
        ref = state_of(a)
        ref_eval = a.evaluate(hubs)["cost"]
    batch = hubga.Batch(tile_config=16)
    with make(inst, stream=batch.stream, **kw) as s:
        batch.set([s])
        batch.step(3)
        got_eval = s.evaluate(hubs)["cost"]          # tile configuration 0: row-major split
        batch.step(3)                                # the batch's folded split again
        batch.synchronize()
        assert same(state_of(s), ref)
    batch.close()
    assert np.array_equal(got_eval, ref_eval)


def test_recomposition_replays_or_recaptures_the_batch_graph():
    """Compositions that shrink (the captured graph replays with idle
    workgroups) and grow beyond its capacity (captured anew), with eager work
    between replays: every member ends where stepping it alone ends."""
    insts = [I.uniform(seed=21, n=200, p=6), I.uniform(seed=22, n=90, p=4), I.uniform(seed=23, n=600, p=12)]
    kw = dict(island_size=64, n1=3, precision="split_bf16")
    pops = [256, 128, 1024]
    steps = [(0, 1), (0, 1), (0,), (0, 1, 2), (2,), (0, 1, 2)]   # members of each batch phase, 2 generations each
    gens = [sum(2 for ph in steps if k in ph) for k in range(3)]
    alone = []
    for k, inst in enumerate(insts):
        with make(inst, population=pops[k], seed=30 + k, **kw) as s:
            s.step(gens[k])
            alone.append(state_of(s))
    batch = hubga.Batch(tile_config=16)
    members = [make(inst, population=pops[k], seed=30 + k, stream=batch.stream, **kw) for k, inst in enumerate(insts)]
    for ph in steps:
        batch.set([members[k] for k in ph])
        batch.step(1)
        members[ph[0]].ancestors()          # eager work and a wait between replays
        batch.step(1)
    batch.synchronize()
    for s, ref in zip(members, alone):
        assert same(state_of(s), ref)
        s.close()
    batch.close()
