"""GPU: the three-part bf16 split (precision SPLIT3_BF16: W = hi + mid + lo,
|W - hi - mid - lo| <= 2^-24 W).  Bars: every cost within its returned bound
of the oracle's in each tile configuration the three-part split runs in
(0, 2, 3, 5), over ragged n and counts, p from 1 to 64, asymmetric and FP32
instances (the measured errors of both splits are printed); GA trajectories
equal to the oracle's; other tile configurations refused."""
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


def make(inst, precision="split3_bf16", **kw):
    return hubga.Solver(inst.C, inst.W, inst.p, chi=inst.chi, alpha=inst.alpha, delta=inst.delta,
                        scale=inst.scale, precision=precision, **kw)


CASES = [("clustered_n1000_p20", lambda: I.clustered(), 256),
         ("ragged_n129_p7_count37", lambda: I.uniform(seed=21, n=129, p=7), 37),
         ("p1_n200", lambda: I.uniform(seed=22, n=200, p=1), 64),
         ("p64_n300", lambda: I.uniform(seed=23, n=300, p=64), 64),
         ("asym_n140_p9", lambda: I.random_asymmetric(seed=24, n=140, p=9), 64),
         ("float32_n384_p50", lambda: I.large(seed=4, n=384, p=50), 64)]


@pytest.mark.parametrize("name,mk,count", CASES, ids=[c[0] for c in CASES])
def test_split3_within_bound_every_config(name, mk, count):
    inst = mk()
    hubs = I.random_hub_sets(5, inst.n, inst.p, count)
    ref, ref_parts = oracle.evaluate(inst.C64(), inst.W64(), hubs, inst.chi, inst.alpha, inst.delta, inst.scale)
    pop = max(2, count + (count % 2))
    with make(inst, precision="split_bf16", population=pop, island_size=2) as s:
        err2 = np.abs(s.evaluate(hubs)["cost"] - ref) / ref
    for cfg in (0, 2, 3, 5):
        with make(inst, population=pop, island_size=2) as s:
            s.set_tile_config(cfg)
            out = s.evaluate(hubs)
        err = np.abs(out["cost"] - ref) / ref
        assert np.all(err <= out["eps"]), (cfg, err.max())
        assert np.allclose(out["parts"][:, [0, 2]], ref_parts[:, [0, 2]], rtol=2.0 ** -23, atol=0)
        print(f"{name} cfg {cfg}: max error three parts {err.max():.3g}, two parts {err2.max():.3g}, "
              f"bound {out['eps'].min():.3g}", flush=True)
        if name.startswith("clustered"):
            assert err.max() <= 1e-7, err.max()


def test_split3_trajectory_equals_oracle():
    inst = I.medium()
    st = oracle.ga_init(inst.C64(), inst.W64(), inst.p, 1024, 64, inst.chi, inst.alpha, inst.delta)
    oracle.ga_run(inst.C64(), inst.W64(), st, 15, S=1024, m=64, n1=5, seed=2, chi=inst.chi, alpha=inst.alpha,
                  delta=inst.delta)
    with make(inst, population=1024, island_size=64, n1=5, seed=2) as s:
        s.step(15)
        anc, anc_cost = s.ancestors()
        best = s.best()
    assert np.array_equal(anc, st.anc) and np.array_equal(anc_cost, st.anc_cost)
    assert np.array_equal(best["hubs"], st.best) and best["cost"] == st.best_cost[0]


def test_split3_refuses_pipelined_configs():
    inst = I.uniform(seed=25, n=100, p=5)
    with make(inst, population=64) as s:
        for cfg in (1, 4, 6, 16, 21):
            with pytest.raises(hubga.HubGAError) as e:
                s.set_tile_config(cfg)
            assert e.value.status == hubga.GA_ERR_INVALID
        s.step(2)                                 # the context keeps working in its configuration
