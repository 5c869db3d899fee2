"""GPU: exhaustive search of the nearest-hub space (ga_enumerate) against the
oracle's enumeration.  Bars: FP64 costs bit-identical; FP32 and split-bf16
costs within their returned bounds; in every precision the returned best
(hub set, exact cost, parts, rank) equals the oracle's argmin with ties to the
lowest rank, over several chunks with a ragged last one, sub-ranges, exact
ties, an asymmetric instance and the full n=100, p=3 space."""
import math

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


def check(inst, precision, population, first=0, count=None):
    C, W = inst.C64(), inst.W64()
    best, hubs, rank, costs = oracle.enumerate_best(C, W, inst.p, inst.chi, inst.alpha, inst.delta, inst.scale,
                                                   first=first, count=count)
    _, ref_parts = oracle.evaluate(C, W, hubs[None], inst.chi, inst.alpha, inst.delta, inst.scale)
    with make(inst, population=population, island_size=2, precision=precision) as s:
        out = s.enumerate(first=first, count=-1 if count is None else count, want_all=True)
    if precision == "fp64":
        assert np.array_equal(out["costs"], costs)
        assert out["rechecks"] == 0
    else:
        err = np.abs(out["costs"] - costs) / costs
        assert np.all(err <= out["eps"]), (err.max(), out["eps"].min())
        assert out["rechecks"] >= 1
    assert out["rank"] == rank and np.array_equal(out["hubs"], hubs)
    assert out["cost"] == best and np.array_equal(out["parts"], ref_parts[0])
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_bf16"])
def test_enumerate_n30_p3_all_sets(precision):
    inst = I.uniform(seed=80, n=30, p=3)      # 4060 sets: 7 full chunks of 512 and one of 476
    out = check(inst, precision, 512)
    assert len(out["costs"]) == math.comb(30, 3)


@pytest.mark.parametrize("precision", ["fp64", "split_bf16"])
def test_enumerate_subrange_and_asymmetric(precision):
    check(I.uniform(seed=81, n=30, p=3), precision, 256, first=1000, count=1500)
    check(I.random_asymmetric(seed=82, n=25, p=2), precision, 64)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_enumerate_exact_ties_go_to_lowest_rank(precision):
    n = 12                                   # a ring with unit flows: rotations cost exactly the same
    i = np.arange(n)
    d = np.abs(i[:, None] - i[None, :])
    C = np.minimum(d, n - d).astype(np.float64)
    W = np.ones((n, n)) - np.eye(n)
    inst = I.Instance("ring", C, W, 3, 1.0, 0.5, 1.0)
    out = check(inst, precision, 64)
    assert out["rechecks"] > 1


def test_enumerate_n100_p3_full_space():
    inst = I.uniform(seed=83, n=100, p=3)    # 161,700 sets through the batched kernel
    out = check(inst, "split_bf16", 4096)
    assert out["rechecks"] < 1000


def test_enumerate_rejects_bad_ranges():
    inst = I.uniform(seed=84, n=20, p=3)
    with make(inst, population=64) as s:
        for first, count in [(-1, 5), (math.comb(20, 3), 1), (0, 0), (10, math.comb(20, 3))]:
            with pytest.raises(hubga.HubGAError) as e:
                s.enumerate(first=first, count=count)
            assert e.value.status == hubga.GA_ERR_INVALID
        assert s.enumerate(first=5, count=3)["rank"] in (5, 6, 7)     # the context survives
    big = I.uniform(seed=85, n=400, p=64)
    with make(big, population=64) as s:
        with pytest.raises(hubga.HubGAError) as e:
            s.enumerate()
        assert e.value.status == hubga.GA_ERR_INVALID
