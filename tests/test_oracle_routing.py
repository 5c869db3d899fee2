"""Pins of the oracle's multi-hop routing (eq. (4) of Sec. 3): the transfer
term read through the all-pairs shortest-path distances of C.

* Floyd-Warshall against scipy's independent shortest-path routines on
  integer non-metric weights (exact arithmetic), symmetric and asymmetric;
* the routed cost against the MIP of Sec. 3 solved for its Y variables by a
  linear program (scipy's HiGHS) with the allocation fixed: objective (1)
  under constraints (4) and Y >= 0;
* with a metric C the routed cost is the direct one; with a triangle
  violation between hubs it is strictly cheaper.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_1704_06258_amd import instances as I


def integer_nonmetric(seed, n, symmetric=True):
    rng = np.random.default_rng(seed)
    C = rng.integers(1, 60, size=(n, n)).astype(np.float64)
    if symmetric:
        C = np.triu(C, 1)
        C = C + C.T
    np.fill_diagonal(C, 0.0)
    return C


@pytest.mark.parametrize("symmetric", [True, False])
def test_shortest_paths_match_scipy_exactly(symmetric):
    for seed in range(4):
        C = integer_nonmetric(seed, 17, symmetric)
        D = oracle.shortest_paths(C)
        assert np.array_equal(D, shortest_path(C, method="D", directed=True))
        assert np.array_equal(D, shortest_path(C, method="FW", directed=True))
        assert np.all(D <= C) and np.array_equal(oracle.shortest_paths(D), D)
        if symmetric:
            assert np.array_equal(D, D.T)


def routed_lp(C, W, a, chi, alpha, delta):
    """Objective (1) with Z fixed by the allocation a, minimised over the
    flows Y_kl^i >= 0 (every arc k != l) subject to the conservation
    constraints (4); returns the optimal value."""
    n = len(a)
    Z = np.zeros((n, n))
    Z[np.arange(n), a] = 1.0
    O, D = W.sum(axis=1), W.sum(axis=0)
    arcs = [(k, l) for k in range(n) for l in range(n) if k != l]
    nv = n * len(arcs)                       # variable (i, arc)
    cost = np.array([alpha * C[k, l] for i in range(n) for (k, l) in arcs])
    A = np.zeros((n * n, nv))
    b = np.zeros(n * n)
    for i in range(n):
        for q, (k, l) in enumerate(arcs):
            A[i * n + k, i * len(arcs) + q] += 1.0       # out of k
            A[i * n + l, i * len(arcs) + q] -= 1.0       # into l
        for k in range(n):
            b[i * n + k] = O[i] * Z[i, k] - W[i] @ Z[:, k]
    res = linprog(cost, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert res.status == 0
    fixed = float((C * Z).sum(axis=1) @ (chi * O + delta * D))
    return fixed + res.fun


def test_routed_cost_is_the_mip_optimum_over_flows():
    rng = np.random.default_rng(5)
    n = 6
    for seed in range(3):
        C = integer_nonmetric(10 + seed, n, symmetric=seed != 1)
        W = rng.integers(0, 9, size=(n, n)).astype(np.float64)
        Cs = oracle.shortest_paths(C)
        for hubs in [(0, 3), (1, 2, 5)]:
            a, _ = oracle.allocate(C, np.array(hubs, np.int32))
            f, _ = oracle.cost_alloc(C, W, a, 2.0, 0.6, 1.5, Ctr=Cs)
            ref = routed_lp(C, W, a, 2.0, 0.6, 1.5)
            assert abs(f - ref) <= 1e-9 * ref, (f, ref)


def test_metric_routing_equals_direct_and_violation_is_cheaper():
    inst = I.small(seed=7, n=20, p=3)
    C, W = inst.C64(), inst.W64()
    hubs = I.random_hub_sets(3, 20, 3, 20)
    direct, _ = oracle.evaluate(C, W, hubs, inst.chi, inst.alpha, inst.delta)
    routed, _ = oracle.evaluate(C, W, hubs, inst.chi, inst.alpha, inst.delta, Ctr=oracle.shortest_paths(C))
    assert np.allclose(routed, direct, rtol=1e-12, atol=0)
    # hubs 0 and 1 far apart directly but close through node 2
    C = np.array([[0, 100, 1, 5], [100, 0, 1, 5], [1, 1, 0, 5], [5, 5, 5, 0]], dtype=np.float64)
    W = np.ones((4, 4)) - np.eye(4)
    h = np.array([[0, 1]], np.int32)
    direct, dp = oracle.evaluate(C, W, h, 1.0, 1.0, 1.0)
    routed, rp = oracle.evaluate(C, W, h, 1.0, 1.0, 1.0, Ctr=oracle.shortest_paths(C))
    assert routed[0] < direct[0] and rp[0, 1] < dp[0, 1]
    assert rp[0, 0] == dp[0, 0] and rp[0, 2] == dp[0, 2]      # collection and distribution use C itself


def test_nonmetric_recipe_violates_triangle_inequality():
    inst = I.nonmetric(n=60)
    C = inst.C64()
    assert np.array_equal(C, C.T) and np.all(np.diag(C) == 0)
    D = oracle.shortest_paths(C)
    assert np.mean(D < C) > 0.2        # many pairs have a shorter detour
