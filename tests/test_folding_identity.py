"""The identity behind the folded batched product (CPU, numpy only).

With C symmetric, T = sum_{i,j} W_ij C[a(i)][a(j)] equals the same sum over
the folded matrix W' (W_ij + W_ji for j > i, W_ii on the diagonal, zero
below), so the matrix-core product may skip every K tile left of a row
tile's diagonal block.  With C asymmetric the identity fails, which is why
asymmetric instances are never folded.
"""
import numpy as np


def folded(W):
    F = np.triu(W + W.T, k=1)
    F[np.diag_indices_from(F)] = np.diag(W)
    return F


def transport(W, C, a):
    return float(np.sum(W * C[np.ix_(a, a)]))


def test_folded_sum_equals_full_sum_for_symmetric_c():
    rng = np.random.default_rng(7)
    for n, p in [(1, 1), (2, 1), (9, 3), (64, 5), (130, 7)]:
        xy = rng.uniform(0, 100, size=(n, 2))
        C = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
        assert np.array_equal(C, C.T)
        W = rng.lognormal(2.0, 1.0, size=(n, n))
        hubs = rng.choice(n, size=p, replace=False)
        a = hubs[np.argmin(C[:, hubs], axis=1)]   # any allocation will do
        full, fold = transport(W, C, a), transport(folded(W), C, a)
        assert abs(full - fold) <= 1e-12 * full


def test_folded_matrix_is_upper_triangular_with_the_same_total():
    rng = np.random.default_rng(8)
    W = rng.uniform(0, 1, size=(50, 50))
    F = folded(W)
    assert np.all(np.tril(F, k=-1) == 0)
    assert abs(F.sum() - W.sum()) <= 1e-12 * W.sum()


def test_asymmetric_c_breaks_the_identity():
    rng = np.random.default_rng(9)
    n = 40
    C = rng.uniform(1, 10, size=(n, n))
    W = rng.uniform(0, 1, size=(n, n))
    a = rng.integers(0, n, size=n)
    assert abs(transport(W, C, a) - transport(folded(W), C, a)) > 1e-6
