"""The factor sweep's host logic (no GPU): the average inter-hub distance
and the grid of cells."""
import numpy as np

from paper_1704_06258_amd import sweep


def test_average_interhub_distance_hand_worked():
    C = np.array([[0, 3, 4, 5],
                  [3, 0, 6, 7],
                  [4, 6, 0, 8],
                  [5, 7, 8, 0]], dtype=np.float64)
    assert sweep.average_interhub_distance(C, [0, 2, 3]) == (4 + 5 + 8) / 3
    assert sweep.average_interhub_distance(C, [1]) == 0.0
    A = C.copy()
    A[0, 1] = 1.0                               # asymmetric: both directions count
    assert sweep.average_interhub_distance(A, [0, 1]) == (1.0 + 3.0) / 2


def test_grid_ties_chi_to_delta():
    cells = sweep.sweep_grid([2, 3, 4], [1.0, 2.0, 3.0], [0.2, 0.4, 0.6, 0.8, 1.0])
    assert len(cells) == 45
    assert all(c[1] == c[3] for c in cells)
    assert cells[0] == (2, 1.0, 0.2, 1.0) and cells[-1] == (4, 3.0, 1.0, 3.0)


def test_autotuner_successive_halving_keeps_the_fastest():
    """The tile search times everything once, the fastest third three more
    times and the last three ten times; a configuration that is only fast on
    its first (noisy) timing does not win."""
    from paper_1704_06258_amd import autotune
    true_ms = {c: 1.0 + 0.05 * ((c * 7) % 22) for c in range(22)}
    calls = []

    def time_fn(c, r):
        calls.append((c, r))
        noise = -0.5 if (c == 13 and r == 1) else 0.0   # looks best once, is not
        return true_ms[c] + noise

    best, times, rounds = autotune.successive_halving(range(22), time_fn)
    assert best == min(true_ms, key=true_ms.get)
    assert [len(x) for x in rounds] == [7, 3, 1]
    assert sum(r for _, r in calls) == 22 * 1 + 7 * 3 + 3 * 10
    assert times[best] == true_ms[best]
