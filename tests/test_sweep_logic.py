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
