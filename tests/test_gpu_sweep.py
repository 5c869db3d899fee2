"""GPU: the chi/delta/alpha sweep (the study of Fig. 3, Sec. 6.2) on the
CAB-sized instance.  Every cell, solved through the batching server beside
the others, equals the oracle's GA for that cell bit for bit (hub set and
exact cost); its average inter-hub distance is that of the oracle's
solution; its exhaustive optimum equals the oracle's enumeration."""
import numpy as np
import pytest

import oracle
from paper_1704_06258_amd import hubga, sweep
from paper_1704_06258_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hubga.lib()
    yield


def test_sweep_cells_equal_oracle():
    inst = I.small()
    C, W = inst.C64(), inst.W64()
    cells = sweep.sweep_grid([2, 3, 4], [1.0, 3.0], [0.2, 1.0])
    G, S, m, n1 = 30, 128, 32, 5
    got, wall = sweep.run_sweep(C, W, cells, generations=G, population=S, island_size=m, n1=n1, seed=1,
                                exhaustive=True)
    assert wall > 0 and len(got) == len(cells)
    for cell, (p, chi, alpha, delta) in zip(got, cells):
        st = oracle.ga_init(C, W, p, S, m, chi, alpha, delta)
        oracle.ga_run(C, W, st, G, S=S, m=m, n1=n1, seed=1, chi=chi, alpha=alpha, delta=delta)
        assert np.array_equal(cell.hubs, st.best), (p, chi, alpha)
        assert cell.cost == st.best_cost[0]
        assert cell.interhub == sweep.average_interhub_distance(C, st.best)
        best, hubs, _, _ = oracle.enumerate_best(C, W, p, chi, alpha, delta)
        assert cell.optimum == best and np.array_equal(cell.optimum_hubs, hubs)
        assert cell.cost >= cell.optimum
    rows = sweep.summary(got)
    assert len(rows) == len(cells) and all(r["optimal"] in (True, False) for r in rows)
