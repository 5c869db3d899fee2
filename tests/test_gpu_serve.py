"""GPU: the continuous-batching server.  Requests of mixed n, p and
population share the GPU (admitted by HBM budget and slots, joining and
leaving at generation boundaries); every result must be bit-identical (hub
set and exact cost) to the same request solved alone."""
import numpy as np
import pytest

from paper_1704_06258_amd import hubga, serve
from paper_1704_06258_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hubga.lib()
    yield


def requests(k=10, gens=30):
    out = []
    sizes = [(50, 3, 256), (100, 5, 512), (200, 10, 256), (150, 20, 256), (120, 2, 256)]
    for r in range(k):
        n, p, S = sizes[r % len(sizes)]
        inst = I.uniform(seed=100 + r, n=n, p=p)
        # arrivals 0.2 ms apart, well inside one request's service time
        out.append(serve.SolveRequest(r, 0.0002 * r, inst.C, inst.W, p, inst.chi, inst.alpha, inst.delta, S,
                                      gens + (r % 3), 7 + r))
    return out


@pytest.mark.parametrize("realtime", [False, True])
def test_served_results_equal_alone(realtime):
    reqs = requests()
    budget = 4 * max(serve.workspace_bytes(r) for r in reqs)
    srv = serve.Server(hbm_budget=budget, max_slots=4)
    res = srv.run(reqs, realtime=realtime)
    srv.close()
    assert sorted(r.rid for r in res) == list(range(len(reqs)))
    assert srv.max_resident > 1            # requests really shared the GPU
    for r in res:
        alone = serve.solve_alone(reqs[r.rid])
        assert np.array_equal(r.hubs, alone["hubs"]), r.rid
        assert r.cost == alone["cost"], r.rid
        assert r.generations == reqs[r.rid].generations
    stats = serve.latency_stats(res)
    assert stats["p99_s"] >= stats["p50_s"] > 0
