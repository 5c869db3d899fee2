"""GPU: the C ABI used from C.  A small C program (tests/c_abi_client.c),
built with gcc against include/hubga.h and libhubga.so, evaluates and solves
an instance with a library-allocated workspace on the null stream; its output
is checked against the FP64 oracle (costs within the returned bounds, GA
result equal to the oracle's trajectory)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1704_06258_amd import hubga
from paper_1704_06258_amd import instances as I

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_client(tmp_path):
    hubga.lib()
    exe = tmp_path / "c_abi_client"
    libdir = os.path.dirname(hubga.LIB_PATH)
    subprocess.run(["gcc", "-O1", "-o", str(exe), os.path.join(ROOT, "tests", "c_abi_client.c"),
                    "-I", os.path.join(ROOT, "include"), "-L", libdir, "-lhubga", "-Wl,-rpath," + libdir],
                   check=True)
    inst = I.uniform(seed=77, n=90, p=6)
    hubs = I.random_hub_sets(3, inst.n, inst.p, 5)
    blob = tmp_path / "inst.bin"
    with open(blob, "wb") as f:
        f.write(np.array([inst.n, inst.p, len(hubs)], np.int32).tobytes())
        f.write(inst.C64().tobytes())
        f.write(inst.W64().tobytes())
        f.write(hubs.astype(np.int32).tobytes())
    out = subprocess.run([str(exe), str(blob), "12"], check=True, capture_output=True, text=True, timeout=120).stdout
    lines = dict()
    costs = []
    for ln in out.splitlines():
        k, _, v = ln.partition(" ")
        if k == "cost":
            _, c, e = v.split()
            costs.append((float(c), float(e)))
        else:
            lines[k] = v
    assert lines["invalid_init"] == "GA_ERR_INVALID" and lines["invalid_eval"] == "GA_ERR_INVALID"
    assert lines["wrong_state"] == "GA_ERR_STATE"
    ref, _ = oracle.evaluate(inst.C64(), inst.W64(), hubs, 3.0, 0.75, 2.0)
    for (c, e), r in zip(costs, ref):
        assert abs(c - r) <= e * r
    st = oracle.ga_init(inst.C64(), inst.W64(), inst.p, 64, 16, 3.0, 0.75, 2.0)
    oracle.ga_run(inst.C64(), inst.W64(), st, 12, S=64, m=16, n1=5, seed=11, chi=3.0, alpha=0.75, delta=2.0)
    assert float(lines["best_cost"]) == st.best_cost[0]
    assert [int(x) for x in lines["best_hubs"].split()] == st.best.tolist()
    assert lines["stats"].split()[0] == "12"
