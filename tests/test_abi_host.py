"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/hubga.h declares, sizes workspaces and rejects invalid
arguments before any device work."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_1704_06258_amd import hubga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hubga.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ga_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hubga.LIB_PATH):
        from paper_1704_06258_amd import build
        build.build()
    return hubga.lib()


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(hubga.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_params_struct_layout_matches_header():
    # int32 n, p; 4 doubles; uint64 seed; 8 int32 -> 80 bytes with natural alignment
    assert ct.sizeof(hubga.ga_params) == 4 * 2 + 8 * 4 + 8 + 4 * 8
    q = hubga.ga_params_default(25, 3)
    assert (q.n, q.p, q.population, q.island_size, q.n1, q.elitist) == (25, 3, 64, 64, 10, 1)
    assert (q.chi, q.alpha, q.delta, q.scale, q.seed) == (3.0, 0.75, 2.0, 1.0, 1)


def test_workspace_bytes(L):
    q = hubga.make_params(1000, 20, chi=3, alpha=0.75, delta=2, population=4096, precision="split_bf16",
                          c_symmetric=True)
    b = hubga.ga_workspace_bytes(q)
    # C and W (binary64) plus the bf16 hi/lo copies padded to 1024 dominate
    assert b > 2 * 8 * 1000 * 1000 + 2 * 2 * 1024 * 1024
    assert b < 80 * 2**20
    q.c_symmetric = 0
    # an asymmetric C keeps its transpose (binary64, one row more)
    ct_bytes = 8 * (1000 * 1000 + 1000)
    diff = hubga.ga_workspace_bytes(q) - b
    assert abs(diff - ct_bytes) < 64 * 1024, diff
    assert hubga.ga_workspace_bytes(q, hubga.GA_DT_F32, hubga.GA_DT_F32) < hubga.ga_workspace_bytes(q)


def test_workspace_breakdown_large_fp32_instance():
    """n=6000, p=50, population 2048, FP32 C and W, C symmetric: C and W in
    their dtype (C's FP32 copy is C itself), one bf16 hi/lo pair of the padded
    W, the epilogue partials, the hub positions, the per-individual hub
    distance tables and the re-evaluation column sums make up the workspace;
    the rest is below 8 MB."""
    n, p, S, n_pad = 6000, 50, 2048, 6016
    q = hubga.make_params(n, p, chi=3, alpha=0.75, delta=2, population=S, precision="split_bf16", c_symmetric=True)
    b = hubga.ga_workspace_bytes(q, hubga.GA_DT_F32, hubga.GA_DT_F32)
    major = {"C": 4 * (n * n + n), "W": 4 * n * n, "W hi/lo": 2 * 2 * n_pad * n_pad,
             "partials": 8 * (n_pad // 64) * S * p, "hub positions": 2 * S * n_pad, "column sums": 8 * 512 * n,
             "hub distance tables": 4 * S * p * p}
    assert 0 <= b - sum(major.values()) < 8e6, (b, sum(major.values()))
    assert b < 600e6


@pytest.mark.parametrize("field,value", [("n", 0), ("p", 0), ("p", 26), ("island_size", 3), ("population", 96),
                                         ("n1", 0), ("elitist", 2), ("chi", -1.0), ("scale", 0.0),
                                         ("alpha", float("nan")), ("precision", 7), ("multihop", 2)])
def test_invalid_params_rejected_on_host(L, field, value):
    q = hubga.make_params(25, 3, chi=1, alpha=0.75, delta=1, population=64)
    setattr(q, field, value)
    assert hubga.ga_workspace_bytes(q) == 0
    C = np.zeros((25, 25))
    h = ct.c_void_p()
    st = L.ga_init(ct.byref(q), C.ctypes.data, 0, C.ctypes.data, 0, None, 0, None, ct.byref(h))
    assert st == hubga.GA_ERR_INVALID and not h.value
    assert L.ga_last_error(None).decode()


def test_invalid_combination_and_matrices_rejected(L):
    q = hubga.make_params(4, 2, chi=1, alpha=1, delta=1, population=4, island_size=2)
    q.kernel = hubga.GA_KERN_BATCHED   # FP64 needs the plain kernel
    assert hubga.ga_workspace_bytes(q) == 0
    q = hubga.make_params(4, 2, chi=1, alpha=1, delta=1, population=4, island_size=2)
    C = np.ones((4, 4))
    W = np.ones((4, 4))
    h = ct.c_void_p()
    W[1, 2] = -1.0
    assert L.ga_init(ct.byref(q), C.ctypes.data, 0, W.ctypes.data, 0, None, 0, None, ct.byref(h)) == \
        hubga.GA_ERR_INVALID
    assert "W" in L.ga_last_error(None).decode()
    W[1, 2] = np.inf
    assert L.ga_init(ct.byref(q), C.ctypes.data, 0, W.ctypes.data, 0, None, 0, None, ct.byref(h)) == \
        hubga.GA_ERR_INVALID
    W[1, 2] = 1.0
    q.c_symmetric = 1
    C[0, 1] = 2.0
    assert L.ga_init(ct.byref(q), C.ctypes.data, 0, W.ctypes.data, 0, None, 0, None, ct.byref(h)) == \
        hubga.GA_ERR_INVALID
    assert "symmetric" in L.ga_last_error(None).decode()


def test_null_context_calls(L):
    assert L.ga_step(None, 1) == hubga.GA_ERR_INVALID
    assert L.ga_status_str(hubga.GA_ERR_STATE) == b"GA_ERR_STATE"
    L.ga_free(None)
