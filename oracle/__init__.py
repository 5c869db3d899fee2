"""FP64 CPU oracle for the USApHMP parallel GA (arXiv 1704.06258).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does.  The
arithmetic lives in ``hub_oracle.c`` (plain C, binary64, no FMA contraction);
this module only compiles it with gcc and marshals numpy arrays through ctypes.

Each wrapper names the passage of the paper it follows:

* ``cost_alloc`` / ``evaluate`` -- objective (1) of Sec. 3 with direct
  hub-to-hub routing, i.e. the per-path cost chi*C_ik + alpha*C_kl + delta*C_jl
  of Sec. 6.2, optionally scaled as in Sec. 4.3;
* ``allocate`` -- nearest-hub allocation, hubs allocated to themselves
  (Sec. 4.1, Sec. 5);
* ``middle_nodes`` -- the initial solution from the p middle nodes (Sec. 4.1);
* ``ga_children`` / ``ga_run`` -- the island GA of Sec. 4.2 and Sec. 5;
* ``enumerate_best`` -- exhaustive search of the nearest-hub solution space,
  the optimum of Sec. 6.2's comparisons over the GA's search space;
* ``shortest_paths`` and the ``Ctr`` argument -- multi-hop routing of the
  inter-hub flow (eq. (4) of Sec. 3, read as routes along shortest paths).
* ``philox`` -- Philox4x64-10 (Salmon et al., SC'11), the counter-based
  generator that both sides implement from its published definition.
"""
from __future__ import annotations

import ctypes as ct
import itertools
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hub_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhub_oracle.so")
_lock = threading.Lock()
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile hub_oracle.c into libhub_oracle.so (gcc, -O2, no FP contraction)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ct.CDLL(_LIB_PATH)
        i32, f64, u64 = ct.c_int, ct.c_double, ct.c_uint64
        lib.oracle_philox4x64_10.argtypes = [_up, _up, _up]
        lib.oracle_philox4x64_10.restype = None
        lib.oracle_mulhi.argtypes = [u64, u64]
        lib.oracle_mulhi.restype = u64
        lib.oracle_ga_draw.argtypes = [u64, u64, u64, u64, u64, _up]
        lib.oracle_ga_draw.restype = None
        lib.oracle_flows.argtypes = [i32, _dp, _dp, _dp]
        lib.oracle_flows.restype = None
        lib.oracle_cost_alloc.argtypes = [i32, _dp, _dp, _ip, f64, f64, f64, f64, _dp]
        lib.oracle_cost_alloc.restype = f64
        lib.oracle_flow_matrix.argtypes = [i32, i32, _dp, _ip, _dp]
        lib.oracle_flow_matrix.restype = None
        lib.oracle_allocate.argtypes = [i32, i32, _dp, _ip, _ip, _ip]
        lib.oracle_allocate.restype = None
        lib.oracle_middle_nodes.argtypes = [i32, i32, _dp, _ip]
        lib.oracle_middle_nodes.restype = None
        lib.oracle_op_swap.argtypes = [i32, _ip, ct.POINTER(ct.c_int), u64, u64]
        lib.oracle_op_swap.restype = None
        lib.oracle_op_crossover.argtypes = [_ip, i32, _ip, i32, i32, _ip]
        lib.oracle_op_crossover.restype = i32
        lib.oracle_op_correct.argtypes = [i32, i32, _ip, ct.POINTER(ct.c_int), _up]
        lib.oracle_op_correct.restype = i32
        lib.oracle_ga_children.argtypes = [i32, i32, i32, i32, u64, u64, _ip, _ip]
        lib.oracle_ga_children.restype = i32
        lib.oracle_evaluate.argtypes = [i32, i32, _dp, _dp, i32, _ip, f64, f64, f64, f64, _dp,
                                        ct.c_void_p, ct.c_void_p]
        lib.oracle_evaluate.restype = i32
        lib.oracle_ga_init.argtypes = [i32, i32, _dp, _dp, i32, i32, f64, f64, f64, f64,
                                       _ip, _dp, _dp, _ip, _dp, _dp, _lp]
        lib.oracle_ga_init.restype = i32
        lib.oracle_ga_run.argtypes = [i32, i32, _dp, _dp, i32, i32, i32, i32, f64, f64, f64, f64, u64, i32,
                                      _ip, _dp, _dp, _ip, _dp, _dp, _lp, ct.c_void_p]
        lib.oracle_ga_run.restype = i32
        lib.oracle_shortest_paths.argtypes = [i32, _dp, _dp]
        lib.oracle_shortest_paths.restype = None
        lib.oracle_cost_alloc_routed.argtypes = [i32, _dp, ct.c_void_p, _dp, _ip, f64, f64, f64, f64, _dp]
        lib.oracle_cost_alloc_routed.restype = f64
        lib.oracle_evaluate_routed.argtypes = [i32, i32, _dp, ct.c_void_p, _dp, i32, _ip, f64, f64, f64, f64, _dp,
                                               ct.c_void_p, ct.c_void_p]
        lib.oracle_evaluate_routed.restype = i32
        lib.oracle_ga_init_routed.argtypes = [i32, i32, _dp, ct.c_void_p, _dp, i32, i32, f64, f64, f64, f64,
                                              _ip, _dp, _dp, _ip, _dp, _dp, _lp]
        lib.oracle_ga_init_routed.restype = i32
        lib.oracle_ga_run_routed.argtypes = [i32, i32, _dp, ct.c_void_p, _dp, i32, i32, i32, i32, f64, f64, f64,
                                             f64, u64, i32, _ip, _dp, _dp, _ip, _dp, _dp, _lp, ct.c_void_p]
        lib.oracle_ga_run_routed.restype = i32
        _lib = lib
        return lib


def set_threads(k: int) -> int:
    """Threads of the oracle's OpenMP loops from now on (the OpenMP runtime the
    library links); returns the number its parallel regions will use."""
    _load()
    gomp = ct.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(int(k))
    gomp.omp_get_max_threads.restype = ct.c_int
    return int(gomp.omp_get_max_threads())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------------ RNG ----

def philox(counter, key) -> np.ndarray:
    """Philox4x64-10 block for a 4-word counter and a 2-word key."""
    out = np.zeros(4, np.uint64)
    _load().oracle_philox4x64_10(np.asarray(counter, np.uint64), np.asarray(key, np.uint64), out)
    return out


def mulhi(w: int, m: int) -> int:
    """floor(w * m / 2**64): a uniform index in [0, m) from a 64-bit word."""
    return int(_load().oracle_mulhi(w, m))


def ga_draw(seed: int, g: int, idx: int, op: int, t: int = 0) -> np.ndarray:
    """The four words for (generation, index, operator, repeat) under ``seed``."""
    out = np.zeros(4, np.uint64)
    _load().oracle_ga_draw(seed, g, idx, op, t, out)
    return out


# ------------------------------------------------------------ evaluation ---

def flows(W):
    """Originating and destined flows O_i = sum_j W_ij, D_j = sum_i W_ij (Sec. 3)."""
    W = _f64(W)
    n = W.shape[0]
    O = np.zeros(n)
    D = np.zeros(n)
    _load().oracle_flows(n, W, O, D)
    return O, D


def _tr(Ctr):
    """(pointer, keep-alive array) of an optional transfer matrix."""
    if Ctr is None:
        return None, None
    Ctr = _f64(Ctr)
    return Ctr.ctypes.data, Ctr


def shortest_paths(C):
    """All-pairs shortest-path distances of C (Floyd-Warshall in binary64):
    the transfer costs of multi-hop routing, eq. (4) of Sec. 3."""
    C = _f64(C)
    out = np.empty_like(C)
    _load().oracle_shortest_paths(C.shape[0], C, out)
    return out


def cost_alloc(C, W, alloc, chi, alpha, delta, scale=1.0, Ctr=None):
    """Cost of an arbitrary allocation (node ids); returns (cost, (Cc, T, Dd)).
    Ctr: transfer matrix of the inter-hub legs (default C: direct routing;
    ``shortest_paths(C)``: multi-hop routing)."""
    C, W = _f64(C), _f64(W)
    parts = np.zeros(3)
    tp, keep = _tr(Ctr)
    f = _load().oracle_cost_alloc_routed(C.shape[0], C, tp, W, _i32(alloc), chi, alpha, delta, scale, parts)
    del keep
    return f, parts


def flow_matrix(W, kpos, p):
    """F = A^T W A for the one-hot allocation A given by hub positions kpos."""
    W = _f64(W)
    F = np.zeros((p, p))
    _load().oracle_flow_matrix(W.shape[0], p, W, _i32(kpos), F)
    return F


def allocate(C, hubs):
    """Nearest-hub allocation of a sorted hub list; returns (node ids, positions)."""
    C = _f64(C)
    h = _i32(np.sort(np.asarray(hubs)))
    n, p = C.shape[0], h.shape[0]
    a = np.zeros(n, np.int32)
    k = np.zeros(n, np.int32)
    _load().oracle_allocate(n, p, C, h, a, k)
    return a, k


def middle_nodes(C, p):
    """The p middle nodes (smallest sum_j C_ij, ties to the smaller index)."""
    C = _f64(C)
    h = np.zeros(p, np.int32)
    _load().oracle_middle_nodes(C.shape[0], p, C, h)
    return h


def evaluate(C, W, hubs, chi, alpha, delta, scale=1.0, want_alloc=False, Ctr=None):
    """Costs of a batch of hub sets (count x p); returns (cost, parts[, alloc]).
    Ctr as in ``cost_alloc``."""
    C, W = _f64(C), _f64(W)
    hubs = _i32(np.atleast_2d(hubs))
    n = C.shape[0]
    count, p = hubs.shape
    cost = np.zeros(count)
    parts = np.zeros((count, 3))
    alloc = np.zeros((count, n), np.int32) if want_alloc else None
    tp, keep = _tr(Ctr)
    rc = _load().oracle_evaluate_routed(n, p, C, tp, W, count, hubs, chi, alpha, delta, scale, cost,
                                        parts.ctypes.data, alloc.ctypes.data if want_alloc else None)
    del keep
    if rc:
        raise ValueError("invalid hub set (out of range or repeated)")
    return (cost, parts, alloc) if want_alloc else (cost, parts)


def enumerate_best(C, W, p, chi, alpha, delta, scale=1.0, first=0, count=None, Ctr=None):
    """Exhaustive search of the nearest-hub solution space (the optimum the
    GA is compared with in Sec. 6.2; allocation rule of Sec. 4.1 and 5): the
    p-subsets of range(n) of lexicographic ranks [first, first + count), each
    evaluated as ``evaluate`` does.  Returns (cost, hubs, rank, costs): the
    smallest cost, the first set (lowest rank) attaining it, its rank, and
    every cost in rank order."""
    C = _f64(C)
    n = C.shape[0]
    total = math.comb(n, p)
    count = total - first if count is None else count
    sets = np.array(list(itertools.islice(itertools.combinations(range(n), p), first, first + count)), np.int32)
    costs, _ = evaluate(C, W, sets, chi, alpha, delta, scale, Ctr=Ctr)
    j = int(np.argmin(costs))          # first occurrence: the lowest rank among equal costs
    return float(costs[j]), sets[j].copy(), first + j, costs


# --------------------------------------------------------------- GA ops ----

def op_swap(n, x, w_pos, w_rank):
    """Hub<->spoke swap on a sorted list (mutation of Sec. 4.2 / perturbation of Sec. 4.1)."""
    buf = np.zeros(len(x) + 1, np.int32)
    buf[: len(x)] = x
    cnt = ct.c_int(len(x))
    _load().oracle_op_swap(n, buf, ct.byref(cnt), w_pos, w_rank)
    return buf[: cnt.value].copy()


def op_crossover(xa, xb, cut):
    """Single-point crossover of two sorted hub lists at node cut (Sec. 4.2)."""
    xa, xb = _i32(xa), _i32(xb)
    out = np.zeros(len(xa) + len(xb) + 1, np.int32)
    c = _load().oracle_op_crossover(xa, len(xa), xb, len(xb), cut, out)
    return out[:c].copy()


def op_correct(n, p, x, draws):
    """Correction to exactly p hubs with the given draw words (Sec. 4.2)."""
    buf = np.zeros(max(len(x), p) + 1, np.int32)
    buf[: len(x)] = x
    cnt = ct.c_int(len(x))
    d = np.zeros(max(abs(len(x) - p), 1), np.uint64)
    d[: len(draws)] = draws
    used = _load().oracle_op_correct(n, p, buf, ct.byref(cnt), d)
    return buf[: cnt.value].copy(), used


def ga_children(n, p, S, m, seed, g, anc):
    """All S children of generation g from the R = S/m island ancestors."""
    anc = _i32(anc)
    out = np.zeros((S, p), np.int32)
    if _load().oracle_ga_children(n, p, S, m, seed, g, anc, out):
        raise ValueError("invalid GA configuration")
    return out


class GAState:
    """Caller-owned GA state: generation, island ancestors, best so far."""

    def __init__(self, R, p):
        self.anc = np.zeros((R, p), np.int32)
        self.anc_cost = np.zeros(R)
        self.anc_parts = np.zeros((R, 3))
        self.best = np.zeros(p, np.int32)
        self.best_cost = np.zeros(1)
        self.best_parts = np.zeros(3)
        self.gen = np.zeros(1, np.int64)

    def copy(self):
        s = GAState(*self.anc.shape)
        for k, v in self.__dict__.items():
            setattr(s, k, v.copy())
        return s


def ga_init(C, W, p, S, m, chi, alpha, delta, scale=1.0, Ctr=None) -> GAState:
    """Every island ancestor set to the middle-node solution P0 (Sec. 4.1, Sec. 5)."""
    C, W = _f64(C), _f64(W)
    st = GAState(S // m, p)
    tp, keep = _tr(Ctr)
    rc = _load().oracle_ga_init_routed(C.shape[0], p, C, tp, W, S, m, chi, alpha, delta, scale, st.anc,
                                       st.anc_cost, st.anc_parts, st.best, st.best_cost, st.best_parts, st.gen)
    del keep
    if rc:
        raise ValueError("invalid GA configuration")
    return st


def ga_run(C, W, st: GAState, generations, *, S, m, n1, seed, chi, alpha, delta, scale=1.0, elitist=1, Ctr=None):
    """Advance the GA state by ``generations``; returns the best-cost trace.
    Ctr as in ``cost_alloc``."""
    C, W = _f64(C), _f64(W)
    n, p = C.shape[0], st.anc.shape[1]
    trace = np.zeros(max(generations, 1))
    tp, keep = _tr(Ctr)
    rc = _load().oracle_ga_run_routed(n, p, C, tp, W, S, m, n1, elitist, chi, alpha, delta, scale, seed,
                                      generations, st.anc, st.anc_cost, st.anc_parts, st.best, st.best_cost,
                                      st.best_parts, st.gen, trace.ctypes.data)
    del keep
    if rc:
        raise ValueError("invalid GA configuration")
    return trace[:generations]
