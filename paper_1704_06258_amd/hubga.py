"""ctypes binding of libhubga.so (C ABI in include/hubga.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  The functions keep the ABI's names; ``Solver`` bundles
them for Python callers, with device memory and streams owned by torch.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhubga.so")

GA_OK, GA_ERR_INVALID, GA_ERR_OOM, GA_ERR_DEVICE, GA_ERR_STATE = range(5)
GA_DT_F64, GA_DT_F32 = 0, 1
GA_PREC_FP64, GA_PREC_FP32, GA_PREC_SPLIT_BF16, GA_PREC_SPLIT3_BF16 = 0, 1, 2, 3
GA_KERN_PLAIN, GA_KERN_BATCHED = 0, 1

PRECISIONS = {"fp64": GA_PREC_FP64, "fp32": GA_PREC_FP32, "split_bf16": GA_PREC_SPLIT_BF16,
              "split3_bf16": GA_PREC_SPLIT3_BF16}
DEFAULT_KERNEL = {GA_PREC_FP64: GA_KERN_PLAIN, GA_PREC_FP32: GA_KERN_PLAIN, GA_PREC_SPLIT_BF16: GA_KERN_BATCHED,
                  GA_PREC_SPLIT3_BF16: GA_KERN_BATCHED}
KERNELS = {"plain": GA_KERN_PLAIN, "batched": GA_KERN_BATCHED}

# Every symbol declared in include/hubga.h.
EXPORTS = ("ga_params_default", "ga_workspace_bytes", "ga_init", "ga_evaluate", "ga_evaluate_dev", "ga_step",
           "ga_best", "ga_solve", "ga_population", "ga_ancestors", "ga_get_state", "ga_set_state", "ga_stats",
           "ga_profile_enable", "ga_profile_read", "ga_tile_config_count", "ga_tile_config_info",
           "ga_set_tile_config", "ga_evaluation_folded", "ga_set_stream", "ga_batch_create", "ga_batch_set", "ga_batch_step", "ga_batch_free",
           "ga_status_str", "ga_last_error", "ga_free", "ga_init_static", "ga_enumerate")


class ga_params(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("p", ct.c_int32), ("chi", ct.c_double), ("alpha", ct.c_double),
                ("delta", ct.c_double), ("scale", ct.c_double), ("seed", ct.c_uint64),
                ("population", ct.c_int32), ("island_size", ct.c_int32), ("n1", ct.c_int32),
                ("elitist", ct.c_int32), ("precision", ct.c_int32), ("kernel", ct.c_int32),
                ("c_symmetric", ct.c_int32), ("multihop", ct.c_int32)]


class HubGAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


_lock = threading.Lock()
_lib = None


def lib():
    """Load libhubga.so (raises if it is missing: there is no fallback path)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1704_06258_amd.build`")
        L = ct.CDLL(LIB_PATH)
        vp, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
        P = ct.POINTER(ga_params)
        L.ga_params_default.argtypes = [P, i32, i32]
        L.ga_params_default.restype = None
        L.ga_workspace_bytes.argtypes = [P, ct.c_int, ct.c_int]
        L.ga_workspace_bytes.restype = sz
        L.ga_init.argtypes = [P, vp, ct.c_int, vp, ct.c_int, vp, sz, vp, ct.POINTER(vp)]
        L.ga_init_static.argtypes = [P, vp, ct.c_int, vp, ct.c_int, vp, ct.POINTER(vp)]
        L.ga_init_static.restype = ct.c_int
        L.ga_evaluate.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.ga_evaluate_dev.argtypes = [vp, vp, i32, vp, vp]
        L.ga_enumerate.argtypes = [vp, i64, i64, vp, ct.POINTER(ct.c_double), vp, ct.POINTER(i64), vp, vp,
                                   ct.POINTER(i64)]
        L.ga_enumerate.restype = ct.c_int
        L.ga_step.argtypes = [vp, i32]
        L.ga_best.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ga_solve.argtypes = [vp, i32, vp, vp, vp]
        L.ga_population.argtypes = [vp, vp, vp]
        L.ga_ancestors.argtypes = [vp, vp, vp]
        L.ga_get_state.argtypes = [vp, vp, ct.POINTER(sz)]
        L.ga_set_state.argtypes = [vp, vp, sz]
        L.ga_stats.argtypes = [vp, vp]
        L.ga_profile_enable.argtypes = [vp, i32]
        L.ga_profile_read.argtypes = [vp, ct.POINTER(ct.c_double), ct.POINTER(i64)]
        for f in ("ga_init", "ga_evaluate", "ga_evaluate_dev", "ga_step", "ga_best", "ga_solve", "ga_population",
                  "ga_ancestors", "ga_get_state", "ga_set_state", "ga_stats", "ga_profile_enable",
                  "ga_profile_read"):
            getattr(L, f).restype = ct.c_int
        L.ga_tile_config_count.argtypes = []
        L.ga_tile_config_count.restype = i32
        L.ga_tile_config_info.argtypes = [i32, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32)]
        L.ga_tile_config_info.restype = ct.c_int
        L.ga_set_stream.argtypes = [vp, vp]
        L.ga_set_stream.restype = ct.c_int
        L.ga_set_tile_config.argtypes = [vp, i32]
        L.ga_set_tile_config.restype = ct.c_int
        L.ga_evaluation_folded.argtypes = [vp, ct.POINTER(i32)]
        L.ga_evaluation_folded.restype = ct.c_int
        L.ga_batch_create.argtypes = [vp, i32, ct.POINTER(vp)]
        L.ga_batch_create.restype = ct.c_int
        L.ga_batch_set.argtypes = [vp, ct.POINTER(vp), i32]
        L.ga_batch_set.restype = ct.c_int
        L.ga_batch_step.argtypes = [vp, i32]
        L.ga_batch_step.restype = ct.c_int
        L.ga_batch_free.argtypes = [vp]
        L.ga_batch_free.restype = None
        L.ga_status_str.argtypes = [ct.c_int]
        L.ga_status_str.restype = ct.c_char_p
        L.ga_last_error.argtypes = [vp]
        L.ga_last_error.restype = ct.c_char_p
        L.ga_free.argtypes = [vp]
        L.ga_free.restype = None
        _lib = L
        return L


def status_name(s) -> str:
    try:
        return lib().ga_status_str(int(s)).decode()
    except ImportError:
        return str(s)


def _check(status, ctx=None):
    if status != GA_OK:
        raise HubGAError(status, lib().ga_last_error(ctx).decode())


def _ptr(a) -> int:
    return a.ctypes.data if isinstance(a, np.ndarray) else int(a.data_ptr())


def tile_configs():
    """[(rows, cols, ktile)] of every tile configuration of the batched kernel."""
    out = []
    for c in range(lib().ga_tile_config_count()):
        r, k, kt = ct.c_int32(), ct.c_int32(), ct.c_int32()
        _check(lib().ga_tile_config_info(c, ct.byref(r), ct.byref(k), ct.byref(kt)))
        out.append((r.value, k.value, kt.value))
    return out


def ga_params_default(n, p) -> ga_params:
    q = ga_params()
    lib().ga_params_default(ct.byref(q), n, p)
    return q


def ga_workspace_bytes(params: ga_params, c_dtype=GA_DT_F64, w_dtype=GA_DT_F64) -> int:
    return int(lib().ga_workspace_bytes(ct.byref(params), c_dtype, w_dtype))


def make_params(n, p, *, chi, alpha, delta, scale=1.0, seed=1, population=64, island_size=None, n1=10,
                elitist=True, precision="fp64", kernel=None, c_symmetric=False, multihop=False) -> ga_params:
    q = ga_params_default(n, p)
    q.chi, q.alpha, q.delta, q.scale, q.seed = chi, alpha, delta, scale, seed
    q.population = population
    q.island_size = island_size if island_size is not None else min(64, population)
    q.n1, q.elitist = n1, int(bool(elitist))
    q.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    q.kernel = DEFAULT_KERNEL[q.precision] if kernel is None else (
        KERNELS[kernel] if isinstance(kernel, str) else int(kernel))
    q.c_symmetric = int(bool(c_symmetric))
    q.multihop = int(bool(multihop))
    return q


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float64:
        return GA_DT_F64
    if a.dtype == np.float32:
        return GA_DT_F32
    raise TypeError("C and W must be float64 or float32")


class Solver:
    """One context: an instance resident on the GPU plus its GA state."""

    def __init__(self, C, W, p, *, chi, alpha, delta, scale=1.0, seed=1, population=64, island_size=None, n1=10,
                 elitist=True, precision="fp64", kernel=None, stream=None, device=0, c_symmetric=None,
                 static_workspace=False, multihop=False):
        """``static_workspace``: build the context with ga_init_static on the
        library's per-device static workspace (no device allocation) instead
        of ga_init on a torch-allocated one."""
        import torch
        C = np.ascontiguousarray(C)
        W = np.ascontiguousarray(W)
        n = C.shape[0]
        if C.shape != (n, n) or W.shape != (n, n):
            raise ValueError("C and W must be n x n")
        self.n, self.p = n, p
        sym = bool(np.array_equal(C, C.T)) if c_symmetric is None else bool(c_symmetric)
        self.params = make_params(n, p, chi=chi, alpha=alpha, delta=delta, scale=scale, seed=seed,
                                  population=population, island_size=island_size, n1=n1, elitist=elitist,
                                  precision=precision, kernel=kernel, c_symmetric=sym, multihop=multihop)
        self.S = self.params.population
        self.R = self.S // self.params.island_size
        cdt, wdt = _dtype_code(C), _dtype_code(W)
        nbytes = ga_workspace_bytes(self.params, cdt, wdt)
        if nbytes == 0:
            raise HubGAError(GA_ERR_INVALID, "invalid parameters")
        self.device = torch.device("cuda", device)
        # a stream of its own (non-null, so generations can be replayed as a graph)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.workspace_bytes = nbytes
        h = ct.c_void_p()
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(lib().ga_init_static(ct.byref(self.params), C.ctypes.data, cdt, W.ctypes.data, wdt,
                                            ct.c_void_p(self.stream.cuda_stream), ct.byref(h)))
        else:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            _check(lib().ga_init(ct.byref(self.params), C.ctypes.data, cdt, W.ctypes.data, wdt,
                                 self.workspace.data_ptr(), nbytes, ct.c_void_p(self.stream.cuda_stream),
                                 ct.byref(h)))
        self.ctx = h

    # -- evaluation -------------------------------------------------------
    def evaluate(self, hubs, want_alloc=False):
        """Costs, parts {Cc, T, Dd}, error bounds (and allocations) of host hub sets."""
        hubs = np.ascontiguousarray(np.atleast_2d(hubs), dtype=np.int32)
        if hubs.shape[1] != self.p:
            raise ValueError("hub sets must have p entries")
        k = hubs.shape[0]
        cost = np.zeros(k)
        parts = np.zeros((k, 3))
        eps = np.zeros(k)
        alloc = np.zeros((k, self.n), np.int32) if want_alloc else None
        _check(lib().ga_evaluate(self.ctx, hubs.ctypes.data, k, cost.ctypes.data, parts.ctypes.data,
                                 alloc.ctypes.data if want_alloc else None, eps.ctypes.data), self.ctx)
        out = dict(cost=cost, parts=parts, eps=eps)
        if want_alloc:
            out["alloc"] = alloc
        return out

    def evaluate_dev(self, d_hubs, d_cost=None, d_kidx=None):
        """Stream-ordered evaluation of sorted device hub sets (torch int32, count x p)."""
        import torch
        k = d_hubs.shape[0]
        if d_cost is None:
            d_cost = torch.empty(k, dtype=torch.float64, device=self.device)
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)          # inputs produced on the caller's stream
        _check(lib().ga_evaluate_dev(self.ctx, d_hubs.data_ptr(), k,
                                     d_kidx.data_ptr() if d_kidx is not None else None, d_cost.data_ptr()),
               self.ctx)
        cur.wait_stream(self.stream)          # outputs consumed on the caller's stream
        for t in (d_hubs, d_cost, d_kidx):
            if t is not None:
                t.record_stream(self.stream)
        return d_cost

    def enumerate(self, first=0, count=-1, want_all=False):
        """Exact best hub set of lexicographic ranks [first, first + count)
        (ga_enumerate); with ``want_all`` also every set's cost and bound."""
        import math
        total = math.comb(self.n, self.p)
        k = (total - first) if count < 0 else count
        hubs = np.zeros(self.p, np.int32)
        cost = ct.c_double()
        parts = np.zeros(3)
        rank = ct.c_int64()
        rechecks = ct.c_int64()
        costs = np.zeros(max(k, 1)) if want_all else None
        eps = np.zeros(max(k, 1)) if want_all else None
        _check(lib().ga_enumerate(self.ctx, int(first), int(count), hubs.ctypes.data, ct.byref(cost),
                                  parts.ctypes.data, ct.byref(rank), costs.ctypes.data if want_all else None,
                                  eps.ctypes.data if want_all else None, ct.byref(rechecks)), self.ctx)
        out = dict(hubs=hubs, cost=cost.value, parts=parts, rank=rank.value, rechecks=rechecks.value)
        if want_all:
            out["costs"], out["eps"] = costs[:k], eps[:k]
        return out

    # -- GA ---------------------------------------------------------------
    def step(self, generations=1):
        _check(lib().ga_step(self.ctx, generations), self.ctx)

    def best(self):
        hubs = np.zeros(self.p, np.int32)
        alloc = np.zeros(self.n, np.int32)
        cost = ct.c_double()
        parts = np.zeros(3)
        gen = ct.c_int64()
        _check(lib().ga_best(self.ctx, hubs.ctypes.data, alloc.ctypes.data, ct.addressof(cost), parts.ctypes.data,
                             ct.addressof(gen)), self.ctx)
        return dict(hubs=hubs, alloc=alloc, cost=cost.value, parts=parts, generation=gen.value)

    def solve(self, generations):
        hubs = np.zeros(self.p, np.int32)
        alloc = np.zeros(self.n, np.int32)
        cost = ct.c_double()
        _check(lib().ga_solve(self.ctx, generations, hubs.ctypes.data, alloc.ctypes.data, ct.addressof(cost)),
               self.ctx)
        return dict(hubs=hubs, alloc=alloc, cost=cost.value)

    def population(self):
        hubs = np.zeros((self.S, self.p), np.int32)
        cost = np.zeros(self.S)
        _check(lib().ga_population(self.ctx, hubs.ctypes.data, cost.ctypes.data), self.ctx)
        return hubs, cost

    def ancestors(self):
        hubs = np.zeros((self.R, self.p), np.int32)
        cost = np.zeros(self.R)
        _check(lib().ga_ancestors(self.ctx, hubs.ctypes.data, cost.ctypes.data), self.ctx)
        return hubs, cost

    def get_state(self) -> bytes:
        n = ct.c_size_t()
        _check(lib().ga_get_state(self.ctx, None, ct.byref(n)), self.ctx)
        buf = ct.create_string_buffer(n.value)
        _check(lib().ga_get_state(self.ctx, buf, ct.byref(n)), self.ctx)
        return buf.raw[: n.value]

    def set_state(self, blob: bytes):
        _check(lib().ga_set_state(self.ctx, blob, len(blob)), self.ctx)

    def stats(self):
        s = np.zeros(4, np.int64)
        _check(lib().ga_stats(self.ctx, s.ctypes.data), self.ctx)
        return dict(generations=int(s[0]), rechecks=int(s[1]), islands_rechecked=int(s[2]), evaluations=int(s[3]))

    def set_stream(self, stream):
        """Issue later work on ``stream`` (ordered after the work already queued)."""
        _check(lib().ga_set_stream(self.ctx, ct.c_void_p(stream.cuda_stream)), self.ctx)
        self.stream = stream

    def set_tile_config(self, config: int):
        _check(lib().ga_set_tile_config(self.ctx, int(config)), self.ctx)

    def folded(self) -> bool:
        """True when the batched evaluation multiplies the folded W (symmetric C)."""
        f = ct.c_int32(0)
        _check(lib().ga_evaluation_folded(self.ctx, ct.byref(f)), self.ctx)
        return bool(f.value)

    def profile_enable(self, on=True):
        _check(lib().ga_profile_enable(self.ctx, int(bool(on))), self.ctx)

    def profile_read(self):
        ms = ct.c_double()
        k = ct.c_int64()
        _check(lib().ga_profile_read(self.ctx, ct.byref(ms), ct.byref(k)), self.ctx)
        return ms.value, k.value

    def close(self):
        if getattr(self, "ctx", None):
            lib().ga_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Several Solvers advanced together (ga_batch_*): a generation of the
    grouped members is one replay of a captured graph of six grouped launches
    (kept across compositions that fit its grids, captured anew otherwise).
    Every member must be on ``batch.stream`` (``Solver.set_stream``)."""

    def __init__(self, device=0, tile_config=7, stream=None):
        import torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        h = ct.c_void_p()
        _check(lib().ga_batch_create(ct.c_void_p(self.stream.cuda_stream), int(tile_config), ct.byref(h)))
        self.handle = h
        self.members = []

    def set(self, solvers):
        arr = (ct.c_void_p * max(1, len(solvers)))(*[s.ctx for s in solvers])
        _check(lib().ga_batch_set(self.handle, arr, len(solvers)))
        self.members = list(solvers)

    def step(self, generations=1):
        _check(lib().ga_batch_step(self.handle, int(generations)))

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "handle", None):
            lib().ga_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
