"""Seeded synthetic USApHMP instances and populations.

These are the only inputs shared by the GPU path and its checks.  The module
holds no part of the method's arithmetic: it draws node coordinates and flows,
forms the Euclidean distance matrix, and draws random hub sets.  The paper's
datasets (CAB, AP, Urand, PlanetLab and the authors' own 1500-6000 node
instances, Sec. 6.1 and Table 5) are not available here; the recipes below are
synthetic stand-ins with the same shapes, sizes and factor values:

* ``small``    n=25, p=3 (CAB-like size): coordinates U[0,1000)^2, integer
  flows U{0..100} with W_ii = 0, chi=1, alpha=0.75, delta=1.
* ``medium``   n=200, p=10 (AP/Urand-like): coordinates U[0,10000)^2,
  lognormal(2, 1) flows normalised to sum 1e6, chi=3, alpha=0.75, delta=2.
* ``clustered`` n=1000, p=20 (Urand-1000-like): 20 Gaussian clusters
  (sigma=300) in [0,10000]^2, lognormal flows as above.
* ``large``    n=6000, p=50 (Table 5 shape): coordinates U[0,10000)^2,
  distances rounded to FP32, flows U[0,1) in FP32 with 5% of the rows
  (a seeded choice) scaled by 100 in FP32.
* ``serving``  n in {50,100,200,500,1000,2000}, p in {3,5,10,20},
  population in {256,512,1024,2048}, uniform coordinates, lognormal flows.
* ``nonmetric`` (PlanetLab-like, Sec. 6.1: delays that break the triangle
  inequality, chi = alpha = delta = 1): Euclidean distances of uniform
  coordinates, each pair scaled by a symmetric lognormal factor exp(0.6 Z),
  zero diagonal; lognormal flows.

Every generator uses ``numpy.random.Generator(Philox(seed))``; the distance
matrix is exactly symmetric with a zero diagonal.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np


@dataclasses.dataclass
class Instance:
    name: str
    C: np.ndarray          # n x n distances (float64 or float32), row-major
    W: np.ndarray          # n x n flows (float64 or float32), row-major
    p: int
    chi: float
    alpha: float
    delta: float
    scale: float = 1.0

    @property
    def n(self) -> int:
        return int(self.C.shape[0])

    def C64(self) -> np.ndarray:
        return np.ascontiguousarray(self.C, dtype=np.float64)

    def W64(self) -> np.ndarray:
        return np.ascontiguousarray(self.W, dtype=np.float64)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.C).tobytes())
        h.update(np.ascontiguousarray(self.W).tobytes())
        return h.hexdigest()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def euclidean(xy: np.ndarray) -> np.ndarray:
    """Pairwise Euclidean distances in float64 (exactly symmetric, zero diagonal)."""
    d = xy[:, None, :] - xy[None, :, :]
    return np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1])


def lognormal_flows(rng: np.random.Generator, n: int, total: float = 1e6) -> np.ndarray:
    """W_ij = exp(2 + Z), Z ~ N(0,1), scaled in float64 so that sum(W) = total."""
    W = np.exp(2.0 + rng.standard_normal((n, n)))
    return W * (total / W.sum())


def small(seed: int = 1, n: int = 25, p: int = 3) -> Instance:
    rng = _rng(seed)
    xy = rng.uniform(0.0, 1000.0, size=(n, 2))
    W = rng.integers(0, 101, size=(n, n)).astype(np.float64)
    np.fill_diagonal(W, 0.0)
    return Instance("small", euclidean(xy), W, p, 1.0, 0.75, 1.0)


def medium(seed: int = 2, n: int = 200, p: int = 10) -> Instance:
    rng = _rng(seed)
    xy = rng.uniform(0.0, 10000.0, size=(n, 2))
    W = lognormal_flows(rng, n)
    return Instance("medium", euclidean(xy), W, p, 3.0, 0.75, 2.0)


def clustered(seed: int = 3, n: int = 1000, p: int = 20, clusters: int = 20, sigma: float = 300.0) -> Instance:
    rng = _rng(seed)
    centres = rng.uniform(0.0, 10000.0, size=(clusters, 2))
    pick = rng.integers(0, clusters, size=n)
    xy = np.clip(centres[pick] + rng.normal(0.0, sigma, size=(n, 2)), 0.0, 10000.0)
    W = lognormal_flows(rng, n)
    return Instance("clustered", euclidean(xy), W, p, 3.0, 0.75, 2.0)


def large(seed: int = 4, n: int = 6000, p: int = 50, heavy_frac: float = 0.05) -> Instance:
    rng = _rng(seed)
    xy = rng.uniform(0.0, 10000.0, size=(n, 2))
    C = euclidean(xy).astype(np.float32)
    W = rng.random((n, n), dtype=np.float32)
    heavy = rng.permutation(n)[: int(round(heavy_frac * n))]
    W[heavy] *= np.float32(100.0)
    return Instance("large", C, W, p, 3.0, 0.75, 2.0)


def uniform(seed: int, n: int, p: int, chi=3.0, alpha=0.75, delta=2.0) -> Instance:
    """Uniform coordinates in [0,10000)^2 and lognormal flows (serving mix)."""
    rng = _rng(seed)
    xy = rng.uniform(0.0, 10000.0, size=(n, 2))
    return Instance("uniform", euclidean(xy), lognormal_flows(rng, n), p, chi, alpha, delta)


def nonmetric(seed: int = 6, n: int = 300, p: int = 10, spread: float = 0.6) -> Instance:
    """Symmetric distances that violate the triangle inequality (Sec. 6.1,
    PlanetLab-like), chi = alpha = delta = 1."""
    rng = _rng(seed)
    xy = rng.uniform(0.0, 10000.0, size=(n, 2))
    z = rng.standard_normal((n, n))
    z = np.triu(z, 1)
    z = z + z.T
    C = euclidean(xy) * np.exp(spread * z)
    np.fill_diagonal(C, 0.0)
    return Instance("nonmetric", C, lognormal_flows(rng, n), p, 1.0, 1.0, 1.0)


def random_asymmetric(seed: int, n: int, p: int, chi=2.0, alpha=0.6, delta=1.5, integer=False) -> Instance:
    """Non-symmetric C and W (for catching transposed operands in checks)."""
    rng = _rng(seed)
    if integer:
        C = rng.integers(0, 50, size=(n, n)).astype(np.float64)
        W = rng.integers(0, 20, size=(n, n)).astype(np.float64)
    else:
        C = rng.uniform(0.0, 100.0, size=(n, n))
        W = rng.uniform(0.0, 10.0, size=(n, n))
    np.fill_diagonal(C, 0.0)
    return Instance("asym", C, W, p, chi, alpha, delta)


def random_hub_sets(seed: int, n: int, p: int, count: int) -> np.ndarray:
    """``count`` uniformly random p-subsets of range(n), each sorted (int32)."""
    rng = _rng(seed)
    keys = rng.random((count, n))
    idx = np.argpartition(keys, p - 1, axis=1)[:, :p] if p < n else np.tile(np.arange(n), (count, 1))
    return np.sort(idx, axis=1).astype(np.int32)


SERVING_N = (50, 100, 200, 500, 1000, 2000)
SERVING_P = (3, 5, 10, 20)
SERVING_S = (256, 512, 1024, 2048)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    n: int
    p: int
    S: int
    generations: int
    instance_seed: int
    ga_seed: int

    def instance(self) -> Instance:
        return uniform(self.instance_seed, self.n, self.p)


def serving_requests(count: int, rate: float = 200.0, seed: int = 5, generations: int = 100, first_id: int = 0):
    """Poisson arrivals at ``rate`` per second with the serving size mix."""
    rng = _rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    ns = rng.choice(SERVING_N, size=count)
    ps = rng.choice(SERVING_P, size=count)
    ss = rng.choice(SERVING_S, size=count)
    out = []
    for k in range(count):
        r = first_id + k
        out.append(Request(r, float(t[k]), int(ns[k]), int(ps[k]), int(ss[k]), generations, 5_000_000 + r, r))
    return out
