"""Seeded synthetic workloads for the p-stable LSH query-workload path.

The paper evaluates on real datasets (Audio, LabelMe, P53, Sift, DeepSat; its
Section 6.1) that are not available here; these generators stand in for them with
the shapes of the five evaluation configurations:

  1  n=10,000    d=128 u8  50-component Gaussian mixture, sigma=20, Q=100 noisy
                            data points (noise variance 4), L=10 k=8  w=400
  2  n=1,000,000 d=128 u8  1,000 components, Q=10,000 noisy points, L=20 k=10 w=400
  3  n=1,000,000 d=960 f32 500 clusters in [0,1], sigma=0.05, Q=1,000 noisy points
                            (noise sigma 0.01), L=16 k=12 w=1.5
  4  n=10,000,000 d=96 u8  10,000 components, Q=100,000 Zipf(s=1.1) queries over
                            1,000 hot centres + noise variance 9, L=24 k=10 w=350
  5  configuration-3 data, Zipf(s=1.1) queries over its 500 centres + N(0,0.05^2):
                            200,000 training queries and 100,000 evaluation queries

Queries drawn near data points follow the paper's choice of queries from dense
regions of the dataset (Section 6.2).  The hash parameters follow the p-stable
family of Section 3: a ~ N(0,1)^d and b ~ U[0,w).  b is produced as
float32(u * w) from uniform draws u in [0,1), so that a sweep over w keeps the
same random offsets in units of w.

This module only draws random numbers; it holds none of the method's arithmetic
(no projection, hashing, distance or selection).  Both the CPU oracle and the GPU
library consume what it returns.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Seed bases: data, hash parameters, queries, training queries.
SEED_DATA, SEED_PARAMS, SEED_QUERIES, SEED_TRAIN = 1000, 2000, 3000, 4000

_CHUNK = 1 << 16  # rows per generation chunk (fixed, so results never depend on memory)


@dataclass
class Params:
    """Hash-function parameters of L layers of k functions over d dimensions."""
    a: np.ndarray          # (L, k, d) float32, entries N(0,1)
    u: np.ndarray          # (L, k) float64 in [0,1): b = float32(u * w)
    w: float

    @property
    def L(self) -> int:
        return self.a.shape[0]

    @property
    def k(self) -> int:
        return self.a.shape[1]

    def b(self, w: Optional[float] = None) -> np.ndarray:
        """Offsets b in [0, w) as float32 (strictly below w after rounding)."""
        w = self.w if w is None else float(w)
        wf = np.float32(w)
        b = (self.u * w).astype(np.float32)
        below = np.nextafter(wf, np.float32(0))
        return np.where(b >= wf, below, b).astype(np.float32)


@dataclass
class Workload:
    name: str
    data: np.ndarray               # (n, d) uint8 or float32, row-major
    queries: np.ndarray            # (Q, d) same dtype
    params: Params
    K: int = 10
    centres: Optional[np.ndarray] = None  # mixture centres (float64), kept for query draws
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.data.shape[0]

    @property
    def d(self) -> int:
        return self.data.shape[1]

    @property
    def Q(self) -> int:
        return self.queries.shape[0]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def hash_params(seed: int, L: int, k: int, d: int, w: float) -> Params:
    rng = _rng(seed)
    a = rng.standard_normal((L, k, d)).astype(np.float32)
    u = rng.random((L, k))
    return Params(a=a, u=u, w=float(w))


def gmm_u8(seed: int, n: int, d: int, ncomp: int, sigma: float):
    """Gaussian mixture in [0,255]^d: centres U[0,255]^d, equal weights, points
    centre + N(0, sigma^2) per coordinate, rounded and clipped to 0..255."""
    rng = _rng(seed)
    centres = rng.uniform(0.0, 255.0, size=(ncomp, d))
    comp = rng.integers(0, ncomp, size=n)
    out = np.empty((n, d), dtype=np.uint8)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        z = rng.standard_normal((e - s, d), dtype=np.float32)
        v = centres[comp[s:e]].astype(np.float32) + np.float32(sigma) * z
        np.clip(np.rint(v), 0, 255, out=v)
        out[s:e] = v.astype(np.uint8)
    return out, centres, comp


def mixture_f32(seed: int, n: int, d: int, ncomp: int, sigma: float):
    """Cluster mixture in [0,1]^d: centres U[0,1]^d, points centre + N(0, sigma^2),
    clipped to [0,1], float32."""
    rng = _rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(ncomp, d))
    comp = rng.integers(0, ncomp, size=n)
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        z = rng.standard_normal((e - s, d), dtype=np.float32)
        v = centres[comp[s:e]].astype(np.float32) + np.float32(sigma) * z
        np.clip(v, 0.0, 1.0, out=v)
        out[s:e] = v
    return out, centres, comp


def noisy_points(seed: int, data: np.ndarray, Q: int, sigma: float) -> np.ndarray:
    """Q queries: uniformly chosen data points plus N(0, sigma^2) noise
    (rounded and clipped to 0..255 for u8 data, clipped to [0,1] for float data)."""
    rng = _rng(seed)
    idx = rng.integers(0, data.shape[0], size=Q)
    z = rng.standard_normal((Q, data.shape[1]), dtype=np.float32)
    v = data[idx].astype(np.float32) + np.float32(sigma) * z
    if data.dtype == np.uint8:
        return np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return np.clip(v, 0.0, 1.0).astype(np.float32)


def zipf_ranks(rng: np.random.Generator, nhot: int, s: float, Q: int) -> np.ndarray:
    """Q draws from the finite Zipf law p(r) proportional to r^-s, r = 1..nhot
    (returned 0-based)."""
    p = np.arange(1, nhot + 1, dtype=np.float64) ** (-s)
    p /= p.sum()
    return rng.choice(nhot, size=Q, p=p)


def zipf_queries(seed: int, centres: np.ndarray, Q: int, nhot: int, s: float,
                 sigma: float, dtype) -> np.ndarray:
    """Q queries around a seeded pick of nhot mixture centres chosen with Zipf(s)
    popularity, plus N(0, sigma^2) noise (rounded/clipped like the data)."""
    rng = _rng(seed)
    nhot = min(nhot, centres.shape[0])
    hot = rng.choice(centres.shape[0], size=nhot, replace=False)
    r = zipf_ranks(rng, nhot, s, Q)
    v = np.empty((Q, centres.shape[1]), dtype=np.float32)
    for st in range(0, Q, _CHUNK):
        e = min(Q, st + _CHUNK)
        z = rng.standard_normal((e - st, centres.shape[1]), dtype=np.float32)
        v[st:e] = centres[hot[r[st:e]]].astype(np.float32) + np.float32(sigma) * z
    if dtype == np.uint8:
        return np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return np.clip(v, 0.0, 1.0).astype(np.float32)


# Full-size shapes of the five configurations.
CONFIGS = {
    1: dict(n=10_000, d=128, dtype="u8", ncomp=50, sigma=20.0, Q=100, qsigma=2.0,
            L=10, k=8, w=400.0, K=10, queries="noisy"),
    2: dict(n=1_000_000, d=128, dtype="u8", ncomp=1000, sigma=20.0, Q=10_000, qsigma=2.0,
            L=20, k=10, w=400.0, K=10, queries="noisy"),
    3: dict(n=1_000_000, d=960, dtype="f32", ncomp=500, sigma=0.05, Q=1_000, qsigma=0.01,
            L=16, k=12, w=1.5, K=10, queries="noisy"),
    4: dict(n=10_000_000, d=96, dtype="u8", ncomp=10_000, sigma=20.0, Q=100_000, qsigma=3.0,
            L=24, k=10, w=350.0, K=10, queries="zipf", nhot=1000, zipf_s=1.1),
    5: dict(n=1_000_000, d=960, dtype="f32", ncomp=500, sigma=0.05, Q=100_000, qsigma=0.05,
            L=16, k=12, w=1.5, K=10, queries="zipf", nhot=500, zipf_s=1.1,
            train_Q=200_000, data_cfg=3),
}


def make_config(cfg: int, *, n: Optional[int] = None, Q: Optional[int] = None,
                w: Optional[float] = None, ncomp: Optional[int] = None,
                nhot: Optional[int] = None, L: Optional[int] = None,
                k: Optional[int] = None, K: Optional[int] = None) -> Workload:
    """Workload of configuration cfg (1..5), optionally shrunk (n, Q, ncomp, nhot)
    for tests.  Seeds: data 1000+c, params 2000+c, queries 3000+c, where c is the
    configuration whose data is drawn (configuration 5 reuses configuration 3's
    data, index parameters and seeds for those, and draws its own queries)."""
    spec = dict(CONFIGS[cfg])
    if n is not None:
        spec["n"] = int(n)
    if Q is not None:
        spec["Q"] = int(Q)
    if ncomp is not None:
        spec["ncomp"] = int(ncomp)
    if nhot is not None:
        spec["nhot"] = int(nhot)
    if L is not None:
        spec["L"] = int(L)
    if k is not None:
        spec["k"] = int(k)
    if K is not None:
        spec["K"] = int(K)
    wv = spec["w"] if w is None else float(w)
    dcfg = spec.get("data_cfg", cfg)
    if spec["dtype"] == "u8":
        data, centres, _ = gmm_u8(SEED_DATA + dcfg, spec["n"], spec["d"], spec["ncomp"], spec["sigma"])
    else:
        data, centres, _ = mixture_f32(SEED_DATA + dcfg, spec["n"], spec["d"], spec["ncomp"], spec["sigma"])
    params = hash_params(SEED_PARAMS + dcfg, spec["L"], spec["k"], spec["d"], wv)
    if spec["queries"] == "noisy":
        queries = noisy_points(SEED_QUERIES + cfg, data, spec["Q"], spec["qsigma"])
    else:
        queries = zipf_queries(SEED_QUERIES + cfg, centres, spec["Q"], spec["nhot"],
                               spec["zipf_s"], spec["qsigma"], data.dtype)
    wl = Workload(name=f"cfg{cfg}", data=data, queries=queries, params=params,
                  K=spec["K"], centres=centres, meta=spec)
    return wl


def training_queries(cfg: int, Q: int, *, ncomp: Optional[int] = None,
                     n: Optional[int] = None, nhot: Optional[int] = None) -> np.ndarray:
    """Training workload for the candidate-count model (seed 4000+cfg), drawn like
    the configuration's own queries but from an independent stream."""
    spec = dict(CONFIGS[cfg])
    if ncomp is not None:
        spec["ncomp"] = int(ncomp)
    if n is not None:
        spec["n"] = int(n)
    if nhot is not None:
        spec["nhot"] = int(nhot)
    dcfg = spec.get("data_cfg", cfg)
    rng = _rng(SEED_DATA + dcfg)
    if spec["dtype"] == "u8":
        centres = rng.uniform(0.0, 255.0, size=(spec["ncomp"], spec["d"]))
        dt = np.uint8
    else:
        centres = rng.uniform(0.0, 1.0, size=(spec["ncomp"], spec["d"]))
        dt = np.float32
    return zipf_queries(SEED_TRAIN + cfg, centres, Q, spec.get("nhot", spec["ncomp"]),
                        spec.get("zipf_s", 1.1), spec["qsigma"], dt)


def random_small(seed: int, n: int, d: int, Q: int, L: int, k: int, w: float,
                 dtype: str = "u8", K: int = 10) -> Workload:
    """Small uniform random workload for edge-case tests (ragged sizes)."""
    rng = _rng(seed)
    if dtype == "u8":
        data = rng.integers(0, 256, size=(n, d), dtype=np.uint8)
        queries = rng.integers(0, 256, size=(Q, d), dtype=np.uint8)
    else:
        data = rng.random((n, d), dtype=np.float32)
        queries = rng.random((Q, d), dtype=np.float32)
    params = hash_params(seed + 1, L, k, d, w)
    return Workload(name=f"rand{seed}", data=data, queries=queries, params=params, K=K)


def boundary_params(seed: int, L: int, k: int, d: int, w: float = 4.0, amax: int = 2):
    """Parameters whose projections land exactly on (or one float32 ulp beside)
    bucket boundaries for integer data: a has small integer entries, w is an
    integer and b is an integer, or an integer minus/plus one ulp.  Returns
    (a float32 (L,k,d), b float32 (L,k), w)."""
    rng = _rng(seed)
    a = rng.integers(-amax, amax + 1, size=(L, k, d)).astype(np.float32)
    base = rng.integers(0, int(w), size=(L, k)).astype(np.float32)
    mode = rng.integers(0, 3, size=(L, k))
    b = base.copy()
    up = np.nextafter(base, np.float32(np.inf))
    dn = np.nextafter(base, np.float32(-np.inf))
    b = np.where(mode == 1, up, b)
    b = np.where((mode == 2) & (base > 0), dn, b)
    return a, b.astype(np.float32), float(w)
