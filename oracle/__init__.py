"""CPU oracle for the p-stable LSH query-workload path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing in the GPU library imports this
package, and this package imports nothing from the library.

Modules:
  qw_oracle.c  -- hashing, per-layer buckets, candidate union (or collision
                  counting with a cap), exact verification, top-K and brute-force
                  kNN in FP64 / int64 (plain C, threads over queries only);
                  loaded here through ctypes.
  mlp.py       -- FP64 forward/backward of the candidate-count regressor.
  collision.py -- the p-stable collision probability of Eq. (1).
  ooc.py       -- the index and data caches of the out-of-core setting
                  (Sections 4 and 5.1): IO counts of a workload answered in
                  batches through a C_I / C_D split with MRU or LRU eviction.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qw_oracle.c")
_LIB = os.path.join(_HERE, "libqworacle.so")
CFLAGS = ["-O2", "-std=gnu11", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
          "-pthread", "-Wall", "-Wextra"]

U8, F32 = 0, 1
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.orc_hash.argtypes = [P, i64, i32, i32, P, P, i32, f64, i32, P]
        lib.orc_lsh_query.argtypes = [P, i64, i32, i32, P, i64, P, P, i32, i32, f64, i32, i32,
                                      P, P, P, P, i32, i32]
        lib.orc_lsh_candidates.argtypes = [P, i64, i32, i32, P, i64, P, P, i32, i32, f64, i32,
                                           P, P, P, i32, i32]
        lib.orc_project.argtypes = [P, i64, i32, i32, P, P, i32, f64, P]
        lib.orc_bruteforce.argtypes = [P, i64, i32, i32, P, i64, i32, i32, P, P, P]
        lib.orc_lsh_build.argtypes = [P, i64, i32, i32, P, P, i32, i32, f64, i32]
        lib.orc_lsh_build.restype = ctypes.c_void_p
        lib.orc_lsh_query_built.argtypes = [P, P, i64, i32, i32, P, P, P, P, i32, i32]
        lib.orc_lsh_query_counting.argtypes = [P, i64, i32, i32, P, i64, P, P, i32, i32, f64,
                                               i32, i32, i32, i32, P, P, P, P]
        lib.orc_lsh_query_counting.restype = ctypes.c_int
        lib.orc_lsh_free.argtypes = [P]
        lib.orc_lsh_free.restype = None
        for f in (lib.orc_hash, lib.orc_lsh_query, lib.orc_lsh_candidates, lib.orc_bruteforce,
                  lib.orc_lsh_query_built):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _threads(nthreads: Optional[int]) -> int:
    if nthreads:
        return int(nthreads)
    return max(1, min(16, os.cpu_count() or 1))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _dtype_code(x: np.ndarray) -> int:
    if x.dtype == np.uint8:
        return U8
    if x.dtype == np.float32:
        return F32
    raise TypeError("oracle supports uint8 and float32 vectors")


def hash_points(x: np.ndarray, a: np.ndarray, b: np.ndarray, w: float,
                nthreads: Optional[int] = None) -> np.ndarray:
    """h[m, f] = floor((a_f . x_m + b_f) / w) in FP64, index order.
    a: (..., d) float32 flattened to (nf, d); b: (...,) float32 flattened to (nf,)."""
    x = np.ascontiguousarray(x)
    d = x.shape[1]
    a2 = np.ascontiguousarray(a, dtype=np.float32).reshape(-1, d)
    b2 = np.ascontiguousarray(b, dtype=np.float32).reshape(-1)
    assert a2.shape[0] == b2.shape[0]
    out = np.empty((x.shape[0], a2.shape[0]), dtype=np.int32)
    rc = _load().orc_hash(_ptr(x), x.shape[0], d, _dtype_code(x), _ptr(a2), _ptr(b2),
                          a2.shape[0], float(np.float32(w)), _threads(nthreads), _ptr(out))
    if rc:
        raise ValueError("orc_hash failed (%d)" % rc)
    return out


def project(x: np.ndarray, a: np.ndarray, b: np.ndarray, w: float) -> np.ndarray:
    """y [m, L*k] float64: (a.x + b) / w in the hashing's FP64 sequence (h = floor(y))."""
    x = np.ascontiguousarray(x)
    a2 = np.ascontiguousarray(a.reshape(-1, a.shape[-1]), dtype=np.float32)
    b2 = np.ascontiguousarray(b.reshape(-1), dtype=np.float32)
    out = np.empty((x.shape[0], a2.shape[0]), dtype=np.float64)
    rc = _load().orc_project(_ptr(x), x.shape[0], x.shape[1], _dtype_code(x), _ptr(a2), _ptr(b2),
                             a2.shape[0], float(np.float32(w)), _ptr(out))
    if rc:
        raise ValueError("orc_project failed (%d)" % rc)
    return out


def lsh_query(data: np.ndarray, queries: np.ndarray, a: np.ndarray, b: np.ndarray,
              w: float, K: int, nthreads: Optional[int] = None, probes: int = 0,
              probe_t: int = 0):
    """Top-K of every query over its LSH candidates (probes=1: also the 2k
    one-step neighbour buckets of every layer; probes=2: the probe_t of them
    with the smallest boundary-distance scores).
    Returns (ids int32 [Q,K], dist [Q,K] int64 (u8) or float64 (f32), counts int64 [Q])."""
    data = np.ascontiguousarray(data)
    queries = np.ascontiguousarray(queries)
    L, k, d = a.shape
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    Q = queries.shape[0]
    ids = np.empty((Q, K), dtype=np.int32)
    cnt = np.empty((Q,), dtype=np.int64)
    dt = _dtype_code(data)
    if dt == U8:
        dist = np.empty((Q, K), dtype=np.int64)
        pi, pf = _ptr(dist), None
    else:
        dist = np.empty((Q, K), dtype=np.float64)
        pi, pf = None, _ptr(dist)
    rc = _load().orc_lsh_query(_ptr(data), data.shape[0], d, dt, _ptr(queries), Q, _ptr(a),
                               _ptr(b), L, k, float(np.float32(w)), int(K), _threads(nthreads),
                               _ptr(ids), pi, pf, _ptr(cnt), int(probes), int(probe_t))
    if rc:
        raise ValueError("orc_lsh_query failed (%d)" % rc)
    return ids, dist, cnt


def lsh_query_counting(data: np.ndarray, queries: np.ndarray, a: np.ndarray, b: np.ndarray,
                       w: float, K: int, theta: int, v: int, nthreads: Optional[int] = None):
    """Collision counting with a candidate cap (Section 3, "Collision Counting"): the points sharing
    a bucket with the query in at least theta layers, ranked by (layer count
    descending, id ascending), the first K + v of them verified, the top K kept.
    Returns (ids int32 [Q,K], dist [Q,K] int64 (u8) or float64 (f32),
    verified int64 [Q])."""
    data = np.ascontiguousarray(data)
    queries = np.ascontiguousarray(queries)
    L, k, d = a.shape
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    Q = queries.shape[0]
    ids = np.empty((Q, K), dtype=np.int32)
    cnt = np.empty((Q,), dtype=np.int64)
    dt = _dtype_code(data)
    if dt == U8:
        dist = np.empty((Q, K), dtype=np.int64)
        pi, pf = _ptr(dist), None
    else:
        dist = np.empty((Q, K), dtype=np.float64)
        pi, pf = None, _ptr(dist)
    rc = _load().orc_lsh_query_counting(_ptr(data), data.shape[0], d, dt, _ptr(queries), Q,
                                        _ptr(a), _ptr(b), L, k, float(np.float32(w)), int(K),
                                        int(theta), int(v), _threads(nthreads), _ptr(ids), pi,
                                        pf, _ptr(cnt))
    if rc:
        raise ValueError("orc_lsh_query_counting failed (%d)" % rc)
    return ids, dist, cnt


def lsh_candidates(data: np.ndarray, queries: np.ndarray, a: np.ndarray, b: np.ndarray,
                   w: float, nthreads: Optional[int] = None, probes: int = 0,
                   probe_t: int = 0) -> List[np.ndarray]:
    """Candidate set C(q) of every query, each as ascending int32 ids (probes=1:
    with the one-step neighbour buckets)."""
    data = np.ascontiguousarray(data)
    queries = np.ascontiguousarray(queries)
    L, k, d = a.shape
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    Q = queries.shape[0]
    lib = _load()
    dt = _dtype_code(data)
    cnt = np.empty((Q,), dtype=np.int64)
    args = (_ptr(data), data.shape[0], d, dt, _ptr(queries), Q, _ptr(a), _ptr(b), L, k,
            float(np.float32(w)), _threads(nthreads))
    rc = lib.orc_lsh_candidates(*args, _ptr(cnt), None, None, int(probes), int(probe_t))
    if rc:
        raise ValueError("orc_lsh_candidates failed (%d)" % rc)
    off = np.zeros(Q + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    ids = np.empty(max(1, int(off[-1])), dtype=np.int32)
    rc = lib.orc_lsh_candidates(*args, _ptr(cnt), _ptr(off), _ptr(ids), int(probes), int(probe_t))
    if rc:
        raise ValueError("orc_lsh_candidates failed (%d)" % rc)
    return [ids[off[i]:off[i + 1]].copy() for i in range(Q)]


def bruteforce(data: np.ndarray, queries: np.ndarray, K: int,
               nthreads: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Exact top-K over all points: (ids int32 [Q,K], dist int64 or float64 [Q,K])."""
    data = np.ascontiguousarray(data)
    queries = np.ascontiguousarray(queries)
    Q, d = queries.shape
    ids = np.empty((Q, K), dtype=np.int32)
    dt = _dtype_code(data)
    if dt == U8:
        dist = np.empty((Q, K), dtype=np.int64)
        pi, pf = _ptr(dist), None
    else:
        dist = np.empty((Q, K), dtype=np.float64)
        pi, pf = None, _ptr(dist)
    rc = _load().orc_bruteforce(_ptr(data), data.shape[0], d, dt, _ptr(queries), Q, int(K),
                                _threads(nthreads), _ptr(ids), pi, pf)
    if rc:
        raise ValueError("orc_bruteforce failed (%d)" % rc)
    return ids, dist


class BuiltIndex:
    """The oracle's index built once (hash + per-layer buckets) and queried later;
    lets the build and query phases be timed separately.  Keeps references to
    the arrays it was built from."""

    def __init__(self, data, a, b, w, nthreads=None):
        self.data = np.ascontiguousarray(data)
        L, k, d = a.shape
        self.a = np.ascontiguousarray(a, dtype=np.float32)
        self.b = np.ascontiguousarray(b, dtype=np.float32)
        self.nthreads = _threads(nthreads)
        self.h = _load().orc_lsh_build(_ptr(self.data), self.data.shape[0], d,
                                       _dtype_code(self.data), _ptr(self.a), _ptr(self.b), L, k,
                                       float(np.float32(w)), self.nthreads)
        if not self.h:
            raise ValueError("orc_lsh_build failed")

    def query(self, queries, K, probes=0, probe_t=0):
        queries = np.ascontiguousarray(queries)
        Q = queries.shape[0]
        ids = np.empty((Q, K), dtype=np.int32)
        cnt = np.empty((Q,), dtype=np.int64)
        if _dtype_code(self.data) == U8:
            dist = np.empty((Q, K), dtype=np.int64)
            pi, pf = _ptr(dist), None
        else:
            dist = np.empty((Q, K), dtype=np.float64)
            pi, pf = None, _ptr(dist)
        rc = _load().orc_lsh_query_built(ctypes.c_void_p(self.h), _ptr(queries), Q, int(K),
                                         self.nthreads, _ptr(ids), pi, pf, _ptr(cnt),
                                         int(probes), int(probe_t))
        if rc:
            raise ValueError("orc_lsh_query_built failed (%d)" % rc)
        return ids, dist, cnt

    def close(self):
        if self.h:
            _load().orc_lsh_free(ctypes.c_void_p(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
