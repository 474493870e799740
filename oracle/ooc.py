"""Out-of-core cache simulation: the index cache C_I and the data cache C_D.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark are the only
callers; nothing in the GPU library imports this module.

The paper keeps index files and data objects on external storage and splits
main memory into a cache C = C_I + C_D: C_I holds index files (bucket data)
and C_D holds data objects (Section 4, the split problem).  Each part evicts by
MRU, and C_I is organised by Strategy 1 or 2 (Section 5.1, Design of qwLSH).
Under Strategy 1, C_I is divided equally among the hash layers and each share
evicts on its own; under Strategy 2, one C_I serves every layer.  IO is
counted as index files and data objects read from storage (the IndexIO and
DataIO of Section 1.2, the cost terms of Sections 4 and 5.2).

Reading used for a workload answered in batches of consecutive queries (a
batch of one query is the paper's query-at-a-time setting):

* An index file is one bucket of one layer; its size is 4 bytes per member
  id.  A data object is one point's row of `row_bytes` bytes.
* Capacity: C_I = floor(cache_bytes * index_percent / 100) bytes hold
  floor(C_I / 4) ids.  Under Strategy 1 each layer's share holds
  floor(ids / L) ids; under Strategy 2 one pool holds them all.
  C_D = cache_bytes - C_I holds floor(C_D / row_bytes) rows.
* Recency: query q's layer-l bucket is used at position q * L + l + 1, and a
  data object in C(q) is used at q + 1.  An item's stamp is its largest use
  so far.  No two buckets share a stamp.  Data objects that share one are
  ordered by id.
* For each batch [q0, q1):
  - Index phase.  N is the set of non-empty buckets of the batch's queries,
    and the misses are the members of N not resident.  For each pool,
    deficit = resident ids + ids of the misses - capacity.  A pool with a
    positive deficit evicts its resident buckets outside N, most recently
    used first (MRU; LRU takes the least recently used first), until the
    evicted ids cover the deficit.  If some pool cannot, the batch fails and
    nothing changes.  Otherwise every miss is read (one index file each) and
    becomes resident, and each member of N takes the largest use the batch
    makes of it as its stamp, if that is larger than the old one.
  - Data phase.  D is the union of C(q) over the batch.  The deficit is
    resident rows + misses - capacity, and it is covered by evicting resident
    rows outside D in the same order, with key (stamp, id).  If they cannot
    cover it, the batch fails; the index phase stays done.  Otherwise the
    misses are read (one data object each) and the stamps are updated to the
    batch's largest use (q + 1).
  - A failed batch of several queries is answered as two batches, the first
    ceil(m / 2) queries and then the rest.  A failed single query is an
    error: the cache cannot hold one query's index files or candidates.

The paper prints no worked example or per-query figure of its cache, so the
counts are pinned to what the definitions fix: compulsory reads with an
unbounded cache, the textbook MRU and LRU sequences on a cyclic trace, the
inclusion property of both policies, Strategy 1 as independent per-layer
caches, and hand-worked eviction, stamp and split cases (tests/test_oracle_ooc.py).
"""
from __future__ import annotations

from typing import Dict, Hashable, List, Sequence, Set, Tuple

import numpy as np

MRU, LRU = 0, 1


class CacheTooSmall(ValueError):
    """One query's index files or candidates do not fit their cache."""


def workload_needs(data: np.ndarray, queries: np.ndarray, a: np.ndarray, b: np.ndarray,
                   w: float) -> List[List[Tuple[int, Hashable, int]]]:
    """Per query, the (layer, bucket key, bucket size) of each layer whose
    bucket holds at least one point (the index files the query reads)."""
    from . import hash_points
    L, k, _ = a.shape
    hd = hash_points(data, a, b, w).reshape(data.shape[0], L, k)
    hq = hash_points(queries, a, b, w).reshape(queries.shape[0], L, k)
    needs: List[List[Tuple[int, Hashable, int]]] = [[] for _ in range(queries.shape[0])]
    for l in range(L):
        size: Dict[bytes, int] = {}
        for row in hd[:, l, :]:
            key = row.tobytes()
            size[key] = size.get(key, 0) + 1
        for q in range(queries.shape[0]):
            key = hq[q, l, :].tobytes()
            s = size.get(key, 0)
            if s:
                needs[q].append((l, key, s))
    return needs


def simulate(index_needs: Sequence[Sequence[Tuple[int, Hashable, int]]],
             data_needs: Sequence[Sequence[int]], L: int, row_bytes: int, cache_bytes: int,
             index_percent: int, strategy: int, policy: int, batch: int) -> Dict[str, int]:
    """IO counts of answering the workload through the cache described in the
    module docstring.  index_needs[q]: (layer, bucket key, size) per non-empty
    bucket of query q; data_needs[q]: the ids of C(q)."""
    if strategy not in (1, 2) or policy not in (MRU, LRU) or batch < 1:
        raise ValueError("strategy 1 or 2, policy MRU or LRU, batch >= 1")
    ci_bytes = cache_bytes * index_percent // 100
    ids_total = ci_bytes // 4
    npools = L if strategy == 1 else 1
    cap_pool = ids_total // L if strategy == 1 else ids_total
    cap_rows = (cache_bytes - ci_bytes) // row_bytes
    Q = len(index_needs)

    res_i: Dict[Tuple[int, Hashable], List[int]] = {}  # (layer, key) -> [size, stamp]
    used = [0] * npools
    res_d: Dict[int, int] = {}                         # id -> stamp
    io = {"index_files": 0, "index_bytes": 0, "data_objects": 0, "data_bytes": 0,
          "batches": 0, "splits": 0}

    def pool(layer: int) -> int:
        return layer if strategy == 1 else 0

    def index_phase(q0: int, q1: int) -> bool:
        need: Dict[Tuple[int, Hashable], List[int]] = {}
        for q in range(q0, q1):
            for (l, key, s) in index_needs[q]:
                u = q * L + l + 1
                item = need.setdefault((l, key), [s, 0])
                item[1] = max(item[1], u)
        miss = [it for it in need if it not in res_i]
        miss_ids = [0] * npools
        for it in miss:
            miss_ids[pool(it[0])] += need[it][0]
        evict: List[Tuple[int, Hashable]] = []
        for p in range(npools):
            deficit = used[p] + miss_ids[p] - cap_pool
            if deficit <= 0:
                continue
            cand = [it for it in res_i if pool(it[0]) == p and it not in need]
            cand.sort(key=lambda it: res_i[it][1], reverse=(policy == MRU))
            freed = 0
            for it in cand:
                if freed >= deficit:
                    break
                evict.append(it)
                freed += res_i[it][0]
            if freed < deficit:
                return False
        for it in evict:
            used[pool(it[0])] -= res_i[it][0]
            del res_i[it]
        for it in miss:
            s = need[it][0]
            res_i[it] = [s, 0]
            used[pool(it[0])] += s
            io["index_files"] += 1
            io["index_bytes"] += 4 * s
        for it, (s, u) in need.items():
            res_i[it][1] = max(res_i[it][1], u)
        return True

    def data_phase(q0: int, q1: int) -> bool:
        need: Dict[int, int] = {}
        for q in range(q0, q1):
            for i in data_needs[q]:
                need[int(i)] = q + 1  # queries in increasing order: the last is the largest
        miss = [i for i in need if i not in res_d]
        deficit = len(res_d) + len(miss) - cap_rows
        if deficit > 0:
            cand = [i for i in res_d if i not in need]
            if len(cand) < deficit:
                return False
            cand.sort(key=lambda i: (res_d[i], i), reverse=(policy == MRU))
            for i in cand[:deficit]:
                del res_d[i]
        for i in miss:
            res_d[i] = 0
            io["data_objects"] += 1
            io["data_bytes"] += row_bytes
        for i, u in need.items():
            res_d[i] = max(res_d[i], u)
        return True

    def run(q0: int, q1: int) -> None:
        stack = [(q0, q1)]
        while stack:
            lo, hi = stack.pop()
            ok = index_phase(lo, hi) and data_phase(lo, hi)
            if ok:
                io["batches"] += 1
                continue
            if hi - lo == 1:
                raise CacheTooSmall(f"query {lo} does not fit the cache")
            io["splits"] += 1
            mid = lo + (hi - lo + 1) // 2
            stack.append((mid, hi))
            stack.append((lo, mid))

    for q0 in range(0, Q, batch):
        run(q0, min(Q, q0 + batch))
    return io


def distinct_reads(index_needs, data_needs, row_bytes: int) -> Dict[str, int]:
    """The compulsory reads: every distinct index file and data object of the
    workload read exactly once (an unbounded cache)."""
    files: Set[Tuple[int, Hashable]] = set()
    fbytes = 0
    for needs in index_needs:
        for (l, key, s) in needs:
            if (l, key) not in files:
                files.add((l, key))
                fbytes += 4 * s
    objs = np.unique(np.concatenate([np.asarray(c, dtype=np.int64) for c in data_needs] +
                                    [np.zeros(0, np.int64)]))
    return {"index_files": len(files), "index_bytes": fbytes,
            "data_objects": int(objs.size), "data_bytes": int(objs.size) * row_bytes}
