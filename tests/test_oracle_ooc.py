"""Pins of the out-of-core cache simulation (oracle/ooc.py) to what the
definitions of the index and data caches fix (Section 4; Strategies 1 and 2
and MRU replacement, Section 5.1).  CPU only."""
import json
import os

import numpy as np
import pytest

from oracle import lsh_candidates
from oracle import ooc

HERE = os.path.dirname(os.path.abspath(__file__))


def unit_trace(trace):
    """One layer; query q reads index file trace[q] (one id) and data object
    trace[q]."""
    return [[(0, int(t), 1)] for t in trace], [[int(t)] for t in trace]


def test_cyclic_trace_golden():
    g = json.load(open(os.path.join(HERE, "golden", "ooc_cyclic.json")))
    ineeds, dneeds = unit_trace(g["trace"])
    for name, pol in (("MRU", ooc.MRU), ("LRU", ooc.LRU)):
        for strategy in (1, 2):
            io = ooc.simulate(ineeds, dneeds, L=1, row_bytes=4, cache_bytes=24, index_percent=50,
                              strategy=strategy, policy=pol, batch=1)
            assert io["index_files"] == g["expected"][name]["index_files"], (name, io)
            assert io["data_objects"] == g["expected"][name]["data_objects"], (name, io)
            assert io["index_bytes"] == 4 * io["index_files"]
            assert io["data_bytes"] == 4 * io["data_objects"]
            assert io["batches"] == 12 and io["splits"] == 0


@pytest.mark.parametrize("pol", [ooc.MRU, ooc.LRU])
def test_inclusion_property(pol):
    """MRU and LRU order victims by last use, which does not depend on the cache
    size, so one item per access obeys the inclusion property: a larger cache
    never reads more."""
    rng = np.random.default_rng(5)
    for trial in range(20):
        trace = rng.integers(0, 9, size=60)
        ineeds, dneeds = unit_trace(trace)
        prev_i = prev_d = None
        for cap in range(1, 11):
            io = ooc.simulate(ineeds, dneeds, L=1, row_bytes=4, cache_bytes=8 * cap,
                              index_percent=50, strategy=2, policy=pol, batch=1)
            if prev_i is not None:
                assert io["index_files"] <= prev_i and io["data_objects"] <= prev_d
            prev_i, prev_d = io["index_files"], io["data_objects"]
        # a cache holding every item reads each item once
        assert prev_i == len(set(trace.tolist())) and prev_d == prev_i


def small_workload(seed=3, n=3000, d=16, Q=60, L=4, k=3):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, 255, size=(20, d))
    data = np.clip(np.rint(centres[rng.integers(0, 20, n)] + rng.normal(0, 12, (n, d))),
                   0, 255).astype(np.uint8)
    queries = np.clip(np.rint(data[rng.integers(0, n, Q)] + rng.normal(0, 2, (Q, d))),
                      0, 255).astype(np.uint8)
    a = rng.normal(size=(L, k, d)).astype(np.float32)
    w = 120.0
    b = (rng.uniform(size=(L, k)) * w).astype(np.float32)
    return data, queries, a, b, w


def test_unbounded_cache_reads_each_item_once():
    data, queries, a, b, w = small_workload()
    L = a.shape[0]
    ineeds = ooc.workload_needs(data, queries, a, b, w)
    cands = lsh_candidates(data, queries, a, b, w)
    # independent count of the compulsory reads
    files = {(l, key) for needs in ineeds for (l, key, _) in needs}
    objs = np.unique(np.concatenate(cands))
    assert len(files) > 20 and objs.size > 200
    for strategy in (1, 2):
        for pol in (ooc.MRU, ooc.LRU):
            for batch in (1, 7, 60):
                io = ooc.simulate(ineeds, cands, L=L, row_bytes=16, cache_bytes=1 << 30,
                                  index_percent=50, strategy=strategy, policy=pol, batch=batch)
                assert io["index_files"] == len(files)
                assert io["data_objects"] == objs.size
                assert io["splits"] == 0
                assert io == dict(ooc.distinct_reads(ineeds, cands, 16),
                                  batches=-(-60 // batch), splits=0)


def test_workload_needs_match_bucket_definition():
    """Bucket sizes against a direct count of the points sharing the query's
    k hash values in that layer (numpy broadcasting over all points)."""
    from oracle import hash_points
    data, queries, a, b, w = small_workload(Q=15)
    L, k, _ = a.shape
    hd = hash_points(data, a, b, w).reshape(-1, L, k)
    hq = hash_points(queries, a, b, w).reshape(-1, L, k)
    needs = ooc.workload_needs(data, queries, a, b, w)
    for q in range(queries.shape[0]):
        got = {l: s for (l, _, s) in needs[q]}
        for l in range(L):
            s = int(np.all(hd[:, l, :] == hq[q, l, :], axis=1).sum())
            assert got.get(l, 0) == s


def test_strategy1_is_independent_layer_caches():
    """Strategy 1 gives every layer its own share and its own MRU list: with no
    split, its reads are the sum of L one-layer caches of that share."""
    data, queries, a, b, w = small_workload(seed=9, Q=80)
    L = a.shape[0]
    ineeds = ooc.workload_needs(data, queries, a, b, w)
    empty = [[] for _ in ineeds]
    biggest = max(s for needs in ineeds for (_, _, s) in needs)
    for pol in (ooc.MRU, ooc.LRU):
        cap_pool = biggest + 40
        cache = cap_pool * L * 8  # index share 50 %: cap_pool * L ids
        io = ooc.simulate(ineeds, empty, L=L, row_bytes=16, cache_bytes=cache,
                          index_percent=50, strategy=1, policy=pol, batch=1)
        assert io["splits"] == 0
        tot = 0
        for l in range(L):
            sub = [[(0, key, s) for (ll, key, s) in needs if ll == l] for needs in ineeds]
            r = ooc.simulate(sub, empty, L=1, row_bytes=16, cache_bytes=8 * cap_pool,
                             index_percent=50, strategy=2, policy=pol, batch=1)
            tot += r["index_files"]
        assert io["index_files"] == tot
        # the per-layer caches are smaller than everything: some files are read twice
        assert tot > len({(l, key) for needs in ineeds for (l, key, _) in needs})


def test_split_hand_example():
    """Two queries: one bucket of four ids shared, disjoint candidates {0, 1}
    and {2, 3}; the data cache holds two rows.  The batch of both fails in its
    data phase (four rows), after its index phase read the bucket.  The first
    query then reads rows 0 and 1; the second evicts both and reads 2 and 3."""
    ineeds = [[(0, "X", 4)], [(0, "X", 4)]]
    dneeds = [[0, 1], [2, 3]]
    # index share 50 % of 64 bytes: 8 ids; data: 32 bytes = 2 rows of 16
    io = ooc.simulate(ineeds, dneeds, L=1, row_bytes=16, cache_bytes=64, index_percent=50,
                      strategy=2, policy=ooc.MRU, batch=2)
    assert io == {"index_files": 1, "index_bytes": 16, "data_objects": 4, "data_bytes": 64,
                  "batches": 2, "splits": 1}
    with pytest.raises(ooc.CacheTooSmall):
        ooc.simulate([[(0, "X", 4)]], [[0, 1, 2]], L=1, row_bytes=16, cache_bytes=64,
                     index_percent=50, strategy=2, policy=ooc.MRU, batch=1)
    with pytest.raises(ooc.CacheTooSmall):  # a bucket of 9 ids in a cache of 8
        ooc.simulate([[(0, "Y", 9)]], [[0]], L=1, row_bytes=16, cache_bytes=64,
                     index_percent=50, strategy=2, policy=ooc.MRU, batch=1)


def test_needed_items_are_never_victims():
    """Query 1 reads buckets A (layer 1) and C (layer 0) after query 0 read A
    (layer 1, use 2) and B (layer 0, use 1).  One pool of two ids: C's miss
    evicts one item, and A, the most recently used, is needed by the same
    query, so B goes.  Three index files; the same holds for rows."""
    ineeds = [[(0, "B", 1), (1, "A", 1)], [(0, "C", 1), (1, "A", 1)]]
    dneeds = [[5, 7], [5, 9]]
    for pol in (ooc.MRU, ooc.LRU):
        io = ooc.simulate(ineeds, dneeds, L=2, row_bytes=4, cache_bytes=16, index_percent=50,
                          strategy=2, policy=pol, batch=1)
        assert io["index_files"] == 3 and io["data_objects"] == 3, io


def test_stamp_is_last_use_within_a_batch():
    """Batches of two.  Batch 1: query 0 reads rows {0, 1}, query 1 reads {0}:
    row 0 was last used by query 1 (stamp 2), row 1 by query 0 (stamp 1).
    Batch 2 (queries 2 and 3 read {2}) must evict one row of a two-row cache;
    MRU takes row 0.  Batch 3 (queries 4 and 5 read {0}) reads row 0 again and
    evicts row 2 (stamp 4).  Four reads.  The index side is built the same
    way: bucket X is used by both queries of batch 1 (last at use 3), bucket Y
    only by query 0 (use 2)."""
    dneeds = [[0, 1], [0], [2], [2], [0], [0]]
    io = ooc.simulate([[] for _ in dneeds], dneeds, L=1, row_bytes=4, cache_bytes=16,
                      index_percent=50, strategy=2, policy=ooc.MRU, batch=2)
    assert io["data_objects"] == 4 and io["batches"] == 3, io
    ineeds = [[(0, "X", 1), (1, "Y", 1)], [(0, "X", 1)], [(0, "Z", 1)], [(0, "Z", 1)],
              [(0, "X", 1)], [(0, "X", 1)]]
    io = ooc.simulate(ineeds, [[] for _ in ineeds], L=2, row_bytes=4, cache_bytes=16,
                      index_percent=50, strategy=2, policy=ooc.MRU, batch=2)
    assert io["index_files"] == 4 and io["batches"] == 3, io


def test_split_halves_round_up():
    """A batch of three that fails splits into the first two queries and the
    last one.  Query 0 alone needs both rows of the cache, so the pair fails
    again: three batches after two splits (a split that took one query first
    would need only one)."""
    dneeds = [[0, 1], [2], [3]]
    io = ooc.simulate([[] for _ in dneeds], dneeds, L=1, row_bytes=4, cache_bytes=16,
                      index_percent=50, strategy=2, policy=ooc.MRU, batch=3)
    assert io["batches"] == 3 and io["splits"] == 2 and io["data_objects"] == 4, io
