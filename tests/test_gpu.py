"""GPU parity tests: the HIP path (through the C ABI) against the CPU oracle.

Bucket ids, candidate sets and top-K ids must be bit-exact; uint8 distances are
exact int32; float distances must lie within 1e-5 relative of the FP64 oracle
(the library returns the FP64 index-order distance rounded once to float32).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1907_11803_amd import lib, synth

pytestmark = pytest.mark.gpu

I32MAX = np.iinfo(np.int32).max
FORMS = [lib.QW_FORM_PLAIN_FP32, lib.QW_FORM_FAST]
SCHEDS = [lib.QW_SCHED_SUM, lib.QW_SCHED_ACTUAL, lib.QW_SCHED_NONE, lib.QW_SCHED_LEARNED]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def build(wl_data, a, b, w, form=lib.QW_FORM_FAST):
    return lib.Index(dev(wl_data), dev(a), dev(b), w, form=form)


def check_topk(ids_g, dist_g, ids_o, dist_o, is_u8):
    ids_g = ids_g.cpu().numpy()
    dist_g = dist_g.cpu().numpy()
    assert np.array_equal(ids_g, ids_o), np.argwhere(ids_g != ids_o)[:5]
    if is_u8:
        want = np.where(dist_o == np.iinfo(np.int64).max, I32MAX, dist_o).astype(np.int64)
        assert np.array_equal(dist_g.astype(np.int64), want)
    else:
        fin = np.isfinite(dist_o)
        assert np.array_equal(np.isfinite(dist_g), fin)
        np.testing.assert_allclose(dist_g[fin], dist_o[fin], rtol=1e-5, atol=0)
        # the library rounds the FP64 distance once
        assert np.array_equal(dist_g[fin], dist_o[fin].astype(np.float32))


@pytest.fixture(scope="module")
def cfg1():
    return synth.make_config(1)


# ---------------------------------------------------------------- hashing

@pytest.mark.parametrize("form", FORMS)
def test_hash_bit_exact_cfg1(cfg1, form):
    p = cfg1.params
    ix = build(cfg1.data, p.a, p.b(), p.w, form)
    for x in (cfg1.data[:3001], cfg1.queries):
        h, rec = ix.hash(dev(x), form)
        want = oracle.hash_points(x, p.a, p.b(), p.w)
        assert np.array_equal(h.cpu().numpy(), want)
        assert 0 <= rec < 0.05 * want.size


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dtype,d", [("u8", 48), ("u8", 150), ("f32", 150)])
def test_hash_boundary_cases(form, dtype, d):
    """Projections exactly on bucket boundaries or one ulp of b beside them
    (float data holds small integers, so its projections hit them too)."""
    L, k = 3, 5
    a, b, w = synth.boundary_params(17, L, k, d, w=4.0)
    rng = np.random.default_rng(18)
    x = rng.integers(0, 256, size=(777, d), dtype=np.uint8)
    if dtype == "f32":
        x = x.astype(np.float32)
    ix = build(x, a, b, w, form)
    h, rec = ix.hash(dev(x), form)
    assert np.array_equal(h.cpu().numpy(), oracle.hash_points(x, a, b, w))
    assert rec > 0  # exact boundary hits must take the FP64 path


@pytest.mark.parametrize("form", FORMS)
def test_hash_float_data_ragged_d(form):
    wl = synth.random_small(23, n=1500, d=37, Q=70, L=3, k=7, w=0.7, dtype="f32")
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w, form)
    h, _ = ix.hash(dev(wl.queries), form)
    assert np.array_equal(h.cpu().numpy(), oracle.hash_points(wl.queries, p.a, p.b(), p.w))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dtype,d", [("f32", 200), ("u8", 300)])
def test_hash_several_k_chunks(form, dtype, d):
    """Rows longer than one staged K chunk, with a ragged last chunk."""
    wl = synth.random_small(29, n=700, d=d, Q=131, L=4, k=9,
                            w=3.0 if dtype == "f32" else 900.0, dtype=dtype)
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w, form)
    for x in (wl.data, wl.queries):
        h, _ = ix.hash(dev(x), form)
        assert np.array_equal(h.cpu().numpy(), oracle.hash_points(x, p.a, p.b(), p.w))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("L,k,d,wb", [(19, 7, 40, 4.0), (20, 8, 128, 4.0), (64, 2, 24, 4.0),
                                      (32, 8, 24, 2.0), (20, 8, 300, 4.0)])
def test_hash_many_rows_several_function_tiles(form, L, k, d, wb):
    """Enough rows that the FP16 matrix-core kernel gives each workgroup several
    64-function tiles of its rows (ragged last row block; 133, 160, 128 and 256
    functions per row: a ragged last tile, and row pitches that are and are
    not a multiple of four values; d = 300 takes three staged chunks per
    tile).  Parameters on bucket boundaries, so some outputs take the FP64
    recomputation in every tile; at w = 2 about half of a workgroup's 16,384
    outputs do, more than its pooled recomputes hold, so each lane
    recomputes its own."""
    a, b, w = synth.boundary_params(31, L, k, d, w=wb)
    rng = np.random.default_rng(32)
    x = rng.integers(0, 256, size=(100_003, d), dtype=np.uint8)
    ix = build(x[:256], a, b, w, form)  # a small index: keys stay within 128 bits
    h, rec = ix.hash(dev(x), form)
    want = oracle.hash_points(x, a, b, w)
    assert np.array_equal(h.cpu().numpy(), want)
    assert rec > 0


# ---------------------------------------------------------------- candidates

@pytest.mark.parametrize("w", [400.0, 1200.0])
def test_candidate_sets_cfg1(cfg1, w):
    p = cfg1.params
    ix = build(cfg1.data, p.a, p.b(w), w)
    q = cfg1.queries
    got = ix.candidate_lists(dev(q))
    want = oracle.lsh_candidates(cfg1.data, q, p.a, p.b(w), w)
    for g, o in zip(got, want):
        assert np.array_equal(g, o)
    cnt = ix.candidate_counts(dev(q)).cpu().numpy()
    assert cnt.tolist() == [len(o) for o in want]
    sizes = ix.bucket_sizes(dev(q)).cpu().numpy()
    assert sizes.shape == (q.shape[0], p.L)
    assert np.all(sizes.sum(axis=1) >= cnt)


# ---------------------------------------------------------------- neighbour probing

@pytest.mark.parametrize("w", [400.0, 900.0])
def test_neighbour_probing_cfg1(cfg1, w):
    """Probing the one-step neighbour buckets: candidate sets, counts, layer
    sums and the top K of both forms and every schedule match the oracle with
    probes=1; switching back restores the plain results.  L = 10, k = 8: 170
    lists per query."""
    p = cfg1.params
    ix = build(cfg1.data, p.a, p.b(w), w)
    q = cfg1.queries
    ix.set_probing(1)
    assert ix.info()["probing"] == 1
    got = ix.candidate_lists(dev(q))
    want = oracle.lsh_candidates(cfg1.data, q, p.a, p.b(w), w, probes=1)
    plain = oracle.lsh_candidates(cfg1.data, q, p.a, p.b(w), w)
    assert sum(len(o) for o in want) > sum(len(o) for o in plain)
    for g, o in zip(got, want):
        assert np.array_equal(g, o)
    cnt = ix.candidate_counts(dev(q)).cpu().numpy()
    assert cnt.tolist() == [len(o) for o in want]
    sizes = ix.bucket_sizes(dev(q)).cpu().numpy()
    assert sizes.shape == (q.shape[0], p.L) and np.all(sizes.sum(axis=1) >= cnt)
    ids_o, dist_o, cnt_o = oracle.lsh_query(cfg1.data, q, p.a, p.b(w), w, cfg1.K, probes=1)
    for form in FORMS:
        ids, dist, st = ix.query(dev(q), cfg1.K, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM),
                                 stats=True)
        check_topk(ids, dist, ids_o, dist_o, True)
        assert st["cand_unique"] == int(cnt_o.sum())
    for sched in SCHEDS:
        for group in (0, 1):
            ids, dist = ix.query(dev(q), cfg1.K, lib.make_opts(sched=sched, group=group))
            check_topk(ids, dist, ids_o, dist_o, True)
    ix.set_probing(0)
    ids_o, dist_o, _ = oracle.lsh_query(cfg1.data, q, p.a, p.b(w), w, cfg1.K)
    ids, dist = ix.query(dev(q), cfg1.K)
    check_topk(ids, dist, ids_o, dist_o, True)


def test_neighbour_probing_float_and_learned():
    """Float data with probing (L = 16, k = 12: 400 lists per query), both
    forms, and a count model trained under probing keeps the results."""
    wl = synth.make_config(3, n=6000, Q=60, ncomp=30, w=4.0)
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w)
    ix.set_probing(1)
    ids_o, dist_o, cnt = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(), p.w, wl.K, probes=1)
    assert cnt.mean() > 20
    for form in FORMS:
        ids, dist = ix.query(dev(wl.queries), wl.K, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
        check_topk(ids, dist, ids_o, dist_o, False)
    train = synth.training_queries(3, 2000, n=6000, ncomp=30)
    ix.train_count_model(dev(train), epochs=2, batch=256, lr=2e-3, seed=1)
    assert ix.info()["has_count_model"] == 1
    for group in (0, 1):
        ids, dist = ix.query(dev(wl.queries), wl.K, lib.make_opts(sched=lib.QW_SCHED_LEARNED,
                                                                   group=group))
        check_topk(ids, dist, ids_o, dist_o, False)
    ix.set_probing(0)
    assert ix.info()["has_count_model"] == 0


@pytest.mark.parametrize("T", [1, 4, 16])
def test_query_directed_probing_cfg1(cfg1, T):
    """Query-directed probing (the T best one-step moves by boundary-distance
    score, from FP64 projections on the GPU): candidate lists and the top K of
    both forms, every schedule and both groupings match the oracle."""
    p = cfg1.params
    w = 600.0
    ix = build(cfg1.data, p.a, p.b(w), w)
    q = cfg1.queries
    ix.set_probing(2, T)
    info = ix.info()
    assert info["probing"] == 2 and info["probes_per_layer"] == T
    want = oracle.lsh_candidates(cfg1.data, q, p.a, p.b(w), w, probes=2, probe_t=T)
    for g, o in zip(ix.candidate_lists(dev(q)), want):
        assert np.array_equal(g, o)
    ids_o, dist_o, _ = oracle.lsh_query(cfg1.data, q, p.a, p.b(w), w, cfg1.K, probes=2, probe_t=T)
    for form in FORMS:
        ids, dist = ix.query(dev(q), cfg1.K, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
        check_topk(ids, dist, ids_o, dist_o, True)
    for sched in SCHEDS:
        for group in (0, 1):
            ids, dist = ix.query(dev(q), cfg1.K, lib.make_opts(sched=sched, group=group))
            check_topk(ids, dist, ids_o, dist_o, True)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
@pytest.mark.parametrize("k", [3, 5, 8, 10, 12, 13, 16, 20, 32])
def test_query_directed_probing_every_k(dtype, k):
    """The move selection for every function count (the kernel is built for
    k = 8, 10, 12 and 16 exactly and for bounds of 8, 16 and 32 otherwise),
    ragged rows, and T up to 2k moves: candidate lists and top K match the
    oracle."""
    d = 37 if dtype == "u8" else 21
    # bucket widths giving about 100-800 candidates per query at T = 3
    mult = {"u8": {3: 0.25, 5: 0.5, 16: 2, 20: 2, 32: 4},
            "f32": {3: 0.5, 5: 1, 8: 2, 10: 2, 12: 4, 13: 4, 16: 4, 20: 4, 32: 8}}[dtype].get(k, 1)
    w = (1500.0 if dtype == "u8" else 1.5) * mult
    wl = synth.random_small(900 + k, 3000, d, 50, 3, k, w, dtype=dtype)
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w)
    for T in sorted({1, 3, 2 * k}):
        ix.set_probing(2, T)
        want = oracle.lsh_candidates(wl.data, wl.queries, p.a, p.b(), p.w, probes=2, probe_t=T)
        for g, o in zip(ix.candidate_lists(dev(wl.queries)), want):
            assert np.array_equal(g, o)
        ids_o, dist_o, _ = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(), p.w, wl.K, probes=2,
                                            probe_t=T)
        ids, dist = ix.query(dev(wl.queries), wl.K, lib.make_opts(sched=lib.QW_SCHED_SUM))
        check_topk(ids, dist, ids_o, dist_o, dtype == "u8")
    ix.close()


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_query_directed_probing_score_ties(dtype):
    """Small integer parameters put projections on quarter steps, so scores
    tie exactly (f = 1/2 scores both moves 1/4; equal fractions across
    functions): ties are broken by move index as the oracle breaks them."""
    L, k, d = 3, 5, 48
    a, b, w = synth.boundary_params(31, L, k, d, w=4.0)
    rng = np.random.default_rng(32)
    x = rng.integers(0, 8, size=(2000, d), dtype=np.uint8)
    qx = rng.integers(0, 8, size=(64, d), dtype=np.uint8)
    if dtype == "f32":
        x, qx = x.astype(np.float32), qx.astype(np.float32)
    ix = build(x, a, b, w)
    for T in (1, 2, 5, 2 * k):
        ix.set_probing(2, T)
        want = oracle.lsh_candidates(x, qx, a, b, w, probes=2, probe_t=T)
        for form in FORMS:
            ix_lists = ix.candidate_lists(dev(qx))
            for g, o in zip(ix_lists, want):
                assert np.array_equal(g, o)
            ids_o, dist_o, _ = oracle.lsh_query(x, qx, a, b, w, 10, probes=2, probe_t=T)
            ids, dist = ix.query(dev(qx), 10, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
            check_topk(ids, dist, ids_o, dist_o, dtype == "u8")
    ix.close()


def test_query_directed_probing_float():
    wl = synth.make_config(3, n=6000, Q=60, ncomp=30, w=4.0)
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w)
    ix.set_probing(2, 5)
    ids_o, dist_o, cnt = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(), p.w, wl.K, probes=2,
                                          probe_t=5)
    assert cnt.mean() > 10
    for form in FORMS:
        ids, dist = ix.query(dev(wl.queries), wl.K, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
        check_topk(ids, dist, ids_o, dist_o, False)
    with pytest.raises(lib.QwError):
        ix.set_probing(2, 2 * p.k + 1)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_neighbour_probing_960_lists(dtype):
    """L = 64, k = 7: 64 * 15 = 960 lists per query, near the 1024-list limit
    (the workgroup prefix uses all four entries per thread, the list search
    all ten steps); both forms and the candidate lists match the oracle."""
    rng = np.random.default_rng(21)
    n, d, Q, L, k = 2500, 16, 40, 64, 7
    if dtype == "u8":
        data = rng.integers(0, 256, size=(n, d), dtype=np.uint8)
        q = np.clip(data[:Q].astype(np.int32) + rng.integers(-3, 4, size=(Q, d)), 0, 255).astype(np.uint8)
        w = 250.0
    else:
        data = rng.random((n, d), dtype=np.float32)
        q = (data[:Q] + rng.normal(0, 0.01, size=(Q, d))).astype(np.float32)
        w = 1.2
    a = rng.standard_normal((L, k, d)).astype(np.float32)
    b = (rng.random((L, k)) * w).astype(np.float32)
    ix = build(data, a, b, w)
    ix.set_probing(1)
    want = oracle.lsh_candidates(data, q, a, b, w, probes=1)
    for g, o in zip(ix.candidate_lists(dev(q)), want):
        assert np.array_equal(g, o)
    ids_o, dist_o, cnt = oracle.lsh_query(data, q, a, b, w, 10, probes=1)
    assert cnt.mean() > 100  # 135 (uint8) and 436 (float) candidates per query
    for form in FORMS:
        ids, dist = ix.query(dev(q), 10, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
        check_topk(ids, dist, ids_o, dist_o, dtype == "u8")


def test_neighbour_probing_limits():
    rng = np.random.default_rng(9)
    data = rng.integers(0, 256, size=(500, 16), dtype=np.uint8)
    L, k, w = 64, 8, 600.0  # 64 * 17 = 1088 lists: beyond 1024
    a = rng.standard_normal((L, k, 16)).astype(np.float32)
    b = (rng.random((L, k)) * w).astype(np.float32)
    ix = build(data, a, b, w)
    with pytest.raises(lib.QwError):
        ix.set_probing(1)
    with pytest.raises(lib.QwError):
        ix.set_probing(2)
    assert ix.info()["probing"] == 0


# ---------------------------------------------------------------- top-K, uint8

@pytest.mark.parametrize("w", [400.0, 1200.0])
@pytest.mark.parametrize("form", FORMS)
def test_topk_cfg1(cfg1, w, form):
    p = cfg1.params
    ix = build(cfg1.data, p.a, p.b(w), w)
    ids_o, dist_o, cnt_o = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, p.b(w), w, cfg1.K)
    opts = lib.make_opts(form=form, sched=lib.QW_SCHED_SUM)
    ids, dist, st = ix.query(dev(cfg1.queries), cfg1.K, opts, stats=True)
    check_topk(ids, dist, ids_o, dist_o, True)
    assert st["cand_unique"] == int(cnt_o.sum())
    assert st["overflow"] == 0


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("group", [0, 1])
def test_fast_form_schedules_identical(cfg1, sched, group):
    p = cfg1.params
    w = 1200.0
    ix = build(cfg1.data, p.a, p.b(w), w)
    ids_o, dist_o, _ = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, p.b(w), w, cfg1.K)
    opts = lib.make_opts(form=lib.QW_FORM_FAST, sched=sched, group=group)
    for rep in range(3):  # graph replays, with eager work in between
        ids, dist = ix.query(dev(cfg1.queries), cfg1.K, opts)
        torch.cuda.synchronize()
        check_topk(ids, dist, ids_o, dist_o, True)
        _ = (torch.arange(1000, device="cuda") * 2).sum().item()


@pytest.mark.parametrize("keep", [-1, 1, 2, 3])
def test_fused_topk_keep_and_fallback(cfg1, keep):
    """In-kernel top K (uint8, K <= 16) and the separate select kernel (keep
    -1) give the oracle's answer; keeping fewer keys per lane sends queries
    to the second selection pass without changing the result.  w = 3000
    gives 1.2K-6.7K unique candidates per query, several per lane."""
    p = cfg1.params
    w = 3000.0
    ix = build(cfg1.data, p.a, p.b(w), w)
    for K in (1, 10, 16):
        ids_o, dist_o, _ = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, p.b(w), w, K)
        for sched in (lib.QW_SCHED_SUM, lib.QW_SCHED_NONE):
            opts = lib.make_opts(sched=sched, topk_keep=keep)
            ids, dist, st = ix.query(dev(cfg1.queries), K, opts, stats=True)
            check_topk(ids, dist, ids_o, dist_o, True)
            if keep == 1 and K == 16:
                assert st["topk_second_pass"] > 0
            if keep == -1:
                assert st["fallback"] == 0 and st["topk_second_pass"] == 0


def test_ragged_u8_and_topk_sizes():
    """d not a multiple of 16, n and Q not multiples of the tile sizes, several K."""
    wl = synth.random_small(31, n=2345, d=53, Q=77, L=4, k=3, w=700.0, dtype="u8")
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w)
    for K in (1, 7, 33, 300):
        ids_o, dist_o, _ = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(), p.w, K)
        for form in FORMS:
            ids, dist = ix.query(dev(wl.queries), K, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
            check_topk(ids, dist, ids_o, dist_o, True)


def test_padding_and_empty_workload():
    wl = synth.random_small(41, n=500, d=16, Q=20, L=2, k=6, w=50.0, dtype="u8")
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w)
    ids_o, dist_o, cnt = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(), p.w, 10)
    assert (cnt < 10).any()  # small w: most queries have few candidates
    ids, dist = ix.query(dev(wl.queries), 10)
    check_topk(ids, dist, ids_o, dist_o, True)
    e_ids, e_dist = ix.query(dev(wl.queries[:0]), 10)
    assert e_ids.shape == (0, 10)


def test_duplicates_tie_break():
    rng = np.random.default_rng(5)
    base = rng.integers(0, 256, size=(300, 24), dtype=np.uint8)
    data = np.concatenate([base, base[:100], base[:50]])  # ids 300.. duplicate 0..
    q = base[:40].copy()
    L, k, w = 3, 2, 2000.0
    a = rng.standard_normal((L, k, 24)).astype(np.float32)
    b = (rng.random((L, k)) * w).astype(np.float32)
    ix = build(data, a, b, w)
    ids_o, dist_o, _ = oracle.lsh_query(data, q, a, b, w, 5)
    for form in FORMS:
        ids, dist = ix.query(dev(q), 5, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
        check_topk(ids, dist, ids_o, dist_o, True)
    assert ids_o[0, :3].tolist() == [0, 300, 400]


# ---------------------------------------------------------------- float data

@pytest.fixture(scope="module")
def cfg3_small():
    return synth.make_config(3, n=6000, Q=60, ncomp=30, w=8.0)


@pytest.mark.parametrize("form", FORMS)
def test_topk_float_cfg3_small(cfg3_small, form):
    wl = cfg3_small
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w)
    ids_o, dist_o, cnt = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(), p.w, wl.K)
    assert cnt.mean() > 50
    ids, dist = ix.query(dev(wl.queries), wl.K, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
    check_topk(ids, dist, ids_o, dist_o, False)


def test_float_fp64_ties_follow_rounded_sequence():
    """Swapped pairs whose FP64 distances tie only without fused multiply-adds:
    both forms and the brute force must order every pair by id, as the oracle."""
    from fp64_ties import tie_workload
    data, queries = tie_workload()
    n = data.shape[0]
    L, k, w = 1, 1, 1.0e4
    rng = np.random.default_rng(3)
    a = rng.standard_normal((L, k, 2)).astype(np.float32)
    b = np.full((L, k), w / 2, np.float32)
    ix = build(data, a, b, w)
    ids_o, dist_o, cnt = oracle.lsh_query(data, queries, a, b, w, n)
    assert (cnt == n).all()
    for form in FORMS:
        ids, dist = ix.query(dev(queries), n, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
        check_topk(ids, dist, ids_o, dist_o, False)
    ids, dist = ix.bruteforce(dev(queries), n)
    check_topk(ids, dist, ids_o, dist_o, False)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_bruteforce_matches_oracle(dtype):
    wl = synth.random_small(51, n=3000, d=40, Q=30, L=1, k=1, w=10.0, dtype=dtype)
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w)
    ids_o, dist_o = oracle.bruteforce(wl.data, wl.queries, 12)
    ids, dist = ix.bruteforce(dev(wl.queries), 12)
    check_topk(ids, dist, ids_o, dist_o, dtype == "u8")


def test_huge_w_equals_bruteforce():
    """Every point in one bucket per layer: LSH top-K equals exact kNN."""
    rng = np.random.default_rng(61)
    data = rng.integers(0, 256, size=(4000, 32), dtype=np.uint8)
    q = rng.integers(0, 256, size=(25, 32), dtype=np.uint8)
    L, k, w = 2, 3, 1.0e7
    a = rng.standard_normal((L, k, 32)).astype(np.float32)
    b = np.full((L, k), w / 2, np.float32)
    ix = build(data, a, b, w)
    ids_o, dist_o = oracle.bruteforce(data, q, 10)
    for form in FORMS:
        ids, dist = ix.query(dev(q), 10, lib.make_opts(form=form, sched=lib.QW_SCHED_SUM))
        check_topk(ids, dist, ids_o, dist_o, True)


# ---------------------------------------------------------------- count model

def test_mlp_gradient_matches_oracle():
    from oracle import mlp
    rng = np.random.default_rng(71)
    L, H, B = 16, 64, 300
    P = lib.qw_mlp_param_count(L)
    params = (rng.standard_normal(P) * 0.2).astype(np.float32)
    feats = np.log1p(rng.integers(0, 800, size=(B, L))).astype(np.float32)
    targets = np.log1p(rng.integers(1, 4000, size=B)).astype(np.float32)
    grad, loss = lib.qw_mlp_loss_grad(dev(params), L, dev(feats), dev(targets))
    W1 = params[:H * L].reshape(H, L).astype(np.float64)
    b1 = params[H * L:H * L + H].astype(np.float64)
    W2 = params[H * L + H:H * L + 2 * H].astype(np.float64)
    b2 = float(params[-1])
    lo, (dW1, db1, dW2, db2) = mlp.loss_and_grad(W1, b1, W2, b2, feats.astype(np.float64), targets)
    want = np.concatenate([dW1.ravel(), db1, dW2, [db2]])
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - lo) <= 1e-4 * abs(lo)
    np.testing.assert_allclose(g, want, rtol=1e-4, atol=1e-4 * np.abs(want).max())


def test_adam_matches_oracle():
    from oracle import mlp
    rng = np.random.default_rng(72)
    P = 500
    p = rng.standard_normal(P).astype(np.float32)
    g = rng.standard_normal(P).astype(np.float32)
    pt, gt = dev(p), dev(g)
    m, v = torch.zeros_like(pt), torch.zeros_like(pt)
    pm, mm, vm = p.astype(np.float64), np.zeros(P), np.zeros(P)
    for step in (1, 2, 3):
        lib.qw_mlp_adam(pt, gt, m, v, step, 1e-2)
        pm, mm, vm = mlp.adam_step(pm, g.astype(np.float64), mm, vm, step, 1e-2)
    np.testing.assert_allclose(pt.cpu().numpy(), pm, rtol=1e-5, atol=1e-6)


def test_mlp_bf16_prediction_close_to_fp64():
    from oracle import mlp
    rng = np.random.default_rng(73)
    L, H, B = 12, 64, 200
    P = lib.qw_mlp_param_count(L)
    params = (rng.standard_normal(P) * 0.2).astype(np.float32)
    feats = np.log1p(rng.integers(0, 800, size=(B, L))).astype(np.float32)
    out = lib.qw_mlp_predict_bf16(dev(params), L, dev(feats)).cpu().numpy()
    W1 = params[:H * L].reshape(H, L)
    y, _ = mlp.forward(W1, params[H * L:H * L + H], params[H * L + H:H * L + 2 * H], params[-1], feats)
    # bf16 operands: 8-bit mantissa, relative error ~2^-8 per operand
    assert np.max(np.abs(out - y)) <= 0.05 * (np.max(np.abs(y)) + 1)


def test_learned_schedule_trains_and_keeps_results(cfg1):
    p = cfg1.params
    w = 1200.0
    ix = build(cfg1.data, p.a, p.b(w), w)
    train = synth.training_queries(1, 3000)
    loss = ix.train_count_model(dev(train), epochs=4, batch=256, lr=3e-3, seed=1)
    assert math.isfinite(loss)
    assert ix.info()["has_count_model"] == 1
    # the sizing margin is calibrated on the training queries: at least 0.05,
    # and about 1 training query in 200 exceeds its sized prediction
    margin = ix.info()["count_margin"]
    assert 0.05 <= margin <= 8.0
    with pytest.raises(lib.QwError):
        ix.set_count_margin(float("nan"))
    with pytest.raises(lib.QwError):
        ix.set_count_margin(9.0)
    ids_o, dist_o, _ = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, p.b(w), w, cfg1.K)
    ids, dist, st = ix.query(dev(cfg1.queries), cfg1.K,
                             lib.make_opts(sched=lib.QW_SCHED_LEARNED), stats=True)
    check_topk(ids, dist, ids_o, dist_o, True)
    # a sabotaged model (predicts 0 candidates) still gives the exact results
    P = lib.qw_mlp_param_count(p.L)
    bad = np.zeros(P, np.float32)
    bad[-1] = -5.0
    ix.set_count_model(bad)
    assert abs(ix.info()["count_margin"] - math.log(1.25)) < 1e-6
    ids, dist, st = ix.query(dev(cfg1.queries), cfg1.K,
                             lib.make_opts(sched=lib.QW_SCHED_LEARNED), stats=True)
    check_topk(ids, dist, ids_o, dist_o, True)
    ix.set_count_margin(-4.0)  # smallest margin: still exact results
    ids, dist, st = ix.query(dev(cfg1.queries), cfg1.K,
                             lib.make_opts(sched=lib.QW_SCHED_LEARNED), stats=True)
    check_topk(ids, dist, ids_o, dist_o, True)
    ix.close()
    # every point a candidate (|C(q)| = n = 10,000): sets chosen from the
    # sabotaged prediction overflow and the queries move up the size classes
    wh = 1e7
    bh = np.full_like(p.b(wh), wh / 2)
    ixh = build(cfg1.data, p.a, bh, wh)
    ixh.set_count_model(bad)
    ids_o, dist_o, cnt_o = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, bh, wh, cfg1.K)
    assert np.all(cnt_o == cfg1.data.shape[0])
    for group in (0, 1):
        ids, dist, st = ixh.query(dev(cfg1.queries), cfg1.K,
                                  lib.make_opts(sched=lib.QW_SCHED_LEARNED, group=group), stats=True)
        check_topk(ids, dist, ids_o, dist_o, True)
        assert st["overflow"] >= cfg1.queries.shape[0]
        assert st["cand_unique"] == int(cnt_o.sum())
    ixh.close()


def test_global_memory_sets():
    """Every one of 30,000 points a candidate of every query, more than the
    largest on-chip set holds (3/4 of 2^15 slots): the workgroup kernel's
    global-memory class answers them, both from its own segment (sizes from
    the bucket-size bound) and from the overflow of the merged on-chip launch
    (a count model that predicts no candidates); the wave kernel takes them in
    id-hash passes."""
    rng = np.random.default_rng(41)
    n, d, Q, L, k = 30_000, 16, 40, 2, 2
    data = rng.integers(0, 256, size=(n, d), dtype=np.uint8)
    queries = rng.integers(0, 256, size=(Q, d), dtype=np.uint8)
    a = synth.hash_params(42, L, k, d, 1e7).a
    wh = 1e7
    bh = np.full((L, k), wh / 2, dtype=np.float32)
    ix = build(data, a, bh, wh)
    ids_o, dist_o, cnt_o = oracle.lsh_query(data, queries, a, bh, wh, 10)
    assert np.all(cnt_o == n)
    q = dev(queries)
    for dedup in (1, 2):
        ids, dist, st = ix.query(q, 10, lib.make_opts(sched=lib.QW_SCHED_SUM, dedup=dedup),
                                 stats=True)
        check_topk(ids, dist, ids_o, dist_o, True)
        assert st["cand_unique"] == n * Q
    bad = np.zeros(lib.qw_mlp_param_count(L), np.float32)
    bad[-1] = -5.0
    ix.set_count_model(bad)
    ids, dist, st = ix.query(q, 10, lib.make_opts(sched=lib.QW_SCHED_LEARNED, dedup=1), stats=True)
    check_topk(ids, dist, ids_o, dist_o, True)
    assert st["overflow"] >= Q
    ix.close()


# ---------------------------------------------------------------- errors

def test_error_paths(cfg1):
    p = cfg1.params
    ix = build(cfg1.data[:1000], p.a, p.b(), p.w)
    q = dev(cfg1.queries)
    with pytest.raises(lib.QwError) as e:
        ix.query(q, 0)
    assert e.value.status == lib.QW_EINVAL
    with pytest.raises(lib.QwError):
        ix.query(q, 5000)
    for keep in (-2, 4):
        with pytest.raises(lib.QwError) as e:
            ix.query(q, 10, lib.make_opts(topk_keep=keep))
        assert e.value.status == lib.QW_EINVAL
    with pytest.raises(lib.QwError):  # w <= 0
        lib.Index(dev(cfg1.data[:100]), dev(p.a), dev(p.b()), 0.0)
    with pytest.raises(lib.QwError):  # keys wider than 128 bits: tiny w, k = 8, huge ranges
        lib.Index(dev(cfg1.data[:2000]), dev(p.a), dev(p.b(0.001)), 0.001)


# ---------------------------------------------------------------- the two dedup kernels

@pytest.mark.parametrize("dedup", [lib.QW_DEDUP_BLOCK, lib.QW_DEDUP_WAVE])
@pytest.mark.parametrize("w", [400.0, 1200.0, 3000.0])
def test_dedup_kernels_match_oracle(cfg1, dedup, w):
    """Both fast-form candidate kernels (one workgroup per query in size
    classes; one wave per query with id-hash passes) against the oracle, for
    every schedule and K of 1, 10 and 16.  At w = 3000 queries hold 1.2K-6.7K
    unique candidates: the wave kernel runs 1-8 passes and splits passes that
    overflow."""
    p = cfg1.params
    ix = build(cfg1.data, p.a, p.b(w), w)
    q = dev(cfg1.queries)
    for K in (1, 10, 16):
        ids_o, dist_o, _ = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, p.b(w), w, K)
        for sched in (lib.QW_SCHED_SUM, lib.QW_SCHED_NONE, lib.QW_SCHED_ACTUAL):
            for group in (0, 1):
                ids, dist, st = ix.query(q, K, lib.make_opts(sched=sched, group=group, dedup=dedup),
                                         stats=True)
                check_topk(ids, dist, ids_o, dist_o, True)
    ix.close()


def test_wave_kernel_splits_passes_of_a_sabotaged_count_model(cfg1):
    """A count model that predicts no candidates puts every query in the
    smallest class: the wave kernel starts with one pass and splits it until
    each pass fits its set (10,000 candidates per query at huge w), with exact
    results and every split counted as an overflow."""
    p = cfg1.params
    wh = 1e7
    bh = np.full_like(p.b(wh), wh / 2)
    ix = build(cfg1.data, p.a, bh, wh)
    P = lib.qw_mlp_param_count(p.L)
    bad = np.zeros(P, np.float32)
    bad[-1] = -5.0
    ix.set_count_model(bad)
    ids_o, dist_o, cnt_o = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, bh, wh, cfg1.K)
    for graph in (0, 1):
        ids, dist, st = ix.query(dev(cfg1.queries), cfg1.K,
                                 lib.make_opts(sched=lib.QW_SCHED_LEARNED, dedup=lib.QW_DEDUP_WAVE,
                                               graph=graph), stats=True)
        check_topk(ids, dist, ids_o, dist_o, True)
        assert st["overflow"] == cfg1.queries.shape[0]
        assert st["cand_unique"] == int(cnt_o.sum())
    ix.close()


@pytest.mark.parametrize("d", [8, 53, 128, 1024])
def test_wave_kernel_row_widths_and_probing(d):
    """The wave kernel for every lanes-per-row width (rows of 1, 4, 8 and 64
    16-byte parts: 1, 2, 4 and 32 lanes per row), ragged n and Q, with
    query-directed probing (L * 3 lists), against the oracle."""
    wl = synth.random_small(91 + d, n=2311, d=d, Q=57, L=6, k=3, w=float(60 * d ** 0.5), dtype="u8")
    p = wl.params
    ix = build(wl.data, p.a, p.b(), p.w)
    for probes in (0, 2):
        if probes:
            ix.set_probing(2, 2)
        ids_o, dist_o, _ = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(), p.w, 10, probes=probes,
                                            probe_t=2 if probes else 0)
        for dedup in (lib.QW_DEDUP_BLOCK, lib.QW_DEDUP_WAVE):
            ids, dist = ix.query(dev(wl.queries), 10, lib.make_opts(sched=lib.QW_SCHED_SUM, dedup=dedup))
            check_topk(ids, dist, ids_o, dist_o, True)
    ix.close()


def test_dedup_option_validation(cfg1):
    p = cfg1.params
    ix = build(cfg1.data[:1000], p.a, p.b(), p.w)
    q = dev(cfg1.queries)
    for kw in ({"dedup": 3}, {"dedup": -1}, {"xchunk": -1}, {"xchunk": 257}, {"stage_split": -2},
               {"stage_split": 100}):
        with pytest.raises(lib.QwError) as e:
            ix.query(q, 10, lib.make_opts(**kw))
        assert e.value.status == lib.QW_EINVAL
    with pytest.raises(lib.QwError) as e:  # the staged kernel takes the fast form only
        ix.query(q, 10, lib.make_opts(stage_split=50, form=lib.QW_FORM_PLAIN_FP32))
    assert e.value.status == lib.QW_EUNSUPPORTED
    ix.set_probing(1)  # 170 lists per query: beyond the staged kernel's 64
    with pytest.raises(lib.QwError) as e:
        ix.query(q, 10, lib.make_opts(stage_split=50))
    assert e.value.status == lib.QW_EUNSUPPORTED
    ix.close()


# ---------------------------------------------------------------- workload invariants and limits

def test_query_permutation_invariance():
    """Answers do not depend on where a query sits in the workload: a permuted
    workload returns the permuted answers, bit for bit, in both forms, both
    candidate kernels and both groupings (the schedule reorders queries by
    size class and candidate overlap)."""
    wl = synth.make_config(2, n=100_000, Q=3000, ncomp=100)
    p = wl.params
    w = 1000.0
    ix = build(wl.data, p.a, p.b(w), w)
    ix.train_count_model(dev(synth.training_queries(2, 5000, ncomp=100)), epochs=2, batch=1024,
                         lr=2e-3, seed=1)
    perm = np.random.default_rng(5).permutation(wl.Q)
    q, qp = dev(wl.queries), dev(wl.queries[perm])
    for probes in (0, 2):
        if probes:
            ix.set_probing(2, 2)
        for o in (lib.make_opts(form=lib.QW_FORM_PLAIN_FP32),
                  lib.make_opts(dedup=lib.QW_DEDUP_BLOCK, group=0),
                  lib.make_opts(dedup=lib.QW_DEDUP_BLOCK, group=1),
                  lib.make_opts(dedup=lib.QW_DEDUP_WAVE, group=0),
                  lib.make_opts(dedup=lib.QW_DEDUP_WAVE, group=1, xchunk=16)):
            ids, dist = ix.query(q, wl.K, o)
            ids_p, dist_p = ix.query(qp, wl.K, o)
            assert np.array_equal(ids.cpu().numpy()[perm], ids_p.cpu().numpy())
            assert np.array_equal(dist.cpu().numpy()[perm], dist_p.cpu().numpy())
    ix.close()


def test_oversized_requests_give_enomem(cfg1):
    """Requests beyond the device's memory are refused with QW_ENOMEM before
    anything is allocated or read (the library checks the device's free memory
    first), and the index keeps answering afterwards."""
    import ctypes
    so = lib.load()
    # an index over 2^31 - 1 rows of 8192 floats (70 TB): refused before the data copy
    a1 = torch.zeros((1, 1, 8192), dtype=torch.float32, device="cuda")
    b1 = torch.zeros((1, 1), dtype=torch.float32, device="cuda")
    small = torch.zeros((4, 8192), dtype=torch.float32, device="cuda")
    out = ctypes.c_void_p()
    rc = so.qw_build_index(small.data_ptr(), 2 ** 31 - 1, 8192, lib.QW_F32, a1.data_ptr(), b1.data_ptr(),
                           1.0, 1, 1, None, None, ctypes.byref(out))
    assert rc == lib.QW_ENOMEM and not out.value
    # a workload of 2^31 - 1 queries (over a TB of workspace) on a small index
    p = cfg1.params
    ix = build(cfg1.data, p.a, p.b(), p.w)
    q = dev(cfg1.queries)
    ids = torch.full((4, cfg1.K), -7, dtype=torch.int32, device="cuda")
    dist = torch.full_like(ids, -7)
    for o in (lib.make_opts(), lib.make_opts(form=lib.QW_FORM_PLAIN_FP32)):
        rc = so.qw_query_workload(ix.handle, q.data_ptr(), 2 ** 31 - 1, cfg1.K, ctypes.byref(o), None,
                                  ids.data_ptr(), dist.data_ptr(), None)
        assert rc == lib.QW_ENOMEM
    torch.cuda.synchronize()
    assert bool((ids == -7).all()) and bool((dist == -7).all())
    ids_o, dist_o, _ = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, p.b(), p.w, cfg1.K)
    ids, dist = ix.query(q, cfg1.K)
    check_topk(ids, dist, ids_o, dist_o, True)
    ix.close()


@pytest.mark.skip(reason="the first staging split (a share of the candidate kernels' list and row "
                         "loads made non-temporal) faulted the GPU on its first run (memory fault "
                         "during this test, cause not found by reading the code); that kernel path "
                         "was removed, and qw_opts.stage_split is now served by the staged LDS "
                         "kernel, tested by test_staged_kernel_keeps_results")
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_staging_split_keeps_results(dtype):
    """The staging split (a share of the bucket lists and of the candidate rows
    loaded non-temporally) changes only cache residency: every split, both
    candidate kernels, both groupings and neighbour probing (more than 64
    lists: the wide-list kernel) return the oracle's results."""
    if dtype == "u8":
        wl = synth.make_config(2, n=50_000, Q=500, ncomp=100)
        w = 1000.0
    else:
        wl = synth.make_config(3, n=8000, Q=80, ncomp=40)
        w = 4.0
    p = wl.params
    ix = build(wl.data, p.a, p.b(w), w)
    q = dev(wl.queries)
    for probes in (0, 1):
        if probes:
            ix.set_probing(1)
        ids_o, dist_o, _ = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(w), w, wl.K, probes=probes)
        for split in (-1, 1, 50, 99):
            for dedup in ((lib.QW_DEDUP_BLOCK, lib.QW_DEDUP_WAVE) if dtype == "u8" else (lib.QW_DEDUP_BLOCK,)):
                for group in (0, 1):
                    ids, dist, st = ix.query(q, wl.K, lib.make_opts(stage_split=split, dedup=dedup, group=group),
                                             stats=True)
                    assert st["split_used"] == split
                    check_topk(ids, dist, ids_o, dist_o, dtype == "u8")
    ix.close()


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_staged_kernel_keeps_results(dtype):
    """The staged candidate kernel (LDS caches of bucket lists and rows kept
    across runs of consecutive queries, split s % / 100 - s %) returns the
    oracle's results at every split, with and without bucket grouping, for
    every schedule, K of 1 and 10, and with query-directed probing (60 lists);
    queries beyond its set go to the fallback."""
    if dtype == "u8":
        wl = synth.make_config(2, n=50_000, Q=400, ncomp=100)
        w = 1000.0
    else:
        wl = synth.make_config(3, n=8000, Q=80, ncomp=40)
        w = 4.0
    p = wl.params
    ix = build(wl.data, p.a, p.b(w), w)
    q = dev(wl.queries)
    for probes in (0, 2):
        if probes:
            ix.set_probing(2, 2)
        for K in (1, wl.K):
            ids_o, dist_o, cnt = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(w), w, K, probes=probes,
                                                  probe_t=2)
            for split in (1, 50, 99):
                for group in (0, 1):
                    for sched in (lib.QW_SCHED_SUM, lib.QW_SCHED_NONE):
                        ids, dist, st = ix.query(q, K, lib.make_opts(stage_split=split, group=group,
                                                                     sched=sched), stats=True)
                        assert st["split_used"] == split
                        assert st["cand_unique"] == int(cnt.sum())
                        check_topk(ids, dist, ids_o, dist_o, dtype == "u8")
    ix.close()


def test_staged_kernel_large_candidate_sets(cfg1):
    """Queries with more bucket entries than the staged kernel's set holds
    (w = 3000 on the small workload: up to 6,700 unique candidates) go to the
    fallback and keep exact results; so do K beyond the fused limit."""
    p = cfg1.params
    w = 3000.0
    ix = build(cfg1.data, p.a, p.b(w), w)
    q = dev(cfg1.queries)
    for K in (10, 40):
        ids_o, dist_o, _ = oracle.lsh_query(cfg1.data, cfg1.queries, p.a, p.b(w), w, K)
        ids, dist = ix.query(q, K, lib.make_opts(stage_split=50))
        check_topk(ids, dist, ids_o, dist_o, True)
    ix.close()
