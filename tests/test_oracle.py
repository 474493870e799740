"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against an independent source: a hand-worked
example, exact rational arithmetic, brute force written separately in numpy, the
closed form and numerical quadrature of Eq. (1), Monte Carlo statistics, or
finite differences.  None of them re-types the oracle's own code path.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import collision, mlp
from paper_1907_11803_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
I64MAX = np.iinfo(np.int64).max


def _np_topk(dist, K):
    """(dist asc, id asc) selection written with numpy's lexsort."""
    order = np.lexsort((np.arange(dist.shape[0]), dist))
    return order[:K]


# ---------------------------------------------------------------- worked example

def test_worked_example_golden():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    a = np.array(g["a"], np.float32)
    b = np.array(g["b"], np.float32)
    data = np.array(g["data"], np.uint8)
    qs = np.array(g["queries"], np.uint8)
    w, K = g["w"], g["K"]
    hd = oracle.hash_points(data, a, b, w)
    hq = oracle.hash_points(qs, a, b, w)
    assert hd.tolist() == g["hashes_data"]
    assert hq.tolist() == g["hashes_queries"]
    cands = oracle.lsh_candidates(data, qs, a, b, w)
    assert [c.tolist() for c in cands] == g["candidates"]
    ids, dist, cnt = oracle.lsh_query(data, qs, a, b, w, K)
    assert ids.tolist() == g["topk_ids"]
    want = [[I64MAX if v == "INT64_MAX" else v for v in row] for row in g["topk_dist"]]
    assert dist.tolist() == want
    assert cnt.tolist() == [len(c) for c in g["candidates"]]


# ---------------------------------------------------------------- hash function

def test_hash_unit_vectors_are_coordinates():
    """a = e_j, b = 0, w = 1 gives h = v_j (the textbook 1-D grid)."""
    rng = np.random.default_rng(5)
    d = 37
    x = rng.integers(0, 256, size=(50, d), dtype=np.uint8)
    a = np.eye(d, dtype=np.float32)
    b = np.zeros(d, np.float32)
    h = oracle.hash_points(x, a, b, 1.0)
    assert np.array_equal(h, x.astype(np.int32))
    # w = 8, b = 0: integer division of the coordinate
    h8 = oracle.hash_points(x, a, b, 8.0)
    assert np.array_equal(h8, x.astype(np.int32) // 8)


def _exact_floor(a_row, v, bj, w):
    s = Fraction(0)
    for ai, vi in zip(a_row.tolist(), v.tolist()):
        s += Fraction(ai) * Fraction(vi)
    return math.floor((s + Fraction(float(bj))) / Fraction(float(w)))


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_hash_matches_exact_rational_floor(dtype):
    """Random inputs: the FP64 oracle equals floor of the exact rational value
    (no integer lies within the FP64 error of these values)."""
    rng = np.random.default_rng(11)
    d, m, nf, w = 24, 40, 12, 3.5
    if dtype == "u8":
        x = rng.integers(0, 256, size=(m, d), dtype=np.uint8)
    else:
        x = rng.random((m, d), dtype=np.float32)
        w = 0.25
    a = rng.standard_normal((nf, d)).astype(np.float32)
    b = (rng.random(nf) * w).astype(np.float32)
    h = oracle.hash_points(x, a, b, w)
    for r in range(m):
        for j in range(nf):
            assert h[r, j] == _exact_floor(a[j], x[r], b[j], np.float32(w)), (r, j)


def test_hash_boundary_cases_exact():
    """Projections exactly on a bucket boundary, or one float32 ulp of b beside it."""
    L, k, d = 3, 5, 16
    a, b, w = synth.boundary_params(7, L, k, d, w=4.0)
    rng = np.random.default_rng(8)
    x = rng.integers(0, 256, size=(64, d), dtype=np.uint8)
    h = oracle.hash_points(x, a, b, w)
    a2, b2 = a.reshape(-1, d), b.reshape(-1)
    on_boundary = 0
    for r in range(x.shape[0]):
        for j in range(a2.shape[0]):
            e = _exact_floor(a2[j], x[r], b2[j], w)
            assert h[r, j] == e
            s = int(np.dot(a2[j].astype(np.int64), x[r].astype(np.int64)))
            if float(b2[j]).is_integer() and (s + int(b2[j])) % 4 == 0:
                on_boundary += 1
    assert on_boundary > 50  # the construction does land on boundaries


def test_hash_rejects_bad_w():
    x = np.zeros((2, 3), np.uint8)
    with pytest.raises(ValueError):
        oracle.hash_points(x, np.ones((1, 3), np.float32), np.zeros(1, np.float32), 0.0)


# ---------------------------------------------------------------- candidates and top-K

def _naive_candidates(hd, hq, L, k):
    """C(q) = {p : exists l, all k hashes of layer l equal}, by broadcasting."""
    n = hd.shape[0]
    hd3 = hd.reshape(n, L, k)
    out = []
    for q in range(hq.shape[0]):
        eq = np.all(hd3 == hq[q].reshape(1, L, k), axis=2)  # [n, L]
        out.append(np.nonzero(eq.any(axis=1))[0].astype(np.int32))
    return out


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_candidates_equal_union_of_bucket_members(dtype):
    wl = synth.make_config(1, n=3000, Q=40, w=900.0) if dtype == "u8" else \
        synth.make_config(3, n=2000, Q=30, ncomp=20, w=8.0)
    a, b, w = wl.params.a, wl.params.b(), wl.params.w
    L, k = wl.params.L, wl.params.k
    cands = oracle.lsh_candidates(wl.data, wl.queries, a, b, w)
    hd = oracle.hash_points(wl.data, a, b, w)
    hq = oracle.hash_points(wl.queries, a, b, w)
    naive = _naive_candidates(hd, hq, L, k)
    assert sum(len(c) for c in cands) > 0
    for c, nv in zip(cands, naive):
        assert np.array_equal(c, nv)


def _naive_probe_candidates(hd, hq, L, k):
    """Neighbour probing written from its definition with numpy broadcasting: p
    is a candidate when, in some layer, its tuple minus the query's is zero or
    has a single non-zero coordinate equal to -1 or +1."""
    hd3 = hd.reshape(hd.shape[0], L, k).astype(np.int64)
    out = []
    for q in range(hq.shape[0]):
        diff = hd3 - hq[q].reshape(1, L, k).astype(np.int64)  # [n, L, k]
        nz = np.count_nonzero(diff, axis=2)
        l1 = np.abs(diff).sum(axis=2)
        ok = (nz == 0) | ((nz == 1) & (l1 == 1))
        out.append(np.nonzero(ok.any(axis=1))[0].astype(np.int32))
    return out


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_neighbour_probing_candidates_match_definition(dtype):
    """Candidates with neighbour probing equal the definition, contain the
    plain candidates, and add some (w chosen so buckets are small)."""
    wl = synth.make_config(1, n=3000, Q=40, w=500.0) if dtype == "u8" else \
        synth.make_config(3, n=2000, Q=30, ncomp=20, w=4.0)
    a, b, w = wl.params.a, wl.params.b(), wl.params.w
    L, k = wl.params.L, wl.params.k
    plain = oracle.lsh_candidates(wl.data, wl.queries, a, b, w)
    probed = oracle.lsh_candidates(wl.data, wl.queries, a, b, w, probes=1)
    hd = oracle.hash_points(wl.data, a, b, w)
    hq = oracle.hash_points(wl.queries, a, b, w)
    naive = _naive_probe_candidates(hd, hq, L, k)
    added = 0
    for c0, c1, nv in zip(plain, probed, naive):
        assert np.array_equal(c1, nv)
        assert np.isin(c0, c1).all()
        added += len(c1) - len(c0)
    assert added > 0


def test_project_floors_to_hash_and_is_close_to_exact():
    """y = (a.x + b) / w from the oracle floors to its hash values and lies within
    a few FP64 ulps of the exact rational value."""
    wl = synth.make_config(1, n=200, Q=5, w=500.0)
    a, b, w = wl.params.a, wl.params.b(), wl.params.w
    y = oracle.project(wl.queries, a, b, w)
    assert np.array_equal(np.floor(y).astype(np.int32), oracle.hash_points(wl.queries, a, b, w))
    af = a.reshape(-1, a.shape[-1])
    for r in range(wl.queries.shape[0]):
        for f in range(0, af.shape[0], 7):
            ex = (sum(Fraction(float(u)) * int(v) for u, v in zip(af[f], wl.queries[r])) +
                  Fraction(float(b.reshape(-1)[f]))) / Fraction(float(np.float32(w)))
            assert abs(y[r, f] - float(ex)) <= 1e-12 * max(1.0, abs(float(ex)))


@pytest.mark.parametrize("T", [1, 3, 6])
def test_query_directed_probing_matches_definition(T):
    """The T best moves by (score, index) with score f^2 for -1 and (1 - f)^2 for
    +1 (f the fractional part of y), selected here with numpy's lexsort from the
    oracle's y, then the candidate set by broadcasting; T = 2k equals probing
    every neighbour."""
    wl = synth.make_config(1, n=3000, Q=25, w=500.0)
    a, b, w = wl.params.a, wl.params.b(), wl.params.w
    L, k = wl.params.L, wl.params.k
    got = oracle.lsh_candidates(wl.data, wl.queries, a, b, w, probes=2, probe_t=T)
    hd = oracle.hash_points(wl.data, a, b, w).reshape(-1, L, k).astype(np.int64)
    hq = oracle.hash_points(wl.queries, a, b, w).reshape(-1, L, k).astype(np.int64)
    y = oracle.project(wl.queries, a, b, w).reshape(-1, L, k)
    for q in range(wl.queries.shape[0]):
        ok = np.zeros(hd.shape[0], dtype=bool)
        for l in range(L):
            fr = y[q, l] - np.floor(y[q, l])
            score = np.empty(2 * k)
            score[0::2] = fr * fr
            score[1::2] = (1.0 - fr) * (1.0 - fr)
            moves = np.lexsort((np.arange(2 * k), score))[:T]
            targets = [hq[q, l].copy()]
            for mv in moves:
                t = hq[q, l].copy()
                t[mv // 2] += 1 if mv % 2 else -1
                targets.append(t)
            for t in targets:
                ok |= np.all(hd[:, l, :] == t, axis=1)
        assert np.array_equal(got[q], np.nonzero(ok)[0].astype(np.int32))
    full = oracle.lsh_candidates(wl.data, wl.queries, a, b, w, probes=2, probe_t=2 * k)
    every = oracle.lsh_candidates(wl.data, wl.queries, a, b, w, probes=1)
    assert all(np.array_equal(x, z) for x, z in zip(full, every))


def test_query_directed_probing_picks_nearest_neighbour_cells():
    """Geometric statement of the query-directed order (Lv et al.): in the
    projected space of a layer (coordinates y_j = (a_j.q + b_j) / w) the query
    lies in the cell prod_j [h_j, h_j + 1); the neighbour bucket that moves
    coordinate j by -1 is the adjacent cell whose nearest point lies y_j - h_j
    away, by +1 the one lying h_j + 1 - y_j away.  The T chosen moves are the T
    adjacent cells nearest to the query's point, computed here in exact rational
    arithmetic from the float32 parameters (no FP64 rounding, no squares).  The
    paper fixes no probe order; this pins the reading, not a printed value."""
    wl = synth.make_config(1, n=1500, Q=8, w=500.0)
    a, b, w = wl.params.a, wl.params.b(), wl.params.w
    L, k, d = a.shape
    hd = oracle.hash_points(wl.data, a, b, w).reshape(-1, L, k).astype(np.int64)
    wf = Fraction(float(np.float32(w)))
    af = [[[Fraction(float(v)) for v in a[l, j]] for j in range(k)] for l in range(L)]
    for T in (1, 4):
        got = oracle.lsh_candidates(wl.data, wl.queries, a, b, w, probes=2, probe_t=T)
        for q in range(wl.queries.shape[0]):
            x = [int(v) for v in wl.queries[q]]
            ok = np.zeros(hd.shape[0], dtype=bool)
            for l in range(L):
                y = [(sum(u * v for u, v in zip(af[l][j], x)) + Fraction(float(b[l, j]))) / wf
                     for j in range(k)]
                h = [math.floor(v) for v in y]
                cells = []
                for j in range(k):
                    cells.append((y[j] - h[j], j, -1))
                    cells.append((h[j] + 1 - y[j], j, +1))
                cells.sort()
                assert all(c0[0] != c1[0] for c0, c1 in zip(cells, cells[1:]))  # no exact ties
                targets = [np.array(h)]
                for _, j, s in cells[:T]:
                    t = np.array(h)
                    t[j] += s
                    targets.append(t)
                for t in targets:
                    ok |= np.all(hd[:, l, :] == t, axis=1)
            assert np.array_equal(got[q], np.nonzero(ok)[0].astype(np.int32))


def test_neighbour_probing_topk_is_topk_of_candidates():
    """The probed top K is the (distance, id) top K of the probed candidate set,
    selected here with numpy's lexsort over int64 distances."""
    wl = synth.make_config(1, n=3000, Q=25, w=500.0)
    a, b, w, K = wl.params.a, wl.params.b(), wl.params.w, 10
    ids, dist, cnt = oracle.lsh_query(wl.data, wl.queries, a, b, w, K, probes=1)
    cands = oracle.lsh_candidates(wl.data, wl.queries, a, b, w, probes=1)
    for q in range(wl.queries.shape[0]):
        c = cands[q]
        assert cnt[q] == len(c)
        dq = ((wl.data[c].astype(np.int64) - wl.queries[q].astype(np.int64)) ** 2).sum(axis=1)
        order = np.lexsort((c, dq))[:K]
        want = np.full(K, -1, np.int32)
        want[:len(order)] = c[order]
        assert np.array_equal(ids[q], want)
        assert np.array_equal(dist[q, :len(order)], dq[order])


def test_huge_w_equals_exact_knn_u8():
    """w huge and b = w/2: every projection lands in bucket 0, so every point is a
    candidate and the result is exact kNN (checked against numpy brute force)."""
    rng = np.random.default_rng(3)
    n, d, Q, L, k, K = 700, 20, 25, 3, 4, 12
    data = rng.integers(0, 256, size=(n, d), dtype=np.uint8)
    data[100] = data[5]   # duplicates exercise the id tie-break
    data[400] = data[5]
    qs = rng.integers(0, 256, size=(Q, d), dtype=np.uint8)
    qs[0] = data[5]
    a = rng.standard_normal((L, k, d)).astype(np.float32)
    w = 1.0e9
    b = np.full((L, k), w / 2, np.float32)
    ids, dist, cnt = oracle.lsh_query(data, qs, a, b, w, K)
    assert np.all(cnt == n)
    for q in range(Q):
        dd = ((data.astype(np.int64) - qs[q].astype(np.int64)) ** 2).sum(axis=1)
        sel = _np_topk(dd, K)
        assert ids[q].tolist() == sel.tolist()
        assert dist[q].tolist() == dd[sel].tolist()
    assert ids[0, :3].tolist() == [5, 100, 400]  # distance 0, ascending ids


def test_huge_w_equals_exact_knn_f32():
    rng = np.random.default_rng(4)
    n, d, Q, L, k, K = 500, 33, 15, 2, 3, 10
    data = rng.random((n, d), dtype=np.float32)
    qs = rng.random((Q, d), dtype=np.float32)
    a = rng.standard_normal((L, k, d)).astype(np.float32)
    w = 1.0e6
    b = np.full((L, k), w / 2, np.float32)
    ids, dist, cnt = oracle.lsh_query(data, qs, a, b, w, K)
    assert np.all(cnt == n)
    for q in range(Q):
        dd = ((data.astype(np.float64) - qs[q].astype(np.float64)) ** 2).sum(axis=1)
        sel = _np_topk(dd, K)
        assert ids[q].tolist() == sel.tolist()
        np.testing.assert_allclose(dist[q], dd[sel], rtol=1e-13)


def test_bruteforce_matches_numpy():
    rng = np.random.default_rng(9)
    data = rng.integers(0, 256, size=(999, 17), dtype=np.uint8)
    qs = rng.integers(0, 256, size=(20, 17), dtype=np.uint8)
    ids, dist = oracle.bruteforce(data, qs, 7)
    for q in range(20):
        dd = ((data.astype(np.int64) - qs[q].astype(np.int64)) ** 2).sum(axis=1)
        sel = _np_topk(dd, 7)
        assert ids[q].tolist() == sel.tolist()
        assert dist[q].tolist() == dd[sel].tolist()


def test_tiny_exhaustive_lsh_topk():
    """n <= 64, d <= 8: top-K of the oracle equals selection over its own naive
    candidate set, computed with numpy."""
    rng = np.random.default_rng(12)
    for trial in range(20):
        n, d = int(rng.integers(1, 65)), int(rng.integers(1, 9))
        Q, L, k, K = 6, int(rng.integers(1, 4)), int(rng.integers(1, 4)), int(rng.integers(1, 9))
        data = rng.integers(0, 8, size=(n, d), dtype=np.uint8)
        qs = rng.integers(0, 8, size=(Q, d), dtype=np.uint8)
        a = rng.standard_normal((L, k, d)).astype(np.float32)
        w = 6.0
        b = (rng.random((L, k)) * w).astype(np.float32)
        ids, dist, cnt = oracle.lsh_query(data, qs, a, b, w, K)
        hd = oracle.hash_points(data, a, b, w)
        hq = oracle.hash_points(qs, a, b, w)
        naive = _naive_candidates(hd, hq, L, k)
        for q in range(Q):
            c = naive[q]
            assert cnt[q] == len(c)
            dd = ((data[c].astype(np.int64) - qs[q].astype(np.int64)) ** 2).sum(axis=1)
            order = np.lexsort((c, dd))[:K]
            want_ids = c[order].tolist() + [-1] * (K - len(order))
            want_d = dd[order].tolist() + [I64MAX] * (K - len(order))
            assert ids[q].tolist() == want_ids
            assert dist[q].tolist() == want_d


def test_padding_when_few_candidates():
    data = np.array([[0, 0], [10, 10]], np.uint8)
    qs = np.array([[0, 1]], np.uint8)
    a = np.array([[[1, 0], [0, 1]]], np.float32)
    b = np.zeros((1, 2), np.float32)
    ids, dist, cnt = oracle.lsh_query(data, qs, a, b, 4.0, 4)
    assert cnt.tolist() == [1]
    assert ids.tolist() == [[0, -1, -1, -1]]
    assert dist.tolist() == [[1, I64MAX, I64MAX, I64MAX]]
    # float data pads with +inf
    ids, distf, _ = oracle.lsh_query(data.astype(np.float32), qs.astype(np.float32), a, b, 4.0, 2)
    assert ids.tolist() == [[0, -1]]
    assert distf[0, 0] == 1.0 and math.isinf(distf[0, 1])


def test_float_distance_close_to_exact_rational():
    rng = np.random.default_rng(21)
    data = rng.random((30, 64), dtype=np.float32)
    q = rng.random((1, 64), dtype=np.float32)
    ids, dist = oracle.bruteforce(data, q, 30)
    for r in range(30):
        p = int(ids[0, r])
        ex = sum((Fraction(float(x)) - Fraction(float(y))) ** 2 for x, y in zip(data[p], q[0]))
        assert abs(dist[0, r] - float(ex)) <= 1e-14 * float(ex)


def test_float_distance_rounds_each_product_and_sum():
    """Pairs whose distances tie with separately rounded products and sums but
    not with a fused multiply-add: the oracle's distances equal the rounded
    sequence written out in Python floats, each pair ties, and the tie goes to
    the smaller id."""
    from fp64_ties import tie_workload
    data, queries = tie_workload()
    n = data.shape[0]
    ids, dist = oracle.bruteforce(data, queries, n)
    for j in range(queries.shape[0]):
        c = float(queries[j, 0])
        want = {}
        for p in range(n):
            tx, ty = float(data[p, 0]) - c, float(data[p, 1]) - c
            want[p] = tx * tx + ty * ty  # each product and the sum rounded once
        for r in range(n):
            assert dist[j, r] == want[int(ids[j, r])]
        pos = {int(p): r for r, p in enumerate(ids[j])}
        for p in range(0, n, 2):  # rows p and p + 1 are a swapped pair
            assert want[p] == want[p + 1]
            assert pos[p] < pos[p + 1]


# ---------------------------------------------------------------- Eq. (1)

def test_eq1_closed_form_matches_quadrature():
    from scipy.integrate import quad

    def integrand(t, r, w):  # Eq. (1) as printed
        return (1.0 / r) * (2.0 / math.sqrt(2.0 * math.pi)) * math.exp(-t * t / (2 * r * r)) * (1 - t / w)

    for r, w in [(1, 1), (1, 4), (250, 400), (300, 400), (2, 1.5), (1, 2.719), (270, 1200), (0.3, 12)]:
        val, err = quad(integrand, 0.0, w, args=(r, w), epsabs=1e-14, epsrel=1e-13, limit=200)
        assert abs(collision.p_collide(r, w) - val) < 1e-12, (r, w)


def test_eq1_family_is_locality_sensitive():
    """P(r) strictly decreasing in r, so P1 = P(r) > P2 = P(cr) for c > 1."""
    rs = np.linspace(0.05, 50, 400)
    ps = [collision.p_collide(r, 4.0) for r in rs]
    assert all(p1 > p2 for p1, p2 in zip(ps, ps[1:]))
    assert abs(collision.p_collide(1e-9, 4.0) - 1.0) < 1e-6
    for c in (1.5, 2.0, 3.0):
        assert collision.p_collide(10.0, 4.0) > collision.p_collide(10.0 * c, 4.0)


def _pair_at_distance(rng, d, r):
    x = rng.random(d) * 4.0
    u = rng.standard_normal(d)
    u /= np.linalg.norm(u)
    y = x + r * u
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    return x32, y32, float(np.linalg.norm(x32.astype(np.float64) - y32.astype(np.float64)))


@pytest.mark.parametrize("r,w", [(1.0, 4.0), (3.0, 4.0), (2.0, 1.5)])
def test_empirical_collision_rate_matches_eq1(r, w):
    """Single functions: over many independent (a, b) draws the oracle's hashes
    of two points at distance r agree with probability P(r), within 5 sigma."""
    rng = np.random.default_rng(31)
    d, nf = 16, 200_000
    x, y, rr = _pair_at_distance(rng, d, r)
    a = rng.standard_normal((nf, d)).astype(np.float32)
    b = (rng.random(nf) * w).astype(np.float32)
    h = oracle.hash_points(np.stack([x, y]), a, b, w)
    rate = float(np.mean(h[0] == h[1]))
    p = collision.p_collide(rr, w)
    sigma = math.sqrt(p * (1 - p) / nf)
    assert abs(rate - p) < 5 * sigma, (rate, p)


def test_empirical_candidate_rate_matches_layers():
    """Layers: a point at distance r is a candidate with probability
    1 - (1 - P(r)^k)^L (conjunction inside a layer, disjunction across layers)."""
    rng = np.random.default_rng(41)
    d, L, k, w, r, trials = 8, 3, 2, 4.0, 2.5, 4000
    x, y, rr = _pair_at_distance(rng, d, r)
    hits = 0
    a_all = rng.standard_normal((trials, L, k, d)).astype(np.float32)
    b_all = (rng.random((trials, L, k)) * w).astype(np.float32)
    for t in range(trials):
        c = oracle.lsh_candidates(y[None, :], x[None, :], a_all[t], b_all[t], w, nthreads=1)
        hits += len(c[0])
    p = collision.p_candidate(rr, w, k, L)
    sigma = math.sqrt(p * (1 - p) / trials)
    assert abs(hits / trials - p) < 5 * sigma, (hits / trials, p)


# ---------------------------------------------------------------- count model

def _rand_mlp(rng, L=6, H=5, B=9):
    W1 = rng.standard_normal((H, L)) * 0.5
    b1 = rng.standard_normal(H) * 0.1
    W2 = rng.standard_normal(H) * 0.5
    b2 = 0.3
    f = mlp.features(rng.integers(0, 500, size=(B, L)))
    t = np.log1p(rng.integers(1, 3000, size=B).astype(np.float64))
    return W1, b1, W2, b2, f, t


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    W1, b1, W2, b2, f, t = _rand_mlp(rng)
    loss, (dW1, db1, dW2, db2) = mlp.loss_and_grad(W1, b1, W2, b2, f, t)
    h = 1e-6

    def L_(W1_, b1_, W2_, b2_):
        return mlp.loss_and_grad(W1_, b1_, W2_, b2_, f, t)[0]

    for idx in np.ndindex(W1.shape):
        P, M = W1.copy(), W1.copy()
        P[idx] += h; M[idx] -= h
        fd = (L_(P, b1, W2, b2) - L_(M, b1, W2, b2)) / (2 * h)
        assert abs(fd - dW1[idx]) <= 1e-6 * max(1.0, abs(fd))
    for i in range(b1.size):
        P, M = b1.copy(), b1.copy()
        P[i] += h; M[i] -= h
        fd = (L_(W1, P, W2, b2) - L_(W1, M, W2, b2)) / (2 * h)
        assert abs(fd - db1[i]) <= 1e-6 * max(1.0, abs(fd))
    for i in range(W2.size):
        P, M = W2.copy(), W2.copy()
        P[i] += h; M[i] -= h
        fd = (L_(W1, b1, P, b2) - L_(W1, b1, M, b2)) / (2 * h)
        assert abs(fd - dW2[i]) <= 1e-6 * max(1.0, abs(fd))
    fd = (L_(W1, b1, W2, b2 + h) - L_(W1, b1, W2, b2 - h)) / (2 * h)
    assert abs(fd - db2) <= 1e-6 * max(1.0, abs(fd))


def test_mlp_forward_hand_example():
    """One hidden unit active, one clipped by the relu; values worked by hand."""
    W1 = np.array([[1.0, 2.0], [-1.0, -1.0]])
    b1 = np.array([0.5, 0.0])
    W2 = np.array([2.0, 3.0])
    b2 = -1.0
    f = np.array([[1.0, 1.0]])
    y, _ = mlp.forward(W1, b1, W2, b2, f)
    # z = [3.5, -2], relu -> [3.5, 0], y = 2*3.5 - 1 = 6
    assert y.tolist() == [6.0]
    loss, (dW1, db1, dW2, db2) = mlp.loss_and_grad(W1, b1, W2, b2, f, np.array([4.0]))
    # r = 2, loss = 4, dy = 4; dW2 = 4*a = [14, 0]; db2 = 4; dz = [8, 0]; dW1 = [[8,8],[0,0]]
    assert loss == 4.0
    assert dW2.tolist() == [14.0, 0.0] and db2 == 4.0
    assert dW1.tolist() == [[8.0, 8.0], [0.0, 0.0]] and db1.tolist() == [8.0, 0.0]


def test_adam_first_step_is_lr_times_sign():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-4)


def test_adam_second_step_hand_worked():
    """Two Adam steps from zero moments, worked by hand with exact fractions.
    beta1 = 9/10, beta2 = 999/1000; gradients g1 = 1 then g2 in {1, -1, 3}:
      m2 = (9/100) g1 + (1/10) g2,   mhat2 = m2 / (1 - 81/100)
      v2 = (999/10^6) g1^2 + (1/1000) g2^2,   vhat2 = v2 / (1 - 998001/10^6)
    g2 = 1: mhat2 = 1, vhat2 = 1; g2 = -1: mhat2 = -1/19, vhat2 = 1;
    g2 = 3: mhat2 = 39/19, vhat2 = 9999/1999.  A dropped bias correction,
    beta1 and beta2 swapped, or the corrections taken at step - 1 fail here."""
    lr, eps = 0.01, 1e-8
    cases = {1.0: (Fraction(1), Fraction(1)), -1.0: (Fraction(-1, 19), Fraction(1)),
             3.0: (Fraction(39, 19), Fraction(9999, 1999))}
    for g2, (mhat, vhat) in cases.items():
        p, m, v = mlp.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, lr)
        p1 = -lr * 1.0 / (1.0 + eps)
        np.testing.assert_allclose(p, [p1], rtol=1e-15)
        np.testing.assert_allclose(m, [0.1], rtol=1e-15)
        np.testing.assert_allclose(v, [0.001], rtol=1e-15)
        p, m, v = mlp.adam_step(p, np.array([g2]), m, v, 2, lr)
        np.testing.assert_allclose(m, [float(Fraction(9, 100) + Fraction(1, 10) * Fraction(g2))],
                                   rtol=1e-14)
        np.testing.assert_allclose(v, [float(Fraction(999, 10**6) + Fraction(1, 1000) * Fraction(g2) ** 2)],
                                   rtol=1e-14)
        want = p1 - lr * float(mhat) / (math.sqrt(float(vhat)) + eps)
        np.testing.assert_allclose(p, [want], rtol=1e-13)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient g the bias-corrected moments equal g and g^2 at
    every step, so each of the first steps moves the parameter by
    lr * g / (|g| + eps)."""
    lr, eps = 0.003, 1e-8
    g = np.array([0.25, -4.0, 2.0e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 7):
        p, m, v = mlp.adam_step(p, g, m, v, step, lr, eps=eps)
        np.testing.assert_allclose(p, -step * lr * g / (np.abs(g) + eps), rtol=1e-9)


def test_built_index_matches_one_shot_query():
    wl = synth.make_config(1, n=2000, Q=30, w=1000.0)
    a, b, w = wl.params.a, wl.params.b(), wl.params.w
    bi = oracle.BuiltIndex(wl.data, a, b, w)
    for probes in (0, 1):
        ids1, d1, c1 = oracle.lsh_query(wl.data, wl.queries, a, b, w, 10, probes=probes)
        ids2, d2, c2 = bi.query(wl.queries, 10, probes=probes)
        assert np.array_equal(ids1, ids2) and np.array_equal(d1, d2) and np.array_equal(c1, c2)
    bi.close()


# ---------------------------------------------------------------- collision counting

def test_counting_hand_example():
    """Three single-function layers reading one coordinate each (a = e_j, b = 0,
    w = 1, so h_j(v) = v_j): the layer counts of the query (0, 0, 0) are 3, 2,
    1, 2, 0 for the five points; the cap keeps the best-counted points and
    breaks equal counts by id, whatever their distances."""
    data = np.array([[0, 0, 0], [0, 0, 5], [0, 5, 5], [5, 0, 0], [5, 5, 5]], np.uint8)
    qs = np.zeros((1, 3), np.uint8)
    a = np.eye(3, dtype=np.float32).reshape(3, 1, 3)
    b = np.zeros((3, 1), np.float32)
    run = lambda K, theta, v: oracle.lsh_query_counting(data, qs, a, b, 1.0, K, theta, v)
    ids, dist, cnt = run(1, 2, 1)
    assert ids.tolist() == [[0]] and dist.tolist() == [[0]] and cnt.tolist() == [2]
    ids, dist, cnt = run(2, 2, 0)  # points 1 and 3 tie on count 2: id 1 is kept
    assert ids.tolist() == [[0, 1]] and dist.tolist() == [[0, 25]] and cnt.tolist() == [2]
    ids, dist, cnt = run(3, 2, 0)
    assert ids.tolist() == [[0, 1, 3]] and dist.tolist() == [[0, 25, 25]]
    ids, dist, cnt = run(3, 1, 10)  # point 2 (count 1) joins; point 4 never does
    assert ids.tolist() == [[0, 1, 3]] and cnt.tolist() == [4]
    ids, dist, cnt = run(2, 3, 5)
    assert ids.tolist() == [[0, -1]] and dist.tolist() == [[0, I64MAX]] and cnt.tolist() == [1]
    ids, dist, cnt = run(2, 4, 5)  # a threshold above L: nothing qualifies
    assert ids.tolist() == [[-1, -1]] and cnt.tolist() == [0]


def _naive_counting(data, qs, hd, hq, L, k, K, theta, v):
    """Collision counting from its definition with numpy: the number of layers
    whose whole k-tuple matches, by broadcasting over all points; a lexsort by
    (count descending, id ascending) for the cap; then (distance, id)."""
    n = hd.shape[0]
    hd3 = hd.reshape(n, L, k)
    out = []
    for q in range(qs.shape[0]):
        col = np.all(hd3 == hq[q].reshape(1, L, k), axis=2).sum(axis=1)
        c = np.nonzero(col >= theta)[0]
        c = c[np.lexsort((c, -col[c]))][:K + v]
        dd = ((data[c].astype(np.int64) - qs[q].astype(np.int64)) ** 2).sum(axis=1)
        order = np.lexsort((c, dd))[:K]
        out.append((c[order].tolist() + [-1] * (K - len(order)), len(c), dd[order].tolist()))
    return out


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_counting_matches_dense_definition(dtype):
    """Small random cases, several thresholds and caps, against the dense count
    over all points (float rows hold small integers, so every distance is exact
    and the float and integer orders agree)."""
    rng = np.random.default_rng(31)
    for trial in range(25):
        n, d = int(rng.integers(1, 200)), int(rng.integers(1, 9))
        Q, L, k = 5, int(rng.integers(1, 7)), int(rng.integers(1, 3))
        K, theta, v = int(rng.integers(1, 9)), int(rng.integers(1, L + 2)), int(rng.integers(0, 12))
        data = rng.integers(0, 8, size=(n, d)).astype(np.uint8)
        qs = rng.integers(0, 8, size=(Q, d)).astype(np.uint8)
        if dtype == "f32":
            data, qs = data.astype(np.float32), qs.astype(np.float32)
        a = rng.standard_normal((L, k, d)).astype(np.float32)
        w = 4.0
        b = (rng.random((L, k)) * w).astype(np.float32)
        ids, dist, cnt = oracle.lsh_query_counting(data, qs, a, b, w, K, theta, v)
        hd = oracle.hash_points(data, a, b, w)
        hq = oracle.hash_points(qs, a, b, w)
        for q, (want_ids, nver, want_d) in enumerate(_naive_counting(data, qs, hd, hq, L, k, K,
                                                                     theta, v)):
            assert ids[q].tolist() == want_ids
            assert cnt[q] == nver
            assert dist[q][:len(want_d)].tolist() == want_d


def test_counting_threshold_one_without_cap_is_the_union():
    wl = synth.make_config(1, n=3000, Q=40, w=900.0)
    a, b, w = wl.params.a, wl.params.b(), wl.params.w
    ids0, dist0, cnt0 = oracle.lsh_query(wl.data, wl.queries, a, b, w, 10)
    ids1, dist1, cnt1 = oracle.lsh_query_counting(wl.data, wl.queries, a, b, w, 10, 1, 3000)
    assert np.array_equal(ids0, ids1) and np.array_equal(dist0, dist1)
    assert np.array_equal(cnt0, cnt1)
    # a tighter threshold or cap verifies fewer points and never a better answer
    ids2, dist2, cnt2 = oracle.lsh_query_counting(wl.data, wl.queries, a, b, w, 10, 2, 100)
    assert np.all(cnt2 <= np.minimum(cnt0, 110))
    assert np.all(dist2 >= dist0)
