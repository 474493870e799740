"""The allocation-free query entry point (qw_query_workload_noalloc), called
through the C ABI: its results equal qw_query_workload's plain form (and the
oracle's) on two calls in a row, the second with a smaller input, for uint8
rows used in place, float rows that need a padded copy, query-directed
probing and collision counting; sizes beyond its scratch are refused with the
outputs untouched.  Collected last: a failure here hides no other test."""
import numpy as np
import pytest
import torch

import oracle
from paper_1907_11803_amd import lib, synth

pytestmark = pytest.mark.gpu

I32MAX = np.iinfo(np.int32).max


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def noalloc(ix, q, K, is_u8):
    ids = torch.full((q.shape[0], K), -7, dtype=torch.int32, device="cuda")
    dist = torch.full((q.shape[0], K), -7, dtype=torch.int32 if is_u8 else torch.float32,
                      device="cuda")
    lib.qw_query_workload_noalloc(ix.handle, q, K, ids, dist)
    torch.cuda.synchronize()
    return ids, dist


def plain(ix, q, K):
    ids, dist = ix.query(q, K, lib.make_opts(form=lib.QW_FORM_PLAIN_FP32))
    torch.cuda.synchronize()
    return ids, dist


def check_oracle(ids, dist, ids_o, dist_o, is_u8):
    assert np.array_equal(ids.cpu().numpy(), ids_o)
    if is_u8:
        want = np.where(dist_o == np.iinfo(np.int64).max, I32MAX, dist_o)
        assert np.array_equal(dist.cpu().numpy().astype(np.int64), want)
    else:
        d = dist.cpu().numpy()
        fin = np.isfinite(dist_o)
        assert np.array_equal(np.isfinite(d), fin)
        assert np.array_equal(d[fin], dist_o[fin].astype(np.float32))


@pytest.mark.parametrize("case", ["u8", "u8_probing", "f32_padded", "u8_counting",
                                  "u8_counting_both_sizes"])
def test_noalloc_matches_query_workload_twice(case):
    if case == "f32_padded":  # d = 100: rows are padded into the scratch
        wl = synth.random_small(71, n=3000, d=100, Q=90, L=8, k=6, w=2.0, dtype="f32")
    elif case == "u8_counting_both_sizes":  # listed totals on both sides of 6,144
        wl = synth.make_config(1, L=32, k=1, w=55.0)
    else:
        wl = synth.make_config(1, w=1200.0)
    p = wl.params
    is_u8 = wl.data.dtype == np.uint8
    ix = lib.Index(dev(wl.data), dev(p.a), dev(p.b()), p.w)
    probes, probe_t = 0, 0
    if case == "u8_probing":
        ix.set_probing(2, 3)
        probes, probe_t = 2, 3
    if case.startswith("u8_counting"):
        ix.set_counting(2, 40)
    K = wl.K
    # two calls in a row, the second with fewer queries: the scratch keeps the
    # first call's contents, which must not leak into the second
    for rows in (np.arange(wl.Q), np.arange(7, wl.Q - 30)):
        q = dev(wl.queries[rows])
        ids, dist = noalloc(ix, q, K, is_u8)
        ids_p, dist_p = plain(ix, q, K)
        assert torch.equal(ids, ids_p) and torch.equal(dist, dist_p)
        if case.startswith("u8_counting"):
            ids_o, dist_o, _ = oracle.lsh_query_counting(wl.data, wl.queries[rows], p.a, p.b(),
                                                         p.w, K, 2, 40)
        else:
            ids_o, dist_o, _ = oracle.lsh_query(wl.data, wl.queries[rows], p.a, p.b(), p.w, K,
                                                probes=probes, probe_t=probe_t)
        check_oracle(ids, dist, ids_o, dist_o, is_u8)
    ix.close()


def test_noalloc_refuses_beyond_its_scratch():
    """A workload whose workspace exceeds the 32 MiB scratch is refused with
    QW_EUNSUPPORTED and the outputs untouched; the index keeps answering
    through both entry points afterwards."""
    wl = synth.make_config(1, w=1200.0)
    p = wl.params
    ix = lib.Index(dev(wl.data), dev(p.a), dev(p.b()), p.w)
    # 80 functions and 10 lists: 4*80 + 8*10 + 8 = 408 bytes per query
    big = dev(np.repeat(wl.queries, 1000, axis=0))  # 100,000 queries, ~40 MB of workspace
    ids = torch.full((big.shape[0], wl.K), -7, dtype=torch.int32, device="cuda")
    dist = torch.full_like(ids, -7)
    with pytest.raises(lib.QwError) as e:
        lib.qw_query_workload_noalloc(ix.handle, big, wl.K, ids, dist)
    assert e.value.status == lib.QW_EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((ids == -7).all()) and bool((dist == -7).all())
    q = dev(wl.queries)
    a = noalloc(ix, q, wl.K, True)
    b = plain(ix, q, wl.K)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    ix.close()
