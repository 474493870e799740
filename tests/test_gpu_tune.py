"""The autotuner of the fast form's scheduling settings: every setting it
times returns the same outputs, the cache it writes is JSON keyed by the GPU
architecture and the workload, and a query that names the cache returns the
untuned query's outputs bit for bit, and the oracle's."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_1907_11803_amd import lib, synth

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("probing,model", [(0, False), (2, True)])
def test_tuned_and_default_outputs_identical(tmp_path, probing, model):
    wl = synth.make_config(1)
    p = wl.params
    ix = lib.Index(dev(wl.data), dev(p.a), dev(p.b()), p.w)
    if probing:
        ix.set_probing(2, 2)
    if model:
        ix.train_count_model(dev(synth.training_queries(1, 4000)), epochs=2, batch=1024, lr=2e-3, seed=1)
    q = dev(wl.queries)
    K = wl.K
    cache = tmp_path / "tune.json"
    r = ix.autotune(q, K, str(cache))
    assert r["candidates"] >= 4
    assert r["dedup"] in (1, 2) and r["group"] in (0, 1)
    assert (r["xchunk"] in (16, 64, 256)) if r["group"] else r["xchunk"] == 0
    assert r["stage_split"] == -1
    assert 0 < r["ms"] <= r["ms_default"]
    doc = json.loads(cache.read_text())
    (e,) = doc["entries"]
    assert e["arch"].startswith("gfx") and len(e["key"]) == 16
    assert (e["dedup"], e["group"], e["xchunk"], e["split"]) == (r["dedup"], r["group"], r["xchunk"],
                                                                 r["stage_split"])

    ids_d, dist_d, st = ix.query(q, K, lib.make_opts(), stats=True)
    assert st["tuned"] == 0 and st["dedup_used"] in (1, 2)
    ids_d, dist_d = ids_d.cpu().numpy(), dist_d.cpu().numpy()
    for graph in (0, 1):
        ids_t, dist_t, st = ix.query(q, K, lib.make_opts(graph=graph, tune_cache=str(cache)), stats=True)
        assert st["tuned"] == 1
        assert (st["dedup_used"], st["group_used"], st["xchunk_used"]) == (r["dedup"], r["group"], r["xchunk"])
        assert st["split_used"] == r["stage_split"]
        assert np.array_equal(ids_t.cpu().numpy(), ids_d)
        assert np.array_equal(dist_t.cpu().numpy(), dist_d)
    # an explicit setting wins over the cache
    _, _, st = ix.query(q, K, lib.make_opts(dedup=1, group=0, stage_split=-1, tune_cache=str(cache)),
                        stats=True)
    assert (st["dedup_used"], st["group_used"], st["xchunk_used"], st["split_used"]) == (1, 0, 0, -1)
    ids_o, dist_o, _ = oracle.lsh_query(wl.data, wl.queries, p.a, p.b(), p.w, K, probes=probing, probe_t=2)
    assert np.array_equal(ids_d, ids_o)
    assert np.array_equal(dist_d.astype(np.int64),
                          np.where(dist_o == np.iinfo(np.int64).max, np.iinfo(np.int32).max, dist_o))

    # a second workload adds an entry; re-tuning the first replaces its entry
    ix.autotune(q[: q.shape[0] // 2].contiguous(), K, str(cache))
    ix.autotune(q, K, str(cache))
    doc = json.loads(cache.read_text())
    assert len(doc["entries"]) == 2
    assert len({x["key"] for x in doc["entries"]}) == 2
    ix.close()


def test_tune_cache_miss_and_bad_paths(tmp_path):
    """A cache without this workload's entry (or no such file) leaves the
    built-in automatic settings; the tuner refuses an unwritable path and
    collision counting."""
    wl = synth.make_config(1, n=20_000, Q=300)
    p = wl.params
    ix = lib.Index(dev(wl.data), dev(p.a), dev(p.b()), p.w)
    q = dev(wl.queries)
    ids_d, dist_d = ix.query(q, wl.K, lib.make_opts())
    for path in (str(tmp_path / "absent.json"), str(tmp_path / "other.json")):
        if path.endswith("other.json"):
            ix.autotune(q[:100], wl.K, path)
        ids_t, dist_t, st = ix.query(q, wl.K, lib.make_opts(tune_cache=path), stats=True)
        assert st["tuned"] == 0
        assert torch.equal(ids_t, ids_d) and torch.equal(dist_t, dist_d)
    with pytest.raises(lib.QwError):
        ix.autotune(q, wl.K, str(tmp_path / "no_such_dir" / "t.json"))
    ix.set_counting(2, 0)
    with pytest.raises(lib.QwError):
        ix.autotune(q, wl.K, str(tmp_path / "t.json"))
    ix.close()
