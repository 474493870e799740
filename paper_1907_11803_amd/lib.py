"""Python binding of libqwlsh (the C ABI in include/qwlsh.h).

Argument marshalling only: every step of the query path runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the current stream.
The functions keep the C names; `Index` is a small owner object around them.

The library must have been built (``python -m paper_1907_11803_amd.build``);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Tuple

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqwlsh.so")

QW_OK, QW_EINVAL, QW_ENOMEM, QW_EDEVICE, QW_EUNSUPPORTED, QW_EINTERNAL = range(6)
QW_U8, QW_F32 = 0, 1
QW_FORM_PLAIN_FP32, QW_FORM_FAST = 0, 1
QW_SCHED_SUM, QW_SCHED_LEARNED, QW_SCHED_ACTUAL, QW_SCHED_NONE = range(4)
QW_MLP_HIDDEN = 64
QW_OOC_MRU, QW_OOC_LRU = 0, 1


class QwError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class qw_opts(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("sched", ctypes.c_int32), ("group", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("topk_keep", ctypes.c_int32), ("dedup", ctypes.c_int32), ("xchunk", ctypes.c_int32),
                ("stage_split", ctypes.c_int32), ("tune_cache", ctypes.c_char_p)]


class qw_stats(ctypes.Structure):
    _fields_ = [("projections", ctypes.c_int64), ("recomputed", ctypes.c_int64),
                ("recompute_frac", ctypes.c_double), ("probes_hit", ctypes.c_int64),
                ("cand_total", ctypes.c_int64), ("cand_unique", ctypes.c_int64),
                ("overflow", ctypes.c_int64), ("fallback", ctypes.c_int64),
                ("topk_second_pass", ctypes.c_int64),
                ("bins", ctypes.c_int64 * 8),
                ("ms_stage", ctypes.c_float * 8),
                ("dedup_used", ctypes.c_int32), ("group_used", ctypes.c_int32),
                ("xchunk_used", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("split_used", ctypes.c_int32),
                ("ooc_index_files", ctypes.c_int64), ("ooc_index_bytes", ctypes.c_int64),
                ("ooc_data_objects", ctypes.c_int64), ("ooc_data_bytes", ctypes.c_int64),
                ("ooc_batches", ctypes.c_int64), ("ooc_splits", ctypes.c_int64)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["bins"] = list(self.bins)
        d["ms_stage"] = list(self.ms_stage)
        return d


class qw_index_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("L", ctypes.c_int32), ("k", ctypes.c_int32), ("w", ctypes.c_float),
                ("key_bits", ctypes.c_int32 * 64), ("buckets", ctypes.c_int64),
                ("max_bucket", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("has_count_model", ctypes.c_int32), ("count_margin", ctypes.c_float),
                ("probing", ctypes.c_int32), ("probes_per_layer", ctypes.c_int32),
                ("count_threshold", ctypes.c_int32), ("count_extra", ctypes.c_int32),
                ("mean_hit_bucket", ctypes.c_double), ("out_of_core", ctypes.c_int32),
                ("ooc_index_percent", ctypes.c_int32), ("host_bytes", ctypes.c_int64)]


class qw_ooc_tune_result(ctypes.Structure):
    _fields_ = [("index_percent", ctypes.c_int32), ("shares", ctypes.c_int32),
                ("percent", ctypes.c_int32 * 11), ("ms", ctypes.c_float * 11),
                ("index_bytes", ctypes.c_int64 * 11), ("data_bytes", ctypes.c_int64 * 11),
                ("batches", ctypes.c_int64 * 11), ("splits", ctypes.c_int64 * 11)]


class qw_ooc_opts(ctypes.Structure):
    _fields_ = [("cache_bytes", ctypes.c_int64), ("index_percent", ctypes.c_int32),
                ("strategy", ctypes.c_int32), ("policy", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("keep", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class qw_tune_result(ctypes.Structure):
    _fields_ = [("dedup", ctypes.c_int32), ("group", ctypes.c_int32), ("xchunk", ctypes.c_int32),
                ("stage_split", ctypes.c_int32),
                ("ms", ctypes.c_float), ("ms_default", ctypes.c_float), ("candidates", ctypes.c_int32)]


# exported symbols and their signatures (restype qw_status unless noted)
_P, _I32, _I64, _F32, _U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_uint64
SIGNATURES = {
    "qw_default_opts": (None, [_P]),
    "qw_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "qw_build_index": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _P, _F32, _I32, _I32, _P, _P, _P]),
    "qw_query_workload": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P, _P, _P]),
    "qw_query_workload_noalloc": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P]),
    "qw_autotune": (ctypes.c_int, [_P, _P, _I64, _I32, _P, ctypes.c_char_p, _P, _P]),
    "qw_free_index": (None, [_P]),
    "qw_get_index_info": (ctypes.c_int, [_P, _P]),
    "qw_hash": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P]),
    "qw_bucket_sizes": (ctypes.c_int, [_P, _P, _I64, _P, _P]),
    "qw_candidate_counts": (ctypes.c_int, [_P, _P, _I64, _P, _P]),
    "qw_candidate_lists": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P]),
    "qw_bruteforce_knn": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P]),
    "qw_mlp_param_count": (_I32, [_I32]),
    "qw_mlp_loss_grad": (ctypes.c_int, [_P, _I32, _P, _P, _I32, _P, _P, _P]),
    "qw_mlp_adam": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I32, _F32, _F32, _F32, _F32, _P]),
    "qw_mlp_predict_bf16": (ctypes.c_int, [_P, _I32, _P, _I32, _P, _P]),
    "qw_train_count_model": (ctypes.c_int, [_P, _P, _I64, _I32, _I32, _F32, _U64, _P, _P]),
    "qw_set_count_model": (ctypes.c_int, [_P, _P, _I32]),
    "qw_get_count_model": (ctypes.c_int, [_P, _P, _I32]),
    "qw_set_count_margin": (ctypes.c_int, [_P, ctypes.c_float]),
    "qw_set_probing": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "qw_set_counting": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "qw_set_out_of_core": (ctypes.c_int, [_P, _P, _P]),
    "qw_autotune_ooc": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libqwlsh.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_1907_11803_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(s: int) -> str:
    try:
        return load().qw_status_string(int(s)).decode()
    except Exception:
        return "status %d" % s


def _check(rc: int, where: str):
    if rc != QW_OK:
        raise QwError(rc, where)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t: torch.Tensor, dtypes, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    return t.contiguous()


def _dtype_code(t: torch.Tensor) -> int:
    return QW_U8 if t.dtype == torch.uint8 else QW_F32


QW_DEDUP_AUTO, QW_DEDUP_BLOCK, QW_DEDUP_WAVE = 0, 1, 2


def make_opts(form: int = QW_FORM_FAST, sched: int = QW_SCHED_LEARNED, group: int = -1,
              graph: int = 1, timing: int = 0, topk_keep: int = 0, dedup: int = 0,
              xchunk: int = 0, tune_cache: Optional[str] = None, stage_split: int = 0) -> qw_opts:
    o = qw_opts()
    load().qw_default_opts(ctypes.byref(o))
    o.form, o.sched, o.group, o.graph, o.timing = form, sched, group, graph, timing
    o.topk_keep, o.dedup, o.xchunk, o.stage_split = topk_keep, dedup, xchunk, stage_split
    # the struct keeps a pointer to the encoded path: hold the bytes on the object
    o._tune_path = tune_cache.encode() if tune_cache else None
    o.tune_cache = o._tune_path
    return o


# ------------------------------------------------------------------ thin wrappers

def qw_build_index(data: torch.Tensor, a: torch.Tensor, b: torch.Tensor, w: float,
                   form: int = QW_FORM_FAST, stream=None) -> ctypes.c_void_p:
    data = _dev(data, (torch.uint8, torch.float32), "data")
    a = _dev(a, (torch.float32,), "a")
    b = _dev(b, (torch.float32,), "b")
    if a.dim() != 3 or b.dim() != 2 or a.shape[:2] != b.shape or a.shape[2] != data.shape[1]:
        raise ValueError("expected a [L,k,d] and b [L,k] matching data [n,d]")
    L, k, d = a.shape
    out = ctypes.c_void_p()
    o = make_opts(form=form)
    rc = load().qw_build_index(_ptr(data), data.shape[0], d, _dtype_code(data), _ptr(a), _ptr(b),
                               float(w), L, k, ctypes.byref(o), _stream(stream), ctypes.byref(out))
    _check(rc, "qw_build_index")
    return out


def qw_query_workload(ix, queries: torch.Tensor, K: int, opts: Optional[qw_opts] = None,
                      stream=None, out_ids: Optional[torch.Tensor] = None,
                      out_dist: Optional[torch.Tensor] = None, stats: bool = False):
    queries = _dev(queries, (torch.uint8, torch.float32), "queries")
    Q = queries.shape[0]
    dev = queries.device
    if out_ids is None:
        out_ids = torch.empty((Q, K), dtype=torch.int32, device=dev)
    if out_dist is None:
        out_dist = torch.empty((Q, K), dtype=torch.int32 if queries.dtype == torch.uint8 else torch.float32,
                               device=dev)
    st = qw_stats() if stats else None
    rc = load().qw_query_workload(ix, _ptr(queries), Q, int(K),
                                  ctypes.byref(opts) if opts is not None else None,
                                  _stream(stream), _ptr(out_ids), _ptr(out_dist),
                                  ctypes.byref(st) if st is not None else None)
    _check(rc, "qw_query_workload")
    return (out_ids, out_dist, st.as_dict()) if stats else (out_ids, out_dist)


def qw_query_workload_noalloc(ix, queries: torch.Tensor, K: int, out_ids: torch.Tensor,
                              out_dist: torch.Tensor, stream=None):
    """The allocation-free plain-form query: the caller passes the outputs."""
    queries = _dev(queries, (torch.uint8, torch.float32), "queries")
    rc = load().qw_query_workload_noalloc(ix, _ptr(queries), queries.shape[0], int(K),
                                          _stream(stream), _ptr(out_ids), _ptr(out_dist))
    _check(rc, "qw_query_workload_noalloc")
    return out_ids, out_dist


def qw_autotune(ix, queries: torch.Tensor, K: int, cache_path: str, opts: Optional[qw_opts] = None,
                stream=None) -> dict:
    """Time the fast form's scheduling settings on this workload and record the
    fastest in the JSON cache at `cache_path`; returns the choice and times."""
    queries = _dev(queries, (torch.uint8, torch.float32), "queries")
    r = qw_tune_result()
    rc = load().qw_autotune(ix, _ptr(queries), queries.shape[0], int(K),
                            ctypes.byref(opts) if opts is not None else None,
                            str(cache_path).encode(), _stream(stream), ctypes.byref(r))
    _check(rc, "qw_autotune")
    return {f: getattr(r, f) for f, _ in r._fields_}


def qw_free_index(ix):
    if ix:
        load().qw_free_index(ix)


def qw_get_index_info(ix) -> dict:
    info = qw_index_info()
    _check(load().qw_get_index_info(ix, ctypes.byref(info)), "qw_get_index_info")
    d = {f: getattr(info, f) for f, _ in info._fields_}
    d["key_bits"] = list(info.key_bits)[: info.L]
    return d


def qw_hash(ix, x: torch.Tensor, nf: int, form: int = QW_FORM_FAST, stream=None):
    x = _dev(x, (torch.uint8, torch.float32), "x")
    out = torch.empty((x.shape[0], nf), dtype=torch.int32, device=x.device)
    rec = ctypes.c_int64(0)
    rc = load().qw_hash(ix, _ptr(x), x.shape[0], int(form), _stream(stream), _ptr(out),
                        ctypes.byref(rec))
    _check(rc, "qw_hash")
    return out, int(rec.value)


def qw_bucket_sizes(ix, queries: torch.Tensor, L: int, stream=None) -> torch.Tensor:
    queries = _dev(queries, (torch.uint8, torch.float32), "queries")
    out = torch.empty((queries.shape[0], L), dtype=torch.int32, device=queries.device)
    _check(load().qw_bucket_sizes(ix, _ptr(queries), queries.shape[0], _stream(stream), _ptr(out)),
           "qw_bucket_sizes")
    return out


def qw_candidate_counts(ix, queries: torch.Tensor, stream=None) -> torch.Tensor:
    queries = _dev(queries, (torch.uint8, torch.float32), "queries")
    out = torch.empty((queries.shape[0],), dtype=torch.int32, device=queries.device)
    _check(load().qw_candidate_counts(ix, _ptr(queries), queries.shape[0], _stream(stream), _ptr(out)),
           "qw_candidate_counts")
    return out


def qw_candidate_lists(ix, queries: torch.Tensor, stream=None) -> List[np.ndarray]:
    """Candidate ids per query (sorted ascending here, on the host)."""
    counts = qw_candidate_counts(ix, queries, stream)
    off = torch.zeros((queries.shape[0] + 1,), dtype=torch.int64, device=queries.device)
    off[1:] = torch.cumsum(counts.to(torch.int64), 0)
    total = int(off[-1].item())
    ids = torch.empty((max(total, 1),), dtype=torch.int32, device=queries.device)
    _check(load().qw_candidate_lists(ix, _ptr(queries.contiguous()), queries.shape[0], _ptr(off),
                                     _stream(stream), _ptr(ids)), "qw_candidate_lists")
    h = ids.cpu().numpy()
    o = off.cpu().numpy()
    return [np.sort(h[o[i]:o[i + 1]]) for i in range(queries.shape[0])]


def qw_bruteforce_knn(ix, queries: torch.Tensor, K: int, stream=None):
    queries = _dev(queries, (torch.uint8, torch.float32), "queries")
    Q = queries.shape[0]
    ids = torch.empty((Q, K), dtype=torch.int32, device=queries.device)
    dist = torch.empty((Q, K), dtype=torch.int32 if queries.dtype == torch.uint8 else torch.float32,
                       device=queries.device)
    _check(load().qw_bruteforce_knn(ix, _ptr(queries), Q, int(K), _stream(stream), _ptr(ids),
                                    _ptr(dist)), "qw_bruteforce_knn")
    return ids, dist


def qw_mlp_param_count(L: int) -> int:
    return int(load().qw_mlp_param_count(int(L)))


def qw_mlp_loss_grad(params: torch.Tensor, L: int, feats: torch.Tensor, targets: torch.Tensor,
                     stream=None):
    params = _dev(params, (torch.float32,), "params")
    feats = _dev(feats, (torch.float32,), "feats")
    targets = _dev(targets, (torch.float32,), "targets")
    grad = torch.empty_like(params)
    loss = torch.empty((1,), dtype=torch.float32, device=params.device)
    _check(load().qw_mlp_loss_grad(_ptr(params), int(L), _ptr(feats), _ptr(targets),
                                   feats.shape[0], _stream(stream), _ptr(grad), _ptr(loss)),
           "qw_mlp_loss_grad")
    return grad, loss


def qw_mlp_adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
                stream=None):
    for t, nm in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _dev(t, (torch.float32,), nm)
    _check(load().qw_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(),
                              int(step), float(lr), float(beta1), float(beta2), float(eps),
                              _stream(stream)), "qw_mlp_adam")


def qw_mlp_predict_bf16(params: torch.Tensor, L: int, feats: torch.Tensor, stream=None):
    params = _dev(params, (torch.float32,), "params")
    feats = _dev(feats, (torch.float32,), "feats")
    out = torch.empty((feats.shape[0],), dtype=torch.float32, device=feats.device)
    _check(load().qw_mlp_predict_bf16(_ptr(params), int(L), _ptr(feats), feats.shape[0],
                                      _stream(stream), _ptr(out)), "qw_mlp_predict_bf16")
    return out


def qw_train_count_model(ix, train_queries: torch.Tensor, epochs: int = 10, batch: int = 1024,
                         lr: float = 1e-3, seed: int = 0, stream=None) -> float:
    train_queries = _dev(train_queries, (torch.uint8, torch.float32), "train_queries")
    loss = ctypes.c_float(float("nan"))
    _check(load().qw_train_count_model(ix, _ptr(train_queries), train_queries.shape[0], int(epochs),
                                       int(batch), float(lr), int(seed), _stream(stream),
                                       ctypes.byref(loss)), "qw_train_count_model")
    return float(loss.value)


def qw_set_count_model(ix, params: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(load().qw_set_count_model(ix, ctypes.c_void_p(p.ctypes.data), p.size), "qw_set_count_model")


def qw_set_count_margin(ix, margin: float):
    _check(load().qw_set_count_margin(ix, float(margin)), "qw_set_count_margin")


def qw_set_probing(ix, mode: int, per_layer: int = 0):
    _check(load().qw_set_probing(ix, int(mode), int(per_layer)), "qw_set_probing")


def qw_set_counting(ix, threshold: int, extra: int = 0):
    _check(load().qw_set_counting(ix, int(threshold), int(extra)), "qw_set_counting")


def qw_set_out_of_core(ix, cache_bytes: Optional[int], index_percent: int = 50, strategy: int = 1,
                       policy: int = QW_OOC_MRU, batch: int = 10000, keep: int = 0, stream=None):
    """Out-of-core mode (cache_bytes None: back in core)."""
    if cache_bytes is None:
        _check(load().qw_set_out_of_core(ix, None, _stream(stream)), "qw_set_out_of_core")
        return
    o = qw_ooc_opts(cache_bytes=int(cache_bytes), index_percent=int(index_percent),
                    strategy=int(strategy), policy=int(policy), batch=int(batch), keep=int(keep),
                    reserved=0)
    _check(load().qw_set_out_of_core(ix, ctypes.byref(o), _stream(stream)), "qw_set_out_of_core")


def qw_autotune_ooc(ix, queries: torch.Tensor, K: int, cache_bytes: int, strategy: int = 1,
                    policy: int = QW_OOC_MRU, batch: int = 10000, keep: int = 0, stream=None) -> dict:
    """Time the eleven index shares (1, 10, ..., 90, 99 %) of an out-of-core
    cache on the workload; the index is left out of core at the fastest."""
    queries = _dev(queries, (torch.uint8, torch.float32), "queries")
    o = qw_ooc_opts(cache_bytes=int(cache_bytes), index_percent=0, strategy=int(strategy),
                    policy=int(policy), batch=int(batch), keep=int(keep), reserved=0)
    r = qw_ooc_tune_result()
    _check(load().qw_autotune_ooc(ix, _ptr(queries), queries.shape[0], int(K), ctypes.byref(o),
                                  _stream(stream), ctypes.byref(r)), "qw_autotune_ooc")
    n = r.shares
    return {"index_percent": r.index_percent,
            "shares": [{"index_percent": r.percent[i], "ms": round(float(r.ms[i]), 3),
                        "index_bytes": r.index_bytes[i], "data_bytes": r.data_bytes[i],
                        "batches": r.batches[i], "splits": r.splits[i]} for i in range(n)]}


def qw_get_count_model(ix, L: int) -> np.ndarray:
    p = np.empty(qw_mlp_param_count(L), dtype=np.float32)
    _check(load().qw_get_count_model(ix, ctypes.c_void_p(p.ctypes.data), p.size), "qw_get_count_model")
    return p


# ------------------------------------------------------------------ owner object

class Index:
    """An LSH index on the current HIP device (owns the library handle)."""

    def __init__(self, data: torch.Tensor, a: torch.Tensor, b: torch.Tensor, w: float,
                 form: int = QW_FORM_FAST, stream=None):
        self.handle = qw_build_index(data, a, b, w, form, stream)
        self.L, self.k, self.d = a.shape
        self.n = data.shape[0]
        self.dtype = data.dtype

    def query(self, queries, K, opts: Optional[qw_opts] = None, stream=None, out_ids=None,
              out_dist=None, stats: bool = False):
        return qw_query_workload(self.handle, queries, K, opts, stream, out_ids, out_dist, stats)

    def autotune(self, queries, K, cache_path, opts: Optional[qw_opts] = None, stream=None) -> dict:
        return qw_autotune(self.handle, queries, K, cache_path, opts, stream)

    def hash(self, x, form: int = QW_FORM_FAST, stream=None):
        return qw_hash(self.handle, x, self.L * self.k, form, stream)

    def bucket_sizes(self, queries, stream=None):
        return qw_bucket_sizes(self.handle, queries, self.L, stream)

    def candidate_counts(self, queries, stream=None):
        return qw_candidate_counts(self.handle, queries, stream)

    def candidate_lists(self, queries, stream=None):
        return qw_candidate_lists(self.handle, queries, stream)

    def bruteforce(self, queries, K, stream=None):
        return qw_bruteforce_knn(self.handle, queries, K, stream)

    def train_count_model(self, train_queries, **kw) -> float:
        return qw_train_count_model(self.handle, train_queries, **kw)

    def set_count_model(self, params):
        qw_set_count_model(self.handle, params)

    def get_count_model(self) -> np.ndarray:
        return qw_get_count_model(self.handle, self.L)

    def set_count_margin(self, margin: float):
        qw_set_count_margin(self.handle, margin)

    def set_probing(self, mode: int, per_layer: int = 0):
        qw_set_probing(self.handle, mode, per_layer)

    def set_counting(self, threshold: int, extra: int = 0):
        """Collision counting: threshold on the layers shared with the query
        (0: the plain union), at most K + extra points verified."""
        qw_set_counting(self.handle, threshold, extra)

    def set_out_of_core(self, cache_bytes: Optional[int], **kw):
        """Lists and rows to pinned host memory with an HBM cache of
        cache_bytes split index_percent / the rest (None: back in HBM)."""
        qw_set_out_of_core(self.handle, cache_bytes, **kw)

    def autotune_ooc(self, queries, K, cache_bytes, **kw) -> dict:
        return qw_autotune_ooc(self.handle, queries, K, cache_bytes, **kw)

    def info(self) -> dict:
        return qw_get_index_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            qw_free_index(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
