#!/usr/bin/env python3
"""Benchmark: queries/sec at recall@10 >= 0.9 on one MI355X.

One step = one pass of the whole query path (pad, project + hash, probe,
schedule, de-duplicated candidate union, exact verification, top-K) over the
full query workload, with the index built and the queries already resident in
HBM.  The headline configuration is the 1M-point uint8 workload: n=1,000,000,
d=128 Gaussian mixture (1,000 components, sigma 20), Q=10,000 noisy data
points, L=20 layers of k=10 functions, K=10.  Its stated bucket width w=400
reaches recall@10 of only ~0.13, so the benchmark runs at w_0.9: the smallest w
on the grid {1, 1.5, 2, 2.5, 3, 4, 6, 8} x 400 whose measured recall@10 (against
GPU brute force over all points) is >= 0.9; L and k are unchanged.

Reported: the fast form (FP16 MFMA + FP64 guard band, bucket grouping,
learned-count binning, persistent verify, HIP graph) as `value`; the plain FP32
form beside it; the verify kernel's achieved HBM bandwidth against the 8 TB/s
peak; and the CPU oracle timed on a bounded query sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_FP16_TFLOPS = 2500.0  # dense FP16 matrix peak (no sparsity)
MFMA_PEAK_FP32_TFLOPS = 157.3   # dense FP32 matrix peak
W_GRID = [1, 1.5, 2, 2.5, 3, 4, 6, 8]
METRIC = "queries/sec at recall@10>=0.9, BF16+learned vs plain FP32 on 1 MI355X"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def recall_at_10(ids_lsh, ids_true, dist_lsh, dist_true):
    """Tie-tolerant recall@10: a returned id counts when it is one of the exact
    top-10 ids or its distance is <= the exact 10th distance."""
    import numpy as np
    K = 10
    hits = 0
    for q in range(ids_lsh.shape[0]):
        truth = set(ids_true[q, :K].tolist())
        d10 = dist_true[q, K - 1]
        for r in range(K):
            i = int(ids_lsh[q, r])
            if i < 0:
                continue
            if i in truth or dist_lsh[q, r] <= d10:
                hits += 1
    return hits / (K * ids_lsh.shape[0])


def kernel_source_hash(files):
    """Identifies a kernel's source: stored HBM traffic is used only while it
    matches."""
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1907_11803_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


FUSED_SOURCES = ("qw_dedup.hip", "qw_dedup.h", "qw_dist.h", "qw_wave.h")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--w", type=float, default=None, help="bucket width (default: search w_0.9)")
    ap.add_argument("--probes", type=int, default=None, choices=[0, 1, 2],
                    help="0: each layer's own bucket; 1: also its 2k one-step neighbour "
                         "buckets; 2: only the --probe-t best of them per query "
                         "(query-directed).  Default: the measured best for the workload")
    ap.add_argument("--probe-t", type=int, default=None, help="moves per layer for --probes 2")
    ap.add_argument("--train-queries", type=int, default=None,
                    help="count-model training queries (default: the configuration's, else 50,000)")
    ap.add_argument("--recall-sample", type=int, default=2000,
                    help="queries whose recall@10 is measured against brute force (0 = all)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle query sample (0 = up to 10,000 uint8 / 1,000 float queries)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--count-theta", type=int, default=None,
                    help="collision-counting leg: threshold on shared layers (0: skip; "
                         "default 3 for config 2, else 0)")
    ap.add_argument("--count-v", type=int, default=800,
                    help="collision-counting leg: extra verified points v (K + v in all)")
    ap.add_argument("--profile", action="store_true",
                    help="only the fast-form timed loop (for rocprofv3 runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this engine has no multi-GPU path (queries or data "
              "would be sharded across GPUs with one gather of Q x K results).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1907_11803_amd import lib, synth
    # probing per workload, as measured at w_0.9 (ms per step, recall@10):
    # 1M x 128 uint8: none 0.509 (0.965), query-directed T=2 0.467 (0.921),
    # T=3 0.492 (0.953), every neighbour 0.644 (0.992); 10M x 96 uint8 Zipf:
    # none 3.19 (0.976), T=2 3.76 (0.983); 1M x 960 float Zipf: none 62.8
    # (0.953), T=2 60.5 (0.983)
    best = {2: (2, 2), 5: (2, 2)}.get(args.config, (0, 0))
    if args.probes is None:
        args.probes, args.probe_t = best[0], (args.probe_t or best[1])
    if args.probe_t is None:
        args.probe_t = 2

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    lib.load()
    t0 = time.time()
    spec = synth.CONFIGS[args.config]
    wl = synth.make_config(args.config)
    log(f"[bench] cfg{args.config}: n={wl.n} d={wl.d} Q={wl.Q} L={wl.params.L} "
        f"k={wl.params.k} generated in {time.time() - t0:.1f}s")
    data_d = torch.from_numpy(wl.data).to(dev)
    q_d = torch.from_numpy(wl.queries).to(dev)
    a_d = torch.from_numpy(wl.params.a).to(dev)
    K = wl.K
    is_u8 = wl.data.dtype == np.uint8

    # ---- choose w_0.9 (recall measured on every query against GPU brute force)
    grid = [args.w] if args.w else [m * spec["w"] for m in W_GRID]
    truth = None
    chosen = None
    tried = []
    for w in grid:
        b_d = torch.from_numpy(wl.params.b(w)).to(dev)
        t1 = time.time()
        ix = lib.Index(data_d, a_d, b_d, w, form=lib.QW_FORM_FAST)
        if args.probes:
            ix.set_probing(args.probes, args.probe_t)
        build_s = time.time() - t1
        if args.profile:  # profiling runs time the query loop only
            chosen = (w, ix, b_d, None, None)
            break
        if truth is None:
            t1 = time.time()
            rs = wl.Q if args.recall_sample <= 0 else min(args.recall_sample, wl.Q)
            rsel = np.sort(np.random.default_rng(11).choice(wl.Q, size=rs, replace=False))
            rsel_d = torch.from_numpy(rsel).to(dev)
            ti, td = ix.bruteforce(q_d[rsel_d].contiguous(), K)
            torch.cuda.synchronize()
            truth = (ti.cpu().numpy(), td.cpu().numpy())
            log(f"[bench] brute-force ground truth for {rs} queries in {time.time() - t1:.1f}s")
        ids, dist, st = ix.query(q_d, K, lib.make_opts(sched=lib.QW_SCHED_SUM, graph=0), stats=True)
        rec = recall_at_10(ids.cpu().numpy()[rsel], truth[0], dist.cpu().numpy()[rsel], truth[1])
        tried.append({"w": w, "recall_at_10": round(rec, 4),
                      "mean_unique_candidates": st["cand_unique"] / wl.Q})
        log(f"[bench] w={w}: recall@10={rec:.4f} unique/q={st['cand_unique'] / wl.Q:.0f} "
            f"sum/q={st['cand_total'] / wl.Q:.0f} build {build_s:.1f}s")
        if rec >= 0.9 or w == grid[-1]:
            chosen = (w, ix, b_d, rec, st)
            break
        ix.close()
    w, ix, b_d, rec, st0 = chosen

    # ---- learned count model, trained on the engine's own features
    t1 = time.time()
    ntrain = args.train_queries or spec.get("train_Q", 50_000)
    train = synth.training_queries(args.config, ntrain)
    train_d = torch.from_numpy(train).to(dev)
    train_loss = ix.train_count_model(train_d, epochs=8, batch=1024, lr=2e-3, seed=1)
    del train_d
    log(f"[bench] count model trained on {ntrain} queries, loss {train_loss:.4f}, "
        f"sizing margin {ix.info()['count_margin']:.3f} "
        f"in {time.time() - t1:.1f}s")
    count_model = None
    if not args.profile:
        # prediction quality on the workload's own queries: log(1 + |C(q)|)
        feats = torch.log1p(ix.bucket_sizes(q_d).to(torch.float32)).contiguous()
        params = torch.from_numpy(ix.get_count_model()).to(dev)
        pred = lib.qw_mlp_predict_bf16(params, wl.params.L, feats).cpu().numpy()
        actual = np.log1p(ix.candidate_counts(q_d).cpu().numpy().astype(np.float64))
        count_model = {"train_queries": int(ntrain), "train_loss": round(float(train_loss), 4),
                       "mae_log": round(float(np.mean(np.abs(pred - actual))), 4),
                       "sizing_margin": round(float(ix.info()["count_margin"]), 4)}
        log(f"[bench] count model on the workload: MAE {count_model['mae_log']} (log space)")

    out_ids = torch.empty((wl.Q, K), dtype=torch.int32, device=dev)
    out_dist = torch.empty((wl.Q, K), dtype=torch.int32 if is_u8 else torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def timed(opts, steps, warmup, index=None):
        index = index or ix
        for _ in range(warmup):
            index.query(q_d, K, opts, out_ids=out_ids, out_dist=out_dist)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(steps):
            index.query(q_d, K, opts, out_ids=out_ids, out_dist=out_dist)
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps

    fast_opts = lib.make_opts(form=lib.QW_FORM_FAST, sched=lib.QW_SCHED_LEARNED, group=-1, graph=1)
    if args.profile:
        # a plain device copy of known size (1 GiB read + 1 GiB written) to
        # calibrate the HBM byte counters of a profiling run
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        ms = timed(fast_opts, args.steps, args.warmup)
        log(f"[bench] profile loop: {ms:.3f} ms/step")
        return

    # the copy rate this GPU reaches: 1 GiB device to device (1 GiB read and
    # 1 GiB written per copy), the best of five, as a measured HBM ceiling
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    copy_gbs = 0.0
    for _ in range(6):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = max(copy_gbs, 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    log(f"[bench] device copy: {copy_gbs:.0f} GB/s")

    # exactness of the timed forms against each other and the brute-force recall
    ref_ids, ref_dist = ix.query(q_d, K, lib.make_opts(form=lib.QW_FORM_PLAIN_FP32))
    ref_ids, ref_dist = ref_ids.cpu().numpy(), ref_dist.cpu().numpy()
    f_ids, f_dist = ix.query(q_d, K, fast_opts)
    identical = bool(np.array_equal(f_ids.cpu().numpy(), ref_ids) and
                     np.array_equal(f_dist.cpu().numpy(), ref_dist))

    # ---- timed regions
    ms_fast = timed(fast_opts, args.steps, args.warmup)
    ms_plain = timed(lib.make_opts(form=lib.QW_FORM_PLAIN_FP32), args.steps, args.warmup)
    # the schedules (count sources) under the automatic grouping, then the
    # learned schedule with each fixed grouping; every one must return the
    # fast form's results exactly
    sched_ms = {}
    sched_identical = True
    variants = [(name, lib.make_opts(sched=sc)) for name, sc in (
        ("sum", lib.QW_SCHED_SUM), ("actual", lib.QW_SCHED_ACTUAL),
        ("none", lib.QW_SCHED_NONE), ("learned", lib.QW_SCHED_LEARNED))]
    variants += [(f"learned_group{g}", lib.make_opts(sched=lib.QW_SCHED_LEARNED, group=g))
                 for g in (0, 1)]
    f_ids_np, f_dist_np = f_ids.cpu().numpy(), f_dist.cpu().numpy()
    for name, o in variants:
        sched_ms[name] = round(timed(o, max(5, args.steps // 2), 2), 4)
        s_ids, s_dist = ix.query(q_d, K, o)
        sched_identical &= bool(np.array_equal(s_ids.cpu().numpy(), f_ids_np) and
                                np.array_equal(s_dist.cpu().numpy(), f_dist_np))
    log(f"[bench] fast {ms_fast:.3f} ms/step, plain {ms_plain:.3f} ms/step, scheds {sched_ms}, "
        f"identical {sched_identical}")

    # ---- per-stage timing of the fast pipeline (events inside the library)
    stage = np.zeros(8)
    nrep = 5
    for _ in range(nrep):
        _, _, s = ix.query(q_d, K, lib.make_opts(sched=lib.QW_SCHED_LEARNED, timing=1, graph=0),
                           out_ids=out_ids, out_dist=out_dist, stats=True)
        stage += np.array(s["ms_stage"])
    stage /= nrep
    st = s
    elem = 1 if is_u8 else 4
    L = wl.params.L
    alg_bytes = (wl.Q * wl.d * elem + 8 * L * wl.Q + 4 * st["cand_total"] +
                 st["cand_unique"] * wl.d * elem + 8 * K * wl.Q)
    # Dominant kernel: the dedup kernel, which also verifies its candidates;
    # algorithmic bytes per query: the bucket ids (4 per entry), each unique
    # candidate's row, the query row, and either each candidate's
    # (distance, id) key for the select kernel or, when the kernel selects the
    # top K itself (uint8 rows of at most 1024 bytes, K <= 16, the library's
    # rule), the K output pairs.  Its time: the dedup stage (all of its
    # launches of one step, on two streams).
    topk_fused = is_u8 and K <= 16 and (wl.d + 15) // 16 <= 64
    kname = "dedup_kernel (dedup + verify + top-K)" if topk_fused else "dedup_kernel (dedup + verify)"
    ksrc, kfile = FUSED_SOURCES, "dedup_verify"
    per_cand = wl.d * elem + (0 if topk_fused else 8)
    kbytes = (4 * st["cand_total"] + st["cand_unique"] * per_cand + wl.Q * wl.d * elem +
              (8 * K * wl.Q if topk_fused else 0))
    kms = float(stage[6])
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"{kfile}_cfg{args.config}_traffic.json")
    if os.path.exists(tfile):
        tj = json.load(open(tfile))
        if (tj.get("source") == kernel_source_hash(ksrc) and abs(tj.get("w", -1) - w) < 1e-9
                and tj.get("probes", 0) == args.probes
                and tj.get("probe_t", 0) == (args.probe_t if args.probes == 2 else 0)):
            traffic = tj.get("bytes_per_launch")

    # ---- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu:
        import oracle
        nthreads = max(1, min(16, os.cpu_count() or 1))
        t1 = time.time()
        bi = oracle.BuiltIndex(wl.data, wl.params.a, wl.params.b(w), w, nthreads=nthreads)
        build_cpu = time.time() - t1
        rng = np.random.default_rng(7)
        ns = min(args.cpu_sample if args.cpu_sample > 0 else (10_000 if is_u8 else 1_000), wl.Q)
        sample = np.sort(rng.choice(wl.Q, size=ns, replace=False))
        t1 = time.time()
        o_ids, o_dist, _ = bi.query(wl.queries[sample], K, probes=args.probes,
                                    probe_t=args.probe_t if args.probes == 2 else 0)
        q_cpu = time.time() - t1
        bi.close()
        cpu_match = bool(np.array_equal(o_ids, ref_ids[sample]))
        cpu_model = None
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
        except OSError:
            pass
        cpu = {"value": round(len(sample) / q_cpu, 2), "unit": "queries/s", "cores": nthreads,
               "kind": "oracle", "cpu_model": cpu_model, "host_threads": os.cpu_count(),
               "sample": f"{len(sample)} of {wl.Q} queries against the full {wl.n}-point index; "
                         f"oracle index build {build_cpu:.1f}s excluded, query phase {q_cpu:.2f}s",
               "matches_gpu": cpu_match}
        log(f"[bench] oracle: {cpu['value']} q/s on {nthreads} threads (build {build_cpu:.1f}s)")

    # ---- collision counting with a candidate cap (Section 3, "Collision Counting") on an index of
    # 64 layers over the same data and queries: the points sharing the query's
    # bucket in at least theta layers, ranked by (count desc, id asc), K + v of
    # them verified; beside it the plain union on that index.  Its kernel's
    # algorithmic bytes: the listed ids (4 each), the verified rows, the query
    # rows and the K output pairs.
    counting = None
    count_theta = args.count_theta if args.count_theta is not None else (3 if args.config == 2 else 0)
    if count_theta > 0:
        cL, cw = 64, 2.5 * spec["w"]
        cp = synth.hash_params(2100 + args.config, cL, wl.params.k, wl.d, cw)
        cix = lib.Index(data_d, torch.from_numpy(cp.a).to(dev), torch.from_numpy(cp.b()).to(dev),
                        cw, form=lib.QW_FORM_FAST)
        try:
            cix.set_counting(count_theta, args.count_v)
            max_listed = int(cix.bucket_sizes(q_d).to(torch.int64).sum(1).max())
            copts = lib.make_opts(form=lib.QW_FORM_FAST, graph=0)
            c_ids, c_dist, cst = cix.query(q_d, K, copts, stats=True)
            c_ids, c_dist = c_ids.cpu().numpy(), c_dist.cpu().numpy()
            crec = recall_at_10(c_ids[rsel], truth[0], c_dist[rsel], truth[1])
            p_ids, p_dist = cix.query(q_d, K, lib.make_opts(form=lib.QW_FORM_PLAIN_FP32))
            c_same = bool(np.array_equal(p_ids.cpu().numpy(), c_ids) and
                          np.array_equal(p_dist.cpu().numpy(), c_dist))
            cms = timed(copts, args.steps, args.warmup, cix)
            kms_c = 0.0
            for _ in range(nrep):
                _, _, cs = cix.query(q_d, K, lib.make_opts(timing=1, graph=0), out_ids=out_ids,
                                     out_dist=out_dist, stats=True)
                kms_c += cs["ms_stage"][3] / nrep
            cbytes = (4 * cst["cand_total"] + cst["cand_unique"] * wl.d * elem + wl.Q * wl.d * elem
                      + 8 * K * wl.Q)
            cix.set_counting(0)
            u_ids, u_dist, ust = cix.query(q_d, K, fast_opts, stats=True)
            urec = recall_at_10(u_ids.cpu().numpy()[rsel], truth[0], u_dist.cpu().numpy()[rsel],
                                truth[1])
            ums = timed(fast_opts, args.steps, args.warmup, cix)
            cach = cbytes / (kms_c * 1e-3) / 1e9 if kms_c > 0 else None
            counting = {
                "index": {"L": cL, "k": wl.params.k, "w": cw}, "theta": count_theta,
                "v": args.count_v, "qps": round(wl.Q / (cms * 1e-3), 1),
                "ms_per_step": round(cms, 4), "recall_at_10": round(crec, 4),
                "verified_per_query": cst["cand_unique"] / wl.Q,
                "listed_per_query": cst["cand_total"] / wl.Q, "max_listed": max_listed,
                "forms_identical": c_same,
                "kernel": {"name": "count_kernel", "ms": round(kms_c, 4),
                           "algorithmic_bytes": int(cbytes),
                           "achieved_gbs": round(cach, 1) if cach else None,
                           "frac": round(cach / HBM_PEAK_GBS, 4) if cach else None},
                "union_same_index": {"qps": round(wl.Q / (ums * 1e-3), 1),
                                     "recall_at_10": round(urec, 4),
                                     "unique_per_query": ust["cand_unique"] / wl.Q},
            }
            log(f"[bench] counting theta={count_theta} v={args.count_v}: {cms:.3f} ms/step, "
                f"recall {crec:.4f}, kernel {kms_c:.3f} ms; union on that index {ums:.3f} ms, "
                f"recall {urec:.4f}")
        except lib.QwError as e:
            counting = {"error": str(e)}
        cix.close()

    # hashing (A1-A2): algorithmic projection flops against the dense MFMA peak
    # of the type the kernel multiplies in (FP16 for uint8 data, FP32 for float)
    hash_flops = 2.0 * wl.d * L * wl.params.k * wl.Q
    hash_peak = MFMA_PEAK_FP16_TFLOPS if is_u8 else MFMA_PEAK_FP32_TFLOPS
    hash_tflops = hash_flops / (stage[0] * 1e-3) / 1e12 if stage[0] > 0 else None
    hash_info = {"kernel": "hash_mfma_f16_kernel" if is_u8 else "hash_mfma_f32_kernel",
                 "ms": round(float(stage[0]), 4),
                 "algorithmic_tflops": round(hash_tflops, 2) if hash_tflops else None,
                 "peak_tflops": hash_peak,
                 "frac": round(hash_tflops / hash_peak, 5) if hash_tflops else None,
                 "index_build_s": round(build_s, 3)}

    qps = wl.Q / (ms_fast * 1e-3)
    line = {
        "metric": METRIC,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_fast, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8" if is_u8 else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"cfg{args.config}: n={wl.n} d={wl.d} {'u8' if is_u8 else 'f32'}, "
                         f"Q={wl.Q} queries, L={L} k={wl.params.k} w={w} (w_0.9), K={K}"
                         + ({0: "", 1: ", one-step neighbour buckets probed",
                             2: f", {args.probe_t} query-directed neighbour probes per layer"}[args.probes])),
            "n": wl.n, "d": wl.d, "Q": wl.Q, "L": L, "k": wl.params.k, "w": w, "K": K,
            "projection": "fp16-mfma+fp64-guard" if is_u8 else "fp32-mfma+fp64-guard",
            "bucket_grouping": "automatic (rows of 1024 bytes or more, or 32768 queries or more)",
            "neighbour_probing": {0: None, 1: "all one-step", 2: f"query-directed, {args.probe_t} per layer"}[args.probes],
            "w_search": tried,
        },
        "recall_at_10": round(rec, 4),
        "plain_fp32_qps": round(wl.Q / (ms_plain * 1e-3), 1),
        "speedup_vs_plain_fp32": round(ms_plain / ms_fast, 3),
        "forms_identical": identical,
        "sched_ms_per_step": sched_ms,
        "sched_identical": sched_identical,
        "collision_counting": counting,
        "stage_ms": {"hash": round(stage[0], 4), "probe": round(stage[1], 4),
                     "schedule": round(stage[2], 4), "dedup": round(stage[6], 4),
                     "select": round(stage[7], 4),
                     "candidates_verify_topk": round(stage[3], 4),
                     "fallback": round(stage[4], 4), "total": round(stage[5], 4)},
        "recompute_frac": st["recompute_frac"],
        "cand_per_query": {"sum_of_buckets": st["cand_total"] / wl.Q,
                           "unique": st["cand_unique"] / wl.Q},
        "overflow_queries": st["overflow"],
        "fallback_queries": st["fallback"],
        "topk_second_pass_queries": st["topk_second_pass"],
        "count_model": count_model,
        "bins": st["bins"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": traffic, "kernel": kname,
                     "measured_copy_gbs": round(copy_gbs, 1),
                     "frac_of_measured_copy": round(achieved / copy_gbs, 4) if achieved else None,
                     # HBM bytes the counters saw over the same kernel time
                     "traffic_achieved": round(traffic / (kms * 1e-3) / 1e9, 1) if traffic and kms > 0 else None,
                     "traffic_frac": round(traffic / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic and kms > 0 else None,
                     "kernel_ms": round(kms, 4),
                     "kernel_algorithmic_bytes": int(kbytes),
                     "path_algorithmic_bytes_per_step": int(alg_bytes)},
        "hash_mfma": hash_info,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ix.close()


if __name__ == "__main__":
    main()
