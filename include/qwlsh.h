/*
 * qwlsh.h -- C ABI of the MI355X (gfx950) engine for p-stable LSH query
 * workloads.
 *
 * The engine answers a whole workload of Q similarity queries against an index
 * of L hash layers, each keyed by k concatenated p-stable functions
 *     h_{a,b}(v) = floor((a.v + b) / w)                  (Section 3; the floor is
 *                                                          that of the cited
 *                                                          scheme of Datar et al.)
 * combined conjunctively inside a layer and disjunctively across layers
 * (Section 1.1).  Per query it projects and hashes, probes every layer's bucket,
 * forms the de-duplicated union of the bucket members (the candidates found by
 * accessing the index, Section 1.2), removes false positives by exact distance
 * and returns the top-K (the c-k-ANN output of Section 3).  The workload is
 * processed as a whole (Sections 4 and 5.1): queries whose candidate sets
 * overlap are scheduled together so shared ids and points are fetched once and
 * reused from cache.  Optionally every layer also probes the neighbouring
 * buckets (qw_set_probing), or the union gives way to collision counting with
 * a cap on the verified points (qw_set_counting).
 *
 * Conventions for every entry point:
 *  - Pointers documented "device" must point to memory of the current HIP
 *    device; "host" pointers to host memory.  No pointer may be NULL unless
 *    documented "nullable".
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *    enqueued on it; unless documented otherwise, calls return before the GPU
 *    finishes and outputs are valid once the stream reaches that point.
 *  - Errors are returned as qw_status; on error, output buffers are left
 *    untouched and no work is enqueued.  No C++ exception crosses the ABI.
 *  - An index is not thread-safe: calls on one index must be serialised by the
 *    caller.  Distinct indexes may be used concurrently.
 *  - Vectors are row-major, dtype QW_U8 (uint8) or QW_F32 (float32).
 *  - Distances are SQUARED Euclidean: int32 exact for QW_U8 data, float32 for
 *    QW_F32 data (the float64 distance of the index-order sum, rounded once).
 *  - Results are sorted by (distance ascending, id ascending); rows with fewer
 *    than K candidates are padded with id -1 and distance INT32_MAX (QW_U8) or
 *    +infinity (QW_F32).
 */
#ifndef QWLSH_H
#define QWLSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QW_OK = 0,
    QW_EINVAL = 1,        /* invalid argument (null pointer, bad size, out-of-range value) */
    QW_ENOMEM = 2,        /* device or host allocation failed */
    QW_EDEVICE = 3,       /* a HIP runtime call failed */
    QW_EUNSUPPORTED = 4,  /* valid request the engine cannot serve (e.g. keys wider than 128 bits) */
    QW_EINTERNAL = 5      /* internal invariant violated */
} qw_status;

typedef enum { QW_U8 = 0, QW_F32 = 1 } qw_dtype;

/* Execution form.  Both forms return identical results. */
typedef enum {
    /* FP32 projections (guard band + FP64 recompute keeps bucket ids exact), one
     * workgroup per query in workload order, one hash-set size for the whole
     * workload. */
    QW_FORM_PLAIN_FP32 = 0,
    /* FP16 (uint8 data) or FP32 (float data) MFMA projections with an FP64 guard
     * band; queries binned by predicted candidate count (and, with grouping,
     * ordered by a min-hash of their candidate sets) into persistent
     * dedup-and-verify kernels that also select the
     * top K (uint8 rows of at most 1024 bytes, K <= 16; otherwise a per-query
     * select kernel does); replayed from a HIP graph. */
    QW_FORM_FAST = 1
} qw_form;

/* Where the fast form takes each query's predicted candidate count from. */
typedef enum {
    QW_SCHED_SUM = 0,     /* sum of the query's bucket sizes (an upper bound, never overflows) */
    QW_SCHED_LEARNED = 1, /* the count model (qw_train_count_model / qw_set_count_model) */
    QW_SCHED_ACTUAL = 2,  /* an extra counting pass gives the exact count */
    QW_SCHED_NONE = 3     /* no binning: one hash-set size for the whole workload */
} qw_sched;

typedef struct {
    int32_t form;      /* qw_form */
    int32_t sched;     /* qw_sched (fast form only) */
    int32_t group;     /* fast form: 1 = order queries within a size class by a min-hash of
                          their candidate sets (the minimum over their buckets of each
                          bucket's smallest mixed id) and deal the order to the XCDs in
                          chunks, so queries with overlapping candidates share an L2,
                          0 = no bucket ordering, -1 = automatic (default): ordering for
                          rows of 1024 bytes or more or workloads of 32768 queries or
                          more, where neighbouring queries share the rows they verify
                          in cache */
    int32_t graph;     /* fast form: 1 = capture/replay the query pipeline as a HIP graph */
    int32_t timing;    /* 1 = record per-stage HIP events and report them in qw_stats (syncs) */
    int32_t topk_keep; /* fast form, uint8 rows of at most 1024 bytes, K <= 16: the dedup kernel
                          selects the top K itself, each lane keeping this many of its
                          candidates' keys (1..3; 0 = all it keeps: 3 in the workgroup
                          kernel, 4 in the wave kernel); a query whose top K that cannot
                          settle takes a second pass or the fallback, so smaller values
                          only send more queries there (diagnostic).  -1 = a separate
                          select kernel. */
    int32_t dedup;     /* fast form, uint8 rows of at most 1024 bytes, K <= 16, at most 64
                          bucket lists per query: 0 = automatic (the tuned choice when
                          tune_cache holds one for this workload, else the wave kernel
                          when a query's expected bucket entries fit one set of the wave
                          kernel), 1 = one workgroup per query in size-class launches,
                          2 = one wave per query (a fixed on-chip set per wave, larger
                          candidate sets in id-hash passes); ignored elsewhere */
    int32_t xchunk;    /* fast form with bucket grouping: consecutive items of the grouped
                          order dealt to one XCD (1..256; 0 = the tuned value or 256) */
    int32_t stage_split; /* fast form: the staged candidate kernel, the GPU form of the
                          split of Sections 4-5 of a fixed cache between index files (C_I)
                          and data objects (C_D).  s in 1..99: each workgroup takes runs of
                          16 consecutive queries of the schedule's order and keeps in its
                          80 KiB of LDS, beside a 32 KiB hash set, a cache of bucket id lists
                          (s % of the rest, lists of at most 32 ids) and a cache of candidate
                          rows (100 - s %), direct-mapped, across the run; a list or row found
                          there is not read from memory.  Keys go to the select kernel; a
                          query of more than 6144 bucket entries goes to the fallback.
                          Needs at most 64 lists per query and rows of at most 4 KiB
                          (QW_EUNSUPPORTED otherwise).  -1 = off (the other kernels), 0 =
                          automatic (the tuned choice when tune_cache holds one, else off).
                          Results are identical for every value. */
    const char *tune_cache; /* nullable: JSON file written by qw_autotune; automatic settings
                               (dedup 0, xchunk 0, group -1) take its entry for this
                               workload, when it has one */
} qw_opts;

/* Filled (host memory) by qw_query_workload when non-NULL; the call then
 * synchronises `stream` before returning. */
typedef struct {
    int64_t projections;   /* (query, function) projections computed */
    int64_t recomputed;    /* of which recomputed in FP64 inside the guard band */
    double recompute_frac; /* recomputed / projections */
    int64_t probes_hit;    /* (query, layer) probes that found a bucket */
    int64_t cand_total;    /* sum over queries and layers of the bucket sizes */
    int64_t cand_unique;   /* sum over queries of |C(q)| */
    int64_t overflow;      /* queries moved to a larger hash set because theirs was sized too small */
    int64_t fallback;      /* fast form: queries answered by the fused per-query path */
    int64_t topk_second_pass; /* fast form, in-kernel top K: queries whose lanes' kept keys did
                                 not settle the top K, selected by a second verify pass */
    int64_t bins[8];       /* queries per hash-set size class (fast form) */
    float ms_stage[8];     /* timing=1: hash, probe, schedule, candidates+verify+top-K,
                              fallback, total, dedup + verify (fast form; with the top K where
                              the kernel selects it), select kernel (fast form) */
    int32_t dedup_used;    /* fast form: the settings the call ran with (automatic ones
                              resolved): dedup kernel (1 or 2), */
    int32_t group_used;    /* bucket grouping (0 or 1), */
    int32_t xchunk_used;   /* XCD chunk (0 without grouping), */
    int32_t tuned;         /* 1 when the tuning cache supplied an automatic setting; all five
                              are 0 in the plain form and under collision counting */
    int32_t split_used;    /* staging split (-1 off, else the index share in percent) */
    /* out-of-core mode (qw_set_out_of_core), this call's reads from host memory: */
    int64_t ooc_index_files;   /* index files (bucket id lists) read into the index cache */
    int64_t ooc_index_bytes;   /* their bytes (4 per id) */
    int64_t ooc_data_objects;  /* data objects (rows) read into the data cache */
    int64_t ooc_data_bytes;    /* their bytes (row_bytes each, the padded row) */
    int64_t ooc_batches;       /* batches answered */
    int64_t ooc_splits;        /* batches that did not fit the cache and were halved */
} qw_stats;

typedef struct {
    int64_t n;
    int32_t d, dtype, L, k;
    float w;
    int32_t key_bits[64];  /* packed key width of each layer (first min(L,64) layers) */
    int64_t buckets;       /* total buckets over all layers */
    int64_t max_bucket;    /* largest bucket size */
    int64_t device_bytes;  /* device memory held by the index */
    int32_t has_count_model;
    float count_margin;    /* log-space margin added to the model's prediction when sizing sets */
    int32_t probing;       /* qw_set_probing mode (0: the query's own bucket per layer) */
    int32_t probes_per_layer; /* neighbour buckets probed per layer (0 without probing) */
    int32_t count_threshold;  /* qw_set_counting threshold (0: plain union) */
    int32_t count_extra;      /* qw_set_counting extra (v) */
    double mean_hit_bucket;   /* mean over layers of sum_b s_b^2 / n: the expected size of the
                                 bucket a data point falls in */
    int32_t out_of_core;      /* 1 while qw_set_out_of_core is on */
    int32_t ooc_index_percent;  /* its index share (0 in core) */
    int64_t host_bytes;       /* pinned host memory held (the out-of-core lists and rows) */
} qw_index_info;

typedef struct qw_index qw_index;

/* Default options: fast form, learned schedule when a model is loaded (else
 * the bucket-size sum), automatic grouping, graph on, timing off, in-kernel top K
 * where it applies (topk_keep 0). */
void qw_default_opts(qw_opts *o);

/*
 * Build the index (Sections 1.1 and 3: L layers of k p-stable functions).
 *  data  device, n x d row-major, dtype `dtype`; copied into the index, so the
 *        caller may free it after the call returns.
 *  a     device, float32 [L][k][d]: the projection vectors a_{l,j}.
 *  b     device, float32 [L][k]: offsets b_{l,j}, expected in [0, w).
 *  w     bucket width, finite and > 0.
 *  o     nullable; selects the projection form used to hash the data (results
 *        are identical either way).
 *  out   host; receives the new index (owned by the library; free with
 *        qw_free_index).
 * Limits: 1 <= n <= 2^31-1, 1 <= d <= 8192, 1 <= L <= 64, 1 <= k <= 32.
 * Errors: QW_EINVAL on bad arguments or when |a.v + b| / w can exceed 2^30
 * (hash values would leave int32); QW_EUNSUPPORTED when a layer's packed key
 * needs more than 128 bits; QW_ENOMEM; QW_EDEVICE.
 * Synchronises `stream` before returning.
 */
qw_status qw_build_index(const void *data, int64_t n, int32_t d, int32_t dtype,
                         const float *a, const float *b, float w, int32_t L, int32_t k,
                         const qw_opts *o, void *stream, qw_index **out);

/*
 * Answer a query workload: for each of the Q queries, the K nearest candidates.
 *  queries   device, Q x d row-major, same dtype as the data.
 *  K         1 <= K <= 1024.
 *  o         nullable (defaults of qw_default_opts).
 *  out_ids   device int32 [Q][K].
 *  out_dist  device [Q][K]: int32 (QW_U8) or float32 (QW_F32).
 *  st        host, nullable.
 * Q = 0 is valid and does nothing.  Workspace is owned by the index and grown
 * on demand (the first call at a new size allocates).
 */
qw_status qw_query_workload(qw_index *ix, const void *queries, int64_t Q, int32_t K,
                            const qw_opts *o, void *stream, int32_t *out_ids, void *out_dist,
                            qw_stats *st);

/*
 * The plain form's query workload without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * output conventions as qw_query_workload with o->form = QW_FORM_PLAIN_FP32
 * (or collision counting when qw_set_counting is active); no options, no
 * statistics.
 * Every workspace buffer (query hashes, bucket ranges, counters, the padded
 * query copy when d is not a multiple of 16 or `queries` is not 16-byte
 * aligned, the query-directed probing moves) comes from one static
 * device array of 32 MiB per GPU, held until the process ends.  The call
 * allocates nothing -- no hipMalloc, no hipFree -- and grows no buffer of the
 * index.  Limits: the workspace of Q queries, about
 * Q * (4*L*k + 8*lists + 8 [+ 4*L with probing] [+ T*L with
 * query-directed probing] [+ 8 with collision counting] [+ d*elem when
 * padded]) bytes plus alignment, must
 * fit 32 MiB, and each query's hash set must fit on-chip memory; otherwise
 * QW_EUNSUPPORTED, with the outputs untouched.
 * Every call on one GPU shares that GPU's array and overwrites it: calls that
 * overlap on one GPU (other streams, other threads, other indexes) race and
 * must be serialised by the caller.  Synchronises `stream` once (the hash-set
 * size is read back from the device).
 */
qw_status qw_query_workload_noalloc(qw_index *ix, const void *queries, int64_t Q, int32_t K,
                                    void *stream, int32_t *out_ids, void *out_dist);

/* Outcome of qw_autotune (host). */
typedef struct {
    int32_t dedup, group, xchunk; /* the fastest setting, explicit values (qw_opts meaning) */
    int32_t stage_split;          /* -1 (off) or the index share in percent */
    float ms;                     /* its time per call (graph replay, mean of 5) */
    float ms_default;             /* the built-in automatic setting's time per call */
    int32_t candidates;           /* settings timed */
} qw_tune_result;

/*
 * Tune the fast form's scheduling settings for one workload and record the
 * fastest in a JSON cache.  The cost-model role of Section 5 (Cost Models and
 * Workflow of qwLSH: a split chosen offline from the data's shape and then
 * applied to every workload of that shape), with measured times in place of
 * a trained model.  Each candidate setting -- the dedup kernel (qw_opts.dedup
 * 1, or 2 where the wave kernel applies), bucket grouping off, or on with an
 * XCD chunk of 16, 64 or 256 -- answers `queries` (device, Q x d) for K
 * neighbours: two warm-up calls, then five timed graph replays on `stream`.
 * All settings return the same ids and distances; a candidate whose outputs
 * differ from the built-in automatic setting's is a library bug and gives
 * QW_EINTERNAL.  Where the staged kernel applies (qw_opts.stage_split), the
 * fastest of them is then timed at splits of 1, 10, 50, 90 and 99 %, and a
 * split that beats it is kept.  `base` (nullable) supplies the remaining
 * options (form must be QW_FORM_FAST; its schedule is part of the cache key).
 *  cache_path  host string: the JSON file, created or updated in place (one
 *              entry per line, keyed by the GPU architecture, e.g. gfx950, and
 *              a hash of n, d, dtype, L, k, w, the probing, Q, K, the schedule
 *              and whether a count model is set).  A call whose
 *              qw_opts.tune_cache names this file takes the entry for its
 *              workload wherever its own settings are automatic.
 *  out         host; the chosen setting and times.
 * Allocates two output buffers of Q*K*4 bytes each and the workspace of the
 * candidates' graphs; synchronises `stream`.  Errors: QW_EINVAL (bad
 * arguments, collision counting active, another device current, or the file
 * cannot be written), QW_ENOMEM, QW_EDEVICE, QW_EINTERNAL as above.
 */
qw_status qw_autotune(qw_index *ix, const void *queries, int64_t Q, int32_t K,
                      const qw_opts *base, const char *cache_path, void *stream,
                      qw_tune_result *out);

/* Release the index and all device memory it holds (NULL is a no-op). */
void qw_free_index(qw_index *ix);

/* Static string naming a status code. */
const char *qw_status_string(qw_status s);

/* Index description (host `info`). */
qw_status qw_get_index_info(const qw_index *ix, qw_index_info *info);

/* ---- introspection (tests and measurements; same ownership rules) ---------- */

/*
 * Hash values of m vectors: out_h device int32 [m][L*k], function order
 * (layer, function).  `form` selects the projection path (qw_form).
 * out_recomputed: host, nullable; receives the number of guard-band recomputes
 * (the call then synchronises `stream`).
 */
qw_status qw_hash(qw_index *ix, const void *x, int64_t m, int32_t form, void *stream,
                  int32_t *out_h, int64_t *out_recomputed);

/* Bucket size of each (query, layer): out_sizes device int32 [Q][L] (0 = miss);
 * with neighbour probing (qw_set_probing) the sum over the layer's probed
 * buckets. */
qw_status qw_bucket_sizes(qw_index *ix, const void *queries, int64_t Q, void *stream,
                          int32_t *out_sizes);

/* |C(q)| of each query: out_counts device int32 [Q]. */
qw_status qw_candidate_counts(qw_index *ix, const void *queries, int64_t Q, void *stream,
                              int32_t *out_counts);

/*
 * Candidate ids of each query, in unspecified order within a query: offsets
 * device int64 [Q+1] (exclusive prefix sums of qw_candidate_counts), out_ids
 * device int32 [offsets[Q]].
 */
qw_status qw_candidate_lists(qw_index *ix, const void *queries, int64_t Q,
                             const int64_t *offsets, void *stream, int32_t *out_ids);

/*
 * Exact kNN of Q queries (device, Q x d) over all n indexed points -- the c-k-ANN
 * problem with every point a candidate (Section 3); the recall ground truth.
 * Same output conventions as qw_query_workload; 1 <= K <= 1024.
 */
qw_status qw_bruteforce_knn(qw_index *ix, const void *queries, int64_t Q, int32_t K,
                            void *stream, int32_t *out_ids, void *out_dist);

/* ---- candidate-count model (steers scheduling only, never results) --------
 *
 * A two-layer perceptron y = W2 relu(W1 f + b1) + b2 over f_l = log(1 + s_l)
 * (s_l = the query's bucket size in layer l) predicting log(1 + |C(q)|).  It
 * plays the part of the paper's offline-trained model that sets resources
 * from data characteristics (Sections 5.2-5.3).  Parameters are packed float32:
 * W1 [H][L], b1 [H], W2 [H], b2 [1]  (H*L + 2H + 1 values, H = 64).
 */
#define QW_MLP_HIDDEN 64

/* Number of packed parameters for L inputs. */
int32_t qw_mlp_param_count(int32_t L);

/*
 * Loss and gradient of one minibatch (mean squared error), FP32 on the GPU.
 *  params device [P]; feats device float32 [B][L]; targets device float32 [B];
 *  grad device [P] (overwritten); loss device float32 [1] (overwritten).
 */
qw_status qw_mlp_loss_grad(const float *params, int32_t L, const float *feats,
                           const float *targets, int32_t B, void *stream,
                           float *grad, float *loss);

/* One Adam step (bias-corrected, step >= 1) on device params / moments m, v. */
qw_status qw_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t P,
                      int32_t step, float lr, float beta1, float beta2, float eps,
                      void *stream);

/* BF16 inference: out device float32 [B] = predicted log(1 + |C(q)|). */
qw_status qw_mlp_predict_bf16(const float *params, int32_t L, const float *feats, int32_t B,
                              void *stream, float *out);

/*
 * Train the index's count model on m training queries (device, m x d): the
 * engine computes features (bucket sizes) and labels (exact |C(q)|) itself and
 * runs `epochs` passes of minibatch Adam.  It then calibrates the sizing
 * margin: the 99.5th percentile of log(1 + |C(q)|) minus the prediction over
 * the training queries (at least 0.05), so that about 1 query in 200 outgrows
 * the set chosen for it.  final_loss: host, nullable.  Synchronises `stream`.
 */
qw_status qw_train_count_model(qw_index *ix, const void *train_queries, int64_t m,
                               int32_t epochs, int32_t batch, float lr, uint64_t seed,
                               void *stream, float *final_loss);

/* Install / read the count model parameters (host float32 [P]).  Installing
 * resets the sizing margin to log(1.25). */
qw_status qw_set_count_model(qw_index *ix, const float *params, int32_t P);
qw_status qw_get_count_model(const qw_index *ix, float *params, int32_t P);

/* Sizing margin: a set is sized for expm1(prediction + margin) + 32 ids
 * (finite, -4 <= margin <= 8; QW_EINVAL otherwise). */
qw_status qw_set_count_margin(qw_index *ix, float margin);

/*
 * Neighbour probing: the multi-probe variant that Section 2 summarises
 * (look into the buckets next to the query's bucket instead of adding
 * layers).
 *  mode 0 (default): each layer contributes the query's own bucket;
 *  mode 1: each layer also contributes the 2k buckets whose k-tuple differs
 *          from the query's in exactly one coordinate by -1 or +1, so
 *          C(q) = { p : exists l, key_l(p) - key_l(q) in {0, -e_j, +e_j} };
 *  mode 2: query-directed (Lv et al.'s ordering): only the per_layer
 *          (1 <= per_layer <= 2k) of those moves with the smallest scores,
 *          where with y_j = (a_j.q + b_j) / w (the hashing's FP64 sequence)
 *          and f_j = y_j - floor(y_j) moving coordinate j by -1 scores
 *          f_j * f_j and by +1 scores (1 - f_j) * (1 - f_j), each operation
 *          rounded in FP64, ties to the smaller j, then to -1.  The GPU
 *          computes these projections in FP64 for the queries.
 * per_layer is ignored for modes 0 and 1.
 * Every later call on the index (queries, candidate counts and lists, bucket
 * sizes -- then the sum over each layer's probed buckets -- and count-model
 * training) uses the mode.  Changing it drops captured graphs and the count
 * model, which was fitted to the other candidate sets.  Needs
 * L * (1 + probes per layer) <= 1024 lists per query (QW_EUNSUPPORTED
 * otherwise); QW_EINVAL for another mode or per_layer out of range.  Not to be
 * called while work on the index is in flight.
 */
qw_status qw_set_probing(qw_index *ix, int32_t mode, int32_t per_layer);

/*
 * Collision counting with a candidate cap (Section 3, "Collision Counting", after C2LSH: the
 * number of layers in which a point shares the query's bucket is counted, a
 * threshold on that count replaces the plain union, and at most k + v points
 * -- the K results plus v allowed false positives -- are verified).
 *  threshold 0 (default): the plain union of Section 1.2;
 *  threshold t in 1..L: #Col(p) = #{ l : key_l(p) == key_l(q) }; the points
 *      with #Col(p) >= t, ranked by (#Col descending, id ascending), are
 *      verified up to the first K + extra of them, and the top K of those by
 *      (distance, id) is returned (padded as on the plain path).  A layer of
 *      one function (k = 1) is C2LSH's single collision test.
 * extra >= 0 is v.  qw_query_workload then answers with both forms (the form
 * only chooses the hashing) through one kernel that holds a query's counts in
 * LDS; it needs neighbour probing off, n < 2^25 - 1, K + extra <= 1024 and at most 12288
 * listed ids (the sum of a query's L bucket sizes) per query, else it returns
 * QW_EUNSUPPORTED with the outputs untouched (the check synchronises the
 * stream).  qw_stats then reports the verified points as cand_unique.
 * QW_EINVAL for a threshold outside 0..L or an extra outside 0..1024.  Not to be
 * called while work on the index is in flight.
 */
qw_status qw_set_counting(qw_index *ix, int32_t threshold, int32_t extra);

/* ---- out-of-core mode -------------------------------------------------------
 *
 * Section 1.2 and Section 4: the index files and the data objects sit on
 * external storage, and a cache C = C_I + C_D in memory holds some of them, C_I
 * index files and C_D data objects.  Section 5.1: each part evicts by MRU, and
 * C_I is either divided equally among the hash functions' layers (Strategy 1)
 * or shared by all of them (Strategy 2).
 * Here host memory is the storage and HBM is the cache.  An index file is one
 * bucket's id list (4 bytes per id).  A data object is one point's padded
 * row (dp elements).  The probe tables and hash parameters stay in HBM.
 *
 * The workload is answered in batches of consecutive queries.  Each batch:
 *  1. reads its missing bucket lists into C_I;
 *  2. reads its candidates' missing rows into C_D;
 *  3. runs the plain form's union, verification and top-K from HBM alone.
 * Eviction and IO counting follow the reading stated in the oracle's cache
 * model; a batch of one query is the paper's query-at-a-time setting.
 *  - An item's recency is its last use.  Query q uses its layer-l bucket at
 *    q*L + l + 1, and a row of C(q) at q + 1; rows used last by the same query
 *    are ordered by id.
 *  - A batch evicts, outside its own needs, the most recently used items
 *    first (QW_OOC_LRU: least recently used first), until its misses fit.
 *  - A batch that does not fit is answered as two halves.
 * Results are those of the in-core index (bit for bit).
 */
typedef enum { QW_OOC_MRU = 0, QW_OOC_LRU = 1 } qw_ooc_policy;

typedef struct {
    int64_t cache_bytes;    /* C, HBM bytes of the two caches; C_I = C * index_percent / 100
                               (floor) holds floor(C_I / 4) ids, C_D = C - C_I holds
                               floor(C_D / row_bytes) rows */
    int32_t index_percent;  /* C_I's share, 1..99 */
    int32_t strategy;       /* 1: C_I split equally among the L layers (floor(ids / L) ids
                               each); 2: one C_I for all layers */
    int32_t policy;         /* qw_ooc_policy */
    int32_t batch;          /* queries per batch, >= 1 */
    int32_t keep;           /* 0: every qw_query_workload call starts with empty caches (a
                               workload on its own, as the paper measures); 1: the caches
                               persist across calls, and a call's queries count as used
                               after the previous call's */
    int32_t reserved;       /* 0 */
} qw_ooc_opts;

/*
 * Move the index's CSR ids ([L][n] int32) and data rows ([n][dp]) to pinned
 * host memory, free their HBM copies, and give HBM to the two caches.
 *  o       host; NULL moves everything back to HBM and frees the caches.
 *  stream  used for the copies; synchronised before returning.
 * Calling it again with new options keeps the host copies and rebuilds the
 * caches empty.
 *
 * While the mode is on:
 *  - qw_query_workload answers through the caches, whichever form it names:
 *    the form's hashing, then the plain form's per-query kernel.  The
 *    statistics' ooc_* fields count the reads.
 *  - qw_hash and qw_bucket_sizes work as before.
 *  - QW_EUNSUPPORTED from the calls that would read the data or the lists
 *    outside the caches: qw_query_workload_noalloc, qw_candidate_counts,
 *    qw_candidate_lists, qw_bruteforce_knn, qw_train_count_model and
 *    qw_autotune; also from qw_set_probing / qw_set_counting with a mode
 *    other than off, and from qw_opts.stage_split > 0.
 *
 * Errors:
 *  - QW_EINVAL on bad options;
 *  - QW_EUNSUPPORTED when probing or counting is on, or when C_I exceeds
 *    2^31 - 1 ids;
 *  - QW_ENOMEM when the caches or the pinned host copies cannot be allocated.
 *    The index is then left as it was.
 * A query workload returns QW_EUNSUPPORTED when one query's bucket lists or
 * candidate rows do not fit their cache, or when its hash set does not fit
 * on-chip memory.  The outputs of the queries before it are written; the rest
 * are unspecified.
 */
qw_status qw_set_out_of_core(qw_index *ix, const qw_ooc_opts *o, void *stream);

/* Outcome of qw_autotune_ooc (host). */
typedef struct {
    int32_t index_percent;     /* the fastest share; the index is left out of core at it */
    int32_t shares;            /* shares timed: 11 */
    int32_t percent[11];       /* 1, 10, 20, ..., 90, 99 */
    float ms[11];              /* one cold workload pass; -1: the share cannot hold one query */
    int64_t index_bytes[11];   /* bytes of index files read from host memory */
    int64_t data_bytes[11];    /* bytes of data objects read from host memory */
    int64_t batches[11];       /* batches answered */
    int64_t splits[11];        /* batches halved */
} qw_ooc_tune_result;

/*
 * Choose the index share of the out-of-core cache by measurement.  The paper
 * evaluates its split against the best of eleven settings of C_I (1, 10, 20,
 * ..., 90, 99 %, Section 6) and predicts it offline from the data's size and
 * dimensionality (Sections 5.2 and 5.3).  Here each setting is timed on the
 * workload itself.
 *  queries  device, Q x d (the workload, or a sample of it).
 *  K        1 <= K <= 1024.
 *  base     host; the cache size, strategy, policy and batch to keep.  The
 *           index share is ignored; keep applies to the final setting, and
 *           every timed pass starts with empty caches.
 *  out      host; every share's time and reads, and the fastest.
 * Each share answers the workload once, cold (qw_set_out_of_core, then
 * qw_query_workload), with the default query options.  The outputs of every
 * share that fits must be identical; otherwise QW_EINTERNAL.  The index is
 * then left out of core at the fastest share.  It may be in core or out of
 * core on entry.
 * Allocates two output buffers of Q*K*4 bytes and synchronises `stream`.
 * Errors:
 *  - QW_EINVAL on bad arguments;
 *  - QW_EUNSUPPORTED when probing or counting is on, or when no share can
 *    hold one query;
 *  - QW_ENOMEM.
 * After an error the index may be left out of core at one of the shares.
 */
qw_status qw_autotune_ooc(qw_index *ix, const void *queries, int64_t Q, int32_t K,
                          const qw_ooc_opts *base, void *stream, qw_ooc_tune_result *out);

#ifdef __cplusplus
}
#endif

#endif /* QWLSH_H */
