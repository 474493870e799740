/*
 * CPU oracle for p-stable LSH query-workload processing.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may build, load or call this file.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * What it computes, step by step, in the paper's order (the paper builds on
 * E2LSH-style layered hashing, Sections 1.1 and 3):
 *
 *  1. Hash functions (Section 3, the p-stable hash of Datar et al.):
 *       h_{a,b}(v) = floor((a.v + b) / w)
 *     The paper prints the quotient without the floor; the floor is the cited
 *     scheme's definition.  Evaluation order is fixed:
 *       acc = 0.0 (double); for i = 0..d-1: acc = acc + (double)a[i]*(double)v[i];
 *       t = acc + (double)b; y = t / (double)w; h = floor(y).
 *     Each product of a float32 and a uint8 (or of two float32 values) is exact
 *     in double, so this sequence does not depend on FMA contraction; the file is
 *     still compiled with -ffp-contract=off.
 *  2. Layers (Section 1.1: several layers of independently chosen functions,
 *     combined conjunctively inside a layer and disjunctively across layers):
 *     layer l's key of v is the k-tuple (h_{l,0}(v), ..., h_{l,k-1}(v)); two
 *     points share a bucket of layer l iff their tuples are equal.
 *  3. Index: per layer, the point ids sorted by (tuple, id); a bucket is a run
 *     of equal tuples.
 *  4. Candidates of query q (Section 1.2 / 5.1: the index yields candidate ids):
 *     C(q) = { p : exists l with key_l(p) == key_l(q) }, as a set.
 *     With neighbour probing (the multi-probe variant of Lv et al. that
 *     Section 2 summarises: look into the buckets next to the query's bucket
 *     instead of adding layers) every layer also contributes the buckets whose
 *     tuple differs from the query's in exactly one coordinate by -1 or +1:
 *     C(q) = { p : exists l with key_l(p) - key_l(q) in {0, -e_j, +e_j} }.
 *     Query-directed (Lv et al.'s ordering of probes by how close the query
 *     lies to each slot boundary): only the T of those 2k neighbours with the
 *     smallest score, where for y_j = (a_j.q + b_j) / w (step 1's FP64
 *     sequence) and f_j = y_j - floor(y_j), moving coordinate j by -1 scores
 *     f_j * f_j and by +1 scores (1 - f_j) * (1 - f_j), each rounded in FP64;
 *     ties go to the smaller j, then to -1.
 *  5. Verification (removing false positives, Section 1.2): exact squared
 *     Euclidean distance; int64 for uint8 data, double accumulated in index
 *     order for float32 data: acc = acc + (x-q)*(x-q) with x-q formed in double.
 *  6. Top-K (c-k-ANN output, Section 3): the K smallest by (distance, id);
 *     when |C(q)| < K the tail is padded with id -1 and distance INT64_MAX
 *     (u8) or +inf (f32).
 *  7. Brute force: step 6 over all n points (exact kNN).
 *  8. Collision counting with a candidate cap (Section 3, "Collision Counting", after C2LSH: each
 *     layer acts as one collision test, a threshold on the number of tests a
 *     point passes replaces the plain union, and at most k + v points -- K
 *     results plus v allowed false positives -- are verified): #Col(p) is the
 *     number of layers l with key_l(p) == key_l(q); the points with
 *     #Col(p) >= theta are ranked by (#Col descending, id ascending), the
 *     first K + v of them are verified (step 5) and the top K taken (step 6).
 *     theta = 1 with a cap above |C(q)| is the plain union of step 4.
 *
 * All entry points return 0 on success and a negative value on bad input.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_U8 = 0, ORC_F32 = 1 };

static double elem(const void *x, int dtype, int64_t idx)
{
    if (dtype == ORC_U8)
        return (double)((const uint8_t *)x)[idx];
    return (double)((const float *)x)[idx];
}

/* ---- step 1: h = floor((a.v + b) / w), FP64 in index order ---------------- */

static double project_one(const void *x, int dtype, int64_t row, int32_t d,
                          const float *a_j, float b_j, double w)
{
    double acc = 0.0;
    for (int32_t i = 0; i < d; ++i)
        acc = acc + (double)a_j[i] * elem(x, dtype, row * (int64_t)d + i);
    double t = acc + (double)b_j;
    return t / w;
}

static int hash_one(const void *x, int dtype, int64_t row, int32_t d,
                    const float *a_j, float b_j, double w, int32_t *out)
{
    double y = project_one(x, dtype, row, d, a_j, b_j, w);
    double f = floor(y);
    if (!(f >= -2147483648.0 && f <= 2147483647.0))
        return -1;
    *out = (int32_t)f;
    return 0;
}

typedef struct {
    const void *x; int dtype; int64_t m; int32_t d;
    const float *a; const float *b; int32_t nf; double w;
    int32_t *out; int tid, nthreads; int err;
} hash_job;

static void *hash_worker(void *p)
{
    hash_job *j = (hash_job *)p;
    for (int64_t r = j->tid; r < j->m; r += j->nthreads)
        for (int32_t f = 0; f < j->nf; ++f)
            if (hash_one(j->x, j->dtype, r, j->d, j->a + (int64_t)f * j->d, j->b[f],
                         j->w, &j->out[r * j->nf + f]))
                j->err = 1;
    return NULL;
}

static int run_threads(void *(*fn)(void *), void *jobs, size_t job_size, int nthreads)
{
    pthread_t th[256];
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, fn, (char *)jobs + t * job_size))
            return -1;
    for (int t = 0; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    return 0;
}

/* y[m][nf] = (a.x + b) / w in step 1's FP64 sequence (the value h floors). */
int orc_project(const void *x, int64_t m, int32_t d, int32_t dtype, const float *a,
                const float *b, int32_t nf, double w, double *out_y)
{
    if (!x || !a || !b || !out_y || m < 0 || d <= 0 || nf <= 0 || !(w > 0) || !isfinite(w))
        return -1;
    for (int64_t r = 0; r < m; ++r)
        for (int32_t f = 0; f < nf; ++f)
            out_y[r * nf + f] = project_one(x, dtype, r, d, a + (int64_t)f * d, b[f], w);
    return 0;
}

/* h[m][nf] for m rows of x (row-major m x d) and nf functions a[nf][d], b[nf]. */
int orc_hash(const void *x, int64_t m, int32_t d, int32_t dtype,
             const float *a, const float *b, int32_t nf, double w,
             int32_t nthreads, int32_t *out_h)
{
    if (!x || !a || !b || !out_h || m < 0 || d <= 0 || nf <= 0 || !(w > 0) || !isfinite(w))
        return -1;
    if (nthreads < 1) nthreads = 1;
    hash_job jobs[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t)
        jobs[t] = (hash_job){x, dtype, m, d, a, b, nf, w, out_h, t, nthreads, 0};
    if (run_threads(hash_worker, jobs, sizeof(hash_job), nthreads))
        return -2;
    for (int t = 0; t < nthreads; ++t)
        if (jobs[t].err)
            return -3;
    return 0;
}

/* ---- steps 2-3: per-layer buckets as id lists sorted by (tuple, id) -------- */

typedef struct { const int32_t *h; int32_t nf, k, off; } tuple_ctx;

static int cmp_tuple(const int32_t *ta, const int32_t *tb, int32_t k)
{
    for (int32_t j = 0; j < k; ++j) {
        if (ta[j] < tb[j]) return -1;
        if (ta[j] > tb[j]) return 1;
    }
    return 0;
}

static int cmp_ids(const void *pa, const void *pb, void *arg)
{
    const tuple_ctx *c = (const tuple_ctx *)arg;
    int32_t ia = *(const int32_t *)pa, ib = *(const int32_t *)pb;
    int r = cmp_tuple(c->h + (int64_t)ia * c->nf + c->off,
                      c->h + (int64_t)ib * c->nf + c->off, c->k);
    if (r) return r;
    return (ia > ib) - (ia < ib);
}

typedef struct {
    int32_t *order;   /* [L][n] ids sorted by (layer tuple, id) */
    const int32_t *h; /* [n][L*k] data hashes */
    int64_t n; int32_t L, k;
} orc_index;

typedef struct { orc_index *ix; int tid, nthreads; } build_job;

static void *build_worker(void *p)
{
    build_job *j = (build_job *)p;
    orc_index *ix = j->ix;
    for (int32_t l = j->tid; l < ix->L; l += j->nthreads) {
        int32_t *o = ix->order + (int64_t)l * ix->n;
        for (int64_t i = 0; i < ix->n; ++i) o[i] = (int32_t)i;
        tuple_ctx c = {ix->h, ix->L * ix->k, ix->k, l * ix->k};
        qsort_r(o, (size_t)ix->n, sizeof(int32_t), cmp_ids, &c);
    }
    return NULL;
}

/* one sorted id list per layer; layers are independent and sorted in parallel */
static int index_build(orc_index *ix, const int32_t *h, int64_t n, int32_t L, int32_t k,
                       int nthreads)
{
    ix->h = h; ix->n = n; ix->L = L; ix->k = k;
    ix->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * L);
    if (!ix->order) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    build_job jobs[256];
    for (int t = 0; t < nthreads; ++t) jobs[t] = (build_job){ix, t, nthreads};
    return run_threads(build_worker, jobs, sizeof(build_job), nthreads) ? -2 : 0;
}

/* first position in layer l whose tuple is >= t; sets *cnt to the run length of t */
static int64_t bucket_find(const orc_index *ix, int32_t l, const int32_t *t, int64_t *cnt)
{
    const int32_t *o = ix->order + (int64_t)l * ix->n;
    int32_t nf = ix->L * ix->k, off = l * ix->k;
    int64_t lo = 0, hi = ix->n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cmp_tuple(ix->h + (int64_t)o[mid] * nf + off, t, ix->k) < 0) lo = mid + 1;
        else hi = mid;
    }
    int64_t e = lo;
    while (e < ix->n && cmp_tuple(ix->h + (int64_t)o[e] * nf + off, t, ix->k) == 0) ++e;
    *cnt = e - lo;
    return lo;
}

/* ---- steps 4-7 ------------------------------------------------------------ */

static int cmp_i32(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

typedef struct { double df; int64_t di; int32_t id; } scored;

static int cmp_scored_i(const void *pa, const void *pb)
{
    const scored *a = (const scored *)pa, *b = (const scored *)pb;
    if (a->di != b->di) return a->di < b->di ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

static int cmp_scored_f(const void *pa, const void *pb)
{
    const scored *a = (const scored *)pa, *b = (const scored *)pb;
    if (a->df != b->df) return a->df < b->df ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

static void distance(const void *data, const void *q, int dtype, int32_t d,
                     int64_t p, int64_t qi, scored *s)
{
    if (dtype == ORC_U8) {
        const uint8_t *x = (const uint8_t *)data + p * d, *v = (const uint8_t *)q + qi * d;
        int64_t acc = 0;
        for (int32_t i = 0; i < d; ++i) {
            int64_t t = (int64_t)x[i] - (int64_t)v[i];
            acc += t * t;
        }
        s->di = acc; s->df = (double)acc;
    } else {
        const float *x = (const float *)data + p * d, *v = (const float *)q + qi * d;
        double acc = 0.0;
        for (int32_t i = 0; i < d; ++i) {
            double t = (double)x[i] - (double)v[i];
            acc = acc + t * t;
        }
        s->df = acc; s->di = 0;
    }
    s->id = (int32_t)p;
}

typedef struct {
    const orc_index *ix; const int32_t *hq; /* [Q][L*k] query hashes (NULL = brute force) */
    int32_t probes; /* 1: also the 2k one-step neighbour buckets of every layer;
                       2: the probe_t of them with the smallest scores */
    int32_t probe_t;
    const float *a, *b; double w; /* for the scores of probes == 2 */
    const void *data; const void *q; int dtype; int32_t d; int64_t Q; int32_t K;
    int32_t *out_ids; int64_t *out_di; double *out_df; int64_t *out_cnt;
    int64_t *cand_off; int32_t *cand_ids; /* optional candidate-list output */
    int tid, nthreads; int err;
    int32_t theta, vextra; /* step 8 when theta >= 1: threshold and extra verified points */
} query_job;

typedef struct { int32_t count, id; } counted;

static int cmp_counted(const void *pa, const void *pb)
{
    const counted *a = (const counted *)pa, *b = (const counted *)pb;
    if (a->count != b->count) return a->count > b->count ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

static void *query_worker(void *p)
{
    query_job *j = (query_job *)p;
    int64_t n = j->ix->n;
    uint8_t *mark = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    scored *sc = (scored *)malloc(sizeof(scored) * (size_t)(n > 0 ? n : 1));
    int32_t *col = j->theta > 0 ? (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t)) : NULL;
    counted *ct = j->theta > 0 ? (counted *)malloc(sizeof(counted) * (size_t)(n > 0 ? n : 1)) : NULL;
    if (!mark || !list || !sc || (j->theta > 0 && (!col || !ct))) {
        j->err = 1; free(mark); free(list); free(sc); free(col); free(ct); return NULL;
    }
    int32_t L = j->ix->L, k = j->ix->k;
    int32_t t[64];
    double score[128];
    int32_t pick[128];
    const int32_t nprobe = j->probes == 2 ? 1 + j->probe_t : (j->probes ? 1 + 2 * k : 1);
    for (int64_t qi = j->tid; qi < j->Q; qi += j->nthreads) {
        int64_t nc = 0;
        if (j->hq) {  /* step 4: union of the query's bucket(s) in every layer */
            for (int32_t l = 0; l < L; ++l) {
                const int32_t *home = j->hq + qi * (int64_t)L * k + (int64_t)l * k;
                if (j->probes == 2) {
                    /* scores of the 2k moves (index 2c + s), then the probe_t
                       smallest by (score, index) */
                    for (int32_t c = 0; c < k; ++c) {
                        const int32_t fn = l * k + c;
                        double y = project_one(j->q, j->dtype, qi, j->d,
                                               j->a + (int64_t)fn * j->d, j->b[fn], j->w);
                        double fr = y - floor(y);
                        double up = 1.0 - fr;
                        score[2 * c] = fr * fr;
                        score[2 * c + 1] = up * up;
                    }
                    for (int32_t u = 0; u < 2 * k; ++u) pick[u] = u;
                    for (int32_t u = 1; u < 2 * k; ++u) {  /* insertion sort by (score, index) */
                        int32_t v = pick[u], z = u;
                        while (z > 0 && (score[pick[z - 1]] > score[v] ||
                                         (score[pick[z - 1]] == score[v] && pick[z - 1] > v))) {
                            pick[z] = pick[z - 1];
                            --z;
                        }
                        pick[z] = v;
                    }
                }
                for (int32_t pr = 0; pr < nprobe; ++pr) {
                    /* probe 0: the home tuple; probe 1 + 2c + s: coordinate c moved
                       by -1 (s = 0) or +1 (s = 1); query-directed: the pr-th pick */
                    for (int32_t c = 0; c < k; ++c) t[c] = home[c];
                    if (pr > 0) {
                        const int32_t mv = j->probes == 2 ? pick[pr - 1] : pr - 1;
                        t[mv / 2] += (mv % 2) ? 1 : -1;
                    }
                    int64_t cnt;
                    int64_t pos = bucket_find(j->ix, l, t, &cnt);
                    const int32_t *o = j->ix->order + (int64_t)l * n;
                    for (int64_t e = pos; e < pos + cnt; ++e) {
                        if (col) ++col[o[e]];
                        if (!mark[o[e]]) { mark[o[e]] = 1; list[nc++] = o[e]; }
                    }
                }
            }
            for (int64_t c = 0; c < nc; ++c) mark[list[c]] = 0;
            if (col) {  /* step 8: threshold, rank by (count desc, id asc), cap at K + v */
                int64_t m = 0;
                for (int64_t c = 0; c < nc; ++c) {
                    if (col[list[c]] >= j->theta) { ct[m].count = col[list[c]]; ct[m].id = list[c]; ++m; }
                    col[list[c]] = 0;
                }
                qsort(ct, (size_t)m, sizeof(counted), cmp_counted);
                const int64_t cap = (int64_t)j->K + j->vextra;
                nc = m < cap ? m : cap;
                for (int64_t c = 0; c < nc; ++c) list[c] = ct[c].id;
            }
        } else {      /* step 7: every point */
            for (int64_t c = 0; c < n; ++c) list[c] = (int32_t)c;
            nc = n;
        }
        if (j->out_cnt) j->out_cnt[qi] = nc;
        if (j->cand_ids) {
            /* ascending ids, for set comparison */
            int64_t base = j->cand_off[qi];
            for (int64_t c = 0; c < nc; ++c) j->cand_ids[base + c] = list[c];
            /* insertion order is layer order; sort ascending */
            qsort(j->cand_ids + base, (size_t)nc, sizeof(int32_t), cmp_i32);
        }
        if (!j->out_ids) continue;
        for (int64_t c = 0; c < nc; ++c)  /* step 5 */
            distance(j->data, j->q, j->dtype, j->d, list[c], qi, &sc[c]);
        qsort(sc, (size_t)nc, sizeof(scored), j->dtype == ORC_U8 ? cmp_scored_i : cmp_scored_f);
        for (int32_t r = 0; r < j->K; ++r) {  /* step 6 */
            int64_t o = qi * j->K + r;
            if (r < nc) {
                j->out_ids[o] = sc[r].id;
                if (j->out_di) j->out_di[o] = sc[r].di;
                if (j->out_df) j->out_df[o] = sc[r].df;
            } else {
                j->out_ids[o] = -1;
                if (j->out_di) j->out_di[o] = INT64_MAX;
                if (j->out_df) j->out_df[o] = INFINITY;
            }
        }
    }
    free(mark); free(list); free(sc); free(col); free(ct);
    return NULL;
}

static int run_queries(query_job *tmpl, int nthreads)
{
    query_job jobs[256];
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *tmpl; jobs[t].tid = t; jobs[t].nthreads = nthreads; jobs[t].err = 0;
    }
    if (run_threads(query_worker, jobs, sizeof(query_job), nthreads)) return -2;
    for (int t = 0; t < nthreads; ++t)
        if (jobs[t].err) return -4;
    return 0;
}

static int check_common(const void *data, int64_t n, int32_t d, const void *q, int64_t Q,
                        const float *a, const float *b, int32_t L, int32_t k, double w)
{
    if (!data || !q || !a || !b || n < 0 || Q < 0 || d <= 0 || L <= 0 || k <= 0)
        return -1;
    if (!(w > 0) || !isfinite(w) || n > INT32_MAX) return -1;
    return 0;
}

/*
 * Full LSH query workload: hash data and queries, build the per-layer buckets,
 * take the candidate union, verify and select the top-K.
 * out_ids [Q][K]; out_di [Q][K] (u8 data) or out_df [Q][K] (f32 data), either
 * may be NULL; out_cnt [Q] = |C(q)| (nullable).
 */
int orc_lsh_query(const void *data, int64_t n, int32_t d, int32_t dtype,
                  const void *q, int64_t Q, const float *a, const float *b,
                  int32_t L, int32_t k, double w, int32_t K, int32_t nthreads,
                  int32_t *out_ids, int64_t *out_di, double *out_df, int64_t *out_cnt,
                  int32_t probes, int32_t probe_t)
{
    if (check_common(data, n, d, q, Q, a, b, L, k, w) || K <= 0 || !out_ids) return -1;
    if (probes < 0 || probes > 2 || k > 64) return -1;
    if (probes == 2 && (probe_t < 1 || probe_t > 2 * k)) return -1;
    int32_t nf = L * k;
    int32_t *hd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * nf);
    int32_t *hq = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Q > 0 ? Q : 1) * nf);
    if (!hd || !hq) { free(hd); free(hq); return -5; }
    int rc = orc_hash(data, n, d, dtype, a, b, nf, w, nthreads, hd);
    if (!rc) rc = orc_hash(q, Q, d, dtype, a, b, nf, w, nthreads, hq);
    orc_index ix = {0};
    if (!rc) rc = index_build(&ix, hd, n, L, k, nthreads);
    if (!rc) {
        query_job t = {&ix, hq, probes, probe_t, a, b, w, data, q, dtype, d, Q, K, out_ids, out_di, out_df,
                       out_cnt, NULL, NULL, 0, 1, 0, 0, 0};
        rc = run_queries(&t, nthreads);
    }
    free(ix.order); free(hd); free(hq);
    return rc;
}

/*
 * Collision counting (step 8) on the plain layers: out_cnt [Q] (nullable)
 * receives the number of points verified, min(K + v, #{p : #Col(p) >= theta}).
 */
int orc_lsh_query_counting(const void *data, int64_t n, int32_t d, int32_t dtype,
                           const void *q, int64_t Q, const float *a, const float *b,
                           int32_t L, int32_t k, double w, int32_t K, int32_t theta,
                           int32_t v, int32_t nthreads, int32_t *out_ids, int64_t *out_di,
                           double *out_df, int64_t *out_cnt)
{
    if (check_common(data, n, d, q, Q, a, b, L, k, w) || K <= 0 || !out_ids) return -1;
    if (theta < 1 || v < 0 || k > 64) return -1;
    int32_t nf = L * k;
    int32_t *hd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * nf);
    int32_t *hq = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Q > 0 ? Q : 1) * nf);
    if (!hd || !hq) { free(hd); free(hq); return -5; }
    int rc = orc_hash(data, n, d, dtype, a, b, nf, w, nthreads, hd);
    if (!rc) rc = orc_hash(q, Q, d, dtype, a, b, nf, w, nthreads, hq);
    orc_index ix = {0};
    if (!rc) rc = index_build(&ix, hd, n, L, k, nthreads);
    if (!rc) {
        query_job t = {&ix, hq, 0, 0, a, b, w, data, q, dtype, d, Q, K, out_ids, out_di, out_df,
                       out_cnt, NULL, NULL, 0, 1, 0, theta, v};
        rc = run_queries(&t, nthreads);
    }
    free(ix.order); free(hd); free(hq);
    return rc;
}

/*
 * Candidate sets only.  Call with cand_ids == NULL to obtain out_cnt [Q]; then
 * with cand_off [Q+1] (exclusive prefix sums of out_cnt) and cand_ids sized
 * cand_off[Q] to receive each query's candidates in ascending id order.
 */
int orc_lsh_candidates(const void *data, int64_t n, int32_t d, int32_t dtype,
                       const void *q, int64_t Q, const float *a, const float *b,
                       int32_t L, int32_t k, double w, int32_t nthreads,
                       int64_t *out_cnt, const int64_t *cand_off, int32_t *cand_ids,
                       int32_t probes, int32_t probe_t)
{
    if (check_common(data, n, d, q, Q, a, b, L, k, w) || !out_cnt) return -1;
    if (probes < 0 || probes > 2 || k > 64) return -1;
    if (probes == 2 && (probe_t < 1 || probe_t > 2 * k)) return -1;
    if (cand_ids && !cand_off) return -1;
    int32_t nf = L * k;
    int32_t *hd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * nf);
    int32_t *hq = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Q > 0 ? Q : 1) * nf);
    if (!hd || !hq) { free(hd); free(hq); return -5; }
    int rc = orc_hash(data, n, d, dtype, a, b, nf, w, nthreads, hd);
    if (!rc) rc = orc_hash(q, Q, d, dtype, a, b, nf, w, nthreads, hq);
    orc_index ix = {0};
    if (!rc) rc = index_build(&ix, hd, n, L, k, nthreads);
    if (!rc) {
        query_job t = {&ix, hq, probes, probe_t, a, b, w, data, q, dtype, d, Q, 0, NULL, NULL, NULL, out_cnt,
                       (int64_t *)cand_off, cand_ids, 0, 1, 0, 0, 0};
        rc = run_queries(&t, nthreads);
    }
    free(ix.order); free(hd); free(hq);
    return rc;
}

/*
 * The same workload split into its two phases so they can be timed apart:
 * orc_lsh_build hashes the data and builds the per-layer buckets (steps 1-3),
 * orc_lsh_query_built answers queries against it (steps 1 and 4-6).
 */
typedef struct {
    orc_index ix; int32_t *hd; const void *data; int64_t n; int32_t d, dtype, L, k;
    const float *a, *b; double w;
} orc_built;

void *orc_lsh_build(const void *data, int64_t n, int32_t d, int32_t dtype, const float *a,
                    const float *b, int32_t L, int32_t k, double w, int32_t nthreads)
{
    if (check_common(data, n, d, data, 0, a, b, L, k, w)) return NULL;
    orc_built *o = (orc_built *)calloc(1, sizeof(orc_built));
    if (!o) return NULL;
    o->hd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * L * k);
    if (!o->hd || orc_hash(data, n, d, dtype, a, b, L * k, w, nthreads, o->hd) ||
        index_build(&o->ix, o->hd, n, L, k, nthreads)) {
        free(o->hd); free(o->ix.order); free(o);
        return NULL;
    }
    o->data = data; o->n = n; o->d = d; o->dtype = dtype; o->L = L; o->k = k;
    o->a = a; o->b = b; o->w = w;
    return o;
}

int orc_lsh_query_built(void *h, const void *q, int64_t Q, int32_t K, int32_t nthreads,
                        int32_t *out_ids, int64_t *out_di, double *out_df, int64_t *out_cnt,
                        int32_t probes, int32_t probe_t)
{
    orc_built *o = (orc_built *)h;
    if (!o || !q || Q < 0 || K <= 0 || !out_ids) return -1;
    if (probes < 0 || probes > 2 || o->k > 64) return -1;
    if (probes == 2 && (probe_t < 1 || probe_t > 2 * o->k)) return -1;
    int32_t *hq = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Q > 0 ? Q : 1) * o->L * o->k);
    if (!hq) return -5;
    int rc = orc_hash(q, Q, o->d, o->dtype, o->a, o->b, o->L * o->k, o->w, nthreads, hq);
    if (!rc) {
        query_job t = {&o->ix, hq, probes, probe_t, o->a, o->b, o->w, o->data, q, o->dtype, o->d, Q, K, out_ids, out_di,
                       out_df, out_cnt, NULL, NULL, 0, 1, 0, 0, 0};
        rc = run_queries(&t, nthreads);
    }
    free(hq);
    return rc;
}

void orc_lsh_free(void *h)
{
    orc_built *o = (orc_built *)h;
    if (!o) return;
    free(o->ix.order); free(o->hd); free(o);
}

/* Exact kNN over all n points (step 7). */
int orc_bruteforce(const void *data, int64_t n, int32_t d, int32_t dtype,
                   const void *q, int64_t Q, int32_t K, int32_t nthreads,
                   int32_t *out_ids, int64_t *out_di, double *out_df)
{
    if (!data || !q || n < 0 || Q < 0 || d <= 0 || K <= 0 || !out_ids || n > INT32_MAX)
        return -1;
    orc_index ix = {NULL, NULL, n, 1, 1};
    query_job t = {&ix, NULL, 0, 0, NULL, NULL, 0.0, data, q, dtype, d, Q, K, out_ids, out_di, out_df, NULL,
                   NULL, NULL, 0, 1, 0, 0, 0};
    return run_queries(&t, nthreads);
}
