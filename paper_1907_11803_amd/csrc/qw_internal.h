// Internal declarations shared by the HIP translation units of libqwlsh.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qwlsh.h"

namespace qw {

constexpr int kXcd = 8;                   // XCDs: workgroup b runs on XCD b % 8
constexpr int kBlock = 256;              // threads per workgroup for every kernel here
// The guard-band recompute count is spread over this many device counters
// (workgroup b adds to slot b % kRecompSlots): one counter shared by every
// workgroup serialises their atomic adds at the end of the hash kernel.
constexpr int kRecompSlots = 32;
// Largest K the fused dedup kernel selects itself (uint8 data).
constexpr int kFusedTopK = 16;
// K chunk of the FP32 matrix-core hashing of float data: each chunk sums in
// FP32, the chunk sums add up in FP64 (the guard band depends on it).
constexpr int kHashChunkF32 = 64;
// Bucket lists per query at most (neighbour probing: L * (2k + 1)).
constexpr int kMaxLists = 1024;
// With bucket grouping the dedup kernel deals its items to the XCDs in chunks
// of this many consecutive positions of the order (each XCD then takes at most
// one chunk more than its share per launch); without, one at a time.
constexpr uint32_t kXcdChunk = 256;
// Automatic bucket grouping orders queries by candidate overlap when a
// candidate's row is at least kGroupRowBytes bytes (the verification reads
// whole rows that neighbouring queries share in L2 and the last-level cache)
// or the workload has at least kGroupQueries queries (the two radix passes
// the ordering costs are then small against the reuse).  Measured: 1M x 960
// float rows gain 36 %, 100K Zipf queries over 10M x 96 uint8 rows 2 %, and
// 10K queries over 1M x 128 uint8 rows lose 17 %.
constexpr int kGroupRowBytes = 1024;
constexpr int64_t kGroupQueries = 32768;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // empty hash-set slot
constexpr int kMaxL = 64;
constexpr int kMaxK = 32;
constexpr int kMaxTopK = 1024;
constexpr int kMaxD = 8192;

// ---------------------------------------------------------------- status plumbing
#define QW_TRY(expr)                          \
    do {                                      \
        qw_status s_ = (expr);                \
        if (s_ != QW_OK) return s_;           \
    } while (0)

#define QW_HIP(expr)                                          \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) {                               \
            ::qw::note_hip_error(e_, #expr, __FILE__, __LINE__); \
            return QW_EDEVICE;                                \
        }                                                     \
    } while (0)

void note_hip_error(hipError_t e, const char *what, const char *file, int line);

// ---------------------------------------------------------------- device buffers
// A device allocation owned by the library, or a view of `bytes` bytes of
// memory owned elsewhere (never freed, never grown: ensure() beyond its size
// fails with QW_EINTERNAL instead of allocating).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = true;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned)
    {
        o.p = nullptr;
        o.bytes = 0;
        o.owned = true;
    }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            owned = o.owned;
            o.p = nullptr;
            o.bytes = 0;
            o.owned = true;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    qw_status ensure(size_t want);  // grows (contents discarded); never shrinks
    void release();
    void view(void *mem, size_t n)
    {
        release();
        p = mem;
        bytes = n;
        owned = false;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------- index
// Probe-table entry: a bucket of one layer, keyed by its packed k-tuple.
struct TabEntry {
    uint64_t klo, khi;
    uint32_t start, size;  // CSR range of the bucket; size == 0 marks an empty slot
    uint32_t mh;           // min over the bucket's ids of id_mix(id) (grouping key)
    uint32_t unused;
};

// A fixed 32-bit mixer of point ids: the minimum of id_mix over a candidate
// set is a min-hash of the set, so two queries share their key with
// probability equal to the Jaccard similarity of their candidate sets.
__host__ __device__ inline uint32_t id_mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

struct Workspace {
    DevBuf qpad, h, bstart, bsize, bmh, lsum, lmh, moves, pred, feats, keys, keys2, vals,
        vals2, hist, order, binoff, counters, ovf, gscratch, mlpout, scan;
    // flat pipeline
    DevBuf ucount, coff, flag, pkeys, fb;
    // the query rows the kernels of the current call read: the caller's own
    // (no padding needed) or qpad
    const void *qrows = nullptr;
};

// Launch plan of the fast form for one top-K size: hash-set size classes and
// persistent grid sizes.
struct Plan {
    int buf = 64;
    int cmax = 10;      // largest LDS class (log2 capacity)
    int cfloor = 10;    // smallest class worth choosing (no occupancy gain below)
    int ncls = 2;       // LDS classes + 1 global class
    int dgrid[16] = {}; // dedup kernel, per class
    int cap_g = 20, grid_g = 1;
    int topk = 0;       // dedup also selects the top K (0: the select kernel does)
    int wgrid = 0;      // one-wave-per-query dedup kernel (0: not applicable)
    bool wave_default = false;  // the automatic choice when nothing is tuned
    int LC = 2048;      // select kernel list capacity (entries)
    float eps = 0.f;    // FP32 distance bound (float data)
};

// One entry of the tuning cache: the fastest explicit fast-form settings for
// one GPU architecture and workload shape, with the times that chose them.
struct TuneEntry {
    std::string arch, key, desc;
    int32_t dedup = 0, group = -1, xchunk = 0, split = -1;
    double ms = 0.0, ms_default = 0.0;
};

// Out-of-core mode: the CSR ids and the padded rows in pinned host memory,
// and the two HBM caches (bucket lists in C_I, rows in C_D) with their
// bookkeeping.  Bucket records live in an open-addressing map keyed by the
// bucket's position in the CSR (layer * n + start), never deleted, whose
// capacity is at least twice the number of buckets.
struct OocState {
    qw_ooc_opts o{};
    int32_t npools = 1;
    int64_t cap_pool = 0;     // ids per C_I pool
    int64_t ids_total = 0;    // npools * cap_pool: the arena
    int64_t cap_rows = 0;     // rows in C_D
    int64_t row_bytes = 0;
    void *host_ids = nullptr, *host_rows = nullptr;  // pinned host copies
    const void *dev_ids = nullptr, *dev_rows = nullptr;  // their device addresses
    size_t host_bytes = 0;
    int64_t mcap = 0;         // map slots (power of two)
    DevBuf arena[2];          // C_I: resident lists, rebuilt into the other arena per batch
    int cur = 0;
    DevBuf mkey, msize, mstamp, moff, mnoff, mneed, mmiss;  // per map slot
    DevBuf rows, owner;       // C_D: cap_rows rows and the id held by each slot (-1 free)
    DevBuf dir, rstamp, rneed, rmiss;  // per point: slot (-1), last use, batch tags
    DevBuf missd, ckeys, cvals, ckeys2, cvals2, csz, cscan, sort_hist, scan_tmp, copyl, freel,
        bstart2, ctr;
    int64_t cand_cap = 0;     // entries of the candidate lists
    uint32_t tag = 0;         // batch attempt counter (tags are never reused)
    int64_t rows_used = 0;    // resident rows (host mirror)
    int64_t qbase = 0;        // queries answered since the caches were emptied (recency offset)
    OocState() = default;
    OocState(const OocState &) = delete;
    OocState &operator=(const OocState &) = delete;
    ~OocState()
    {
        if (host_ids) (void)hipHostFree(host_ids);
        if (host_rows) (void)hipHostFree(host_rows);
    }
};

// Reads of one out-of-core query call.
struct OocIo {
    int64_t index_files = 0, index_bytes = 0, data_objects = 0, data_bytes = 0, batches = 0,
            splits = 0;
};

struct GraphKey {
    const void *q; int64_t Q; int32_t K; int32_t *ids; void *dist;
    int32_t form, sched, group, topk_keep, dedup, xchunk, split;
    bool operator<(const GraphKey &o) const {
        return std::memcmp(this, &o, sizeof(GraphKey)) < 0;
    }
};

}  // namespace qw

struct qw_index {
    int device = 0;
    int cus = 256;
    size_t lds_max = 65536;
    int64_t n = 0;
    int32_t d = 0, dp = 0, dtype = 0, L = 0, k = 0, nf = 0, nf_pad = 0;
    // bucket lists per layer (1, or 2k + 1 with neighbour probing), lists per
    // query (L * nprobe) and the layer-of-list multiplier (0 without probing)
    int32_t nprobe = 1, nl = 0;
    uint32_t pmagic = 0;
    int32_t count_theta = 0, count_extra = 0;  // qw_set_counting: 0 = plain union
    int32_t probe_mode = 0;  // qw_set_probing mode: 2 = query-directed (nprobe - 1 moves)
    float w = 0.f;
    // hash parameters (device)
    qw::DevBuf a32;      // float [nf_pad][dp], zero padded
    qw::DevBuf a64l;     // double [L][dp][k]: a32 in FP64, layer-major (query-directed probing)
    qw::DevBuf b32;      // float [nf]
    qw::DevBuf a_hi;     // _Float16 [nf_pad][dp]  (uint8 data, MFMA path)
    qw::DevBuf a_lo;     // _Float16 [nf_pad][dp]
    qw::DevBuf gb_plain; // double [nf]: guard-band coefficient of the FP32 VALU path
    qw::DevBuf gb_fast;  // double [nf]: guard-band coefficient of the MFMA path
    bool fast_f16 = true;  // uint8 data with |a| < 2^15 uses the FP16 hi/lo split
    // data copy, rows padded to dp elements
    qw::DevBuf data;
    // key packing per function
    qw::DevBuf hmin, hmax, shift;  // int32 [nf]
    std::vector<int32_t> key_bits;  // per layer
    // CSR ids [L][n] and probe tables
    qw::DevBuf ids;
    qw::DevBuf tab;        // TabEntry, all layers concatenated
    qw::DevBuf tab_off;    // int64 [L] first entry of each layer
    qw::DevBuf tab_mask;   // uint32 [L]
    int64_t buckets = 0, max_bucket = 0;
    // mean over layers of sum_b s_b^2 / n: the expected size of the bucket a
    // point of the data falls in (queries near the data see about this much)
    double mean_hit_bucket = 0.0;
    // count model
    std::vector<float> mlp;  // packed host copy (empty = none)
    float mlp_margin = 0.22314355f;  // log-space sizing margin, log(1.25) until calibrated
    qw::DevBuf mlp_dev;
    qw::DevBuf mlp_lane;   // the model's inference registers, one record per lane
    // query workspace and captured graphs
    qw::Workspace ws;
    std::map<qw::GraphKey, hipGraphExec_t> graphs;
    std::map<int, qw::Plan> plans;  // by K
    hipEvent_t ev[8] = {};
    bool ev_init = false;
    // side stream (default priority) and fork/join events: the larger size
    // classes run beside the merged launch
    hipStream_t side = nullptr;
    hipEvent_t fork[2] = {};
    // tuning cache: the file last named by a call, read once, and the
    // device's architecture name
    std::string tune_path, tune_arch;
    std::vector<qw::TuneEntry> tune_entries;
    // out-of-core mode (null: data and lists in HBM)
    std::unique_ptr<qw::OocState> ooc;

    qw_index() = default;
    qw_index(const qw_index &) = delete;
    qw_index &operator=(const qw_index &) = delete;
    ~qw_index()
    {
        for (auto &e : fork)
            if (e) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
    }
};

namespace qw {

// ---------------------------------------------------------------- tuning
// Key of a workload in the tuning cache (a hash of the index's shape and
// settings, Q, K and the schedule); desc (nullable) receives a readable form.
std::string tune_key(const qw_index *ix, int64_t Q, int32_t K, int32_t sched, std::string *desc);
// The cache entry at `path` for this workload on this GPU's architecture.
bool tune_lookup(qw_index *ix, const char *path, int64_t Q, int32_t K, int32_t sched, TuneEntry *out);
// The fast form's automatic settings (dedup 0, group -1, xchunk 0) resolved
// to the explicit values a call uses: the tuning cache's entry when
// o->tune_cache names one for this workload, else the built-in rules.
// wave_ok (nullable): whether the one-wave-per-query kernel applies.
// Returns whether the cache supplied a setting.
bool resolve_fast_auto(qw_index *ix, int64_t Q, int32_t K, qw_opts *o, bool *wave_ok);

// ---------------------------------------------------------------- kernels (launch wrappers)
// Copy m rows of d elements into rows of dp elements (zero padding).
qw_status launch_pad_rows(const void *src, int64_t m, int32_t d, int32_t dp, int32_t dtype,
                          void *dst, hipStream_t s);

// Hash m padded rows for functions [f0, f0+nfun): out[row][f - f0] (row stride out_ld).
// form 0: FP32 VALU, form 1: MFMA.  recomputed: kRecompSlots device counters
// whose sum is the recompute count (nullable).
qw_status launch_hash(const qw_index *ix, const void *xpad, int64_t m, int32_t f0, int32_t nfun,
                      int32_t form, int32_t *out, int32_t out_ld,
                      unsigned long long *recomputed, hipStream_t s);

// Query-directed probing: each layer's T chosen moves [Q][L][T]
// (T = nprobe - 1) from the FP64 projections of the query rows; hout
// (nullable) receives their floors, the exact hash values [Q][L*k].  clear
// (nullable): nclear words the kernel zeroes before any later kernel runs.
qw_status launch_probe_moves(const qw_index *ix, const void *xpad, int64_t Q, uint8_t *moves,
                             int32_t *hout, hipStream_t s, uint32_t *clear = nullptr,
                             int32_t nclear = 0);

// Probe every list of every query: bstart/bsize [Q][L][P] (bsize 0 = miss);
// bmh (nullable) the bucket's min-hash; moves (query-directed probing) each
// layer's chosen moves.  Per layer [Q][L], each nullable: feats log(1 + s),
// lsum s, lmh the min-hash over the layer's probes (s: the layer's size summed
// over its probes).
qw_status launch_probe(const qw_index *ix, const int32_t *h, int64_t Q, uint32_t *bstart,
                       uint32_t *bsize, float *feats, uint32_t *bmh, const uint8_t *moves,
                       uint32_t *lsum, uint32_t *lmh, hipStream_t s);

// Generic fills.
qw_status launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s);
qw_status launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t count,
                          hipStream_t s);
qw_status launch_iota(int32_t *p, int64_t count, hipStream_t s);

// Exclusive prefix sum of count uint32 values into uint64 out (out has count+1 entries).
qw_status launch_scan_u32_to_u64(const uint32_t *in, int64_t count, unsigned long long *out,
                                 DevBuf &scratch, hipStream_t s);

// Scratch bytes radix_sort_pairs needs for `count` pairs.
size_t radix_sort_scratch_bytes(int64_t count);
// Stable LSD radix sort of (key, value) pairs on key bits [bit_lo, bits).
qw_status radix_sort_pairs(unsigned long long *keys, int32_t *vals, int64_t count, int bit_lo,
                           int bits,
                           unsigned long long *keys_alt, int32_t *vals_alt, DevBuf &hist,
                           hipStream_t s, bool *result_in_alt);

// ---------------------------------------------------------------- verify kernel
// TOPK: top-K of the LSH candidates; COUNT: |C(q)| only; LIST: the candidate ids;
// ALL: top-K over every indexed point (exact kNN, no dedup phase).
enum VerifyMode { VM_TOPK = 0, VM_COUNT = 1, VM_LIST = 2, VM_ALL = 3 };

struct VerifyArgs {
    const int32_t *order;        // item -> query (nullable: identity)
    const unsigned long long *seg;  // nullable: {begin, end} of the items this launch serves
    int64_t nitems;              // used when seg == nullptr and nitems_dev == nullptr
    const uint32_t *nitems_dev;  // nullable: item count read from device memory
    uint32_t *counter;           // persistent work counter (nullable = one item per workgroup)
    const uint32_t *bstart, *bsize;  // [Q][nl] bucket lists (layer-relative starts)
    const int32_t *ids;
    int64_t n;
    int32_t nl;                  // lists per query (L, or L * P with neighbour probing)
    uint32_t pmagic;             // 0, or ceil(2^20 / P): list i belongs to layer (i * pmagic) >> 20
    int32_t d, dp, dtype, K, mode;
    const void *data, *queries;
    uint32_t cap_log2;           // hash-set capacity 2^cap_log2
    uint32_t limit;              // abort when more unique ids than this (overflow); <= 3/4 capacity
    uint32_t buf;                // top-K buffer entries (power of two)
    int32_t global_tab;          // 1: hash set in global scratch
    int32_t short_probe;         // 1: bounded probing (only where an overflow moves the query on)
    uint32_t *gscratch;          // global scratch (global_tab): 2^cap_log2 words per workgroup
    uint32_t *ovf_count;         // queue receiving queries whose set overflowed
    int32_t *ovf_list;
    const uint32_t *in_count;    // nullable: queue of queries this launch serves after its segment
    const int32_t *in_list;
    int32_t *out_ids;            // TOPK: [Q][K]; LIST: concatenated lists
    void *out_dist;              // TOPK
    int32_t *out_counts;         // COUNT
    const long long *offsets;    // LIST
    uint32_t *ucount_out;        // nullable: |C(q)| of each answered query
    const int32_t *row_slot;     // nullable: row of point id is data + row_slot[id] * row bytes
                                 // (the out-of-core data cache); LDS hash sets only
};

// Collision counting (one workgroup per query; plain layer lists, no probing).
struct CountArgs {
    const uint32_t *bstart, *bsize;  // [Q][L] bucket lists (layer-relative starts)
    const int32_t *ids;
    int64_t n;
    int32_t L, theta, K, extra;      // count threshold; K + extra ids verified at most
    int32_t ncap;                    // kept-id buffer entries (even, >= K + extra)
    int32_t dtype, dp;
    uint32_t cap_log2;               // set slots 2^cap_log2, at least 4/3 of the listed ids
    const void *data, *queries;
    int32_t *out_ids;                // [Q][K]
    void *out_dist;                  // [Q][K] int32 (uint8 data) or float
    uint32_t *out_counts;            // nullable: [Q] ids verified
    const int32_t *qlist;            // nullable: workgroup b answers query qlist[b] (else b)
    int32_t id_top, key_top;         // radix selects start at these bits (ids < 2^(id_top + 8),
                                     // distance keys' high words < 2^(key_top + 8))
};
size_t count_lds_bytes(int cap_log2, int ncap);
// Splits the Q queries by the sum of their L list lengths (<= limit: list0,
// else list1); cnt (zeroed, device): n0, n1, the largest sum of each list.
qw_status launch_count_split(const uint32_t *bsize, int64_t Q, int32_t L, uint32_t limit,
                             int32_t *list0, int32_t *list1, uint32_t *cnt, hipStream_t s);
// `grid` workgroups of 512 threads (large: 1024).
qw_status launch_count(const CountArgs &a, int64_t grid, bool large, hipStream_t s);
// Largest sum of one query's L list lengths the counting set takes (3/4 of
// the largest set, 2^14 slots); queries up to kCountSmallListed (3/4 of 2^13)
// run in the smaller workgroups.
constexpr uint32_t kCountMaxListed = 12288;
constexpr uint32_t kCountSmallListed = 6144;
constexpr int kCountMaxSetLog2 = 14;
// Ids share a set word with their count (7 bits), so counting needs n below this.
constexpr int64_t kCountMaxN = (int64_t(1) << 25) - 1;

size_t verify_lds_bytes(int cap_log2, int buf, int global_tab, int L, int dp, int dtype);
qw_status launch_verify(const VerifyArgs &a, int grid, hipStream_t s);

// ---------------------------------------------------------------- out-of-core mode
// Host copies and empty caches for options `o` (validated by the caller).
qw_status ooc_enable(qw_index *ix, const qw_ooc_opts &o, hipStream_t s);
// Everything back in HBM, caches freed.
qw_status ooc_disable(qw_index *ix, hipStream_t s);
// Empty both caches.
qw_status ooc_reset(qw_index *ix, hipStream_t s);
// Answer Q probed queries (ws.bstart / ws.bsize hold their buckets) in
// batches through the caches.  `tmpl` carries the verify launch's settings
// (mode, K, set size, buffers); the per-batch pointers are filled here.
// out_dist_elem: bytes per distance.  Synchronises s per batch.
qw_status ooc_answer(qw_index *ix, int64_t Q, const VerifyArgs &tmpl, const void *qrows,
                     int32_t *out_ids, void *out_dist, hipStream_t s, OocIo *io);
// Candidates processed per workgroup iteration (sizes the top-K buffer).
int verify_per_iter(int dp, int dtype);
// Resident workgroups per CU of the verify kernel with `lds` bytes of LDS.
int verify_blocks_per_cu(int dp, int dtype, size_t lds);

// ---------------------------------------------------------------- scheduling
qw_status launch_classify(int64_t Q, int32_t L, int64_t n,
                          const uint32_t *bmh, const uint32_t *bsize, const int32_t *exact,
                          const float *pred_log, float margin, int32_t force_max, int32_t cmin,
                          int32_t cfloor, int32_t cmax, int32_t ncls, int32_t group,
                          unsigned long long *keys,
                          int32_t *vals, unsigned long long *class_count, hipStream_t s);
qw_status launch_segments(const unsigned long long *class_count, int32_t ncls,
                          unsigned long long *seg, hipStream_t s);
// Classes without bucket grouping in one kernel: class c's queries to
// order[c * Q ..) (any order), counts added to class_count, seg[2c], seg[2c+1]
// = [c * Q, c * Q + count_c).  done: a zeroed counter.  mlp_lane (nullable):
// the count model's lane records, run in the kernel on log(1 + s_l) for the
// queries whose bound class lies above cfloor (the only ones it can move).
qw_status launch_classify_bin(int64_t Q, int32_t L, int64_t n, const uint32_t *bsize,
                              const int32_t *exact, const uint32_t *mlp_lane, float margin,
                              int32_t force_max, int32_t cmin, int32_t cfloor, int32_t cmax,
                              int32_t ncls, int32_t *order, unsigned long long *class_count,
                              uint32_t *done, unsigned long long *seg, hipStream_t s);
qw_status launch_max_u32(const uint32_t *v, int64_t count, uint32_t *out, hipStream_t s);
qw_status launch_max_bucket_sum(const uint32_t *bsize, int64_t Q, int32_t L, uint32_t *out,
                                hipStream_t s);
qw_status launch_probe_stats(const uint32_t *bsize, int64_t count, unsigned long long *hits,
                             unsigned long long *total, hipStream_t s);
qw_status launch_gather_batch(const float *feats, const float *labels, const int32_t *perm,
                              int32_t L, int32_t B, float *fb, float *tb, hipStream_t s);
qw_status launch_labels(const int32_t *counts, int64_t m, float *out, hipStream_t s);

// ---------------------------------------------------------------- build
qw_status build_index(const void *data, int64_t n, int32_t d, int32_t dtype, const float *a,
                      const float *b, float w, int32_t L, int32_t k, int32_t form,
                      hipStream_t s, qw_index **out);

// ---------------------------------------------------------------- flat pipeline
struct DedupArgs {
    const int32_t *order;            // scheduled query order
    const unsigned long long *seg;   // {begin, end} of every class in the order (gaps allowed)
    int32_t cls_lo, cls_hi;          // this launch serves classes cls_lo..cls_hi
    int32_t queue_only;              // serve only the in_list queue (no segment)
    int32_t cap_base;                // class c uses a set of 2^(cap_base + c) slots
    uint32_t xchunk;                 // items dealt to each XCD in turn (1 .. kXcdChunk)
    uint32_t *xwork;                 // [kXcd] work counters, one per XCD (zero on entry)
    const uint32_t *in_count;        // nullable: queue of overflowed queries served after the segment
    const int32_t *in_list;
    uint32_t *ovf_count;             // queue receiving this class's overflows
    int32_t *ovf_list;
    const uint32_t *bstart, *bsize;  // [Q][nl] bucket lists (layer-relative starts)
    const int32_t *ids;
    int64_t n;
    int32_t nl;                      // lists per query (L, or L * P with neighbour probing)
    uint32_t pmagic;                 // 0, or ceil(2^20 / P): list i belongs to layer (i * pmagic) >> 20
    uint32_t cap_log2, limit;
    int32_t global_tab;
    uint32_t *gscratch;              // 2^cap_log2 words per workgroup (global_tab)
    int32_t count_only;              // write |C(q)| only
    // the key list (select kernel) is cut into kXcd regions of `region` keys;
    // region x is filled by the workgroups of XCD x (blockIdx % kXcd) through
    // its own bump allocator alloc[x]; fail[x] keeps the complement of the
    // lowest offset refused there (0 = none), so region x holds the granted
    // lists in [x * region, x * region + min(alloc[x], ~fail[x]))
    unsigned long long *alloc;       // [kXcd]
    unsigned long long *fail;        // [kXcd]
    unsigned long long region;
    uint32_t *ucount;                // |C(q)|
    unsigned long long *coff;        // offset of each query's keys
    uint32_t *flag;                  // 1 = answer q with the fallback
    // every unique candidate is verified in place: keys[coff + i] =
    // (squared distance << 32) | id, or the fused top K below
    int32_t dp, dtype;
    int32_t addr32;                  // n * row bytes < 2^32 and n < 2^24: 32-bit row offsets
    const void *data, *queries;
    unsigned long long *keys;
    // fused top-K (uint8, topk = K in 1..kFusedTopK, rows of at most 64
    // parts): the kernel selects the K nearest itself and writes the output;
    // no keys, no list space.  Queries it cannot settle go to fb_list.
    int32_t topk;
    int32_t topk_keep;               // keys kept per lane, 1..3 (fewer only reach the fallback more)
    int32_t *out_ids;
    void *out_dist;
    uint32_t *fb_count;
    int32_t *fb_list;
    uint32_t *topk2_count;           // queries that took the second selection pass
};


struct SelectArgs {
    const unsigned long long *keys;
    const unsigned long long *coff;
    const uint32_t *ucount;
    const uint32_t *flag;
    int32_t K, LC, dtype, dp, d;
    float eps;
    uint32_t *fb_count;
    int32_t *fb_list;
    int32_t *out_ids;
    void *out_dist;
    const void *data, *queries;
};

// Staged candidate kernel (qw_opts.stage_split): one workgroup per run of
// `chunk` consecutive items of the order (classes largest first), LDS caches
// of bucket id lists (icn slots of kStageIps ids) and rows (dcn slots) kept
// across them; keys for the select kernel, flag[q] = 1 for queries left to
// the fallback.
constexpr int kStageIps = 32;                        // ids per index-cache slot
constexpr size_t kStageLdsBytes = 80 * 1024;         // two workgroups per CU
constexpr int kStageMaxRow = 4096;                   // row bytes at most
struct StageArgs {
    const int32_t *order;
    const unsigned long long *seg;  // {begin, end} of each class in the order
    int32_t ncls;
    uint32_t *counter;              // run counter (zero on entry)
    uint32_t chunk;                 // items per run
    const uint32_t *bstart, *bsize;
    const int32_t *ids;
    int64_t n;
    int32_t nl;                     // lists per query (at most 64)
    uint32_t pmagic;
    int32_t dp, dtype;
    const void *data, *queries;
    unsigned long long *keys, *alloc, *fail;
    unsigned long long region;
    uint32_t *ucount;
    unsigned long long *coff;
    uint32_t *flag;
    uint32_t icn, dcn;              // index / data cache slots
};
// LDS bytes of the staged kernel for rows of row_bytes at an index share of
// `split` percent; icn/dcn receive the cache slots.
size_t stage_lds_bytes(int row_bytes, int32_t split, uint32_t *icn, uint32_t *dcn);
qw_status launch_stage(const StageArgs &a, int grid, hipStream_t s);

size_t dedup_lds_bytes(int cap_log2, int global_tab, int L, int row_bytes);
int dedup_blocks_per_cu(size_t lds, int dtype);
qw_status launch_dedup(const DedupArgs &a, int grid, hipStream_t s);
// One wave per query (uint8, fused top K, at most 64 lists): the whole
// workload in one launch over classes cls_lo..cls_hi (no queue), each XCD's
// items dealt to its waves in rounds; a query's class sets how many id-hash
// passes it starts with (cap_base + class - 11 doublings), a pass that
// overflows splits in place (counted in *ovf_count); unsettled top K to
// fb_list (counted in *topk2_count too).
int dedup_wave_applies(int dtype, int dp, int nl, int topk);
int dedup_wave_blocks_per_cu();
size_t dedup_wave_lds_bytes();
int dedup_wave_keep();      // keys kept per lane (topk_keep 0)
uint32_t dedup_wave_set_limit();  // unique ids one pass of the wave kernel takes
qw_status launch_dedup_wave(const DedupArgs &a, int grid, hipStream_t s);
size_t select_lds_bytes(int LC, int dtype, int dp);
qw_status launch_select(const SelectArgs &a, int64_t Q, hipStream_t s);
// Scratch bytes launch_scan_u32_to_u64 needs for `count` values.
size_t scan_scratch_bytes(int64_t count);

// ---------------------------------------------------------------- model
qw_status launch_mlp_features(const uint32_t *bsize, int64_t Q, int32_t L, float *feats,
                              hipStream_t s);
qw_status launch_mlp_predict_bf16(const float *params, int32_t L, const float *feats,
                                  int64_t B, float *out, hipStream_t s);
qw_status launch_mlp_loss_grad(const float *params, int32_t L, const float *feats,
                               const float *targets, int32_t B, float *grad, float *loss,
                               hipStream_t s);
qw_status launch_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t P,
                          int32_t step, float lr, float b1, float b2, float eps,
                          hipStream_t s);

// ---------------------------------------------------------------- misc
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int ceil_log2(uint64_t v) {
    int r = 0;
    while ((1ull << r) < v) ++r;
    return r;
}

}  // namespace qw
