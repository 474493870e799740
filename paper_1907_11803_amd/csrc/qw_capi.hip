// C ABI of libqwlsh: argument validation, workspace, and the two execution forms
// of the query-workload pipeline (hash -> probe -> schedule -> verify/top-K).
#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <new>
#include <random>
#include <vector>

#include "qw_internal.h"
#include "qw_mlp.h"

using namespace qw;

// Device scratch of qw_query_workload_noalloc (see carve_plain_ws below): one
// copy per GPU, held until the process ends.  Host code never passes this
// name to a kernel or a copy: it takes the device address from
// hipGetSymbolAddress once per device and uses that.
constexpr size_t kNoAllocBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kCmin = 10;
constexpr int kMaxClasses = 16;

// counters buffer: u64 [kC64] then u32 [kC32]
enum {
    C_UNUSED = 0, C_UNIQUE, C_PROBEHIT, C_CANDTOT, C_CLASS /* .. C_CLASS+15 */,
    C_ALLOC = 20 /* .. +kXcd-1 */, C_FAIL = 28 /* .. +kXcd-1 */, C_SPARE = 36,
    C_RECOMP = 40 /* .. +kRecompSlots-1 */, kC64 = C_RECOMP + kRecompSlots
};
// u32: overflow-queue lengths per class (queue i holds queries that overflowed
// class i-1), fallback queue, misc, then kXcd work counters per class
enum { W_CLSDONE = 0, W_TOPK2 = 1, W_WORK = 2 /* .. 5: counting split counts; .. 15 unused */, W_QCNT = 16 /* .. 32 */, W_SIMPLE = 33, W_MAX = 34,
       W_DUMMY = 35, W_QMERGED = 36, W_FB = 44, W_FBWORK = 45, W_STAGE = 46, W_XWORK = 48,
       kC32 = W_XWORK + kXcd * (kMaxClasses + 1) };
constexpr int kQueueMerged = kMaxClasses + 1;  // overflow queue of the merged launch
constexpr uint32_t kStageChunk = 16;   // staged kernel: consecutive items per workgroup run
constexpr int kStageBlocksPerCu = 2;   // its LDS (80 KiB) allows two workgroups per CU
constexpr int64_t kCandPerQuery = 4096;  // pair space reserved per query (beyond: fallback)


inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned long long *c64(qw_index *ix) { return ix->ws.counters.as<unsigned long long>(); }
inline uint32_t *c32(qw_index *ix) { return reinterpret_cast<uint32_t *>(c64(ix) + kC64); }

int pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

void drop_graphs(qw_index *ix)
{
    for (auto &g : ix->graphs) (void)hipGraphExecDestroy(g.second);
    ix->graphs.clear();
}

Plan make_plan(qw_index *ix, int K)
{
    auto hit = ix->plans.find(K);
    if (hit != ix->plans.end()) return hit->second;
    Plan p;
    p.buf = pow2_at_least(std::max(64, 2 * (K + verify_per_iter(ix->dp, ix->dtype))));
    const int rbytes = ix->dp * (ix->dtype == QW_U8 ? 1 : 4);
    int c = kCmin;
    while (c + 1 < 30 && (int)(c + 1 - kCmin) < kMaxClasses - 1 &&
           dedup_lds_bytes(c + 1, 0, ix->nl, rbytes) <= ix->lds_max)
        ++c;
    p.cmax = c;
    p.ncls = (p.cmax - kCmin + 1) + 1;
    // largest LDS set that does not lower the dedup kernel's occupancy (its
    // registers bound it first): smaller sets save nothing
    p.cfloor = kCmin;
    {
        const int nb0 = dedup_blocks_per_cu(dedup_lds_bytes(kCmin, 0, ix->nl, rbytes), ix->dtype);
        while (p.cfloor < p.cmax &&
               dedup_blocks_per_cu(dedup_lds_bytes(p.cfloor + 1, 0, ix->nl, rbytes), ix->dtype) >= nb0)
            ++p.cfloor;
    }
    const uint64_t bound = std::min<uint64_t>((uint64_t)ix->nl * (uint64_t)std::max<int64_t>(1, ix->max_bucket),
                                              (uint64_t)ix->n);
    p.cap_g = p.cmax + 1;
    while ((3ull << p.cap_g) < 4 * bound) ++p.cap_g;  // load factor <= 3/4
    const double per_wg = std::ldexp(4.0, p.cap_g);
    const double budget = 2.0 * 1024 * 1024 * 1024;
    p.grid_g = (int)std::max(1.0, std::min((double)ix->cus, std::floor(budget / per_wg)));
    for (int i = 0; i + 1 < p.ncls; ++i)
        p.dgrid[i] = dedup_blocks_per_cu(dedup_lds_bytes(kCmin + i, 0, ix->nl, rbytes), ix->dtype) * ix->cus;
    p.dgrid[p.ncls - 1] = p.grid_g;
    // select list: a few K keys in the usual case (512 entries at K <= 128;
    // a list beyond it sends the query to the fallback); K <= 1024 keeps
    // LC <= 4096 (32 KiB of keys, 64 KiB with the FP64 re-rank of float data)
    static_assert(kMaxTopK <= 1024 && kBlock <= 1024, "select list sizing");
    p.LC = pow2_at_least(std::max(512, 4 * K));
    // uint8 rows of at most 64 parts and small K: the dedup kernel selects
    // the top K itself
    p.topk = (ix->dtype == QW_U8 && K <= kFusedTopK && rbytes / 16 <= 64) ? K : 0;
    p.wgrid = dedup_wave_applies(ix->dtype, ix->dp, ix->nl, p.topk) ? dedup_wave_blocks_per_cu() * ix->cus : 0;
    // the wave kernel's set takes 1536 unique ids per pass; a query's lists
    // hold about nl * mean_hit_bucket entries, of which duplicates across
    // layers remove a good part: the wave kernel while that stays within two
    // sets' worth (beyond, extra passes re-read the ids and the workgroup
    // kernel's larger sets pay)
    p.wave_default = p.wgrid > 0 && (double)ix->nl * ix->mean_hit_bucket <= 2.0 * dedup_wave_set_limit();
    {  // FP32 distance bound of the dedup kernel's verification (float data)
        const int parts = ix->dp * (ix->dtype == QW_U8 ? 1 : 4) / 16;
        int G = 1;
        while (G < parts && G < 64) G <<= 1;
        const int P = (parts + G - 1) / G;
        p.eps = (float)((4 * P + 16) * std::ldexp(1.0, -24) + (ix->d + 2) * std::ldexp(1.0, -52));
    }
    ix->plans[K] = p;
    return p;
}

// Grow the query workspace for Q queries (keys: the key list of the select
// kernel); drops captured graphs when any buffer moves.
qw_status ensure_ws(qw_index *ix, int64_t Q, const Plan *plan, bool keys = false)
{
    Workspace &w = ix->ws;
    auto ptrs = [&w]() {
        return std::vector<void *>{w.qpad.p, w.h.p, w.bstart.p, w.bsize.p, w.bmh.p, w.lsum.p,
                                   w.lmh.p, w.moves.p, w.pred.p,
                                   w.feats.p, w.keys.p, w.keys2.p, w.vals.p, w.vals2.p,
                                   w.binoff.p, w.counters.p, w.ovf.p, w.gscratch.p, w.mlpout.p,
                                   w.order.p,
                                   w.hist.p, w.scan.p, w.ucount.p, w.coff.p, w.flag.p,
                                   w.pkeys.p, w.fb.p};
    };
    const std::vector<void *> before = ptrs();
    // two passes: the first adds up what the buffers must grow by and refuses
    // a workload beyond the device's free memory before anything is
    // allocated; the second grows them
    size_t extra = 0;
    bool dry = true;
    auto grow = [&](DevBuf &b, size_t want) -> qw_status {
        if (!dry) {
            const qw_status rc = b.ensure(want);
            if (rc != QW_OK) drop_graphs(ix);  // a buffer may have moved before the failure
            return rc;
        }
        if (!b.p || want > b.bytes) extra += want - std::min(want, b.bytes) + 256;
        return QW_OK;
    };
    for (int pass = 0; pass < 2; ++pass, dry = false) {
        if (!dry) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && extra > free_b) return QW_ENOMEM;
            (void)hipGetLastError();
        }
        const size_t elem = ix->dtype == QW_U8 ? 1 : 4;
        const int64_t q = std::max<int64_t>(Q, 1);
        QW_TRY(grow(w.qpad, elem * (size_t)q * ix->dp));
        QW_TRY(grow(w.h, sizeof(int32_t) * (size_t)q * ix->nf));
        QW_TRY(grow(w.bstart, sizeof(uint32_t) * (size_t)q * ix->nl));
        QW_TRY(grow(w.bsize, sizeof(uint32_t) * (size_t)q * ix->nl));
        QW_TRY(grow(w.bmh, sizeof(uint32_t) * (size_t)q * ix->nl));
        if (ix->nprobe > 1) {
            QW_TRY(grow(w.lsum, sizeof(uint32_t) * (size_t)q * ix->L));
            QW_TRY(grow(w.lmh, sizeof(uint32_t) * (size_t)q * ix->L));
        }
        if (ix->probe_mode == 2) QW_TRY(grow(w.moves, (size_t)q * ix->L * (ix->nprobe - 1)));
        QW_TRY(grow(w.pred, sizeof(int32_t) * q));
        QW_TRY(grow(w.feats, sizeof(float) * (size_t)q * ix->L));
        QW_TRY(grow(w.mlpout, sizeof(float) * q));
        QW_TRY(grow(w.keys, sizeof(unsigned long long) * q));
        QW_TRY(grow(w.keys2, sizeof(unsigned long long) * q));
        QW_TRY(grow(w.vals, sizeof(int32_t) * q));
        QW_TRY(grow(w.vals2, sizeof(int32_t) * q));
        QW_TRY(grow(w.ovf, sizeof(int32_t) * q * (kQueueMerged + 1)));  // one queue per class + merged
        QW_TRY(grow(w.binoff, sizeof(unsigned long long) * 2 * kMaxClasses));
        QW_TRY(grow(w.order, sizeof(int32_t) * (size_t)kMaxClasses * q));  // per-class lists
        QW_TRY(grow(w.counters, sizeof(unsigned long long) * kC64 + sizeof(uint32_t) * kC32));
        QW_TRY(grow(w.hist, radix_sort_scratch_bytes(q)));
        QW_TRY(grow(w.scan, scan_scratch_bytes(q)));
        QW_TRY(grow(w.ucount, sizeof(uint32_t) * q));  // |C(q)|, written on every path
        if (plan) {
            const size_t g = (size_t)plan->grid_g * (size_t(1) << plan->cap_g) * 4;
            QW_TRY(grow(w.gscratch, g));
            // one equal region per XCD, each with room for its share of the
            // queries plus one chunk of items per dedup launch (at most ncls + 1)
            const int64_t slack = (int64_t)kXcd * kXcdChunk * (plan->ncls + 1);
            const int64_t cand_cap = std::max<int64_t>((q + slack) * kCandPerQuery, 1 << 20);
            QW_TRY(grow(w.coff, sizeof(unsigned long long) * q));
            QW_TRY(grow(w.flag, sizeof(uint32_t) * q));
            if (keys) QW_TRY(grow(w.pkeys, sizeof(unsigned long long) * cand_cap));
            QW_TRY(grow(w.fb, sizeof(int32_t) * q));
        }
    }
    if (before != ptrs()) drop_graphs(ix);
    return QW_OK;
}

VerifyArgs base_args(qw_index *ix, int K, int mode)
{
    VerifyArgs a;
    std::memset(&a, 0, sizeof(a));
    a.bstart = ix->ws.bstart.as<uint32_t>();
    a.bsize = ix->ws.bsize.as<uint32_t>();
    a.ids = ix->ids.as<int32_t>();
    a.n = ix->n;
    a.nl = ix->nl;
    a.pmagic = ix->pmagic;
    a.d = ix->d;
    a.dp = ix->dp;
    a.dtype = ix->dtype;
    a.K = K;
    a.mode = mode;
    a.data = ix->data.p;
    a.queries = ix->ws.qrows;
    a.ovf_count = c32(ix) + W_DUMMY;  // callers that can overflow set a real queue
    a.ovf_list = ix->ws.ovf.as<int32_t>();
    a.ucount_out = ix->ws.ucount.as<uint32_t>();
    return a;
}

// The query rows the kernels read: the caller's own rows when they need no
// padding (d a multiple of 16 elements, 16-byte aligned address), else a
// zero-padded copy in the workspace.  Sets ix->ws.qrows.
qw_status stage_query_rows(qw_index *ix, const void *x, int64_t m, hipStream_t s)
{
    if (ix->d == ix->dp && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        ix->ws.qrows = x;
        return QW_OK;
    }
    QW_TRY(launch_pad_rows(x, m, ix->d, ix->dp, ix->dtype, ix->ws.qpad.p, s));
    ix->ws.qrows = ix->ws.qpad.p;
    return QW_OK;
}

// Per (query, layer) bucket sizes and min-hashes, as the schedule and the
// count model read them: the lists themselves without neighbour probing, the
// sums (smallest min-hash) over each layer's lists with it.
const uint32_t *layer_sizes(qw_index *ix)
{
    return ix->nprobe > 1 ? ix->ws.lsum.as<uint32_t>() : ix->ws.bsize.as<uint32_t>();
}
const uint32_t *layer_mh(qw_index *ix)
{
    return ix->nprobe > 1 ? ix->ws.lmh.as<uint32_t>() : ix->ws.bmh.as<uint32_t>();
}

// stage rows -> hash -> probe for Q queries (counters must already be cleared);
// feats (nullable) receives the count-model inputs log(1 + s_{q,l}) (s: the
// layer's size), bmh (nullable) the buckets' min-hashes
// Words of the counters buffer (zeroed at the start of every call).
constexpr int64_t kCounterWords = (int64_t)(sizeof(unsigned long long) * kC64 + sizeof(uint32_t) * kC32) / 4;

// clear_in_moves: the caller has not zeroed the counters; the query-directed
// move kernel, the first kernel of this path to run, zeroes them (the fast
// form with query-directed probing only).
qw_status front(qw_index *ix, const void *queries, int64_t Q, int form, hipStream_t s,
                hipEvent_t *ev = nullptr, float *feats = nullptr, uint32_t *bmh = nullptr,
                bool clear_in_moves = false)
{
    QW_TRY(stage_query_rows(ix, queries, Q, s));
    const bool probed = ix->nprobe > 1;
    uint32_t *lsum = probed ? ix->ws.lsum.as<uint32_t>() : nullptr;
    uint32_t *lmh = probed && bmh ? ix->ws.lmh.as<uint32_t>() : nullptr;
    // query-directed probing chooses its moves from FP64 index-order
    // projections, whose floors are the exact hash values: the fast form
    // takes them from there and runs no other hashing
    const bool moves_hash = ix->probe_mode == 2 && form == QW_FORM_FAST;
    if (clear_in_moves && !moves_hash) return QW_EINTERNAL;
    if (!moves_hash)
        QW_TRY(launch_hash(ix, ix->ws.qrows, Q, 0, ix->nf, form, ix->ws.h.as<int32_t>(), ix->nf,
                           c64(ix) + C_RECOMP, s));
    const uint8_t *moves = nullptr;
    if (ix->probe_mode == 2) {
        QW_TRY(launch_probe_moves(ix, ix->ws.qrows, Q, ix->ws.moves.as<uint8_t>(),
                                  moves_hash ? ix->ws.h.as<int32_t>() : nullptr, s,
                                  clear_in_moves ? ix->ws.counters.as<uint32_t>() : nullptr,
                                  clear_in_moves ? (int32_t)kCounterWords : 0));
        moves = ix->ws.moves.as<uint8_t>();
    }
    if (ev) QW_HIP(hipEventRecord(ev[1], s));
    QW_TRY(launch_probe(ix, ix->ws.h.as<int32_t>(), Q, ix->ws.bstart.as<uint32_t>(),
                        ix->ws.bsize.as<uint32_t>(), feats, bmh, moves, lsum, lmh, s));
    return QW_OK;
}

qw_status clear_counters(qw_index *ix, hipStream_t s)
{
    return launch_fill_u32(ix->ws.counters.as<uint32_t>(), 0u, kCounterWords, s);
}

// One hash-set size for all queries (from the largest bound), one workgroup per
// query.  Used by the plain form and by the introspection calls.  Syncs.
// may_alloc = false (the allocation-free entry point): a set beyond LDS, which
// would need global scratch, returns QW_EUNSUPPORTED before any verification.
qw_status verify_simple(qw_index *ix, int64_t Q, int K, int mode, hipStream_t s,
                        int32_t *out_ids, void *out_dist, int32_t *out_counts,
                        const long long *offsets, hipEvent_t ev_sched = nullptr,
                        bool may_alloc = true)
{
    uint32_t *mx = c32(ix) + W_MAX;
    QW_TRY(launch_fill_u32(mx, 0u, 1, s));
    QW_TRY(launch_max_bucket_sum(layer_sizes(ix), Q, ix->L, mx, s));
    uint32_t maxsum = 0;
    QW_HIP(hipMemcpyAsync(&maxsum, mx, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    if (ev_sched) QW_HIP(hipEventRecord(ev_sched, s));
    const uint64_t bound = std::min<uint64_t>(maxsum, (uint64_t)ix->n);
    int cap = kCmin;
    while ((3ull << cap) < 4 * bound) ++cap;  // load factor <= 3/4: never overflows
    VerifyArgs a = base_args(ix, K, mode);
    const int buf = pow2_at_least(std::max(64, 2 * (K + verify_per_iter(ix->dp, ix->dtype))));
    a.buf = (uint32_t)buf;
    a.nitems = Q;
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    a.out_counts = out_counts;
    a.offsets = offsets;
    if (verify_lds_bytes(cap, buf, 0, ix->nl, ix->dp, ix->dtype) <= ix->lds_max) {
        a.cap_log2 = (uint32_t)cap;
        a.limit = (1u << cap) / 4 * 3;
        return launch_verify(a, (int)Q, s);
    }
    // very large candidate sets: hash sets in global scratch, persistent workgroups
    if (!may_alloc) return QW_EUNSUPPORTED;
    const int grid = (int)std::min<int64_t>(Q, ix->cus);
    void *old = ix->ws.gscratch.p;
    QW_TRY(ix->ws.gscratch.ensure((size_t)grid * (size_t(1) << cap) * 4));
    if (ix->ws.gscratch.p != old) drop_graphs(ix);  // captured graphs hold the old pointer
    a.cap_log2 = (uint32_t)cap;
    a.limit = (1u << cap) / 4 * 3;
    a.global_tab = 1;
    a.gscratch = ix->ws.gscratch.as<uint32_t>();
    a.counter = c32(ix) + W_SIMPLE;
    QW_TRY(launch_fill_u32(a.counter, 0u, 1, s));
    return launch_verify(a, grid, s);
}

// Collision counting: one set size for all queries (from the largest list
// total), one workgroup per query.  Checks the limits before anything is
// written to the outputs; syncs.
qw_status count_query(qw_index *ix, int64_t Q, int K, hipStream_t s, int32_t *out_ids,
                      void *out_dist, hipEvent_t ev_sched)
{
    if (ix->nprobe != 1 || (int64_t)K + ix->count_extra > kMaxTopK || ix->n >= kCountMaxN)
        return QW_EUNSUPPORTED;
    // the queries split by their listed ids (the smaller sets let more
    // workgroups share a CU); both lists' sizes and largest sums read back
    uint32_t *cnt = c32(ix) + W_WORK;  // n0, n1, max0, max1
    if (!ix->ws.order.p || ix->ws.order.bytes < sizeof(int32_t) * 2 * (size_t)Q) return QW_EINTERNAL;
    int32_t *list0 = ix->ws.order.as<int32_t>(), *list1 = list0 + Q;
    QW_TRY(launch_fill_u32(cnt, 0u, 4, s));
    QW_TRY(launch_count_split(ix->ws.bsize.as<uint32_t>(), Q, ix->L, kCountSmallListed, list0, list1,
                              cnt, s));
    uint32_t h[4] = {0, 0, 0, 0};
    QW_HIP(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    if (ev_sched) QW_HIP(hipEventRecord(ev_sched, s));
    if (h[0] + h[1] != (uint64_t)Q || h[2] > kCountSmallListed) return QW_EINTERNAL;
    if (h[3] > kCountMaxListed) return QW_EUNSUPPORTED;
    auto cap_for = [](uint32_t listed) {
        int c = 8;
        while ((3ull << c) < 4ull * listed) ++c;  // load factor <= 3/4
        return c;
    };
    CountArgs a;
    std::memset(&a, 0, sizeof(a));
    a.bstart = ix->ws.bstart.as<uint32_t>();
    a.bsize = ix->ws.bsize.as<uint32_t>();
    a.ids = ix->ids.as<int32_t>();
    a.n = ix->n;
    a.L = ix->L;
    a.theta = ix->count_theta;
    a.K = K;
    a.extra = ix->count_extra;
    a.ncap = (K + ix->count_extra + 1) & ~1;
    a.dtype = ix->dtype;
    a.dp = ix->dp;
    a.data = ix->data.p;
    a.queries = ix->ws.qrows;
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    a.out_counts = ix->ws.ucount.as<uint32_t>();
    // the radix selects skip bytes no value reaches: ids are below n; a uint8
    // squared distance is at most dp * 255^2; a float key's high word is that
    // of a non-negative FP64 value (below 2^31)
    auto top_byte = [](uint64_t bound) {  // 8 * floor(log2(bound) / 8)
        int b = 0;
        while (b < 24 && (bound >> (b + 8)) != 0) b += 8;
        return b;
    };
    a.id_top = top_byte((uint64_t)std::max<int64_t>(1, ix->n - 1));
    a.key_top = ix->dtype == QW_U8 ? top_byte((uint64_t)ix->dp * 65025ull) : 24;
    const int cap0 = cap_for(h[2]), cap1 = cap_for(h[3]);
    for (int c : {cap0, cap1})  // both checked before either writes an output
        if (c > kCountMaxSetLog2 || count_lds_bytes(c, a.ncap) > ix->lds_max) return QW_EUNSUPPORTED;
    a.cap_log2 = (uint32_t)cap0;
    a.qlist = list0;
    QW_TRY(launch_count(a, h[0], false, s));
    a.cap_log2 = (uint32_t)cap1;
    a.qlist = list1;
    return launch_count(a, h[1], true, s);
}

// Out-of-core answer of Q probed queries: one hash-set size for all queries
// (from the largest list total, read back: the call synchronises), then the
// batches through the caches.  Refuses a set beyond on-chip memory.
qw_status ooc_query(qw_index *ix, int64_t Q, int K, hipStream_t s, int32_t *out_ids,
                    void *out_dist, OocIo *io, hipEvent_t ev_sched)
{
    uint32_t *mx = c32(ix) + W_MAX;
    QW_TRY(launch_fill_u32(mx, 0u, 1, s));
    QW_TRY(launch_max_bucket_sum(ix->ws.bsize.as<uint32_t>(), Q, ix->L, mx, s));
    uint32_t maxsum = 0;
    QW_HIP(hipMemcpyAsync(&maxsum, mx, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    if (ev_sched) QW_HIP(hipEventRecord(ev_sched, s));
    const uint64_t bound = std::min<uint64_t>(maxsum, (uint64_t)ix->n);
    int cap = kCmin;
    while ((3ull << cap) < 4 * bound) ++cap;  // load factor <= 3/4: never overflows
    VerifyArgs a = base_args(ix, K, VM_TOPK);
    const int buf = pow2_at_least(std::max(64, 2 * (K + verify_per_iter(ix->dp, ix->dtype))));
    if (verify_lds_bytes(cap, buf, 0, ix->nl, ix->dp, ix->dtype) > ix->lds_max)
        return QW_EUNSUPPORTED;
    a.buf = (uint32_t)buf;
    a.cap_log2 = (uint32_t)cap;
    a.limit = (1u << cap) / 4 * 3;
    return ooc_answer(ix, Q, a, ix->ws.qrows, out_ids, out_dist, s, io);
}

qw_status check_index(const qw_index *ix)
{
    if (!ix) return QW_EINVAL;
    int dev = -1;
    QW_HIP(hipGetDevice(&dev));
    if (dev != ix->device) return QW_EINVAL;
    return QW_OK;
}

// Fast form: exact MFMA hashing, probe, schedule (size classes from the
// selected count source, optional bucket grouping), per-class dedup kernels
// that verify their candidates and either select the top K themselves or
// write keys into per-XCD regions for the select kernel, then the fallback.
qw_status enqueue_fast(qw_index *ix, const Plan &plan, const void *queries, int64_t Q, int K,
                       const qw_opts &o, hipStream_t s, int32_t *out_ids, void *out_dist,
                       hipEvent_t *ev)
{
    Workspace &w = ix->ws;
    if (ev) QW_HIP(hipEventRecord(ev[0], s));
    // with query-directed probing the move kernel runs first and zeroes the
    // counters itself (one launch fewer per call)
    const bool clear_in_moves = ix->probe_mode == 2;
    if (!clear_in_moves) QW_TRY(clear_counters(ix, s));
    // the staged kernel writes keys for the select kernel
    const bool stage = o.stage_split > 0;
    const int topk = !stage && o.topk_keep >= 0 ? plan.topk : 0;  // in-kernel top K
    const bool learned = o.sched == QW_SCHED_LEARNED && !ix->mlp.empty();
    // the binning kernel runs the count model itself; the grouped schedule
    // takes the predictions from the inference kernel
    QW_TRY(front(ix, queries, Q, QW_FORM_FAST, s, ev,
                 learned && o.group ? w.feats.as<float>() : nullptr,
                 o.group ? w.bmh.as<uint32_t>() : nullptr, clear_in_moves));
    if (ev) QW_HIP(hipEventRecord(ev[2], s));
    unsigned long long *seg = w.binoff.as<unsigned long long>();
    unsigned long long *ccount = c64(ix) + C_CLASS;
    int32_t *queues = w.ovf.as<int32_t>();
    const int64_t cand_cap = (int64_t)(w.pkeys.bytes / sizeof(unsigned long long));
    auto schedule = [&](const int32_t *ex, const float *pl, int force_max,
                        const int32_t **order) -> qw_status {
        if (!o.group) {  // classes only: one binning kernel (with the count model)
            QW_TRY(launch_classify_bin(Q, ix->L, ix->n, layer_sizes(ix), ex,
                                       learned && !ex ? ix->mlp_lane.as<uint32_t>() : nullptr,
                                       ix->mlp_margin, force_max, kCmin, plan.cfloor, plan.cmax,
                                       plan.ncls, w.order.as<int32_t>(), ccount,
                                       c32(ix) + W_CLSDONE, seg, s));
            *order = w.order.as<int32_t>();
            return QW_OK;
        }
        QW_TRY(launch_classify(Q, ix->L, ix->n, layer_mh(ix),
                               layer_sizes(ix), ex, pl, ix->mlp_margin, force_max, kCmin,
                               plan.cfloor, plan.cmax, plan.ncls, o.group, w.keys.as<unsigned long long>(),
                               w.vals.as<int32_t>(), ccount, s));
        bool alt = false;
        QW_TRY(radix_sort_pairs(w.keys.as<unsigned long long>(), w.vals.as<int32_t>(), Q,
                                o.group ? 0 : 16, 24, w.keys2.as<unsigned long long>(),
                                w.vals2.as<int32_t>(), w.hist, s, &alt));
        *order = alt ? w.vals2.as<int32_t>() : w.vals.as<int32_t>();
        QW_TRY(launch_segments(ccount, plan.ncls, seg, s));
        return QW_OK;
    };
    // Classes run from the smallest hash set to the global one.  Each launch
    // serves its segment of the order, then the queue of queries that
    // overflowed the previous class; its own overflows go to the next queue.
    // One launch serves every LDS class up to cfloor (their sets cost no
    // occupancy, so the launch is sized for the largest; queries go largest
    // first).  The larger classes run beside it on the side stream, one launch
    // each, each serving its segment and then the queue of queries that
    // overflowed the class before it; queries that overflow the merged launch
    // are served afterwards by the global class.
    auto dedup_classes = [&](const int32_t *order, int count_only) -> qw_status {
        if (stage && !count_only) {  // index/data caches in LDS at the chosen split
            StageArgs a;
            std::memset(&a, 0, sizeof(a));
            a.order = order;
            a.seg = seg;
            a.ncls = plan.ncls;
            a.counter = c32(ix) + W_STAGE;
            a.chunk = kStageChunk;
            a.bstart = w.bstart.as<uint32_t>();
            a.bsize = w.bsize.as<uint32_t>();
            a.ids = ix->ids.as<int32_t>();
            a.n = ix->n;
            a.nl = ix->nl;
            a.pmagic = ix->pmagic;
            a.dp = ix->dp;
            a.dtype = ix->dtype;
            a.data = ix->data.p;
            a.queries = w.qrows;
            a.keys = w.pkeys.as<unsigned long long>();
            a.alloc = c64(ix) + C_ALLOC;
            a.fail = c64(ix) + C_FAIL;
            a.region = (unsigned long long)(cand_cap / kXcd);
            a.ucount = w.ucount.as<uint32_t>();
            a.coff = w.coff.as<unsigned long long>();
            a.flag = w.flag.as<uint32_t>();
            (void)stage_lds_bytes(ix->dp * (ix->dtype == QW_U8 ? 1 : 4), o.stage_split, &a.icn, &a.dcn);
            return launch_stage(a, kStageBlocksPerCu * ix->cus, s);
        }
        // gpart (global class only): 0 = the whole grid and scratch, 1 / 2 =
        // the first / second half of them, so two global-class launches can
        // run at once on disjoint sets
        auto launch_range = [&](int lo, int hi, const int32_t *in_list, const uint32_t *in_count,
                                int32_t *ovf_list, uint32_t *ovf_count, int slot, int queue_only,
                                hipStream_t st, int gpart = 0) -> qw_status {
            DedupArgs a;
            std::memset(&a, 0, sizeof(a));
            a.order = order;
            a.seg = seg;
            a.cls_lo = lo;
            a.cls_hi = hi;
            a.queue_only = queue_only;
            a.cap_base = kCmin;
            a.xchunk = o.group ? (o.xchunk > 0 ? (uint32_t)o.xchunk : kXcdChunk) : 1u;
            a.xwork = c32(ix) + W_XWORK + kXcd * slot;
            a.in_list = in_list;
            a.in_count = in_count;
            a.ovf_list = ovf_list;
            a.ovf_count = ovf_count;
            a.bstart = w.bstart.as<uint32_t>();
            a.bsize = w.bsize.as<uint32_t>();
            a.ids = ix->ids.as<int32_t>();
            a.n = ix->n;
            a.nl = ix->nl;
            a.pmagic = ix->pmagic;
            a.count_only = count_only;
            a.alloc = c64(ix) + C_ALLOC;
            a.fail = c64(ix) + C_FAIL;
            a.region = (unsigned long long)(cand_cap / kXcd);
            a.dp = ix->dp;
            a.dtype = ix->dtype;
            a.data = ix->data.p;
            a.queries = w.qrows;
            {
                const uint64_t rb = (uint64_t)ix->dp * (ix->dtype == QW_U8 ? 1 : 4);
                a.addr32 = (uint64_t)ix->n * rb < (1ull << 32) && ix->n < (1ll << 24) ? 1 : 0;
            }
            a.keys = w.pkeys.as<unsigned long long>();
            a.topk = topk;
            a.topk_keep = o.topk_keep == 0 ? 3 : o.topk_keep;
            a.out_ids = out_ids;
            a.out_dist = out_dist;
            a.fb_count = c32(ix) + W_FB;
            a.fb_list = w.fb.as<int32_t>();
            a.topk2_count = c32(ix) + W_TOPK2;
            a.ucount = w.ucount.as<uint32_t>();
            a.coff = w.coff.as<unsigned long long>();
            a.flag = w.flag.as<uint32_t>();
            if (hi == plan.ncls - 1) {
                a.cap_log2 = (uint32_t)plan.cap_g;
                a.limit = (1u << plan.cap_g) / 4 * 3;
                a.global_tab = 1;
                const int half = plan.grid_g / 2;
                a.gscratch = w.gscratch.as<uint32_t>() +
                             (gpart == 2 ? (size_t)half << plan.cap_g : size_t(0));
                if (gpart) return launch_dedup(a, gpart == 1 ? half : plan.grid_g - half, st);
            } else {
                a.cap_log2 = (uint32_t)(kCmin + hi);  // LDS size; also the queue's class
                a.limit = 0xFFFFFFFFu;                 // each set's own 3/4 bound
            }
            return launch_dedup(a, plan.dgrid[hi], st);
        };
        const bool wave = plan.wgrid > 0 && o.dedup == 2;  // o: settings resolved by the caller
        if (wave && topk && !count_only) {
            // one wave per query over every class, largest first; sets that
            // overflow split into id-hash passes inside the kernel
            DedupArgs a;
            std::memset(&a, 0, sizeof(a));
            a.order = order;
            a.seg = seg;
            a.cls_lo = 0;
            a.cls_hi = plan.ncls - 1;
            a.cap_base = kCmin;
            a.xchunk = o.group ? (o.xchunk > 0 ? (uint32_t)o.xchunk : kXcdChunk) : 1u;
            a.ovf_count = c32(ix) + W_QMERGED;
            a.bstart = w.bstart.as<uint32_t>();
            a.bsize = w.bsize.as<uint32_t>();
            a.ids = ix->ids.as<int32_t>();
            a.n = ix->n;
            a.nl = ix->nl;
            a.pmagic = ix->pmagic;
            a.dp = ix->dp;
            a.dtype = ix->dtype;
            a.data = ix->data.p;
            a.queries = w.qrows;
            a.addr32 = (uint64_t)ix->n * (uint64_t)ix->dp < (1ull << 32) && ix->n < (1ll << 24) ? 1 : 0;
            a.topk = topk;
            a.topk_keep = o.topk_keep == 0 ? dedup_wave_keep() : o.topk_keep;
            a.out_ids = out_ids;
            a.out_dist = out_dist;
            a.fb_count = c32(ix) + W_FB;
            a.fb_list = w.fb.as<int32_t>();
            a.topk2_count = c32(ix) + W_TOPK2;
            a.ucount = w.ucount.as<uint32_t>();
            return launch_dedup_wave(a, plan.wgrid, s);
        }
        const int merged = std::max(0, std::min(plan.cfloor - kCmin, plan.ncls - 2));
        const int glob = plan.ncls - 1;
        // with two or more global-class workgroups, the side stream's global
        // class and the merged launch's overflow each take half of them (and
        // of their scratch sets), so the latter follows the merged launch on
        // its own stream instead of waiting for the side stream first
        const int gsplit = plan.grid_g >= 2 ? 1 : 0;
        QW_HIP(hipEventRecord(ix->fork[0], s));
        QW_HIP(hipStreamWaitEvent(ix->side, ix->fork[0], 0));
        for (int i = merged + 1; i < plan.ncls; ++i) {
            const bool first = i == merged + 1;
            QW_TRY(launch_range(i, i, first ? nullptr : queues + (int64_t)i * Q,
                                first ? nullptr : c32(ix) + W_QCNT + i,
                                queues + (int64_t)(i + 1) * Q, c32(ix) + W_QCNT + i + 1, i, 0,
                                ix->side, i == glob ? gsplit : 0));
        }
        QW_TRY(launch_range(0, merged, nullptr, nullptr, queues + (int64_t)kQueueMerged * Q,
                            c32(ix) + W_QMERGED, merged, 0, s));
        QW_HIP(hipEventRecord(ix->fork[1], ix->side));
        if (!gsplit) QW_HIP(hipStreamWaitEvent(s, ix->fork[1], 0));
        // overflow of the merged launch (usually none): the global class, queue only
        QW_TRY(launch_range(glob, glob, queues + (int64_t)kQueueMerged * Q, c32(ix) + W_QMERGED,
                            queues + (int64_t)(glob + 1) * Q, c32(ix) + W_DUMMY, kMaxClasses, 1, s,
                            gsplit ? 2 : 0));
        if (gsplit) QW_HIP(hipStreamWaitEvent(s, ix->fork[1], 0));
        return QW_OK;
    };
    const int32_t *order = nullptr;
    const int32_t *exact = nullptr;
    const float *pred_log = nullptr;
    if (o.sched == QW_SCHED_ACTUAL) {  // extra counting pass: exact |C(q)|
        QW_TRY(schedule(nullptr, nullptr, 0, &order));
        QW_TRY(dedup_classes(order, 1));
        QW_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ccount), 0u, 2 * kMaxClasses, s));
        QW_TRY(launch_fill_u32(c32(ix) + W_CLSDONE, 0u, W_SIMPLE - W_CLSDONE, s));
        QW_TRY(launch_fill_u32(c32(ix) + W_XWORK, 0u, kXcd * (kMaxClasses + 1), s));
        QW_TRY(launch_fill_u32(c32(ix) + W_QMERGED, 0u, 1, s));
        exact = reinterpret_cast<const int32_t *>(w.ucount.p);
    } else if (learned && o.group) {
        QW_TRY(launch_mlp_predict_bf16(ix->mlp_dev.as<float>(), ix->L, w.feats.as<float>(), Q,
                                       w.mlpout.as<float>(), s));
        pred_log = w.mlpout.as<float>();
    }
    QW_TRY(schedule(exact, pred_log, o.sched == QW_SCHED_NONE, &order));
    if (!topk) QW_TRY(launch_fill_u32(w.flag.as<uint32_t>(), 0u, Q, s));  // read by the select kernel
    if (ev) QW_HIP(hipEventRecord(ev[3], s));
    QW_TRY(dedup_classes(order, 0));
    if (ev) QW_HIP(hipEventRecord(ev[6], s));
    SelectArgs m;
    std::memset(&m, 0, sizeof(m));
    m.keys = w.pkeys.as<unsigned long long>();
    m.coff = w.coff.as<unsigned long long>();
    m.ucount = w.ucount.as<uint32_t>();
    m.flag = w.flag.as<uint32_t>();
    m.K = K;
    m.LC = plan.LC;
    m.dtype = ix->dtype;
    m.dp = ix->dp;
    m.d = ix->d;
    m.eps = plan.eps;
    m.fb_count = c32(ix) + W_FB;
    m.fb_list = w.fb.as<int32_t>();
    m.out_ids = out_ids;
    m.out_dist = out_dist;
    m.data = ix->data.p;
    m.queries = w.qrows;
    if (!topk) QW_TRY(launch_select(m, Q, s));
    if (ev) QW_HIP(hipEventRecord(ev[4], s));
    // queries flagged on the way (list space, ties or band wider than the list):
    // the fused per-query kernel with a global hash set answers them
    VerifyArgs a = base_args(ix, K, VM_TOPK);
    a.nitems = 0;
    a.in_list = w.fb.as<int32_t>();
    a.in_count = c32(ix) + W_FB;
    a.counter = c32(ix) + W_FBWORK;
    a.buf = (uint32_t)plan.buf;
    a.cap_log2 = (uint32_t)plan.cap_g;
    a.limit = (1u << plan.cap_g) / 4 * 3;
    a.global_tab = 1;
    a.gscratch = w.gscratch.as<uint32_t>();
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    QW_TRY(launch_verify(a, plan.grid_g, s));
    if (ev) QW_HIP(hipEventRecord(ev[5], s));
    return QW_OK;
}

qw_status fill_stats(qw_index *ix, int64_t Q, hipStream_t s, qw_stats *st, hipEvent_t *ev,
                     bool fast)
{
    std::memset(st, 0, sizeof(*st));
    if (Q <= 0) return QW_OK;
    QW_TRY(launch_probe_stats(ix->ws.bsize.as<uint32_t>(), Q * ix->nl, c64(ix) + C_PROBEHIT,
                              c64(ix) + C_CANDTOT, s));
    // |C(q)| of every query, written by whichever kernel answered it
    QW_TRY(launch_probe_stats(ix->ws.ucount.as<uint32_t>(), Q, c64(ix) + C_SPARE,
                              c64(ix) + C_UNIQUE, s));
    unsigned long long h64[kC64];
    uint32_t h32[kC32];
    QW_HIP(hipMemcpyAsync(h64, c64(ix), sizeof(h64), hipMemcpyDeviceToHost, s));
    QW_HIP(hipMemcpyAsync(h32, c32(ix), sizeof(h32), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    st->projections = Q * ix->nf;
    for (int i = 0; i < kRecompSlots; ++i) st->recomputed += (int64_t)h64[C_RECOMP + i];
    st->recompute_frac = (double)st->recomputed / (double)st->projections;
    st->probes_hit = (int64_t)h64[C_PROBEHIT];
    st->cand_total = (int64_t)h64[C_CANDTOT];
    st->cand_unique = (int64_t)h64[C_UNIQUE];
    st->overflow = 0;
    if (fast) {
        for (int i = 1; i <= kMaxClasses; ++i) st->overflow += (int64_t)h32[W_QCNT + i];
        st->overflow += (int64_t)h32[W_QMERGED];
    }
    st->fallback = fast ? (int64_t)h32[W_FB] : 0;
    st->topk_second_pass = fast ? (int64_t)h32[W_TOPK2] : 0;
    if (fast)
        for (int i = 0; i < 8; ++i) st->bins[i] = (int64_t)h64[C_CLASS + i];
    if (ev) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) st->ms_stage[0] = ms;
        if (hipEventElapsedTime(&ms, ev[1], ev[2]) == hipSuccess) st->ms_stage[1] = ms;
        if (hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess) st->ms_stage[2] = ms;
        if (hipEventElapsedTime(&ms, ev[3], ev[4]) == hipSuccess) st->ms_stage[3] = ms;
        if (hipEventElapsedTime(&ms, ev[4], ev[5]) == hipSuccess) st->ms_stage[4] = ms;
        if (hipEventElapsedTime(&ms, ev[0], ev[5]) == hipSuccess) st->ms_stage[5] = ms;
        if (fast) {  // dedup (with the verification, and the top K where fused), select
            if (hipEventElapsedTime(&ms, ev[3], ev[6]) == hipSuccess) st->ms_stage[6] = ms;
            if (hipEventElapsedTime(&ms, ev[6], ev[4]) == hipSuccess) st->ms_stage[7] = ms;
        }
        (void)hipGetLastError();
    }
    return QW_OK;
}

qw_status ensure_events(qw_index *ix)
{
    if (ix->ev_init) return QW_OK;
    for (auto &e : ix->ev) QW_HIP(hipEventCreate(&e));
    ix->ev_init = true;
    return QW_OK;
}

qw_status check_vectors(const qw_index *ix, const void *x, int64_t m)
{
    if (m < 0 || (m > 0 && !x)) return QW_EINVAL;
    if (m > INT32_MAX) return QW_EINVAL;
    (void)ix;
    return QW_OK;
}

// ---------------------------------------------------------------- allocation-free queries
// Device scratch of qw_query_workload_noalloc: every workspace buffer of the
// plain form's pipeline is carved from it, so that entry point allocates
// nothing.  Each GPU the library runs on holds its own copy until the process
// ends; its device address is taken once per device (hipGetSymbolAddress, with
// the device current) and only that address is handed to kernels and fills.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

qw_status scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return QW_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        QW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return QW_EDEVICE;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return QW_OK;
}

// Workspace views into `base` (kNoAllocBytes bytes) for the plain form over Q
// queries: the buffers front(), verify_simple() and count_query() read.
// Returns false when they do not fit.
bool carve_plain_ws(const qw_index *ix, int64_t Q, bool pad, unsigned char *base, Workspace &w)
{
    size_t off = 0;
    bool ok = true;
    auto take = [&](DevBuf &b, size_t bytes) {
        const size_t at = (off + 255) & ~size_t(255);
        if (!ok || bytes > kNoAllocBytes || at > kNoAllocBytes - bytes) {
            ok = false;
            return;
        }
        b.view(base + at, bytes ? bytes : 16);
        off = at + (bytes ? bytes : 16);
    };
    const size_t q = (size_t)Q;
    const size_t elem = ix->dtype == QW_U8 ? 1 : 4;
    take(w.counters, sizeof(unsigned long long) * kC64 + sizeof(uint32_t) * kC32);
    if (pad) take(w.qpad, elem * q * (size_t)ix->dp);
    take(w.h, sizeof(int32_t) * q * (size_t)ix->nf);
    take(w.bstart, sizeof(uint32_t) * q * (size_t)ix->nl);
    take(w.bsize, sizeof(uint32_t) * q * (size_t)ix->nl);
    if (ix->nprobe > 1) take(w.lsum, sizeof(uint32_t) * q * (size_t)ix->L);
    if (ix->probe_mode == 2) take(w.moves, q * (size_t)ix->L * (size_t)(ix->nprobe - 1));
    take(w.ucount, sizeof(uint32_t) * q);
    take(w.ovf, sizeof(int32_t) * q);
    if (ix->count_theta > 0) take(w.order, sizeof(int32_t) * 2 * q);  // counting's two query lists
    return ok;
}

}  // namespace

bool qw::resolve_fast_auto(qw_index *ix, int64_t Q, int32_t K, qw_opts *o, bool *wave_ok)
{
    const Plan plan = make_plan(ix, K);
    if (wave_ok) *wave_ok = plan.wgrid > 0;
    TuneEntry e;
    bool tuned = false;
    if (o->tune_cache && (o->dedup == 0 || o->group < 0 || o->xchunk == 0 || o->stage_split == 0) &&
        tune_lookup(ix, o->tune_cache, Q, K, o->sched, &e)) {
        tuned = true;
        const bool grp = o->group < 0 ? e.group != 0 : o->group != 0;
        if (o->dedup == 0) o->dedup = e.dedup;
        if (o->group < 0) o->group = e.group;
        // the tuned chunk belongs to the tuned grouping
        if (o->xchunk == 0 && grp && e.group) o->xchunk = e.xchunk;
        if (o->stage_split == 0) o->stage_split = e.split;
    }
    if (o->stage_split == 0) o->stage_split = -1;  // off unless tuned or asked for
    if (o->dedup == 0) o->dedup = plan.wgrid > 0 && plan.wave_default ? 2 : 1;
    if (o->group < 0)
        o->group = ix->dp * (ix->dtype == QW_U8 ? 1 : 4) >= kGroupRowBytes || Q >= kGroupQueries;
    if (o->xchunk == 0 && o->group) o->xchunk = (int32_t)kXcdChunk;
    if (!o->group) o->xchunk = 0;  // unused without grouping
    return tuned;
}

// ============================================================================ ABI

extern "C" {

void qw_default_opts(qw_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->form = QW_FORM_FAST;
    o->sched = QW_SCHED_LEARNED;
    o->group = -1;  // automatic: kGroupRowBytes or kGroupQueries
    o->graph = 1;
    o->timing = 0;
}

const char *qw_status_string(qw_status s)
{
    switch (s) {
    case QW_OK: return "ok";
    case QW_EINVAL: return "invalid argument";
    case QW_ENOMEM: return "out of memory";
    case QW_EDEVICE: return "HIP device error";
    case QW_EUNSUPPORTED: return "unsupported request";
    case QW_EINTERNAL: return "internal error";
    }
    return "unknown status";
}

qw_status qw_build_index(const void *data, int64_t n, int32_t d, int32_t dtype, const float *a,
                         const float *b, float w, int32_t L, int32_t k, const qw_opts *o,
                         void *stream, qw_index **out)
{
    if (!data || !a || !b || !out) return QW_EINVAL;
    if (n < 1 || n > INT32_MAX || d < 1 || d > kMaxD || L < 1 || L > kMaxL || k < 1 || k > kMaxK)
        return QW_EINVAL;
    if (dtype != QW_U8 && dtype != QW_F32) return QW_EINVAL;
    if (!std::isfinite(w) || !(w > 0.f)) return QW_EINVAL;
    if ((uint64_t)n * (uint64_t)L >= (1ull << 31)) return QW_EUNSUPPORTED;
    const int form = o ? o->form : QW_FORM_FAST;
    if (form != QW_FORM_PLAIN_FP32 && form != QW_FORM_FAST) return QW_EINVAL;
    try {
        return build_index(data, n, d, dtype, a, b, w, L, k, form, S(stream), out);
    } catch (const std::bad_alloc &) {
        return QW_ENOMEM;
    } catch (...) {
        return QW_EINTERNAL;
    }
}

void qw_free_index(qw_index *ix)
{
    if (!ix) return;
    (void)hipDeviceSynchronize();
    drop_graphs(ix);
    if (ix->ev_init)
        for (auto &e : ix->ev) (void)hipEventDestroy(e);
    delete ix;  // the destructor releases the side stream and its events
}

qw_status qw_get_index_info(const qw_index *ix, qw_index_info *info)
{
    if (!ix || !info) return QW_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->n = ix->n;
    info->d = ix->d;
    info->dtype = ix->dtype;
    info->L = ix->L;
    info->k = ix->k;
    info->w = ix->w;
    for (int l = 0; l < ix->L && l < 64; ++l) info->key_bits[l] = ix->key_bits[l];
    info->buckets = ix->buckets;
    info->max_bucket = ix->max_bucket;
    const DevBuf *bufs[] = {&ix->a32, &ix->b32, &ix->a_hi, &ix->a_lo, &ix->gb_plain,
                            &ix->gb_fast, &ix->data, &ix->hmin, &ix->hmax, &ix->shift,
                            &ix->ids, &ix->tab, &ix->tab_off, &ix->tab_mask, &ix->mlp_dev,
                            &ix->mlp_lane};
    for (const DevBuf *b : bufs) info->device_bytes += (int64_t)b->bytes;
    info->has_count_model = ix->mlp.empty() ? 0 : 1;
    info->count_margin = ix->mlp_margin;
    info->probing = ix->probe_mode;
    info->probes_per_layer = ix->nprobe - 1;
    info->count_threshold = ix->count_theta;
    info->count_extra = ix->count_extra;
    info->mean_hit_bucket = ix->mean_hit_bucket;
    info->out_of_core = ix->ooc ? 1 : 0;
    info->ooc_index_percent = ix->ooc ? ix->ooc->o.index_percent : 0;
    info->host_bytes = ix->ooc ? (int64_t)ix->ooc->host_bytes : 0;
    if (ix->ooc) {
        const OocState &o = *ix->ooc;
        for (const DevBuf *b : {&o.arena[0], &o.arena[1], &o.rows, &o.mkey, &o.msize, &o.mstamp,
                                &o.moff, &o.mnoff, &o.mneed, &o.owner, &o.freel, &o.dir,
                                &o.rstamp, &o.rneed, &o.missd, &o.copyl, &o.ckeys,
                                &o.ckeys2, &o.cvals, &o.cvals2, &o.csz, &o.cscan, &o.sort_hist,
                                &o.scan_tmp, &o.bstart2, &o.ctr})
            info->device_bytes += (int64_t)b->bytes;
    }
    return QW_OK;
}

qw_status qw_query_workload(qw_index *ix, const void *queries, int64_t Q, int32_t K,
                            const qw_opts *o, void *stream, int32_t *out_ids, void *out_dist,
                            qw_stats *st)
{
    QW_TRY(check_index(ix));
    QW_TRY(check_vectors(ix, queries, Q));
    if (K < 1 || K > kMaxTopK || (Q > 0 && (!out_ids || !out_dist))) return QW_EINVAL;
    qw_opts opt;
    if (o) opt = *o; else qw_default_opts(&opt);
    if (opt.form != QW_FORM_PLAIN_FP32 && opt.form != QW_FORM_FAST) return QW_EINVAL;
    if (opt.sched < QW_SCHED_SUM || opt.sched > QW_SCHED_NONE) return QW_EINVAL;
    if (opt.topk_keep < -1 || opt.topk_keep > 3) return QW_EINVAL;
    if (opt.group < -1 || opt.group > 1) return QW_EINVAL;
    if (opt.dedup < 0 || opt.dedup > 2 || opt.xchunk < 0 || opt.xchunk > (int32_t)kXcdChunk)
        return QW_EINVAL;
    if (opt.stage_split < -1 || opt.stage_split > 99) return QW_EINVAL;
    if (ix->ooc && opt.stage_split > 0) return QW_EUNSUPPORTED;
    // the staged kernel: fast form, at most 64 lists per query, rows of at most 4 KiB
    if (opt.stage_split > 0) {
        const int rb = ix->dp * (ix->dtype == QW_U8 ? 1 : 4);
        uint32_t icn = 0, dcn = 0;
        if (opt.form != QW_FORM_FAST || ix->nl > 64 || ix->count_theta > 0 || rb > kStageMaxRow ||
            stage_lds_bytes(rb, opt.stage_split, &icn, &dcn) > ix->lds_max)
            return QW_EUNSUPPORTED;
    }
    if (Q == 0) {
        if (st) std::memset(st, 0, sizeof(*st));
        return QW_OK;
    }
    hipStream_t s = S(stream);
    try {
        if (opt.timing) QW_TRY(ensure_events(ix));
        if (ix->ooc) {  // out of core: either form's hashing, then batches through the caches
            QW_TRY(ensure_ws(ix, Q, nullptr));
            hipEvent_t *ev = opt.timing ? ix->ev : nullptr;
            if (ev) QW_HIP(hipEventRecord(ev[0], s));
            QW_TRY(clear_counters(ix, s));
            QW_TRY(front(ix, queries, Q, opt.form, s, ev));
            if (ev) QW_HIP(hipEventRecord(ev[2], s));
            OocIo io;
            QW_TRY(ooc_query(ix, Q, K, s, out_ids, out_dist, &io, ev ? ev[3] : nullptr));
            if (ev) {
                QW_HIP(hipEventRecord(ev[4], s));
                QW_HIP(hipEventRecord(ev[5], s));
            }
            if (st) {
                QW_TRY(fill_stats(ix, Q, s, st, ev, false));
                st->ooc_index_files = io.index_files;
                st->ooc_index_bytes = io.index_bytes;
                st->ooc_data_objects = io.data_objects;
                st->ooc_data_bytes = io.data_bytes;
                st->ooc_batches = io.batches;
                st->ooc_splits = io.splits;
            }
            return QW_OK;
        }
        if (ix->count_theta > 0) {  // collision counting, either form's hashing
            QW_TRY(ensure_ws(ix, Q, nullptr));
            hipEvent_t *ev = opt.timing ? ix->ev : nullptr;
            if (ev) QW_HIP(hipEventRecord(ev[0], s));
            QW_TRY(clear_counters(ix, s));
            QW_TRY(front(ix, queries, Q, opt.form, s, ev));
            if (ev) QW_HIP(hipEventRecord(ev[2], s));
            QW_TRY(count_query(ix, Q, K, s, out_ids, out_dist, ev ? ev[3] : nullptr));
            if (ev) {
                QW_HIP(hipEventRecord(ev[4], s));
                QW_HIP(hipEventRecord(ev[5], s));
            }
            if (st) QW_TRY(fill_stats(ix, Q, s, st, ev, false));
            return QW_OK;
        }
        if (opt.form == QW_FORM_PLAIN_FP32) {
            QW_TRY(ensure_ws(ix, Q, nullptr));
            hipEvent_t *ev = opt.timing ? ix->ev : nullptr;
            if (ev) QW_HIP(hipEventRecord(ev[0], s));
            QW_TRY(clear_counters(ix, s));
            QW_TRY(front(ix, queries, Q, QW_FORM_PLAIN_FP32, s, ev));
            if (ev) QW_HIP(hipEventRecord(ev[2], s));
            QW_TRY(verify_simple(ix, Q, K, VM_TOPK, s, out_ids, out_dist, nullptr, nullptr,
                                 ev ? ev[3] : nullptr));
            if (ev) {
                QW_HIP(hipEventRecord(ev[4], s));
                QW_HIP(hipEventRecord(ev[5], s));
            }
            if (st) QW_TRY(fill_stats(ix, Q, s, st, ev, false));
            return QW_OK;
        }
        const Plan plan = make_plan(ix, K);
        const bool learned = opt.sched == QW_SCHED_LEARNED && !ix->mlp.empty();
        const int sched = opt.sched == QW_SCHED_LEARNED && !learned ? QW_SCHED_SUM : opt.sched;
        qw_opts eff = opt;
        eff.sched = sched;
        const bool tuned = resolve_fast_auto(ix, Q, K, &eff, nullptr);
        // a tuned split applies only where the staged kernel does
        if (eff.stage_split > 0) {
            const int rb = ix->dp * (ix->dtype == QW_U8 ? 1 : 4);
            uint32_t icn = 0, dcn = 0;
            if (ix->nl > 64 || rb > kStageMaxRow || stage_lds_bytes(rb, eff.stage_split, &icn, &dcn) > ix->lds_max)
                eff.stage_split = -1;
        }
        QW_TRY(ensure_ws(ix, Q, &plan, !(eff.topk_keep >= 0 && plan.topk) || eff.stage_split > 0));
        if (opt.timing || !opt.graph) {
            QW_TRY(enqueue_fast(ix, plan, queries, Q, K, eff, s, out_ids, out_dist,
                                opt.timing ? ix->ev : nullptr));
        } else {
            GraphKey key;
            std::memset(&key, 0, sizeof(key));
            key.q = queries; key.Q = Q; key.K = K; key.ids = out_ids; key.dist = out_dist;
            key.form = eff.form; key.sched = eff.sched; key.group = eff.group;
            key.topk_keep = eff.topk_keep;
            key.dedup = eff.dedup;
            key.xchunk = eff.xchunk;
            key.split = eff.stage_split;
            auto it = ix->graphs.find(key);
            if (it == ix->graphs.end()) {
                hipStream_t cs;
                QW_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                hipGraph_t g = nullptr;
                qw_status rc = QW_OK;
                if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    (void)hipStreamDestroy(cs);
                    return QW_EDEVICE;
                }
                rc = enqueue_fast(ix, plan, queries, Q, K, eff, cs, out_ids, out_dist, nullptr);
                hipError_t ec = hipStreamEndCapture(cs, &g);
                (void)hipStreamDestroy(cs);
                if (rc != QW_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc;
                }
                if (ec != hipSuccess || !g) return QW_EDEVICE;
                hipGraphExec_t ex = nullptr;
                hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ei != hipSuccess) return QW_EDEVICE;
                it = ix->graphs.emplace(key, ex).first;
            }
            QW_HIP(hipGraphLaunch(it->second, s));
        }
        if (st) {
            QW_TRY(fill_stats(ix, Q, s, st, opt.timing ? ix->ev : nullptr, true));
            st->dedup_used = eff.dedup;
            st->group_used = eff.group;
            st->xchunk_used = eff.xchunk;
            st->tuned = tuned;
            st->split_used = eff.stage_split;
        }
        return QW_OK;
    } catch (const std::bad_alloc &) {
        return QW_ENOMEM;
    } catch (...) {
        return QW_EINTERNAL;
    }
}

qw_status qw_query_workload_noalloc(qw_index *ix, const void *queries, int64_t Q, int32_t K,
                                    void *stream, int32_t *out_ids, void *out_dist)
{
    QW_TRY(check_index(ix));
    QW_TRY(check_vectors(ix, queries, Q));
    if (K < 1 || K > kMaxTopK || (Q > 0 && (!out_ids || !out_dist))) return QW_EINVAL;
    if (ix->ooc) return QW_EUNSUPPORTED;  // the lists and rows are in host memory
    if (Q == 0) return QW_OK;
    void *base = nullptr;
    QW_TRY(scratch_address(ix->device, &base));
    const bool pad = !(ix->d == ix->dp && (reinterpret_cast<uintptr_t>(queries) & 15) == 0);
    Workspace view;
    if (!carve_plain_ws(ix, Q, pad, static_cast<unsigned char *>(base), view))
        return QW_EUNSUPPORTED;  // the workspace of Q queries exceeds the scratch
    hipStream_t s = S(stream);
    // the index's own workspace steps aside for the call and comes back on
    // every path; nothing below grows a buffer (a view refuses to)
    std::swap(ix->ws, view);
    struct Restore {
        qw_index *ix;
        Workspace *saved;
        ~Restore() { std::swap(ix->ws, *saved); }
    } restore{ix, &view};
    try {
        QW_TRY(clear_counters(ix, s));
        QW_TRY(front(ix, queries, Q, QW_FORM_PLAIN_FP32, s));
        if (ix->count_theta > 0) return count_query(ix, Q, K, s, out_ids, out_dist, nullptr);
        return verify_simple(ix, Q, K, VM_TOPK, s, out_ids, out_dist, nullptr, nullptr, nullptr,
                             false);
    } catch (...) {
        return QW_EINTERNAL;
    }
}

qw_status qw_hash(qw_index *ix, const void *x, int64_t m, int32_t form, void *stream,
                  int32_t *out_h, int64_t *out_recomputed)
{
    QW_TRY(check_index(ix));
    QW_TRY(check_vectors(ix, x, m));
    if (form != QW_FORM_PLAIN_FP32 && form != QW_FORM_FAST) return QW_EINVAL;
    if (m > 0 && !out_h) return QW_EINVAL;
    if (m == 0) {
        if (out_recomputed) *out_recomputed = 0;
        return QW_OK;
    }
    hipStream_t s = S(stream);
    QW_TRY(ensure_ws(ix, m, nullptr));
    QW_TRY(clear_counters(ix, s));
    QW_TRY(stage_query_rows(ix, x, m, s));
    QW_TRY(launch_hash(ix, ix->ws.qrows, m, 0, ix->nf, form, out_h, ix->nf, c64(ix) + C_RECOMP, s));
    if (out_recomputed) {
        unsigned long long r[kRecompSlots];
        QW_HIP(hipMemcpyAsync(r, c64(ix) + C_RECOMP, sizeof(r), hipMemcpyDeviceToHost, s));
        QW_HIP(hipStreamSynchronize(s));
        int64_t tot = 0;
        for (int i = 0; i < kRecompSlots; ++i) tot += (int64_t)r[i];
        *out_recomputed = tot;
    }
    return QW_OK;
}

qw_status qw_bucket_sizes(qw_index *ix, const void *queries, int64_t Q, void *stream,
                          int32_t *out_sizes)
{
    QW_TRY(check_index(ix));
    QW_TRY(check_vectors(ix, queries, Q));
    if (Q > 0 && !out_sizes) return QW_EINVAL;
    if (Q == 0) return QW_OK;
    hipStream_t s = S(stream);
    QW_TRY(ensure_ws(ix, Q, nullptr));
    QW_TRY(clear_counters(ix, s));
    QW_TRY(front(ix, queries, Q, QW_FORM_FAST, s));
    QW_HIP(hipMemcpyAsync(out_sizes, layer_sizes(ix), sizeof(int32_t) * Q * ix->L,
                          hipMemcpyDeviceToDevice, s));
    return QW_OK;
}

qw_status qw_candidate_counts(qw_index *ix, const void *queries, int64_t Q, void *stream,
                              int32_t *out_counts)
{
    QW_TRY(check_index(ix));
    QW_TRY(check_vectors(ix, queries, Q));
    if (Q > 0 && !out_counts) return QW_EINVAL;
    if (ix->ooc) return QW_EUNSUPPORTED;
    if (Q == 0) return QW_OK;
    hipStream_t s = S(stream);
    QW_TRY(ensure_ws(ix, Q, nullptr));
    QW_TRY(clear_counters(ix, s));
    QW_TRY(front(ix, queries, Q, QW_FORM_FAST, s));
    return verify_simple(ix, Q, 1, VM_COUNT, s, nullptr, nullptr, out_counts, nullptr);
}

qw_status qw_candidate_lists(qw_index *ix, const void *queries, int64_t Q, const int64_t *offsets,
                             void *stream, int32_t *out_ids)
{
    QW_TRY(check_index(ix));
    QW_TRY(check_vectors(ix, queries, Q));
    if (Q > 0 && (!offsets || !out_ids)) return QW_EINVAL;
    if (ix->ooc) return QW_EUNSUPPORTED;
    if (Q == 0) return QW_OK;
    hipStream_t s = S(stream);
    QW_TRY(ensure_ws(ix, Q, nullptr));
    QW_TRY(clear_counters(ix, s));
    QW_TRY(front(ix, queries, Q, QW_FORM_FAST, s));
    return verify_simple(ix, Q, 1, VM_LIST, s, out_ids, nullptr, nullptr,
                         reinterpret_cast<const long long *>(offsets));
}

qw_status qw_bruteforce_knn(qw_index *ix, const void *queries, int64_t Q, int32_t K,
                            void *stream, int32_t *out_ids, void *out_dist)
{
    QW_TRY(check_index(ix));
    QW_TRY(check_vectors(ix, queries, Q));
    if (K < 1 || K > kMaxTopK || (Q > 0 && (!out_ids || !out_dist))) return QW_EINVAL;
    if (ix->ooc) return QW_EUNSUPPORTED;
    if (Q == 0) return QW_OK;
    hipStream_t s = S(stream);
    QW_TRY(ensure_ws(ix, Q, nullptr));
    QW_TRY(stage_query_rows(ix, queries, Q, s));
    VerifyArgs a = base_args(ix, K, VM_ALL);
    a.nl = 0;  // no bucket lists: every point
    a.pmagic = 0;
    a.nitems = Q;
    a.cap_log2 = 1;
    a.limit = 1;
    a.buf = (uint32_t)pow2_at_least(std::max(64, 2 * (K + verify_per_iter(ix->dp, ix->dtype))));
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    return launch_verify(a, (int)Q, s);
}

// ---------------------------------------------------------------- count model

int32_t qw_mlp_param_count(int32_t L) { return QW_MLP_HIDDEN * L + 2 * QW_MLP_HIDDEN + 1; }

qw_status qw_mlp_loss_grad(const float *params, int32_t L, const float *feats,
                           const float *targets, int32_t B, void *stream, float *grad,
                           float *loss)
{
    if (!params || !feats || !targets || !grad || !loss || L < 1 || L > kMaxL || B < 1)
        return QW_EINVAL;
    return launch_mlp_loss_grad(params, L, feats, targets, B, grad, loss, S(stream));
}

qw_status qw_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t P,
                      int32_t step, float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!params || !grad || !m || !v || P < 1 || step < 1) return QW_EINVAL;
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return QW_EINVAL;
    return launch_mlp_adam(params, grad, m, v, P, step, lr, beta1, beta2, eps, S(stream));
}

qw_status qw_mlp_predict_bf16(const float *params, int32_t L, const float *feats, int32_t B,
                              void *stream, float *out)
{
    if (!params || !feats || !out || L < 1 || L > kMaxL || B < 0) return QW_EINVAL;
    return launch_mlp_predict_bf16(params, L, feats, B, out, S(stream));
}

qw_status qw_set_count_model(qw_index *ix, const float *params, int32_t P)
{
    if (!ix || !params || P != qw_mlp_param_count(ix->L)) return QW_EINVAL;
    for (int32_t i = 0; i < P; ++i)
        if (!std::isfinite(params[i])) return QW_EINVAL;
    QW_TRY(ix->mlp_dev.ensure(sizeof(float) * P));
    QW_HIP(hipMemcpy(ix->mlp_dev.p, params, sizeof(float) * P, hipMemcpyHostToDevice));
    std::vector<uint32_t> lanes(64 * kMlpLaneWords);
    mlp_pack_lanes(params, ix->L, lanes.data());
    QW_TRY(ix->mlp_lane.ensure(sizeof(uint32_t) * lanes.size()));
    QW_HIP(hipMemcpy(ix->mlp_lane.p, lanes.data(), sizeof(uint32_t) * lanes.size(),
                     hipMemcpyHostToDevice));
    ix->mlp.assign(params, params + P);
    ix->mlp_margin = 0.22314355f;
    drop_graphs(ix);
    return QW_OK;
}

qw_status qw_set_count_margin(qw_index *ix, float margin)
{
    if (!ix || !std::isfinite(margin) || margin < -4.f || margin > 8.f) return QW_EINVAL;
    ix->mlp_margin = margin;
    drop_graphs(ix);
    return QW_OK;
}

qw_status qw_set_probing(qw_index *ix, int32_t mode, int32_t per_layer)
{
    QW_TRY(check_index(ix));
    if (mode < 0 || mode > 2) return QW_EINVAL;
    if (mode == 2 && (per_layer < 1 || per_layer > 2 * ix->k)) return QW_EINVAL;
    if (ix->ooc && mode != 0) return QW_EUNSUPPORTED;  // out of core: each layer's own bucket
    const int32_t P = mode == 2 ? 1 + per_layer : (mode ? 2 * ix->k + 1 : 1);
    if ((int64_t)ix->L * P > kMaxLists) return QW_EUNSUPPORTED;
    uint32_t magic = 0;
    if (P > 1) {  // layer of list i: (i * magic) >> 20, checked over every list index
        magic = ((1u << 20) + (uint32_t)P - 1) / (uint32_t)P;
        for (int i = 0; i < kMaxLists; ++i)
            if ((int)(((uint32_t)i * magic) >> 20) != i / P) return QW_EINTERNAL;
    }
    if (P == ix->nprobe && mode == ix->probe_mode) return QW_OK;
    drop_graphs(ix);
    ix->plans.clear();
    ix->probe_mode = mode;
    ix->nprobe = P;
    ix->nl = ix->L * P;
    ix->pmagic = magic;
    ix->mlp.clear();
    return QW_OK;
}

qw_status qw_set_counting(qw_index *ix, int32_t threshold, int32_t extra)
{
    QW_TRY(check_index(ix));
    if (threshold < 0 || threshold > ix->L || extra < 0 || extra > kMaxTopK) return QW_EINVAL;
    if (ix->ooc && threshold != 0) return QW_EUNSUPPORTED;
    ix->count_theta = threshold;
    ix->count_extra = threshold ? extra : 0;
    return QW_OK;
}

qw_status qw_set_out_of_core(qw_index *ix, const qw_ooc_opts *o, void *stream)
{
    QW_TRY(check_index(ix));
    hipStream_t s = S(stream);
    try {
        if (!o) {
            if (!ix->ooc) return QW_OK;
            drop_graphs(ix);
            return ooc_disable(ix, s);
        }
        if (o->cache_bytes <= 0 || o->index_percent < 1 || o->index_percent > 99 ||
            (o->strategy != 1 && o->strategy != 2) ||
            (o->policy != QW_OOC_MRU && o->policy != QW_OOC_LRU) || o->batch < 1 ||
            (o->keep != 0 && o->keep != 1) || o->reserved != 0)
            return QW_EINVAL;
        if (ix->nprobe != 1 || ix->count_theta > 0) return QW_EUNSUPPORTED;
        drop_graphs(ix);  // captured graphs read the in-core lists and rows
        return ooc_enable(ix, *o, s);
    } catch (const std::bad_alloc &) {
        return QW_ENOMEM;
    } catch (...) {
        return QW_EINTERNAL;
    }
}

qw_status qw_get_count_model(const qw_index *ix, float *params, int32_t P)
{
    if (!ix || !params || ix->mlp.empty() || P != (int32_t)ix->mlp.size()) return QW_EINVAL;
    std::memcpy(params, ix->mlp.data(), sizeof(float) * P);
    return QW_OK;
}

qw_status qw_train_count_model(qw_index *ix, const void *train_queries, int64_t m, int32_t epochs,
                               int32_t batch, float lr, uint64_t seed, void *stream,
                               float *final_loss)
{
    QW_TRY(check_index(ix));
    QW_TRY(check_vectors(ix, train_queries, m));
    if (m < 1 || epochs < 1 || batch < 1 || !(lr > 0.f)) return QW_EINVAL;
    if (ix->ooc) return QW_EUNSUPPORTED;  // the labels need the candidate sets
    hipStream_t s = S(stream);
    const int32_t L = ix->L, P = qw_mlp_param_count(L);
    const int32_t B = (int32_t)std::min<int64_t>(batch, m);
    try {
        // features and labels computed by the engine itself
        QW_TRY(ensure_ws(ix, m, nullptr));
        QW_TRY(clear_counters(ix, s));
        QW_TRY(front(ix, train_queries, m, QW_FORM_FAST, s));
        QW_TRY(verify_simple(ix, m, 1, VM_COUNT, s, nullptr, nullptr, ix->ws.pred.as<int32_t>(),
                             nullptr));
        DevBuf feats, labels, perm, fb, tb, params, grad, mom, vel, loss;
        QW_TRY(feats.ensure(sizeof(float) * (size_t)m * L));
        QW_TRY(labels.ensure(sizeof(float) * m));
        QW_TRY(perm.ensure(sizeof(int32_t) * m));
        QW_TRY(fb.ensure(sizeof(float) * (size_t)B * L));
        QW_TRY(tb.ensure(sizeof(float) * B));
        QW_TRY(params.ensure(sizeof(float) * P));
        QW_TRY(grad.ensure(sizeof(float) * P));
        QW_TRY(mom.ensure(sizeof(float) * P));
        QW_TRY(vel.ensure(sizeof(float) * P));
        const int64_t steps_per_epoch = (m + B - 1) / B;
        QW_TRY(loss.ensure(sizeof(float) * steps_per_epoch));
        QW_TRY(launch_mlp_features(layer_sizes(ix), m, L, feats.as<float>(), s));
        QW_TRY(launch_labels(ix->ws.pred.as<int32_t>(), m, labels.as<float>(), s));
        std::vector<float> hl(m);
        QW_HIP(hipMemcpyAsync(hl.data(), labels.p, sizeof(float) * m, hipMemcpyDeviceToHost, s));
        QW_HIP(hipStreamSynchronize(s));
        double mean = 0.0;
        for (float v : hl) mean += v;
        mean /= (double)m;
        // He-style initialisation from the seed
        std::mt19937_64 rng(seed);
        std::normal_distribution<double> nd(0.0, 1.0);
        std::vector<float> p0(P, 0.f);
        const int H = QW_MLP_HIDDEN;
        for (int i = 0; i < H * L; ++i) p0[i] = (float)(nd(rng) * std::sqrt(2.0 / L));
        for (int i = 0; i < H; ++i) p0[H * L + i] = 0.01f;
        for (int i = 0; i < H; ++i) p0[H * L + H + i] = (float)(nd(rng) * std::sqrt(1.0 / H));
        p0[P - 1] = (float)mean;
        QW_HIP(hipMemcpyAsync(params.p, p0.data(), sizeof(float) * P, hipMemcpyHostToDevice, s));
        QW_TRY(launch_fill_u32(mom.as<uint32_t>(), 0u, P, s));
        QW_TRY(launch_fill_u32(vel.as<uint32_t>(), 0u, P, s));
        std::vector<int32_t> order(m);
        for (int64_t i = 0; i < m; ++i) order[i] = (int32_t)i;
        int32_t step = 0;
        std::vector<float> hloss(steps_per_epoch);
        for (int32_t e = 0; e < epochs; ++e) {
            std::shuffle(order.begin(), order.end(), rng);
            QW_HIP(hipMemcpyAsync(perm.p, order.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
            int64_t st_i = 0;
            for (int64_t off = 0; off + B <= m; off += B, ++st_i) {
                QW_TRY(launch_gather_batch(feats.as<float>(), labels.as<float>(),
                                           perm.as<int32_t>() + off, L, B, fb.as<float>(),
                                           tb.as<float>(), s));
                QW_TRY(launch_mlp_loss_grad(params.as<float>(), L, fb.as<float>(), tb.as<float>(),
                                            B, grad.as<float>(), loss.as<float>() + st_i, s));
                QW_TRY(launch_mlp_adam(params.as<float>(), grad.as<float>(), mom.as<float>(),
                                       vel.as<float>(), P, ++step, lr, 0.9f, 0.999f, 1e-8f, s));
            }
            QW_HIP(hipStreamSynchronize(s));  // the host permutation buffer is reused
            if (e == epochs - 1 && st_i > 0) {
                QW_HIP(hipMemcpy(hloss.data(), loss.p, sizeof(float) * st_i, hipMemcpyDeviceToHost));
                double acc = 0.0;
                for (int64_t i = 0; i < st_i; ++i) acc += hloss[i];
                if (final_loss) *final_loss = (float)(acc / (double)st_i);
            }
        }
        std::vector<float> hp(P);
        QW_HIP(hipMemcpy(hp.data(), params.p, sizeof(float) * P, hipMemcpyDeviceToHost));
        QW_TRY(qw_set_count_model(ix, hp.data(), P));
        // calibrate the sizing margin on the training queries, with the same
        // BF16 inference the schedule uses
        DevBuf pred;
        QW_TRY(pred.ensure(sizeof(float) * m));
        for (int64_t off = 0; off < m; off += INT32_MAX) {
            const int32_t cnt = (int32_t)std::min<int64_t>(m - off, INT32_MAX);
            QW_TRY(launch_mlp_predict_bf16(ix->mlp_dev.as<float>(), L, feats.as<float>() + off * L, cnt,
                                           pred.as<float>() + off, s));
        }
        std::vector<float> hpred(m);
        QW_HIP(hipMemcpyAsync(hpred.data(), pred.p, sizeof(float) * m, hipMemcpyDeviceToHost, s));
        QW_HIP(hipStreamSynchronize(s));
        std::vector<float> res(m);
        for (int64_t i = 0; i < m; ++i) res[i] = hl[i] - hpred[i];
        const int64_t at = std::min<int64_t>(m - 1, (int64_t)std::ceil(0.995 * (double)m) - 1);
        std::nth_element(res.begin(), res.begin() + std::max<int64_t>(0, at), res.end());
        float margin = res[std::max<int64_t>(0, at)];
        if (!std::isfinite(margin)) margin = 0.22314355f;
        ix->mlp_margin = std::min(8.f, std::max(0.05f, margin));
        return QW_OK;
    } catch (const std::bad_alloc &) {
        return QW_ENOMEM;
    }
}

}  // extern "C"
