// The fast form's candidate work for uint8 rows of at most 64 16-byte parts,
// K <= kFusedTopK and at most 64 bucket lists per query, one wave per query:
// the wave forms C(q), the union of the query's buckets (Sections 1.2 and
// 5.1), in its own LDS hash set, verifies every unique candidate by its exact
// squared distance (the false-positive removal of Section 1.2) and keeps the
// K nearest (the c-k-ANN output of Section 3).
//
// Persistent single-wave workgroups, sixteen per CU, each take a fixed deal of
// the XCD's queries (no shared counter: a contended atomic's latency would
// stall the loads queued behind it); nothing in a query waits on another
// wave, so the CU always has waves gathering rows while others load ids or
// insert them.  Every wave owns
// a set of 2^11 slots.  A query whose candidate set may exceed 3/4 of it is
// processed in passes over a partition of the point ids by a mixed hash
// (pass p holds the ids whose hash has p in its top bits); a pass that still
// overflows is split in two in place, so the set size never changes a result
// and no query moves to another launch.  Each unique candidate belongs to
// exactly one pass and is verified once.
//
// A query whose top K the lanes' kept keys cannot settle goes to the fallback
// queue (the fused per-query kernel answers it after this launch).
#include "qw_dedup.h"
#include "qw_dist.h"
#include "qw_internal.h"

namespace qw {
namespace {

constexpr int kW = 64;                                      // threads per workgroup: one wave
constexpr int kWSetLog2 = 11;                               // set slots of a pass
constexpr uint32_t kWSetLimit = (1u << kWSetLog2) / 4 * 3;  // unique ids per pass (load <= 3/4)
constexpr int kWRound = 8;                                  // listed ids per lane per load round
constexpr int kWTopR = 4;                                   // keys kept per lane
constexpr uint32_t kWList = 512;                            // selection list (u64 entries)

__host__ __device__ constexpr size_t wa16(size_t v) { return (v + 15) & ~size_t(15); }

// set [2^11 u32] | list starts of a 4096-position chunk, one 64-bit word
// per block of 64 positions [64 u64] | offsets of the non-empty lists [64 u32]
constexpr int kWChunkLog2 = 12;  // positions per chunk of start words
constexpr size_t kWMasks = size_t(4) << kWSetLog2;
constexpr size_t kWCoff = kWMasks + 8 * 64;
constexpr size_t kWLdsBytes = kWCoff + wa16(4 * 64);

// Orders this wave's LDS accesses around a point where lanes read what other
// lanes of the wave wrote (the wave's LDS operations complete in order).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// v of lane (lane ^ M), M < 32: DPP quad permutes for 1 and 2, ds_swizzle
// (bitmask mode: and 0x1F, or 0, xor M) above; neither needs an address
// register.
template <int M>
__device__ inline uint32_t xor_lane(uint32_t v)
{
    static_assert(M >= 1 && M < 32, "within 32 lanes");
    if constexpr (M == 1)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    else if constexpr (M == 2)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    else
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (M << 10) | 0x1F);
}

// Sum over aligned groups of G lanes (G a power of two, at most 32), in every
// lane of the group.
template <int G>
__device__ inline uint32_t group_sum(uint32_t v)
{
    if constexpr (G >= 32) v += xor_lane<16>(v);
    if constexpr (G >= 16) v += xor_lane<8>(v);
    if constexpr (G >= 8) v += xor_lane<4>(v);
    if constexpr (G >= 4) v += xor_lane<2>(v);
    if constexpr (G >= 2) v += xor_lane<1>(v);
    return v;
}

// Sum over the wave (uniform).
__device__ inline uint32_t wave_sum(uint32_t v)
{
    v = group_sum<32>(v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
}

// Inclusive prefix sum over the wave: a scan inside each row of 16 lanes by
// DPP row shifts (lanes shifted in from outside the row read 0), then the
// totals of the rows before.
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    const int row = (int)(threadIdx.x >> 4);
    return v + (row >= 1 ? r0 : 0u) + (row >= 2 ? r1 : 0u) + (row >= 3 ? r2 : 0u);
}

__device__ inline unsigned long long lane_u64(unsigned long long v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

// The K-th smallest of the wave's 64 values (duplicates counted) by a radix
// search from the top bit: one ballot per bit.
__device__ inline uint32_t wave_kth(uint32_t v, int K)
{
    uint32_t prefix = 0;
    int k = K;
#pragma unroll
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t above = bit == 31 ? 0u : ~0u << (bit + 1);
        const bool zero = ((v ^ prefix) & above) == 0u && ((v >> bit) & 1u) == 0u;
        const int cnt = __popcll(__ballot(zero));
        if (cnt < k) {
            prefix |= 1u << bit;
            k -= cnt;
        }
    }
    return prefix;
}

// Each lane's kWTopR smallest (distance << 32 | id) keys of its own stream
// of candidates, ascending, and the smallest key it had to drop (~0: none).
struct WTop {
    unsigned long long k[kWTopR];
    unsigned long long dmin;
};

__device__ inline void wtop_insert(WTop &t, unsigned long long key, bool mine)
{
    unsigned long long v = mine ? key : ~0ull;
#pragma unroll
    for (int r = 0; r < kWTopR; ++r) {
        const bool lt = v < t.k[r];
        const unsigned long long lo = lt ? v : t.k[r];
        v = lt ? t.k[r] : v;
        t.k[r] = lo;
    }
    t.dmin = v < t.dmin ? v : t.dmin;
}

// A key of this lane's stream: inserted when it beats the last kept key (the
// wave skips the insertion when no lane's does), else only counted as dropped.
__device__ inline void wtop_offer(WTop &t, unsigned long long key, bool mine)
{
    const bool better = mine && key < t.k[kWTopR - 1];
    if (mine && !better) t.dmin = key < t.dmin ? key : t.dmin;
    if (__ballot(better) != 0ull) wtop_insert(t, key, better);
}

// Whole wave: the U ids list[0..U) against the query (parts 16-byte parts;
// this lane's query parts q0, q1; qq = |q|^2), every distance into the lanes'
// streams.  A group of G lanes (a power of two, at least half the parts) holds
// one row, two parts per lane; two rows per group per step; the next step's
// rows load while the current ones are reduced.  Row u of a step belongs to
// the stream of lane (step * 2 + u) mod G of its group.
template <int G>
__device__ inline void wverify(const DedupArgs &A, const uint32_t *list, uint32_t U, int parts,
                               uint4 q0, uint4 q1, uint32_t qq, WTop &top)
{
    constexpr int UN = 2;
    const int lane = threadIdx.x;
    const int NG = kW / G;
    const uint32_t PI = (uint32_t)(NG * UN);
    const int grp = lane / G, j = lane % G;
    const int p0 = 2 * j, p1 = 2 * j + 1;
    const bool in0 = p0 < parts, in1 = p1 < parts;
    const int c0 = in0 ? p0 : parts - 1, c1 = in1 ? p1 : parts - 1;
    const uint32_t row_bytes = (uint32_t)parts * 16u;
    const unsigned char *dbase = reinterpret_cast<const unsigned char *>(A.data);
    auto row_part = [&](uint32_t id, int c) -> uint4 {
        if (A.addr32)
            return *reinterpret_cast<const uint4 *>(dbase + (uint32_t)(__umul24(id, row_bytes) + (uint32_t)c * 16u));
        return reinterpret_cast<const uint4 *>(A.data)[(int64_t)id * parts + c];
    };
    struct Step {
        uint32_t id[UN];
        uint4 x0[UN], x1[UN];
    };
    auto load = [&](Step &st, uint32_t base) {
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const uint32_t i = base + (uint32_t)(grp + NG * u);
            st.id[u] = list[i < U ? i : 0u];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            st.x0[u] = row_part(st.id[u], c0);
            st.x1[u] = row_part(st.id[u], c1);
        }
    };
    auto compute = [&](const Step &st, uint32_t base, uint32_t step) {
        uint32_t acc[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const uint32_t a0 = part_dot_u8(st.x0[u], st.x0[u], 0u) - 2u * part_dot_u8(st.x0[u], q0, 0u);
            const uint32_t a1 = part_dot_u8(st.x1[u], st.x1[u], 0u) - 2u * part_dot_u8(st.x1[u], q1, 0u);
            acc[u] = (in0 ? a0 : 0u) + (in1 ? a1 : 0u);
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) acc[u] = group_sum<G>(acc[u]);
        // every lane of the group holds both sums
        if constexpr (G >= UN) {  // the row of this lane's stream, if any
            const uint32_t u = (uint32_t)(j - (int)(step * UN)) & (uint32_t)(G - 1);
            const uint32_t i = base + (uint32_t)grp + (uint32_t)NG * u;
            const bool mine = u < (uint32_t)UN && i < U;
            uint32_t dist = acc[0], id = st.id[0];
#pragma unroll
            for (int k = 1; k < UN; ++k) {
                dist = u == (uint32_t)k ? acc[k] : dist;
                id = u == (uint32_t)k ? st.id[k] : id;
            }
            wtop_offer(top, ((unsigned long long)(dist + qq) << 32) | id, mine);
        } else {  // one lane per row: the lane's stream takes both
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const uint32_t i = base + (uint32_t)(grp + NG * u);
                wtop_offer(top, ((unsigned long long)(acc[u] + qq) << 32) | st.id[u], i < U);
            }
        }
    };
    if (U == 0) return;
    Step sa, sb;
    load(sa, 0);
    uint32_t step = 0;
    for (uint32_t base = 0; base < U; base += 2 * PI) {
        const uint32_t b1 = base + PI;
        load(sb, b1 < U ? b1 : base);  // a step past the end reloads a valid one
        __builtin_amdgcn_sched_barrier(0);
        compute(sa, base, step);
        ++step;
        if (b1 >= U) break;
        const uint32_t b2 = b1 + PI;
        load(sa, b2 < U ? b2 : b1);
        __builtin_amdgcn_sched_barrier(0);
        compute(sb, b1, step);
        ++step;
    }
}

// The start words of chunk c: bit j of word b is set when a non-empty list
// starts at position 4096 c + 64 b + j.  Each lane holding a non-empty list
// (has) sets the bit of its start.  Whole wave.
__device__ inline void wstarts(unsigned long long *masks, bool has, uint32_t start, uint32_t c)
{
    masks[threadIdx.x] = 0ull;
    wave_lds_sync();
    if (has && (start >> kWChunkLog2) == c)
        atomicOr(&masks[(start >> 6) & 63u], 1ull << (start & 63u));
    wave_lds_sync();
}

// Positions 512 r + 64 j + lane (j < kWRound) of the query's concatenated
// lists into id[j], valid bits in the result.  A position's list is the number
// of list starts at or before it, less one: the starts before its block
// (*cum, running over the blocks in order) plus those in its block up to its
// lane, read from the block's start word.  coff[i] + p is the index in ids of
// position p of the i-th non-empty list.  Every lane issues every load, with
// no branch (a position at or past T reads ids[0]), so the loads' waits can be
// counted exactly.
__device__ inline uint32_t wload_ids(const int32_t *__restrict__ ids, const unsigned long long *masks,
                                     const uint32_t *coff, uint32_t T, uint32_t r, uint32_t &cum,
                                     uint32_t (&id)[kWRound])
{
    const uint32_t lane = threadIdx.x;
    uint32_t valid = 0;
#pragma unroll
    for (int j = 0; j < kWRound; ++j) {
        const uint32_t b = r * kWRound + (uint32_t)j;
        const unsigned long long M = masks[b & 63u];
        const uint32_t lo = (uint32_t)M, hi = (uint32_t)(M >> 32);
        // starts in this block at lanes up to this one
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
        const uint32_t own = (uint32_t)(M >> lane) & 1u;
        const int list = (int)(cum + below + own) - 1;
        cum += (uint32_t)__builtin_popcount(__builtin_amdgcn_readfirstlane((int)lo)) +
               (uint32_t)__builtin_popcount(__builtin_amdgcn_readfirstlane((int)hi));
        const uint32_t p = b * kW + lane;
        const bool ok = p < T;
        const uint32_t at = coff[list < 0 ? 0 : list] + p;
        id[j] = (uint32_t)ids[ok ? at : 0u];
        valid |= ok ? 1u << j : 0u;
    }
    return valid;
}

// Inserts the ids id[r] whose bit r of `valid` is set (any subset) into the
// set tab (2^kWSetLog2 slots, double hashing) and returns how many were new;
// `full` is set when an id found no slot within kShortProbe probes.  Two
// chains per lane (ids 0-3 and 4-7), one id of each at a time, keep two LDS
// compare-and-swaps in flight; an id is done when its slot was free (new) or
// held it already.
__device__ inline uint32_t winsert(uint32_t *tab, const uint32_t (&id)[kWRound], uint32_t valid, bool &full)
{
    static_assert(kWRound == 8, "two chains of four");
    constexpr uint32_t mask = (1u << kWSetLog2) - 1u;
    uint32_t nnew = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t a = id[k], b = id[k + 4];
        bool da = !((valid >> k) & 1u), db = !((valid >> (k + 4)) & 1u);
        uint32_t sa = hash_id(a, kWSetLog2), sb = hash_id(b, kWSetLog2);
        const uint32_t ta = hash_step(a, kWSetLog2), tb = hash_step(b, kWSetLog2);
        for (uint32_t np = 0; !(da && db); ++np) {
            if (np >= kShortProbe) {
                full = true;
                break;
            }
            const uint32_t oa = da ? 0u : atomicCAS(&tab[sa], kEmpty, a);
            const uint32_t ob = db ? 0u : atomicCAS(&tab[sb], kEmpty, b);
            if (!da) {
                nnew += oa == kEmpty ? 1u : 0u;
                da = oa == kEmpty || oa == a;
                sa = (sa + ta) & mask;
            }
            if (!db) {
                nnew += ob == kEmpty ? 1u : 0u;
                db = ob == kEmpty || ob == b;
                sb = (sb + tb) & mask;
            }
        }
    }
    return nnew;
}

// ids of pass p out of 2^lp (top lp bits of a mixed id)
__device__ inline uint32_t pass_mask(const uint32_t (&id)[kWRound], uint32_t valid, int lp, uint32_t p)
{
    if (lp == 0) return valid;
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < kWRound; ++r) m |= (id_mix(id[r]) >> (32 - lp)) == p ? 1u << r : 0u;
    return valid & m;
}

// G: lanes per verified row (a power of two, at least half the row's parts)
template <int G>
__global__ __launch_bounds__(kW, 4) void dedup_wave_kernel(DedupArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *tab = reinterpret_cast<uint32_t *>(smem);
    unsigned long long *masks = reinterpret_cast<unsigned long long *>(smem + kWMasks);
    uint32_t *coff = reinterpret_cast<uint32_t *>(smem + kWCoff);
    const int lane = threadIdx.x;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int nl = A.nl;
    const int parts = A.dp / 16;
    const int K = A.topk;
    int32_t nseg = 0;
    for (int c = A.cls_lo; c <= A.cls_hi; ++c) nseg += (int32_t)(A.seg[2 * c + 1] - A.seg[2 * c]);
    const int xcd = blockIdx.x % kXcd;
    // items: the launch's classes, largest first (each class's segment of the
    // order from its end)
    auto locate = [&](int32_t it, int &cls) -> int32_t {
        for (int c = A.cls_hi; c > A.cls_lo; --c) {
            const int32_t len = (int32_t)(A.seg[2 * c + 1] - A.seg[2 * c]);
            if (it < len) {
                cls = c;
                return (int32_t)A.seg[2 * c + 1] - 1 - it;
            }
            it -= len;
        }
        cls = A.cls_lo;
        return (int32_t)A.seg[2 * A.cls_lo + 1] - 1 - it;
    };
    // static deal: the XCD's waves (W of them, this one w) take the XCD's
    // items in rounds, round j giving slot j W + w (even j) or j W + W - 1 - w
    // (odd j), so the largest items go first and the sums even out
    const uint32_t W = gridDim.x / kXcd;
    const uint32_t wv = blockIdx.x / kXcd;
    auto item_of = [&](uint32_t k) -> int32_t {
        const uint32_t c = A.xchunk;
        const int64_t it = ((int64_t)(k / c) * kXcd + xcd) * c + (int64_t)(k % c);
        return it < (int64_t)nseg ? (int32_t)it : nseg;
    };
    auto uni = [](uint32_t v) -> uint32_t { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
    uint32_t round = 0;
    auto deal = [&]() -> uint32_t {  // this wave's next slot of the XCD
        const uint32_t k = round * W + ((round & 1u) ? W - 1u - wv : wv);
        ++round;
        return k;
    };

    int32_t item = (int32_t)uni((uint32_t)item_of(deal()));
    if (item >= nseg) return;  // uniform
    int cls = 0;
    int32_t q = (int32_t)uni((uint32_t)A.order[locate(item, cls)]);
    uint32_t pf_start = 0, pf_size = 0;  // lanes < nl: the bucket ranges of query q
    if (lane < nl) {
        pf_start = A.bstart[(int64_t)q * nl + lane];
        pf_size = A.bsize[(int64_t)q * nl + lane];
    }
    int32_t item1 = (int32_t)uni((uint32_t)item_of(deal()));
    while (true) {  // uniform: item < nseg
        // the item after next: its slot is only read at the end of this query
        const uint32_t k2 = deal();
        // the next query: its order entry loads now, its bucket ranges once the
        // first ids are on their way
        int cls1 = 0;
        int32_t q1raw = -1;
        if (item1 < nseg) q1raw = A.order[locate(item1, cls1)];
        // list prefix and offsets
        const uint32_t incl = wave_incl_scan(lane < nl ? pf_size : 0u);
        const uint32_t T = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        // the non-empty lists in order: their offsets by rank, their starts in
        // this lane (the start words are set from these per chunk)
        const uint32_t my_start = incl - (lane < nl ? pf_size : 0u);
        const bool has = lane < nl && pf_size > 0;
        const unsigned long long hm = __ballot(has);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(hm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)hm, 0u));
        if (has) coff[rank] = list_offset(lane, pf_start, my_start, A.n, A.pmagic);
        uint32_t nb_start = 0, nb_size = 0;
        int32_t q1 = item1 < nseg ? -1 : -2;  // -2: no next query
        wave_lds_sync();
        // passes: the class's set size over the wave's, at most what the list
        // total can need
        const uint32_t need = T < (uint64_t)A.n ? T : (uint32_t)A.n;
        int lp_t = 0;
        while ((kWSetLimit << lp_t) < need) ++lp_t;
        int lp = A.cap_base + cls - kWSetLog2;
        lp = lp < 0 ? 0 : lp;
        lp = lp < lp_t ? lp : lp_t;
        WTop top;
#pragma unroll
        for (int r = 0; r < kWTopR; ++r) top.k[r] = ~0ull;
        top.dmin = ~0ull;
        uint32_t U = 0;
        bool split = false;
        for (uint32_t p = 0; p < (1u << lp);) {
            // clear the set
            for (uint32_t i = 4 * (uint32_t)lane; i < (1u << kWSetLog2); i += 4 * kW)
                *reinterpret_cast<uint4 *>(tab + i) = uint4{kEmpty, kEmpty, kEmpty, kEmpty};
            wave_lds_sync();
            // insert this pass's ids, the next round's loads in flight
            uint32_t cnt = 0;
            bool full = false;
            uint32_t ida[kWRound], idb[kWRound];
            uint32_t cum = 0;  // list starts before the next block to load
            wstarts(masks, has, my_start, 0u);
            uint32_t va = wload_ids(A.ids, masks, coff, T, 0u, cum, ida);
            if (p == 0 && q1 < 0) {  // the next query's ranges, behind the first ids
                q1 = (int32_t)uni((uint32_t)q1raw);
                const int32_t qn = q1 < 0 ? q : q1;  // a valid row for the unconditional loads
                nb_start = A.bstart[(int64_t)qn * nl + (lane < nl ? lane : 0)];
                nb_size = A.bsize[(int64_t)qn * nl + (lane < nl ? lane : 0)];
            }
            const uint32_t rounds = (T + kWRound * kW - 1) / (kWRound * kW);
            constexpr uint32_t kRoundsPerChunk = (1u << kWChunkLog2) / (kWRound * kW);
            for (uint32_t r = 0; r < rounds; r += 2) {
                // the next round flies while this one is inserted (past the
                // last round the loads repeat valid positions nobody uses)
                if ((r + 1) % kRoundsPerChunk == 0) wstarts(masks, has, my_start, (r + 1) / kRoundsPerChunk);
                const uint32_t vb = wload_ids(A.ids, masks, coff, T, r + 1, cum, idb);
                cnt += winsert(tab, ida, pass_mask(ida, va, lp, p), full);
                if (r + 1 >= rounds) break;
                if ((r + 2) % kRoundsPerChunk == 0) wstarts(masks, has, my_start, (r + 2) / kRoundsPerChunk);
                va = wload_ids(A.ids, masks, coff, T, r + 2, cum, ida);
                cnt += winsert(tab, idb, pass_mask(idb, vb, lp, p), full);
            }
            const uint32_t Up = uni(wave_sum(cnt));
            if (__ballot(full) != 0ull || Up > kWSetLimit) {
                // split this pass in two at the next bit, redo its first half
                split = true;
                ++lp;
                p = 2 * p;
                wave_lds_sync();
                continue;
            }
            // compact the set in place: tab[0..Up) = this pass's unique ids
            wave_lds_sync();
            // eight rounds of slots read together; every write lands below the
            // slots already read
            uint32_t cpos = 0;
            for (uint32_t b = 0; b < (1u << kWSetLog2); b += 8 * kW) {
                uint32_t v[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) v[r] = tab[b + (uint32_t)(r * kW + lane)];
                wave_lds_sync();
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const bool occ = v[r] != kEmpty;
                    const unsigned long long m = __ballot(occ);
                    if (occ) tab[cpos + (uint32_t)__popcll(m & lt_mask)] = v[r];
                    cpos += (uint32_t)__popcll(m);
                }
            }
            wave_lds_sync();
            {
                // this query's row parts (two per lane of a group) and |q|^2
                const uint4 *qrow = reinterpret_cast<const uint4 *>(A.queries) + (int64_t)q * parts;
                const int j = lane % G;
                const int p0 = 2 * j, p1 = 2 * j + 1;
                const uint4 q0 = qrow[p0 < parts ? p0 : parts - 1];
                const uint4 q1v = qrow[p1 < parts ? p1 : parts - 1];
                const uint32_t qp = (p0 < parts ? part_dot_u8(q0, q0, 0u) : 0u) +
                                    (p1 < parts ? part_dot_u8(q1v, q1v, 0u) : 0u);
                wverify<G>(A, tab, Up, parts, q0, q1v, group_sum<G>(qp), top);
            }
            U += Up;
            ++p;
            wave_lds_sync();
        }
        if (lane == 0) {
            A.ucount[q] = U;
            if (split) atomicAdd(A.ovf_count, 1u);
        }
#pragma unroll
        for (int r = 1; r < kWTopR; ++r)  // a diagnostic: fewer kept keys only unsettle more queries
            if (r >= A.topk_keep) {
                top.dmin = top.k[r] < top.dmin ? top.k[r] : top.dmin;
                top.k[r] = ~0ull;
            }
        // the top K from the lanes' kept keys: the K-th smallest lane minimum
        // bounds the K-th key of their union; the kept keys at or below it are
        // ranked
        const uint32_t dw = wave_kth((uint32_t)(top.k[0] >> 32), K);  // all ones: fewer than K kept
        const unsigned long long B = dw == 0xFFFFFFFFu ? ~0ull : (((unsigned long long)dw << 32) | 0xFFFFFFFFull);
        unsigned long long *lst = reinterpret_cast<unsigned long long *>(tab);
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < kWTopR; ++r) {
            const bool take = top.k[r] != ~0ull && top.k[r] <= B;
            const unsigned long long m = __ballot(take);
            const uint32_t pos = c + (uint32_t)__popcll(m & lt_mask);
            if (take && pos < kWList) lst[pos] = top.k[r];
            c += (uint32_t)__popcll(m);
        }
        wave_lds_sync();
        bool fallback = c > kWList;
        unsigned long long kth = ~0ull;  // the K-th key of the union (~0: fewer than K)
        if (!fallback) {
            if (c <= 64) {
                const unsigned long long v = lane < (int)c ? lst[lane] : ~0ull;
                int rk = 0;
                for (uint32_t e = 0; e < c; ++e) rk += lane_u64(v, (int)e) < v ? 1 : 0;
                const unsigned long long kb = __ballot(lane < (int)c && rk == K - 1);
                if (kb) kth = lane_u64(v, __builtin_ctzll(kb));
                const bool unsure = top.dmin != ~0ull && top.dmin <= kth;
                fallback = __ballot(unsure) != 0ull;
                if (!fallback) {
                    if (lane >= (int)c) rk = lane;  // padding positions c .. K-1
                    if (rk < K) {
                        const int64_t o = (int64_t)q * K + rk;
                        const bool has = lane < (int)c;
                        A.out_ids[o] = has ? (int32_t)(uint32_t)v : -1;
                        reinterpret_cast<int32_t *>(A.out_dist)[o] = has ? (int32_t)(v >> 32) : INT32_MAX;
                    }
                }
            } else {
                // long lists (many equal distances at the bound): rank by scanning
                for (uint32_t i = lane; i < c; i += kW) {
                    const unsigned long long v = lst[i];
                    int rk = 0;
                    for (uint32_t e = 0; e < c; ++e) rk += lst[e] < v ? 1 : 0;
                    if (rk == K - 1) kth = v;
                }
                const unsigned long long kb = __ballot(kth != ~0ull);
                if (kb) kth = lane_u64(kth, __builtin_ctzll(kb));
                const bool unsure = top.dmin != ~0ull && top.dmin <= kth;
                fallback = __ballot(unsure) != 0ull;
                if (!fallback) {
                    for (uint32_t i = lane; i < c; i += kW) {
                        const unsigned long long v = lst[i];
                        int rk = 0;
                        for (uint32_t e = 0; e < c; ++e) rk += lst[e] < v ? 1 : 0;
                        if (rk < K) {
                            const int64_t o = (int64_t)q * K + rk;
                            A.out_ids[o] = (int32_t)(uint32_t)v;
                            reinterpret_cast<int32_t *>(A.out_dist)[o] = (int32_t)(v >> 32);
                        }
                    }
                    // c > 64 >= K: no padding
                }
            }
        }
        if (fallback && lane == 0) {
            A.fb_list[atomicAdd(A.fb_count, 1u)] = q;
            atomicAdd(A.topk2_count, 1u);
        }
        wave_lds_sync();  // the list is read before the next query clears the set
        if (item1 >= nseg) break;  // uniform
        item = item1;
        q = q1;
        cls = cls1;
        pf_start = nb_start;
        pf_size = nb_size;
        item1 = (int32_t)uni((uint32_t)item_of(uni(k2)));
    }
}

}  // namespace

uint32_t dedup_wave_set_limit() { return kWSetLimit; }

size_t dedup_wave_lds_bytes() { return kWLdsBytes; }
int dedup_wave_keep() { return kWTopR; }

namespace {
int wave_group(int dp)  // lanes per row for rows of dp bytes: two 16-byte parts per lane
{
    int G = 1;
    while (2 * G < dp / 16) G <<= 1;
    return G;
}
}  // namespace

int dedup_wave_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)dedup_wave_kernel<4>, kW,
                                                     kWLdsBytes) != hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb > 0 ? nb : 1;
}

int dedup_wave_applies(int dtype, int dp, int nl, int topk)
{
    return dtype == QW_U8 && topk >= 1 && topk <= kFusedTopK && dp % 16 == 0 && dp / 16 <= 64 &&
                   nl >= 1 && nl <= 64
               ? 1
               : 0;
}

qw_status launch_dedup_wave(const DedupArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    if (!dedup_wave_applies(a.dtype, a.dp, a.nl, a.topk) || a.xchunk < 1 || a.xchunk > kXcdChunk ||
        a.cls_lo < 0 || a.cls_hi < a.cls_lo || a.in_count || a.count_only || a.topk_keep < 1 ||
        a.topk_keep > kWTopR || a.nl < 1)
        return QW_EINVAL;
    switch (wave_group(a.dp)) {
    case 1: dedup_wave_kernel<1><<<grid, kW, kWLdsBytes, s>>>(a); break;
    case 2: dedup_wave_kernel<2><<<grid, kW, kWLdsBytes, s>>>(a); break;
    case 4: dedup_wave_kernel<4><<<grid, kW, kWLdsBytes, s>>>(a); break;
    case 8: dedup_wave_kernel<8><<<grid, kW, kWLdsBytes, s>>>(a); break;
    case 16: dedup_wave_kernel<16><<<grid, kW, kWLdsBytes, s>>>(a); break;
    default: dedup_wave_kernel<32><<<grid, kW, kWLdsBytes, s>>>(a); break;
    }
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
