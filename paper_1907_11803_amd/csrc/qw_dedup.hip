// Candidate dedup of the fast form: one workgroup per query builds C(q)
// (the union of the query's buckets, Sections 1.2 and 5.1) in an LDS hash set
// sized by its size class, then verifies its unique candidates itself --
// gathers their rows, computes the exact squared distances (the false-
// positive removal of Section 1.2) and either selects the K nearest itself
// (uint8, small K) or writes one (distance, id) key per candidate into the
// query's range of its XCD's key region for the select kernel.  Queries whose
// set overflows move to the next size class; queries the region cannot hold,
// or whose top K the fused selection cannot settle, go to the fallback.
#include "qw_dedup.h"
#include "qw_dist.h"
#include "qw_internal.h"
#include "qw_wave.h"

namespace qw {

enum {
    D_UCOUNT = 0, D_OVF, D_CPOS, D_T, D_CAP, D_OFF = 6 /* u64 */,
    D_WT = 8 /* per-wave counts, kBlock / 64 */, D_NEXT = 12, D_LCNT = 13, D_BAD = 14,
    D_BOUND = 16 /* u64 */, D_KTH = 18 /* u64 */, D_NSCAL = 20
};
constexpr int kRegIds = 12;  // ids per thread of the register-resident path

__host__ __device__ inline size_t a16(size_t v) { return (v + 15) & ~size_t(15); }

// set | list prefix | list starts | scalars | query row
size_t dedup_lds_bytes(int cap_log2, int global_tab, int nl, int row_bytes)
{
    return (global_tab ? 0 : (size_t(4) << cap_log2)) + a16(size_t(nl + 1) * 4) +
           a16(size_t(nl) * 4) + a16(D_NSCAL * 4) + a16((size_t)row_bytes);
}

// Exclusive prefix of the per-wave counts in scal[D_WT..]: the wave's base and
// the workgroup total.  Call after the barrier that publishes the counts.
__device__ inline uint32_t wave_base(const uint32_t *scal, int wave, uint32_t *total)
{
    uint32_t b = 0, t = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        const uint32_t c = scal[D_WT + w];
        b += w < wave ? c : 0u;
        t += c;
    }
    *total = t;
    return b;
}

// Fused top K: every lane keeps the kTopR smallest keys of its own stream of
// candidates (a stream is every G-th row its group verifies), in ascending
// order, and the smallest key it had to drop (~0: none).
constexpr int kTopR = 3;
constexpr uint32_t kTopList = 512;  // list capacity, 8-byte entries in the set's memory

struct LaneTop {
    unsigned long long k[kTopR];
    unsigned long long dmin;
};

__device__ inline void lane_top_insert(LaneTop &t, unsigned long long key, bool mine)
{
    unsigned long long v = mine ? key : ~0ull;
#pragma unroll
    for (int r = 0; r < kTopR; ++r) {
        const bool lt = v < t.k[r];
        const unsigned long long lo = lt ? v : t.k[r];
        v = lt ? t.k[r] : v;
        t.k[r] = lo;
    }
    t.dmin = v < t.dmin ? v : t.dmin;  // the key pushed out of the list, if any
}

// verify_list for rows of at most 64 parts.  A lane holds two consecutive
// parts of a row (G = pow2 >= parts / 2 lanes per row), UN2 rows per group
// per step; the loop is unrolled twice so the two steps in flight alternate
// between register sets.  Row addresses: a 24-bit multiply into a 32-bit
// offset from the uniform data pointer when the data allows (A.addr32).
// MODE: kVerifyKeys writes every key to keys[i]; kVerifyTop feeds the lanes'
// streams into `top`; kVerifyCollect appends every key at or below `bound` to
// keys[] through the LDS counter *lcnt (entries past `cap` are counted, not
// written).
enum { kVerifyKeys = 0, kVerifyTop = 1, kVerifyCollect = 2 };

template <int DT, int MODE>
__device__ inline void verify_small(const DedupArgs &A, const uint32_t *list, uint32_t U,
                                    const uint4 *qrow, int parts, unsigned long long *keys,
                                    uint32_t qq, LaneTop &top, unsigned long long bound = 0,
                                    uint32_t *lcnt = nullptr, uint32_t cap = 0)
{
    constexpr int UN2 = 2;
    const int tid = threadIdx.x;
    const int pl = (parts + 1) / 2;  // lanes' worth of part pairs
    int G = 1;
    while (G < pl) G <<= 1;
    const int NG = kBlock / G;
    const uint32_t PI = (uint32_t)(NG * UN2);
    const int grp = tid / G, j = tid % G;
    const int lg_ng = __builtin_ctz((unsigned)NG);
    const int p0 = 2 * j, p1 = 2 * j + 1;
    const bool in0 = p0 < parts, in1 = p1 < parts;
    const int c0 = in0 ? p0 : parts - 1, c1 = in1 ? p1 : parts - 1;
    const uint4 q0 = qrow[c0], q1 = qrow[c1];
    const int row_bytes = parts * 16;
    const unsigned char *dbase = reinterpret_cast<const unsigned char *>(A.data);
    auto row_part = [&](uint32_t id, int c) -> uint4 {
        if (A.addr32)
            return *reinterpret_cast<const uint4 *>(dbase + (uint32_t)(__umul24(id, (uint32_t)row_bytes) + (uint32_t)c * 16u));
        return reinterpret_cast<const uint4 *>(A.data)[(int64_t)id * parts + c];
    };
    struct Step {
        uint32_t id[UN2];
        uint4 x0[UN2], x1[UN2];
    };
    auto load = [&](Step &st, uint32_t base) {
#pragma unroll
        for (int u = 0; u < UN2; ++u) {
            const uint32_t i = base + (uint32_t)(grp + NG * u);
            st.id[u] = list[i < U ? i : 0u];
        }
#pragma unroll
        for (int u = 0; u < UN2; ++u) {
            st.x0[u] = row_part(st.id[u], c0);
            st.x1[u] = row_part(st.id[u], c1);
        }
    };
    auto compute = [&](const Step &st, uint32_t base) {
        uint32_t accu[UN2];
        float accf[UN2];
#pragma unroll
        for (int u = 0; u < UN2; ++u) {
            accu[u] = 0;
            accf[u] = 0.f;
            if (DT == QW_U8) {
                const uint32_t a0 = part_dot_u8(st.x0[u], st.x0[u], 0u) - 2u * part_dot_u8(st.x0[u], q0, 0u);
                const uint32_t a1 = part_dot_u8(st.x1[u], st.x1[u], 0u) - 2u * part_dot_u8(st.x1[u], q1, 0u);
                accu[u] = (in0 ? a0 : 0u) + (in1 ? a1 : 0u);
            } else {
                uint32_t du = 0;
                float f0 = 0.f, f1 = 0.f;
                part_dist<DT>(st.x0[u], q0, du, f0);
                part_dist<DT>(st.x1[u], q1, du, f1);
                accf[u] = (in0 ? f0 : 0.f) + (in1 ? f1 : 0.f);
            }
        }
#pragma unroll
        for (int u = 0; u < UN2; ++u)
            for (int o = G >> 1; o > 0; o >>= 1) {
                if (DT == QW_U8)
                    accu[u] += (uint32_t)__shfl_xor((int)accu[u], o);
                else
                    accf[u] += __shfl_xor(accf[u], o);
            }
        if (MODE == kVerifyCollect) {
            if (j == 0)
#pragma unroll
                for (int u = 0; u < UN2; ++u) {
                    const uint32_t i = base + (uint32_t)(grp + NG * u);
                    const unsigned long long key = ((unsigned long long)(accu[u] + qq) << 32) | st.id[u];
                    if (i < U && key <= bound) {
                        const uint32_t pos = atomicAdd(lcnt, 1u);
                        if (pos < cap) keys[pos] = key;
                    }
                }
        } else if (MODE == kVerifyTop) {
            // row u of this step belongs to the stream of lane (base / NG + u) mod G
            // of the group (every lane of the group holds the reduced distance);
            // with G >= UN2 a lane owns at most one row of the step
            if (G >= UN2) {
                const uint32_t u = (uint32_t)(j - (int)(base >> lg_ng)) & (uint32_t)(G - 1);
                const uint32_t i = base + (uint32_t)grp + (uint32_t)NG * u;
                const bool mine = u < (uint32_t)UN2 && i < U;
                const uint32_t dist = (u == 0 ? accu[0] : accu[UN2 - 1]) + qq;
                const uint32_t id = u == 0 ? st.id[0] : st.id[UN2 - 1];
                lane_top_insert(top, ((unsigned long long)dist << 32) | id, mine);
            } else {
#pragma unroll
                for (int u = 0; u < UN2; ++u) {
                    const uint32_t i = base + (uint32_t)(grp + NG * u);
                    lane_top_insert(top, ((unsigned long long)(accu[u] + qq) << 32) | st.id[u], i < U);
                }
            }
        } else if (j == 0) {
#pragma unroll
            for (int u = 0; u < UN2; ++u) {
                const uint32_t i = base + (uint32_t)(grp + NG * u);
                if (i < U) {
                    const uint32_t hi = DT == QW_U8 ? accu[u] + qq : __float_as_uint(accf[u]);
                    keys[i] = ((unsigned long long)hi << 32) | st.id[u];
                }
            }
        }
    };
    if (U == 0) return;
    Step sa, sb;
    load(sa, 0);
    for (uint32_t base = 0; base < U; base += 2 * PI) {
        const uint32_t b1 = base + PI;
        load(sb, b1 < U ? b1 : base);  // a step past the end reloads a valid one
        __builtin_amdgcn_sched_barrier(0);
        compute(sa, base);
        if (b1 >= U) break;
        const uint32_t b2 = b1 + PI;
        load(sa, b2 < U ? b2 : b1);
        __builtin_amdgcn_sched_barrier(0);
        compute(sb, b1);
    }
}

// Whole workgroup: keys[i] = (squared distance << 32) | id for the U ids
// list[0..U) against the query row qrow (parts 16-byte parts, in LDS), or
// the fused top K's modes of verify_small.  A
// group of G lanes (a power of two >= parts, at most 64) holds one row, P
// parts per lane; UN rows per group per step.  uint8 distances are
// sum over parts of (|x|^2 - 2 x.q) plus |q|^2 taken once per query (exact in
// wrapping uint32 arithmetic, d * 255^2 < 2^31); float distances sum FP32
// squares of differences.  Rows of one part per lane: the
// next step's rows are loaded before the current step is reduced, so two
// steps are in flight.  No barriers.
template <int DT, int MODE>
__device__ inline void verify_list(const DedupArgs &A, const uint32_t *list, uint32_t U,
                                   const uint4 *qrow, int parts, unsigned long long *keys,
                                   LaneTop &top, unsigned long long bound = 0,
                                   uint32_t *lcnt = nullptr, uint32_t cap = 0)
{
    constexpr int UN = 4;
    const int tid = threadIdx.x;
    int G = 1;
    while (G < parts && G < 64) G <<= 1;
    const int P = (parts + G - 1) / G;
    const int NG = kBlock / G;
    const uint32_t PI = (uint32_t)(NG * UN);
    const int grp = tid / G, j = tid % G;
    const uint4 *drows = reinterpret_cast<const uint4 *>(A.data);
    // |q|^2 (uint8), the same in every group
    uint32_t qq = 0;
    if (DT == QW_U8) {
        for (int p = 0; p < P; ++p) {
            const int part = j + G * p;
            if (part < parts) {
                const uint4 v = qrow[part];
                qq = part_dot_u8(v, v, qq);
            }
        }
        for (int o = G >> 1; o > 0; o >>= 1) qq += (uint32_t)__shfl_xor((int)qq, o);
    }
    auto finish = [&](uint32_t base, const uint32_t (&id)[UN], uint32_t (&accu)[UN],
                      float (&accf)[UN]) {
#pragma unroll
        for (int u = 0; u < UN; ++u)
            for (int o = G >> 1; o > 0; o >>= 1) {
                if (DT == QW_U8)
                    accu[u] += (uint32_t)__shfl_xor((int)accu[u], o);
                else
                    accf[u] += __shfl_xor(accf[u], o);
            }
        if (j == 0)
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const uint32_t i = base + (uint32_t)(grp + NG * u);
                if (i < U) {
                    const uint32_t hi = DT == QW_U8 ? accu[u] + qq : __float_as_uint(accf[u]);
                    keys[i] = ((unsigned long long)hi << 32) | id[u];
                }
            }
    };
    if (P == 1 || MODE != kVerifyKeys) {  // the fused top K runs only on rows of at most 64 parts
        verify_small<DT, MODE>(A, list, U, qrow, parts, keys, qq, top, bound, lcnt, cap);
        return;
    }
    for (uint32_t base = 0; base < U; base += PI) {
        uint32_t id[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const uint32_t i = base + (uint32_t)(grp + NG * u);
            id[u] = list[i < U ? i : 0u];
        }
        uint32_t accu[UN];
        float accf[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            accu[u] = 0;
            accf[u] = 0.f;
        }
        for (int p = 0; p < P; ++p) {
            const int part = j + G * p;
            const int pc = part < parts ? part : parts - 1;
            uint4 xv[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) xv[u] = drows[(int64_t)id[u] * parts + pc];
            const uint4 qv = qrow[pc];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                uint32_t au = 0;
                float af = 0.f;
                if (DT == QW_U8) au = part_dot_u8(xv[u], xv[u], 0u) - 2u * part_dot_u8(xv[u], qv, 0u);
                else part_dist<DT>(xv[u], qv, au, af);
                accu[u] += part < parts ? au : 0u;
                accf[u] += part < parts ? af : 0.f;
            }
        }
        finish(base, id, accu, accf);
    }
}

// Lane l's value (l uniform) in every lane.
__device__ inline unsigned long long readlane_u64(unsigned long long v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

// The K-th smallest of the wave's 64 values v (duplicates counted), by a
// radix search from the top bit: 32 ballots, no shuffles.
__device__ inline uint32_t wave_kth_u32(uint32_t v, int K)
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

// Whole workgroup, fused top K of query q (uint8: a key's high word is the
// exact squared distance) from the lanes' kept keys.  tab holds the U unique
// ids; the selection list follows them in the same memory (cap_words words
// in all), so the ids stay readable for a second pass.  scal[D_LCNT],
// scal[D_BAD], the bound and the K-th key are reset before the verification.
//  1. the K-th smallest lane-minimum distance D_w of a wave bounds the K-th
//     key of the union of kept keys (K lanes hold a key of distance at most
//     D_w); B = every key of distance at most the smallest D_w of the waves;
//  2. the kept keys at or below B are collected and ranked; ranks below K are
//     the output, padded with (-1, INT32_MAX) below K entries;
//  3. the union's top K is the query's top K unless some lane dropped a key
//     below the union's K-th key T (or fewer than K were kept while a lane
//     dropped any).  Then a second pass verifies the candidates again and
//     collects every key at or below T (T is at least the true K-th key, so
//     that set holds the top K) and ranks those.  A list beyond its capacity
//     sends the query to the fallback.
// A.topk_keep < kTopR keeps fewer keys per lane (a diagnostic: more queries
// take the second pass; the result does not change).
template <bool GLOB, int DT>
__device__ inline void fused_topk(const DedupArgs &A, int64_t q, LaneTop t, const uint32_t *tab,
                                  uint32_t U, uint32_t cap_words, const uint4 *qrow, int parts,
                                  uint32_t *scal)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const int K = A.topk;
#pragma unroll
    for (int r = 1; r < kTopR; ++r)
        if (r >= A.topk_keep) {
            t.dmin = t.k[r] < t.dmin ? t.k[r] : t.dmin;
            t.k[r] = ~0ull;
        }
    const uint32_t loff = (U + 1u) & ~1u;  // 8-byte aligned
    unsigned long long *lst = reinterpret_cast<unsigned long long *>(const_cast<uint32_t *>(tab) + loff);
    const uint32_t lcap = min(kTopList, (cap_words - loff) / 2u);
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    unsigned long long *s_bound = reinterpret_cast<unsigned long long *>(&scal[D_BOUND]);
    unsigned long long *s_kth = reinterpret_cast<unsigned long long *>(&scal[D_KTH]);
    auto sync = [&]() {
        if (GLOB) __threadfence();
        __syncthreads();
    };
    // ranks of the c keys lst[0..c) (unique) below K to the output; the K-th
    // key to *s_kth (left unchanged when c < K)
    auto rank_write = [&](uint32_t c) {
        if (c <= 64) {  // the usual case: one wave, ranks by broadcast compares
            if (tid < 64) {
                const unsigned long long v = lane < (int)c ? lst[lane] : ~0ull;
                int r = 0;
                for (uint32_t e = 0; e < c; ++e) r += readlane_u64(v, (int)e) < v ? 1 : 0;
                if (lane >= (int)c) r = lane;  // padding positions c .. K-1
                if (r < K) {
                    const int64_t o = q * K + r;
                    const bool has = lane < (int)c;
                    A.out_ids[o] = has ? (int32_t)(uint32_t)v : -1;
                    reinterpret_cast<int32_t *>(A.out_dist)[o] = has ? (int32_t)(v >> 32) : INT32_MAX;
                }
                if (lane < (int)c && r == K - 1) *s_kth = v;
            }
            return;
        }
        for (uint32_t i = tid; i < c; i += kBlock) {
            const unsigned long long k = lst[i];
            int r = 0;
            for (uint32_t e = 0; e < c; ++e) r += lst[e] < k;
            if (r < K) {
                const int64_t o = q * K + r;
                A.out_ids[o] = (int32_t)(uint32_t)k;
                reinterpret_cast<int32_t *>(A.out_dist)[o] = (int32_t)(k >> 32);
            }
            if (r == K - 1) *s_kth = k;  // keys are unique: one writer
        }
        for (int r = (int)c + tid; r < K; r += kBlock) {
            const int64_t o = q * K + r;
            A.out_ids[o] = -1;
            reinterpret_cast<int32_t *>(A.out_dist)[o] = INT32_MAX;
        }
    };
    const uint32_t dw = wave_kth_u32((uint32_t)(t.k[0] >> 32), K);  // 0xFFFFFFFF: < K kept
    if (lane == 0 && dw != 0xFFFFFFFFu) atomicMin(s_bound, ((unsigned long long)dw << 32) | 0xFFFFFFFFull);
    sync();
    const unsigned long long B = *s_bound;
#pragma unroll
    for (int r = 0; r < kTopR; ++r) {
        const bool take = t.k[r] != ~0ull && t.k[r] <= B;
        const unsigned long long m = __ballot(take);
        uint32_t wb = 0;
        if (lane == 0 && m) wb = atomicAdd(&scal[D_LCNT], (uint32_t)__popcll(m));
        wb = (uint32_t)__shfl((int)wb, 0);
        const uint32_t pos = wb + (uint32_t)__popcll(m & lt_mask);
        if (take && pos < lcap) lst[pos] = t.k[r];
    }
    sync();
    const uint32_t c = scal[D_LCNT];
    if (c > lcap) {  // uniform
        if (tid == 0) A.fb_list[atomicAdd(A.fb_count, 1u)] = (int32_t)q;
        return;
    }
    rank_write(c);
    sync();
    const unsigned long long T = *s_kth;  // ~0 when fewer than K were kept
    const bool unsure = t.dmin != ~0ull && t.dmin <= T;
    if (__ballot(unsure) != 0ull && lane == 0) scal[D_BAD] = 1;
    sync();
    if (!scal[D_BAD]) return;  // uniform
    // second pass: every key at or below T
    sync();  // every thread has read D_BAD and the list
    if (tid == 0) {
        scal[D_LCNT] = 0;
        atomicAdd(A.topk2_count, 1u);
    }
    sync();
    LaneTop unused;
    verify_list<DT, kVerifyCollect>(A, tab, U, qrow, parts, lst, unused, T, &scal[D_LCNT], lcap);
    sync();
    const uint32_t c2 = scal[D_LCNT];
    if (c2 > lcap) {
        if (tid == 0) A.fb_list[atomicAdd(A.fb_count, 1u)] = (int32_t)q;
        return;
    }
    rank_write(c2);
}

// One workgroup per query (persistent).  The items form chunks of A.xchunk
// consecutive positions of the order, dealt to the XCDs in turn; the
// workgroups of XCD x take the items of its chunks one by one through that
// XCD's own counter (a single shared counter would serialise every
// workgroup's atomic on one address), so neighbouring queries of the order --
// grouped by candidate overlap -- share one XCD's L2.  Each workgroup fetches
// its next item while the current one runs.  Queries with
// at most kRegIds * kBlock (12 x 256)
// bucket entries in an LDS set keep their ids in registers from the load to
// the write; larger ones (and the global-memory class, GLOB) go through the
// set and read the unique ids back from it.
// At most 128 registers: four workgroups per CU (the fused top K would
// otherwise cost one).
// MP: neighbour probing (more than 64 lists per query): the list ranges load
// at the start of each query instead of during the previous one, the list
// prefix takes the whole workgroup and the list search ten steps.
template <bool GLOB, int DT, bool MP>
__global__ __launch_bounds__(kBlock, 4) void dedup_kernel(DedupArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    constexpr bool glob = GLOB;
    const size_t tab_bytes = glob ? 0 : (size_t(4) << A.cap_log2);
    uint32_t *lpref = reinterpret_cast<uint32_t *>(smem + tab_bytes);
    uint32_t *lstart = reinterpret_cast<uint32_t *>(smem + tab_bytes + a16(size_t(A.nl + 1) * 4));
    uint32_t *scal = reinterpret_cast<uint32_t *>(smem + tab_bytes + a16(size_t(A.nl + 1) * 4) +
                                                  a16(size_t(A.nl) * 4));
    constexpr int kTop = MP ? kMaxLists / 2 : 32;  // list search steps: log2(kTop) + 1
    const int row_bytes = A.dp * (DT == QW_U8 ? 1 : 4);
    const int parts = row_bytes / 16;
    uint4 *qrow = reinterpret_cast<uint4 *>(reinterpret_cast<unsigned char *>(scal) + a16(D_NSCAL * 4));
    uint32_t *tab = GLOB ? A.gscratch + (size_t)blockIdx.x * (size_t(1) << A.cap_log2)
                         : reinterpret_cast<uint32_t *>(smem);
    unsigned long long *soff = reinterpret_cast<unsigned long long *>(&scal[D_OFF]);
    int64_t nseg = 0;
    if (!A.queue_only)
        for (int c = A.cls_lo; c <= A.cls_hi; ++c) nseg += (int64_t)(A.seg[2 * c + 1] - A.seg[2 * c]);
    const int64_t nin = A.in_count ? (int64_t)*A.in_count : 0;
    const int64_t nall = nseg + nin;
    const int xcd = blockIdx.x % kXcd;
    const unsigned long long rbase = (unsigned long long)xcd * A.region;
    // the launch's classes, largest first (each class's segment of the order
    // from its end), then the queue of queries that overflowed a smaller class
    auto locate = [&](int64_t it, int &cls) -> int64_t {
        for (int c = A.cls_hi; c > A.cls_lo; --c) {
            const int64_t len = (int64_t)(A.seg[2 * c + 1] - A.seg[2 * c]);
            if (it < len) {
                cls = c;
                return (int64_t)A.seg[2 * c + 1] - 1 - it;
            }
            it -= len;
        }
        cls = A.cls_lo;
        return (int64_t)A.seg[2 * A.cls_lo + 1] - 1 - it;
    };
    auto query_of = [&](int64_t it) -> int64_t {
        int c;
        return it < nseg ? (int64_t)A.order[locate(it, c)] : (int64_t)A.in_list[it - nseg];
    };
    auto class_cap = [&](int64_t it) -> int {
        if (it >= nseg) return (int)A.cap_log2;
        int c;
        (void)locate(it, c);
        return A.cap_base + c;
    };
    // LDS sets only need LDS made visible at a barrier: outstanding global
    // loads (ids, the next query's bucket ranges) stay in flight across it
    auto bar = [&]() {
        if (GLOB) {
            __syncthreads();
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        }
    };
    // the k-th item of this XCD
    auto item_of = [&](uint32_t k) -> int64_t {
        const uint32_t c = A.xchunk;
        return ((int64_t)(k / c) * kXcd + xcd) * c + (int64_t)(k % c);
    };
    if (tid == 0) scal[D_NEXT] = atomicAdd(A.xwork + xcd, 1u);
    __syncthreads();
    int64_t item = item_of(scal[D_NEXT]);
    uint32_t pf_start = 0, pf_size = 0;  // threads < nl: bucket range of the next query
    if (!MP && item < nall && tid < A.nl) {
        const int64_t q0 = query_of(item);
        pf_start = A.bstart[q0 * A.nl + tid];
        pf_size = A.bsize[q0 * A.nl + tid];
    }

    while (item < nall) {  // uniform: every thread holds the same item
        uint32_t next = 0;
        if (tid == 0) next = atomicAdd(A.xwork + xcd, 1u);  // published at the end of the iteration
        const int64_t q = query_of(item);
        if (MP) {
            for (int i = tid; i < A.nl; i += kBlock) {
                lstart[i] = A.bstart[q * A.nl + i];
                lpref[i + 1] = A.bsize[q * A.nl + i];
            }
        } else if (tid < A.nl) {
            lstart[tid] = pf_start;
            lpref[tid + 1] = pf_size;
        }
        for (int i = tid; i < parts; i += kBlock)  // the query row, for the verification
            qrow[i] = reinterpret_cast<const uint4 *>(A.queries)[q * parts + i];
        if (tid == 0) {
            scal[D_UCOUNT] = 0;
            scal[D_OVF] = 0;
            scal[D_CPOS] = 0;
        }
        bar();
        uint32_t run = 0;
        if (MP) run = block_list_prefix(lpref, lstart, A.nl, A.n, A.pmagic, &scal[D_WT]);  // every thread
        else if (tid < 64) run = wave_layer_prefix(lpref, lstart, A.nl, A.n, A.pmagic);
        if (tid < 64) {
            if (tid == 0) {
                scal[D_T] = run;
                int c = glob ? (int)A.cap_log2 : class_cap(item);
                if (glob) {  // set sized from the exact bound min(sum_l s_{q,l}, n)
                    const uint64_t bound = min((uint64_t)run, (uint64_t)A.n);
                    c = 10;
                    while (c < (int)A.cap_log2 && (3ull << c) < 4 * bound) ++c;
                }
                scal[D_CAP] = (uint32_t)c;
            }
        }
        bar();
        const uint32_t T = scal[D_T];
        const int cap_log2 = (int)scal[D_CAP];
        const uint32_t cap = 1u << cap_log2;
        const uint32_t set_limit = (cap >> 2) * 3;
        const uint32_t limit = glob ? set_limit : (A.limit < set_limit ? A.limit : set_limit);
        const uint32_t max_probe = glob ? 0xFFFFFFFFu : kShortProbe;
        const bool in_regs = !glob && T <= (uint32_t)(kRegIds * kBlock);
        uint32_t idr[kRegIds];
        uint32_t pend = 0;
        if (in_regs)  // the id loads fly while the set is cleared
            pend = load_ids<kRegIds, kTop>(A.ids, A.nl, lpref, lstart, T, 0u, idr);
        for (uint32_t i = 4 * tid; i < cap; i += 4 * kBlock)  // cap >= 1024: whole 16-byte stores
            *reinterpret_cast<uint4 *>(tab + i) = uint4{kEmpty, kEmpty, kEmpty, kEmpty};
        if (glob) __threadfence();
        bar();
        uint32_t newm = 0;
        uint32_t U = 0, wbase = 0;
        bool ovf = false;
        if (in_regs) {
            bool full = false;
            newm = insert_streams<kRegIds, 4>(tab, cap_log2, idr, pend, max_probe, full);
            // this lane's position among the wave's new ids
            uint32_t cnt = (uint32_t)__popc(newm), incl = cnt;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
                if (lane >= off) incl += t;
            }
            wbase = incl - cnt;
            if (lane == 63) scal[D_WT + wave] = incl;
            if (__ballot(full) != 0ull && lane == 0) scal[D_OVF] = 1;
            bar();
            uint32_t tot = 0;
            wbase += wave_base(scal, wave, &tot);
            U = tot;
            ovf = scal[D_OVF] != 0 || U > limit;
        } else {
            set_union<kTop>(A.ids, A.nl, lpref, lstart, T, tab, cap_log2, limit, glob, max_probe,
                      true, &scal[D_UCOUNT], &scal[D_OVF], &scal[D_CPOS]);
            U = scal[D_UCOUNT];
            ovf = scal[D_OVF] != 0 || U > limit;
        }
        if (tid == 0) {
            unsigned long long off = ~0ull;
            if (ovf) {  // on to the next size class
                const uint32_t o = atomicAdd(A.ovf_count, 1u);
                A.ovf_list[o] = (int32_t)q;
            } else if (A.count_only) {
                A.ucount[q] = U;
            } else if (A.topk) {  // no key list: the top K is selected here
                A.ucount[q] = U;
                off = 0;
            } else {
                off = atomicAdd(A.alloc + xcd, (unsigned long long)U);
                if (off + U > A.region) {  // no list space: answered by the fallback
                    atomicMax(A.fail + xcd, ~off);
                    A.flag[q] = 1;
                    A.ucount[q] = 0;
                    off = ~0ull;
                } else {
                    off += rbase;
                    A.ucount[q] = U;
                    A.coff[q] = off;
                }
            }
            *soff = off;
            scal[D_NEXT] = next;
            // the fused top K's state (read after the verification)
            scal[D_LCNT] = 0;
            scal[D_BAD] = 0;
            *reinterpret_cast<unsigned long long *>(&scal[D_BOUND]) = ~0ull;
            *reinterpret_cast<unsigned long long *>(&scal[D_KTH]) = ~0ull;
        }
        bar();
        const unsigned long long off = *soff;
        item = item_of(scal[D_NEXT]);
        if (!MP && item < nall && tid < A.nl) {  // the next query's bucket ranges fly during the writes
            const int64_t qn = query_of(item);
            pf_start = A.bstart[qn * A.nl + tid];
            pf_size = A.bsize[qn * A.nl + tid];
        }
        if (off != ~0ull) {
            // the unique ids into tab[0..U) (the set path compacted already)
            if (in_regs) {
                uint32_t e = wbase;
#pragma unroll
                for (int g = 0; g < kRegIds / 4; ++g)
                    if ((uint32_t)(4 * g * kBlock) < T)  // uniform: groups that held ids
#pragma unroll
                        for (int r = 4 * g; r < 4 * g + 4; ++r)
                            if ((newm >> r) & 1u) tab[e++] = idr[r];
                bar();
            }
            LaneTop top;
#pragma unroll
            for (int r = 0; r < kTopR; ++r) top.k[r] = ~0ull;
            top.dmin = ~0ull;
            if (DT == QW_U8 && A.topk) {
                verify_list<DT, kVerifyTop>(A, tab, U, qrow, parts, nullptr, top);
                // the selection list goes into the set's memory after the ids
                fused_topk<GLOB, DT>(A, q, top, tab, U, 1u << A.cap_log2, qrow, parts, scal);
            } else {
                verify_list<DT, kVerifyKeys>(A, tab, U, qrow, parts, A.keys + off, top);
            }
        }
        bar();  // scal and the set are rewritten by the next item
    }
}

qw_status launch_dedup(const DedupArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    // the fused top K: uint8 rows of at most 64 parts, 1 <= K <= kFusedTopK
    if (a.xchunk < 1 || a.xchunk > kXcdChunk) return QW_EINVAL;
    if (a.topk && (a.dtype != QW_U8 || a.dp > 64 * 16 || a.topk > kFusedTopK || a.topk < 0 ||
                   a.topk_keep < 1 || a.topk_keep > kTopR))
        return QW_EINVAL;
    if (a.nl < 1 || a.nl > kMaxLists || (a.nl > 64 && !a.pmagic)) return QW_EINVAL;
    const size_t lds = dedup_lds_bytes((int)a.cap_log2, a.global_tab, a.nl,
                                       a.dp * (a.dtype == QW_U8 ? 1 : 4));
    const bool mp = a.nl > 64;  // the wide-list instantiation only where 64 lists do not suffice
    if (a.dtype == QW_U8) {
        if (mp) {
            if (a.global_tab) dedup_kernel<true, QW_U8, true><<<grid, kBlock, lds, s>>>(a);
            else dedup_kernel<false, QW_U8, true><<<grid, kBlock, lds, s>>>(a);
        } else {
            if (a.global_tab) dedup_kernel<true, QW_U8, false><<<grid, kBlock, lds, s>>>(a);
            else dedup_kernel<false, QW_U8, false><<<grid, kBlock, lds, s>>>(a);
        }
    } else {
        if (mp) {
            if (a.global_tab) dedup_kernel<true, QW_F32, true><<<grid, kBlock, lds, s>>>(a);
            else dedup_kernel<false, QW_F32, true><<<grid, kBlock, lds, s>>>(a);
        } else {
            if (a.global_tab) dedup_kernel<true, QW_F32, false><<<grid, kBlock, lds, s>>>(a);
            else dedup_kernel<false, QW_F32, false><<<grid, kBlock, lds, s>>>(a);
        }
    }
    QW_HIP(hipGetLastError());
    return QW_OK;
}

int dedup_blocks_per_cu(size_t lds, int dtype)
{
    int nb = 0;
    const void *fn = dtype == QW_U8 ? (const void *)dedup_kernel<false, QW_U8, false>
                                    : (const void *)dedup_kernel<false, QW_F32, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, lds) != hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb > 0 ? nb : 1;
}

}  // namespace qw
