// Collision counting with a candidate cap (Section 3, "Collision Counting", after C2LSH): every
// layer of the index is one collision test, a point is a candidate when it
// shares the query's bucket in at least theta layers, and at most K + v of the
// candidates are verified -- the K results plus v allowed false positives --
// namely the first K + v by (layer count descending, id ascending).  The
// verified points then give the top K by (distance, id) as on the plain path.
//
// One workgroup per query, all state in LDS:
//   1. the query's L bucket lists go into an open-addressing set of 2^c slots,
//      each holding an id (below 2^25 - 1) and its count (<= L <= 64) in one
//      word;
//   2. a histogram of the counts >= theta gives the count c* at which the
//      ranking crosses K + v: every id counted above c* is kept, and of the
//      ids counted exactly c* the `need` smallest, found by a 4-pass radix
//      select on the id bytes (ids are distinct in the set);
//   3. the kept ids are verified (uint8: exact integer; float: the FP64
//      rounded sequence of the plain path) and ranked by (distance, id) by
//      counting, for each one, the kept ids before it.
// Queries are split by their listed ids first: those with at most
// kCountSmallListed (sets of at most 2^13 slots, 37 KB of LDS) run in
// 512-thread workgroups, four to a CU; the rest in 1024-thread workgroups
// with sets of up to 2^14 slots, two to a CU.  The kept ids' keys and the
// survivors of the final selection reuse the set's LDS once it is read.
#include "qw_dedup.h"
#include "qw_dist.h"
#include "qw_exact.h"

namespace qw {

namespace {

constexpr int kHistBins = kMaxL + 2;
// Threads per workgroup: a query's phases are short and each waits on LDS
// atomics or dependent loads, so a CU needs several queries in flight.
// Two 1024-thread workgroups fill a CU's waves; four 512-thread ones do too
// where their sets leave room (measured on 10K queries of 4,784 listed ids
// each, two workgroups per CU: 256 threads 1.05 ms, 512 0.72 ms, 1024 0.61 ms).
constexpr int kCountBlockSmall = 512, kCountBlockLarge = 1024;

// The set (tab) is read until the kept ids are compacted into cid; the keys
// of the kept ids (ckey) and the survivors of the final selection (surv) are
// written after that, in the set's bytes.
struct CountLayout {
    size_t tab, cid, ckey, surv, hist, radix, scal, total;
};

__host__ __device__ inline CountLayout count_layout(int cap_log2, int ncap)
{
    CountLayout o;
    const size_t set = size_t(4) << cap_log2, keys = size_t(ncap) * 12;
    o.tab = 0;
    o.ckey = 0;                               // 8-byte keys over the set
    o.surv = size_t(ncap) * 8;                // then the survivors (ncap even)
    o.cid = set > keys ? set : keys;
    o.hist = o.cid + size_t(ncap) * 4;
    o.radix = o.hist + kHistBins * 4;
    o.scal = o.radix + 256 * 4;
    o.total = o.scal + 8 * 4;
    return o;
}

enum { SC_CSTAR = 0, SC_NEED, SC_PREFIX, SC_REM, SC_NCAND, SC_NSURV };

// inclusive prefix sum over the 64 lanes of a wave
__device__ inline uint32_t wave_inclusive_sum(uint32_t v)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)v, off);
        if ((threadIdx.x & 63) >= (unsigned)off) v += t;
    }
    return v;
}

// A set slot holds (count << kCountShift) | (id + 1); 0 is a free slot.
constexpr int kCountShift = 25;
constexpr uint32_t kSlotId = (1u << kCountShift) - 1u;
__device__ inline uint32_t slot_id(uint32_t w) { return (w & kSlotId) - 1u; }
__device__ inline uint32_t slot_count(uint32_t w) { return w >> kCountShift; }

// Whole workgroup.  Among the items i < nitems with pred(i), the need-th
// smallest of the 32-bit values val(i) (1 <= need <= that many items), one
// byte per pass, most significant first from bit `top` + 7 (every value is
// below 2^(top + 8); top a multiple of 8): each pass counts the values that
// share the bytes chosen so far in 256 bins, and the first wave finds the bin
// in which the count reaches the rank still wanted.
template <int B, typename Val, typename Pred>
__device__ inline uint32_t block_select(uint32_t nitems, uint32_t need, Val val, Pred pred,
                                        uint32_t *radix, uint32_t *scal, int top)
{
    const int tid = threadIdx.x;
    __syncthreads();  // earlier readers of scal are done
    if (tid == 0) {
        scal[SC_PREFIX] = 0u;
        scal[SC_REM] = need;
    }
    for (int shift = top; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += B) radix[b] = 0u;
        __syncthreads();
        const uint32_t prefix = scal[SC_PREFIX];
        const uint32_t hmask = shift == top ? 0u : (0xFFFFFFFFu << (shift + 8));
        for (uint32_t i = tid; i < nitems; i += B)
            if (pred(i)) {
                const uint32_t v = val(i);
                if ((v & hmask) == prefix) atomicAdd(&radix[(v >> shift) & 255u], 1u);
            }
        __syncthreads();
        if (tid < 64) {  // lane i: bins 4i..4i+3; the lane whose range reaches rem
            const uint32_t rem = scal[SC_REM];
            const uint32_t r0 = radix[4 * tid], r1 = radix[4 * tid + 1];
            const uint32_t r2 = radix[4 * tid + 2], r3 = radix[4 * tid + 3];
            const uint32_t sum = r0 + r1 + r2 + r3;
            const uint32_t inc = wave_inclusive_sum(sum);
            uint32_t cum = inc - sum;
            if (cum < rem && inc >= rem) {  // exactly one lane
                uint32_t b = 0;
                if (cum + r0 < rem) {
                    cum += r0;
                    b = 1;
                    if (cum + r1 < rem) {
                        cum += r1;
                        b = 2;
                        if (cum + r2 < rem) {
                            cum += r2;
                            b = 3;
                        }
                    }
                }
                scal[SC_PREFIX] = prefix | ((4u * (uint32_t)tid + b) << shift);
                scal[SC_REM] = rem - cum;
            }
        }
        __syncthreads();
    }
    return scal[SC_PREFIX];
}

template <int DT, int B>
__global__ __launch_bounds__(B) void count_kernel(const CountArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const CountLayout lay = count_layout((int)A.cap_log2, A.ncap);
    uint32_t *tab = reinterpret_cast<uint32_t *>(smem + lay.tab);
    uint32_t *cid = reinterpret_cast<uint32_t *>(smem + lay.cid);
    uint64_t *ckey = reinterpret_cast<uint64_t *>(smem + lay.ckey);
    uint32_t *surv = reinterpret_cast<uint32_t *>(smem + lay.surv);
    uint32_t *hist = reinterpret_cast<uint32_t *>(smem + lay.hist);
    uint32_t *radix = reinterpret_cast<uint32_t *>(smem + lay.radix);
    uint32_t *scal = reinterpret_cast<uint32_t *>(smem + lay.scal);

    __shared__ uint32_t lpref[kMaxL + 1], lstart[kMaxL];
    const int tid = threadIdx.x;
    const int64_t q = A.qlist ? (int64_t)A.qlist[blockIdx.x] : (int64_t)blockIdx.x;

    // list offsets: an exclusive prefix of the L list sizes over the first wave
    if (tid < 64) {
        uint32_t sz = 0, st = 0;
        if (tid < A.L) {
            sz = A.bsize[q * A.L + tid];
            st = A.bstart[q * A.L + tid];
        }
        const uint32_t inc = wave_inclusive_sum(sz);
        lpref[tid] = inc - sz;
        lstart[tid] = st;
        if (tid == 63) lpref[kMaxL] = inc;
    }
    __syncthreads();
    const uint32_t total = lpref[kMaxL];
    // this query's set: at least 4/3 of its listed ids (<= the launch's size)
    int c = 4;
    while ((3u << c) < 4u * total && c < (int)A.cap_log2) ++c;
    const uint32_t cap = 1u << c, mask = cap - 1u;

    for (uint32_t s = tid; s < cap; s += B) tab[s] = 0u;
    for (int s = tid; s < kHistBins; s += B) hist[s] = 0u;
    if (tid == 0) scal[SC_NCAND] = 0u;
    __syncthreads();

    // 1. count: one insert per listed id (a point lies in one bucket per
    // layer); kCountLoads positions of the concatenated lists per thread are
    // located (binary search over the prefix) and loaded together
    constexpr int kCountLoads = 4;
    for (uint32_t base = 0; base < total; base += kCountLoads * B) {
        uint32_t id[kCountLoads];
#pragma unroll
        for (int r = 0; r < kCountLoads; ++r) {
            const uint32_t pos = base + (uint32_t)(r * B + tid);
            id[r] = kEmpty;
            if (pos < total) {
                int lo = 0;  // largest layer with lpref <= pos (its list holds pos)
#pragma unroll
                for (int step = kMaxL / 2; step > 0; step >>= 1) {
                    const int m = lo + step;
                    if (m < A.L && lpref[m] <= pos) lo = m;
                }
                id[r] = (uint32_t)A.ids[(int64_t)lo * A.n + lstart[lo] + (pos - lpref[lo])];
            }
        }
#pragma unroll
        for (int r = 0; r < kCountLoads; ++r) {
            if (id[r] == kEmpty) continue;
            uint32_t h = hash_id(id[r], c);
            const uint32_t step = hash_step(id[r], c);
            // the set holds at most 3/4 of its slots, so some slot of the
            // odd-step sequence is free or holds the id
            for (uint32_t t = 0; t < cap; ++t) {
                const uint32_t key = id[r] + 1u;
                const uint32_t prev = atomicCAS(&tab[h], 0u, key | (1u << kCountShift));
                if (prev == 0u) break;  // new, counted once
                if ((prev & kSlotId) == key) {
                    atomicAdd(&tab[h], 1u << kCountShift);
                    break;
                }
                h = (h + step) & mask;
            }
        }
    }
    __syncthreads();

    // 2. counts >= theta, the crossing count c* and how many ids it contributes
    for (uint32_t s = tid; s < cap; s += B)
        if (tab[s] != 0u) {
            const uint32_t k = slot_count(tab[s]);
            if (k >= (uint32_t)A.theta) atomicAdd(&hist[k], 1u);
        }
    __syncthreads();
    if (tid < 64) {
        // lane i holds the ids counted L - i (descending counts); the lane
        // whose inclusive sum first reaches K + v holds c*
        const uint32_t capn = (uint32_t)(A.K + A.extra);
        const int k = A.L - tid;
        const uint32_t v = k >= A.theta ? hist[k] : 0u;
        const uint32_t inc = wave_inclusive_sum(v);
        const uint32_t excl = inc - v;
        if (excl < capn && inc >= capn) {  // at most one lane
            scal[SC_CSTAR] = (uint32_t)k;
            scal[SC_NEED] = capn - excl;
        }
        if (tid == 63 && inc < capn) {  // fewer than K + v qualify: all of them
            scal[SC_CSTAR] = (uint32_t)A.theta;
            scal[SC_NEED] = hist[A.theta];
        }
    }
    __syncthreads();
    const uint32_t cstar = scal[SC_CSTAR];
    uint32_t last = 0xFFFFFFFFu;  // largest id kept among those counted c*
    if (scal[SC_NEED] < hist[cstar])  // the need-th smallest id counted exactly c*
        last = block_select<B>(
            cap, scal[SC_NEED], [&](uint32_t s) { return slot_id(tab[s]); },
            [&](uint32_t s) { return tab[s] != 0u && slot_count(tab[s]) == cstar; }, radix, scal,
            A.id_top);

    // kept: counted above c*, or counted c* with an id up to `last`
    // (one LDS atomic per wave and round, not one per kept id on one address)
    for (uint32_t s0 = 0; s0 < cap; s0 += B) {
        const uint32_t s = s0 + (uint32_t)tid;
        const uint32_t w = s < cap ? tab[s] : 0u;
        const uint32_t id = slot_id(w), k = slot_count(w);
        const bool keep = w != 0u && (k > cstar || (k == cstar && id <= last));
        const unsigned long long m = __ballot(keep);
        const int lane = tid & 63;
        uint32_t at = 0;
        if (lane == 0 && m) at = atomicAdd(&scal[SC_NCAND], (uint32_t)__popcll(m));
        at = (uint32_t)__shfl((int)at, 0);
        if (keep) cid[at + (uint32_t)__popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull))] = id;
    }
    __syncthreads();
    const int nc = (int)scal[SC_NCAND];

    // 3. verify the kept ids
    for (int i = tid; i < nc; i += B) {
        const uint32_t id = cid[i];
        if constexpr (DT == QW_U8) {
            const uint4 *x = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(A.data) +
                                                             (int64_t)id * A.dp);
            const uint4 *qv = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(A.queries) +
                                                              q * A.dp);
            uint32_t acc = 0;
            float unused = 0.f;
            const int n16 = A.dp / 16;
            for (int p0 = 0; p0 < n16; p0 += 8) {  // eight 16-byte parts in flight
                uint4 xv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) xv[u] = x[p0 + u < n16 ? p0 + u : n16 - 1];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (p0 + u < n16) part_dist<QW_U8>(xv[u], qv[p0 + u], acc, unused);
            }
            ckey[i] = ((uint64_t)acc << 32) | id;
        } else {
            const float *x = static_cast<const float *>(A.data) + (int64_t)id * A.dp;
            const float *qv = static_cast<const float *>(A.queries) + q * A.dp;
            ckey[i] = (uint64_t)__double_as_longlong(exact_dist_row(x, qv, A.dp));
        }
    }
    __syncthreads();
    // the K-th smallest high word of the keys (uint8: the distance; float: the
    // high word of the non-negative FP64 distance, which orders as the value
    // does): a key with a larger high word is not in the top K
    uint32_t hbound = 0xFFFFFFFFu;
    if (nc > A.K)
        hbound = block_select<B>(
            (uint32_t)nc, (uint32_t)A.K, [&](uint32_t i) { return (uint32_t)(ckey[i] >> 32); },
            [&](uint32_t) { return true; }, radix, scal, A.key_top);
    if (tid == 0) scal[SC_NSURV] = 0u;
    __syncthreads();
    for (int i = tid; i < nc; i += B)
        if ((uint32_t)(ckey[i] >> 32) <= hbound) surv[atomicAdd(&scal[SC_NSURV], 1u)] = (uint32_t)i;
    __syncthreads();
    const int ns = (int)scal[SC_NSURV];
    // rank of each survivor under (distance, id) among the survivors (at least
    // K of them; every key of the top K is one); the keys are distinct
    for (int a = tid; a < ns; a += B) {
        const uint32_t i = surv[a];
        const uint64_t ki = ckey[i];
        const uint32_t ii = cid[i];
        int r = 0;
        for (int b = 0; b < ns; ++b) {
            const uint32_t j = surv[b];
            const uint64_t kj = ckey[j];
            if constexpr (DT == QW_U8) {
                r += kj < ki;
            } else {  // non-negative FP64 bit patterns order as the values do
                r += kj < ki || (kj == ki && cid[j] < ii);
            }
        }
        if (r < A.K) {
            const int64_t o = q * A.K + r;
            A.out_ids[o] = (int32_t)ii;
            if constexpr (DT == QW_U8)
                reinterpret_cast<int32_t *>(A.out_dist)[o] = (int32_t)(ki >> 32);
            else
                reinterpret_cast<float *>(A.out_dist)[o] = (float)__longlong_as_double((long long)ki);
        }
    }
    for (int r = nc + tid; r < A.K; r += B) {
        const int64_t o = q * A.K + r;
        A.out_ids[o] = -1;
        if constexpr (DT == QW_U8)
            reinterpret_cast<int32_t *>(A.out_dist)[o] = INT32_MAX;
        else
            reinterpret_cast<float *>(A.out_dist)[o] = INFINITY;
    }
    if (tid == 0 && A.out_counts) A.out_counts[q] = (uint32_t)nc;
}

}  // namespace

size_t count_lds_bytes(int cap_log2, int ncap) { return count_layout(cap_log2, ncap).total; }

// Per query, the sum of its L list lengths: class 0 when at most `limit`,
// else class 1.  Appends the query to its class's list (one atomic per class
// per workgroup; the lists' order is immaterial) and keeps each class's
// largest sum.  cnt: [n0, n1, max0, max1], zeroed by the caller.
__global__ __launch_bounds__(kBlock) void count_split_kernel(const uint32_t *__restrict__ bsize,
                                                             int64_t Q, int32_t L, uint32_t limit,
                                                             int32_t *__restrict__ list0,
                                                             int32_t *__restrict__ list1,
                                                             uint32_t *cnt)
{
    __shared__ uint32_t wc[2][kBlock / 64], wm[2][kBlock / 64], base[2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t q = (int64_t)blockIdx.x * kBlock + tid;
    uint64_t t = 0;
    if (q < Q)
        for (int32_t l = 0; l < L; ++l) t += bsize[q * L + l];
    const uint32_t tot = (uint32_t)min(t, (uint64_t)0xFFFFFFFFu);
    const bool c1 = q < Q && tot > limit, c0 = q < Q && !c1;
    const unsigned long long b0 = __ballot(c0), b1 = __ballot(c1);
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint32_t m0 = c0 ? tot : 0u, m1 = c1 ? tot : 0u;
    for (int off = 32; off > 0; off >>= 1) {
        m0 = max(m0, (uint32_t)__shfl_xor((int)m0, off));
        m1 = max(m1, (uint32_t)__shfl_xor((int)m1, off));
    }
    if (lane == 0) {
        wc[0][wave] = (uint32_t)__popcll(b0);
        wc[1][wave] = (uint32_t)__popcll(b1);
        wm[0][wave] = m0;
        wm[1][wave] = m1;
    }
    __syncthreads();
    if (tid < 2) {
        uint32_t n = 0, m = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            n += wc[tid][w];
            m = max(m, wm[tid][w]);
        }
        base[tid] = n ? atomicAdd(&cnt[tid], n) : 0u;
        if (m) atomicMax(&cnt[2 + tid], m);
    }
    __syncthreads();
    uint32_t o0 = base[0], o1 = base[1];
    for (int w = 0; w < wave; ++w) {
        o0 += wc[0][w];
        o1 += wc[1][w];
    }
    if (c0) list0[o0 + (uint32_t)__popcll(b0 & lt)] = (int32_t)q;
    if (c1) list1[o1 + (uint32_t)__popcll(b1 & lt)] = (int32_t)q;
}

qw_status launch_count_split(const uint32_t *bsize, int64_t Q, int32_t L, uint32_t limit,
                             int32_t *list0, int32_t *list1, uint32_t *cnt, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    if (Q > 0x7FFFFFFF) return QW_EINTERNAL;
    count_split_kernel<<<(unsigned)ceil_div(Q, kBlock), kBlock, 0, s>>>(bsize, Q, L, limit, list0,
                                                                       list1, cnt);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

qw_status launch_count(const CountArgs &a, int64_t grid, bool large, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    if (a.L < 1 || a.L > kMaxL || a.theta < 1 || a.theta > a.L || a.K < 1 || a.extra < 0 ||
        a.K + a.extra > a.ncap || (a.ncap & 1) || a.cap_log2 < 4 || a.cap_log2 > 16 ||
        grid > 0x7FFFFFFF)
        return QW_EINTERNAL;
    const size_t lds = count_lds_bytes((int)a.cap_log2, a.ncap);
    const unsigned g = (unsigned)grid;
    if (a.dtype == QW_U8) {
        if (large) count_kernel<QW_U8, kCountBlockLarge><<<g, kCountBlockLarge, lds, s>>>(a);
        else count_kernel<QW_U8, kCountBlockSmall><<<g, kCountBlockSmall, lds, s>>>(a);
    } else {
        if (large) count_kernel<QW_F32, kCountBlockLarge><<<g, kCountBlockLarge, lds, s>>>(a);
        else count_kernel<QW_F32, kCountBlockSmall><<<g, kCountBlockSmall, lds, s>>>(a);
    }
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
