// Out-of-core mode: host memory as the external storage, HBM as the cache.
//
// The paper keeps index files and data objects on external storage and splits
// the memory that caches them into C_I (index files) and C_D (data objects)
// (Section 4); each part evicts by MRU, and C_I is divided equally among the
// hash layers (Strategy 1) or shared (Strategy 2) (Section 5.1).  The reads of
// index files and data objects are the IndexIO and DataIO of Section 1.2.
//
// Here the CSR ids ([L][n] int32) and the padded rows live in pinned host
// memory.  An index file is one bucket's id list; a data object is one row.
// The workload is answered in batches of consecutive queries, each in three
// steps that run on the GPU:
//  1. index phase: mark the batch's buckets in a map of bucket records (keyed
//     by the bucket's CSR position layer * n + start); count the misses per
//     pool; when a pool's resident ids plus its misses exceed its share,
//     evict resident buckets outside the batch in recency order (a radix sort
//     of (pool, stamp) keys, then a prefix sum of their sizes), and rebuild
//     the arena: survivors copied from the old arena, misses read from host
//     memory, each pool packed into its own region;
//  2. data phase: mark the rows the batch's buckets list; evict resident rows
//     outside the batch in (stamp, id) recency order when the misses do not
//     fit; read the missing rows from host memory into free slots;
//  3. the plain form's per-query kernel (union, verification, top-K) reads
//     the lists from the arena and the rows through the slot directory.
// Recency: query q's layer-l bucket is used at q * L + l + 1, a row of C(q) at
// q + 1, q counting the queries answered since the caches were last emptied
// (across calls when they persist); an item's stamp is its largest use.  The host reads a few counters
// back after each marking step (misses, resident totals, candidates) to decide
// whether the batch fits; a batch that does not fit is answered as two halves
// (the index phase of a batch whose rows did not fit stays done).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "qw_internal.h"

namespace qw {

namespace {

constexpr unsigned long long kMapEmpty = ~0ull;
constexpr int kMaxPools = 64;
constexpr int kOocBlock = 256;
constexpr int kOocGrid = 2048;  // grid-stride launches

// device counters (uint64)
enum {
    O_USED = 0,                  // resident ids per pool
    O_MISS = O_USED + kMaxPools, // ids of this batch's missing buckets per pool
    O_CIDS = O_MISS + kMaxPools, // ids of the eviction candidates per pool
    O_CCNT = O_CIDS + kMaxPools, // eviction candidates per pool
    O_FILL = O_CCNT + kMaxPools, // arena rebuild: ids placed per pool
    O_IMISS = O_FILL + kMaxPools,// missing buckets
    O_ICAND,                     // bucket eviction candidates
    O_COPY,                      // buckets placed in the new arena
    O_RMISS,                     // missing rows
    O_RCAND,                     // row eviction candidates
    O_FREE,                      // free row slots
    O_WORDS
};

__device__ inline unsigned long long map_mix(unsigned long long g)
{
    g ^= g >> 33;
    g *= 0xFF51AFD7ED558CCDull;
    g ^= g >> 33;
    g *= 0xC4CEB9FE1A85EC53ull;
    g ^= g >> 33;
    return g;
}

// Slot of bucket key g (inserting it when `insert`), or -1 when absent.  The
// map holds at least twice as many slots as there are buckets and keys are
// never removed, so every probe sequence reaches g or an empty slot.
__device__ inline int64_t map_slot(unsigned long long *key, unsigned long long mask,
                                   unsigned long long g, bool insert)
{
    unsigned long long h = map_mix(g) & mask;
    for (unsigned long long it = 0; it <= mask; ++it) {
        const unsigned long long k = __hip_atomic_load(&key[h], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        if (k == g) return (int64_t)h;
        if (k == kMapEmpty) {
            if (!insert) return -1;
            const unsigned long long prev = atomicCAS(&key[h], kMapEmpty, g);
            if (prev == kMapEmpty || prev == g) return (int64_t)h;
        }
        h = (h + 1) & mask;
    }
    return -1;
}

// The scans below give each block one contiguous range of the items, so a
// block reserves the places of all its items with one atomic (one per wave
// would serialise thousands of atomics on one address).
constexpr int kScanGrid = 256;

__device__ inline void block_range(int64_t N, int64_t *lo, int64_t *hi)
{
    const int64_t per = (N + gridDim.x - 1) / gridDim.x;
    *lo = (int64_t)blockIdx.x * per;
    *hi = *lo + per < N ? *lo + per : N;
    if (*lo > N) *lo = N;
}

// Whole block: the sum of v over its threads (barriers inside).
__device__ inline unsigned long long block_sum(unsigned long long v, unsigned long long *red)
{
    for (int off = 32; off > 0; off >>= 1) v += (unsigned long long)__shfl_xor((long long)v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0ull;
    for (int w = 0; w < kOocBlock / 64; ++w) t += red[w];
    return t;
}

// Order-preserving compaction of the items i of [lo, hi) with pred(i): pass
// one counts them and reserves their places at *counter with one atomic,
// pass two calls emit(place, i) with places increasing with i.  Whole block.
template <class Pred, class Emit>
__device__ inline void block_compact(int64_t lo, int64_t hi, unsigned long long *counter, Pred pred,
                                     Emit emit)
{
    __shared__ unsigned long long red[kOocBlock / 64];
    __shared__ unsigned long long bbase;
    __shared__ uint32_t wc[kOocBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    unsigned long long c = 0ull;
    for (int64_t i = lo + tid; i < hi; i += kOocBlock) c += pred(i) ? 1ull : 0ull;
    const unsigned long long tot = block_sum(c, red);
    if (tid == 0) bbase = tot ? atomicAdd(counter, tot) : 0ull;
    __syncthreads();
    if (tot == 0ull) return;  // uniform
    unsigned long long run = bbase;
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t i0 = lo; i0 < hi; i0 += kOocBlock) {
        const int64_t i = i0 + tid;
        const bool p = i < hi && pred(i);
        const unsigned long long m = __ballot(p);
        if (lane == 0) wc[wid] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < kOocBlock / 64; ++w) {
            before += w < wid ? wc[w] : 0u;
            all += wc[w];
        }
        __syncthreads();  // wc is rewritten next round
        if (p) emit(run + before + (unsigned long long)__popcll(m & lt), i);
        run += all;
    }
}

// Index phase, marking: every (query, layer) of the batch with a non-empty
// bucket finds or inserts its bucket's record, tags it as needed by this
// batch and, when it is not resident, counts it once as a miss.
__global__ __launch_bounds__(kOocBlock) void mark_index_kernel(
    const uint32_t *__restrict__ bstart, const uint32_t *__restrict__ bsize, int64_t nql,
    int32_t L, int64_t n, int32_t strategy, uint32_t tag, unsigned long long *mkey,
    unsigned long long mask, uint32_t *msize, const long long *__restrict__ moff, uint32_t *mneed,
    unsigned long long *ctr)
{
    __shared__ unsigned long long pmiss[kMaxPools];
    if (threadIdx.x < kMaxPools) pmiss[threadIdx.x] = 0ull;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nql; base += stride) {
        const int64_t i = base + threadIdx.x;
        bool miss = false;
        int64_t slot = -1;
        uint32_t s = 0;
        int l = 0;
        if (i < nql) {
            s = bsize[i];
            if (s) {
                l = (int)(i % L);
                const unsigned long long g = (unsigned long long)l * (unsigned long long)n + bstart[i];
                slot = map_slot(mkey, mask, g, true);
                if (slot >= 0) {
                    msize[slot] = s;  // every writer stores the bucket's size
                    if (mneed[slot] != tag && atomicExch(&mneed[slot], tag) != tag)
                        miss = moff[slot] < 0;
                }
            }
        }
        const unsigned long long mb = __ballot(miss);
        if (mb && (threadIdx.x & 63) == __ffsll((long long)mb) - 1)
            atomicAdd(&ctr[O_IMISS], (unsigned long long)__popcll(mb));
        if (miss) atomicAdd(&pmiss[strategy == 1 ? l : 0], (unsigned long long)s);
    }
    __syncthreads();
    if (threadIdx.x < kMaxPools && pmiss[threadIdx.x])
        atomicAdd(&ctr[O_MISS + threadIdx.x], pmiss[threadIdx.x]);
}

// Eviction candidates of the index cache: resident buckets this batch does
// not need, keyed (pool, recency) so that an ascending sort puts each pool's
// first victim first.
__global__ __launch_bounds__(kOocBlock) void index_cands_kernel(
    const unsigned long long *__restrict__ mkey, int64_t mcap, int64_t n, int32_t strategy,
    int32_t policy, uint32_t tag, int32_t sbits, const uint32_t *__restrict__ msize,
    const unsigned long long *__restrict__ mstamp, const long long *__restrict__ moff,
    const uint32_t *__restrict__ mneed, unsigned long long *ckeys, int32_t *cvals,
    unsigned long long *ctr)
{
    __shared__ unsigned long long pids[kMaxPools], pcnt[kMaxPools];
    if (threadIdx.x < kMaxPools) {
        pids[threadIdx.x] = 0ull;
        pcnt[threadIdx.x] = 0ull;
    }
    __syncthreads();
    int64_t lo, hi;
    block_range(mcap, &lo, &hi);
    const unsigned long long smax = (1ull << sbits) - 1ull;  // stamps below 2^sbits
    auto cand = [&](int64_t slot) {
        const unsigned long long g = mkey[slot];
        return g != kMapEmpty && moff[slot] >= 0 && mneed[slot] != tag;
    };
    block_compact(lo, hi, &ctr[O_ICAND], cand, [&](unsigned long long o, int64_t slot) {
        const unsigned long long g = mkey[slot];
        const int p = strategy == 1 ? (int)(g / (unsigned long long)n) : 0;
        const unsigned long long st = mstamp[slot];
        ckeys[o] = ((unsigned long long)p << sbits) | (policy == QW_OOC_MRU ? smax - st : st);
        cvals[o] = (int32_t)slot;
        atomicAdd(&pids[p], (unsigned long long)msize[slot]);
        atomicAdd(&pcnt[p], 1ull);
    });
    __syncthreads();
    if (threadIdx.x < kMaxPools) {
        if (pids[threadIdx.x]) atomicAdd(&ctr[O_CIDS + threadIdx.x], pids[threadIdx.x]);
        if (pcnt[threadIdx.x]) atomicAdd(&ctr[O_CCNT + threadIdx.x], pcnt[threadIdx.x]);
    }
}

__global__ void gather_sizes_kernel(const int32_t *__restrict__ cvals, int64_t count,
                                    const uint32_t *__restrict__ msize, uint32_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = msize[cvals[i]];
}

struct PoolCut {
    long long start[kMaxPools];    // first candidate of the pool in sorted order
    long long deficit[kMaxPools];  // ids the pool must free (<= 0: none)
};

// Evict, in each pool, the shortest prefix of its sorted candidates whose
// sizes cover the pool's deficit.
__global__ void evict_index_kernel(const unsigned long long *__restrict__ ckeys,
                                   const int32_t *__restrict__ cvals, int64_t count, int32_t sbits,
                                   const unsigned long long *__restrict__ prefix, PoolCut cut,
                                   long long *moff)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int p = (int)(ckeys[i] >> sbits);
    const long long d = cut.deficit[p];
    if (d <= 0) return;
    const unsigned long long before = prefix[i] - prefix[cut.start[p]];
    if ((long long)before < d) moff[cvals[i]] = -1;
}

// Arena rebuild, placement: every resident bucket and every miss of this
// batch gets a place in its pool's region of the new arena.  Each block
// reserves its pools' ids and its copy-list entries once.
__global__ __launch_bounds__(kOocBlock) void place_index_kernel(
    const unsigned long long *__restrict__ mkey, int64_t mcap, int64_t n, int32_t strategy,
    uint32_t tag, int64_t cap_pool, const uint32_t *__restrict__ msize,
    const long long *__restrict__ moff, const uint32_t *__restrict__ mneed, long long *mnoff,
    int32_t *copyl, unsigned long long *ctr)
{
    __shared__ unsigned long long lsum[kMaxPools], lbase[kMaxPools], lrun[kMaxPools];
    if (threadIdx.x < kMaxPools) {
        lsum[threadIdx.x] = 0ull;
        lrun[threadIdx.x] = 0ull;
    }
    __syncthreads();
    int64_t lo, hi;
    block_range(mcap, &lo, &hi);
    auto placed = [&](int64_t slot) {
        const unsigned long long g = mkey[slot];
        return g != kMapEmpty && (moff[slot] >= 0 || mneed[slot] == tag);
    };
    auto pool = [&](int64_t slot) {
        return strategy == 1 ? (int)(mkey[slot] / (unsigned long long)n) : 0;
    };
    for (int64_t i = lo + threadIdx.x; i < hi; i += kOocBlock)
        if (placed(i)) atomicAdd(&lsum[pool(i)], (unsigned long long)msize[i]);
    __syncthreads();
    if (threadIdx.x < kMaxPools && lsum[threadIdx.x])
        lbase[threadIdx.x] = atomicAdd(&ctr[O_FILL + threadIdx.x], lsum[threadIdx.x]);
    __syncthreads();
    block_compact(lo, hi, &ctr[O_COPY], placed, [&](unsigned long long o, int64_t slot) {
        const int p = pool(slot);
        const unsigned long long local = atomicAdd(&lrun[p], (unsigned long long)msize[slot]);
        mnoff[slot] = (long long)((unsigned long long)p * (unsigned long long)cap_pool + lbase[p] +
                                  local);
        copyl[o] = (int32_t)slot;
    });
}

// Arena rebuild, copy: one wave per placed bucket; survivors from the old
// arena, misses from the host copy of the CSR (the index IO).
__global__ __launch_bounds__(kOocBlock) void copy_index_kernel(
    const int32_t *__restrict__ copyl, const unsigned long long *__restrict__ ctr,
    const unsigned long long *__restrict__ mkey, const uint32_t *__restrict__ msize,
    const long long *__restrict__ moff, const long long *__restrict__ mnoff,
    const int32_t *__restrict__ old_arena, const int32_t *__restrict__ host_ids,
    int32_t *__restrict__ new_arena, int64_t ids_total)
{
    const int64_t count = (int64_t)ctr[O_COPY];
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); e < count;
         e += nw) {
        const int32_t slot = copyl[e];
        const uint32_t s = msize[slot];
        const long long o = moff[slot];
        const int32_t *src = o >= 0 ? old_arena + o : host_ids + mkey[slot];
        const long long no = mnoff[slot];
        if (no < 0 || no + (long long)s > ids_total) continue;  // placement never exceeds a pool
        int32_t *dst = new_arena + no;
        for (uint32_t j = (uint32_t)lane; j < s; j += 64) dst[j] = src[j];
    }
}

__global__ __launch_bounds__(kOocBlock) void finish_index_kernel(
    const int32_t *__restrict__ copyl, long long *moff, const long long *__restrict__ mnoff,
    unsigned long long *ctr, int32_t npools)
{
    const int64_t count = (int64_t)ctr[O_COPY];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
        const int32_t slot = copyl[e];
        moff[slot] = mnoff[slot];
    }
    if (blockIdx.x == 0 && threadIdx.x < npools) {
        ctr[O_USED + threadIdx.x] = ctr[O_FILL + threadIdx.x];
        ctr[O_FILL + threadIdx.x] = 0ull;
    }
}

// Index phase, commit: stamps of the batch's buckets (largest use) and their
// arena ranges for the verify kernel (a bucket that is not resident, which
// the capacity check rules out, would read as an empty list).
__global__ __launch_bounds__(kOocBlock) void commit_index_kernel(
    const uint32_t *__restrict__ bstart, const uint32_t *__restrict__ bsize, int64_t nql,
    int32_t L, int64_t n, int64_t q0, unsigned long long *mkey, unsigned long long mask,
    unsigned long long *mstamp, const long long *__restrict__ moff, uint32_t *bstart2,
    uint32_t *bsize2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nql) return;
    const uint32_t s = bsize[i];
    uint32_t off = 0u, size = 0u;
    if (s) {
        const int l = (int)(i % L);
        const unsigned long long g = (unsigned long long)l * (unsigned long long)n + bstart[i];
        const int64_t slot = map_slot(mkey, mask, g, false);
        if (slot >= 0 && moff[slot] >= 0) {
            const unsigned long long u = (unsigned long long)(q0 + i / L) * (unsigned long long)L +
                                         (unsigned long long)l + 1ull;
            atomicMax(&mstamp[slot], u);
            off = (uint32_t)moff[slot];
            size = s;
        }
    }
    bstart2[i] = off;
    bsize2[i] = size;
}

// Data phase, marking: every id in the batch's lists is tagged as needed
// (plain stores: every writer stores the same tag).
__global__ __launch_bounds__(kOocBlock) void mark_rows_kernel(
    const uint32_t *__restrict__ bstart2, const uint32_t *__restrict__ bsize, int64_t nql,
    const int32_t *__restrict__ arena, uint32_t tag, uint32_t *rneed)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); e < nql;
         e += nw) {
        const uint32_t s = bsize[e];
        const int32_t *lst = arena + bstart2[e];
        for (uint32_t j = (uint32_t)lane; j < s; j += 64) rneed[lst[j]] = tag;
    }
}

// Data phase, misses: the tagged rows that are not resident, listed in runs
// of increasing id (each block appends its range of ids in order), so rows
// next to each other in host memory are read together.
__global__ __launch_bounds__(kOocBlock) void miss_rows_kernel(const uint32_t *__restrict__ rneed,
                                                              const int32_t *__restrict__ dir,
                                                              int64_t n, uint32_t tag,
                                                              int32_t *missd, unsigned long long *ctr)
{
    int64_t lo, hi;
    block_range(n, &lo, &hi);
    block_compact(
        lo, hi, &ctr[O_RMISS], [&](int64_t id) { return rneed[id] == tag && dir[id] < 0; },
        [&](unsigned long long o, int64_t id) { missd[o] = (int32_t)id; });
}

// Eviction candidates of the data cache: resident rows this batch does not
// need, keyed (stamp, id) in recency order.
__global__ __launch_bounds__(kOocBlock) void row_cands_kernel(
    const int32_t *__restrict__ owner, int64_t cap_rows, const uint32_t *__restrict__ rneed,
    const uint32_t *__restrict__ rstamp, uint32_t tag, int32_t policy, int32_t idbits,
    int32_t kbits, unsigned long long *ckeys, int32_t *cvals, unsigned long long *ctr)
{
    int64_t lo, hi;
    block_range(cap_rows, &lo, &hi);
    auto cand = [&](int64_t slot) {
        const int32_t id = owner[slot];
        return id >= 0 && rneed[id] != tag;
    };
    block_compact(lo, hi, &ctr[O_RCAND], cand, [&](unsigned long long o, int64_t slot) {
        const int32_t id = owner[slot];
        // (stamp, id) in kbits bits, ids below 2^idbits
        unsigned long long key = ((unsigned long long)rstamp[id] << idbits) | (uint32_t)id;
        if (policy == QW_OOC_MRU) key = ((1ull << kbits) - 1ull) - key;
        ckeys[o] = key;
        cvals[o] = (int32_t)slot;
    });
}

__global__ void evict_rows_kernel(const int32_t *__restrict__ cvals, int64_t count,
                                  int32_t *owner, int32_t *dir)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int32_t slot = cvals[i];
    dir[owner[slot]] = -1;
    owner[slot] = -1;
}

__global__ __launch_bounds__(kOocBlock) void free_rows_kernel(const int32_t *__restrict__ owner,
                                                              int64_t cap_rows, int32_t *freel,
                                                              unsigned long long *ctr)
{
    int64_t lo, hi;
    block_range(cap_rows, &lo, &hi);
    block_compact(
        lo, hi, &ctr[O_FREE], [&](int64_t slot) { return owner[slot] < 0; },
        [&](unsigned long long o, int64_t slot) { freel[o] = (int32_t)slot; });
}

// Data phase, reads: from the host copy into free slots (the data IO).  A
// wave takes 64 / parts rows at once when rows are short (so every lane
// moves 16 bytes), else one row in 64-lane strides.
__global__ __launch_bounds__(kOocBlock) void fill_rows_kernel(
    const int32_t *__restrict__ missd, const int32_t *__restrict__ freel,
    const unsigned long long *__restrict__ ctr, int64_t parts, const uint4 *__restrict__ host_rows,
    uint4 *__restrict__ rows, int32_t *owner, int32_t *dir, int64_t cap_rows)
{
    // the eviction leaves at least as many free slots as misses
    const int64_t count = (int64_t)min(ctr[O_RMISS], ctr[O_FREE]);
    const int lane = threadIdx.x & 63;
    // rows per wave: a power of two with rpw * parts <= 64 (1 for long rows)
    int rpw = 1;
    while (rpw * 2 * parts <= 64) rpw *= 2;
    const int lpr = 64 / rpw;  // lanes per row
    const int r = lane / lpr, j0 = lane % lpr;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t e0 = ((int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * rpw;
         e0 < count; e0 += nw * rpw) {
        const int64_t e = e0 + r;
        if (e >= count) continue;
        const int32_t id = missd[e];
        const int32_t slot = freel[e];
        if (slot < 0 || slot >= cap_rows) continue;
        const uint4 *src = host_rows + (int64_t)id * parts;
        uint4 *dst = rows + (int64_t)slot * parts;
        for (int64_t j = j0; j < parts; j += lpr) dst[j] = src[j];
        if (j0 == 0) {
            owner[slot] = id;
            dir[id] = slot;
        }
    }
}

// Data phase, commit: each listed row takes the batch's last use of it.
__global__ __launch_bounds__(kOocBlock) void commit_rows_kernel(
    const uint32_t *__restrict__ bstart2, const uint32_t *__restrict__ bsize, int64_t nql,
    int32_t L, int64_t q0, const int32_t *__restrict__ arena, uint32_t *rstamp)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); e < nql;
         e += nw) {
        const uint32_t s = bsize[e];
        const int32_t *lst = arena + bstart2[e];
        const uint32_t u = (uint32_t)(q0 + e / L + 1);
        for (uint32_t j = (uint32_t)lane; j < s; j += 64) {
            const int32_t id = lst[j];
            if (rstamp[id] < u) atomicMax(&rstamp[id], u);
        }
    }
}

unsigned grid_for(int64_t items, int per_block)
{
    const int64_t b = (items + per_block - 1) / per_block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kOocGrid));
}

unsigned grid_exact(int64_t items)
{
    return (unsigned)std::max<int64_t>(1, (items + kOocBlock - 1) / kOocBlock);
}

enum BatchResult { B_OK = 0, B_INDEX_FULL, B_DATA_FULL };

qw_status read_ctr(OocState &st, std::vector<unsigned long long> &h, hipStream_t s)
{
    h.resize(O_WORDS);
    QW_HIP(hipMemcpyAsync(h.data(), st.ctr.p, sizeof(unsigned long long) * O_WORDS,
                          hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    return QW_OK;
}

// Bits needed for values up to v.
int bit_width(unsigned long long v)
{
    int b = 0;
    while (b < 64 && (v >> b) != 0ull) ++b;
    return b;
}

// Sort the candidate keys of `bits` low bits (8 per pass).
qw_status sort_cands(qw_index *ix, int64_t count, int bits, bool *alt, hipStream_t s)
{
    OocState &st = *ix->ooc;
    return radix_sort_pairs(st.ckeys.as<unsigned long long>(), st.cvals.as<int32_t>(), count, 0,
                            bits, st.ckeys2.as<unsigned long long>(), st.cvals2.as<int32_t>(),
                            st.sort_hist, s, alt);
}

// One batch [q0, q0 + nq): the index phase, then the data phase.
qw_status run_batch(qw_index *ix, int64_t q0, int64_t nq, hipStream_t s, OocIo *io,
                    BatchResult *res)
{
    OocState &st = *ix->ooc;
    const int32_t L = ix->L;
    const int64_t n = ix->n;
    const int64_t nql = nq * L;
    const uint32_t *bs = ix->ws.bstart.as<uint32_t>() + q0 * L;
    const uint32_t *bz = ix->ws.bsize.as<uint32_t>() + q0 * L;
    auto *ctr = st.ctr.as<unsigned long long>();
    auto *mkey = st.mkey.as<unsigned long long>();
    const unsigned long long mask = (unsigned long long)st.mcap - 1ull;
    auto *moff = st.moff.as<long long>();
    std::vector<unsigned long long> h;
    const uint32_t tag = ++st.tag;
    *res = B_OK;

    // ---- index phase
    QW_TRY(launch_fill_u64(ctr + O_MISS, 0ull, O_WORDS - O_MISS, s));
    mark_index_kernel<<<grid_for(nql, kOocBlock), kOocBlock, 0, s>>>(
        bs, bz, nql, L, n, st.o.strategy, tag, mkey, mask, st.msize.as<uint32_t>(), moff,
        st.mneed.as<uint32_t>(), ctr);
    QW_HIP(hipGetLastError());
    QW_TRY(read_ctr(st, h, s));
    PoolCut cut;
    std::memset(&cut, 0, sizeof(cut));
    bool any = false;
    unsigned long long miss_ids = 0;
    for (int p = 0; p < st.npools; ++p) {
        miss_ids += h[O_MISS + p];
        cut.deficit[p] = (long long)h[O_USED + p] + (long long)h[O_MISS + p] - st.cap_pool;
        any |= cut.deficit[p] > 0;
    }
    // widths of the sort keys: bucket stamps up to (queries so far) * L, rows'
    // stamps up to the queries so far, ids below n
    const int64_t qnow = st.qbase + q0 + nq;
    const int sbits = bit_width((unsigned long long)qnow * (unsigned long long)L);
    const int pbits = bit_width((unsigned long long)(st.npools - 1));
    if (any) {
        index_cands_kernel<<<kScanGrid, kOocBlock, 0, s>>>(
            mkey, st.mcap, n, st.o.strategy, st.o.policy, tag, sbits, st.msize.as<uint32_t>(),
            st.mstamp.as<unsigned long long>(), moff, st.mneed.as<uint32_t>(),
            st.ckeys.as<unsigned long long>(), st.cvals.as<int32_t>(), ctr);
        QW_HIP(hipGetLastError());
        QW_TRY(read_ctr(st, h, s));
        long long start = 0;
        for (int p = 0; p < st.npools; ++p) {
            if (cut.deficit[p] > 0 && (long long)h[O_CIDS + p] < cut.deficit[p]) {
                *res = B_INDEX_FULL;  // nothing has changed
                return QW_OK;
            }
            cut.start[p] = start;
            start += (long long)h[O_CCNT + p];
        }
        const int64_t count = (int64_t)h[O_ICAND];
        bool alt = false;
        QW_TRY(sort_cands(ix, count, sbits + pbits, &alt, s));
        const unsigned long long *keys = alt ? st.ckeys2.as<unsigned long long>()
                                             : st.ckeys.as<unsigned long long>();
        const int32_t *vals = alt ? st.cvals2.as<int32_t>() : st.cvals.as<int32_t>();
        gather_sizes_kernel<<<grid_exact(count), kOocBlock, 0, s>>>(vals, count,
                                                                   st.msize.as<uint32_t>(),
                                                                   st.csz.as<uint32_t>());
        QW_HIP(hipGetLastError());
        QW_TRY(launch_scan_u32_to_u64(st.csz.as<uint32_t>(), count,
                                      st.cscan.as<unsigned long long>(), st.scan_tmp, s));
        evict_index_kernel<<<grid_exact(count), kOocBlock, 0, s>>>(
            keys, vals, count, sbits, st.cscan.as<unsigned long long>(), cut, moff);
        QW_HIP(hipGetLastError());
    }
    const int64_t imiss = (int64_t)h[O_IMISS];
    if (imiss > 0) {
        int32_t *old_arena = st.arena[st.cur].as<int32_t>();
        int32_t *new_arena = st.arena[st.cur ^ 1].as<int32_t>();
        place_index_kernel<<<kScanGrid, kOocBlock, 0, s>>>(
            mkey, st.mcap, n, st.o.strategy, tag, st.cap_pool, st.msize.as<uint32_t>(), moff,
            st.mneed.as<uint32_t>(), st.mnoff.as<long long>(), st.copyl.as<int32_t>(), ctr);
        QW_HIP(hipGetLastError());
        copy_index_kernel<<<kOocGrid, kOocBlock, 0, s>>>(
            st.copyl.as<int32_t>(), ctr, mkey, st.msize.as<uint32_t>(), moff,
            st.mnoff.as<long long>(), old_arena, static_cast<const int32_t *>(st.dev_ids),
            new_arena, st.ids_total);
        QW_HIP(hipGetLastError());
        finish_index_kernel<<<grid_for(st.mcap, kOocBlock), kOocBlock, 0, s>>>(
            st.copyl.as<int32_t>(), moff, st.mnoff.as<long long>(), ctr, st.npools);
        QW_HIP(hipGetLastError());
        st.cur ^= 1;
    }
    io->index_files += imiss;
    io->index_bytes += 4 * (int64_t)miss_ids;
    uint32_t *bs2 = st.bstart2.as<uint32_t>();
    uint32_t *bz2 = bs2 + nql;  // resolved sizes
    const int64_t uq0 = st.qbase + q0;  // recency of this batch's first query
    commit_index_kernel<<<grid_exact(nql), kOocBlock, 0, s>>>(
        bs, bz, nql, L, n, uq0, mkey, mask, st.mstamp.as<unsigned long long>(), moff, bs2, bz2);
    QW_HIP(hipGetLastError());

    // ---- data phase
    const int32_t *arena = st.arena[st.cur].as<int32_t>();
    QW_TRY(launch_fill_u64(ctr + O_RMISS, 0ull, O_WORDS - O_RMISS, s));
    mark_rows_kernel<<<grid_for(nql, kOocBlock / 64), kOocBlock, 0, s>>>(
        bs2, bz2, nql, arena, tag, st.rneed.as<uint32_t>());
    QW_HIP(hipGetLastError());
    miss_rows_kernel<<<kScanGrid, kOocBlock, 0, s>>>(
        st.rneed.as<uint32_t>(), st.dir.as<int32_t>(), n, tag, st.missd.as<int32_t>(), ctr);
    QW_HIP(hipGetLastError());
    QW_TRY(read_ctr(st, h, s));
    const int64_t rmiss = (int64_t)h[O_RMISS];
    const int64_t deficit = st.rows_used + rmiss - st.cap_rows;
    if (deficit > 0) {
        const int idbits = bit_width((unsigned long long)(n - 1));
        const int kbits = idbits + bit_width((unsigned long long)qnow);
        row_cands_kernel<<<kScanGrid, kOocBlock, 0, s>>>(
            st.owner.as<int32_t>(), st.cap_rows, st.rneed.as<uint32_t>(),
            st.rstamp.as<uint32_t>(), tag, st.o.policy, idbits, kbits,
            st.ckeys.as<unsigned long long>(), st.cvals.as<int32_t>(), ctr);
        QW_HIP(hipGetLastError());
        QW_TRY(read_ctr(st, h, s));
        const int64_t count = (int64_t)h[O_RCAND];
        if (count < deficit) {
            *res = B_DATA_FULL;  // the index phase stays done
            return QW_OK;
        }
        bool alt = false;
        QW_TRY(sort_cands(ix, count, kbits, &alt, s));
        const int32_t *vals = alt ? st.cvals2.as<int32_t>() : st.cvals.as<int32_t>();
        evict_rows_kernel<<<grid_exact(deficit), kOocBlock, 0, s>>>(vals, deficit,
                                                                    st.owner.as<int32_t>(),
                                                                    st.dir.as<int32_t>());
        QW_HIP(hipGetLastError());
    }
    if (rmiss > 0) {
        free_rows_kernel<<<kScanGrid, kOocBlock, 0, s>>>(
            st.owner.as<int32_t>(), st.cap_rows, st.freel.as<int32_t>(), ctr);
        QW_HIP(hipGetLastError());
        fill_rows_kernel<<<kOocGrid, kOocBlock, 0, s>>>(
            st.missd.as<int32_t>(), st.freel.as<int32_t>(), ctr, st.row_bytes / 16,
            static_cast<const uint4 *>(st.dev_rows), st.rows.as<uint4>(), st.owner.as<int32_t>(),
            st.dir.as<int32_t>(), st.cap_rows);
        QW_HIP(hipGetLastError());
    }
    st.rows_used += rmiss - std::max<int64_t>(deficit, 0);
    io->data_objects += rmiss;
    io->data_bytes += rmiss * st.row_bytes;
    commit_rows_kernel<<<grid_for(nql, kOocBlock / 64), kOocBlock, 0, s>>>(
        bs2, bz2, nql, L, uq0, arena, st.rstamp.as<uint32_t>());
    QW_HIP(hipGetLastError());
    return QW_OK;
}

int64_t pow2_ceil(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

qw_status ooc_reset(qw_index *ix, hipStream_t s)
{
    OocState &st = *ix->ooc;
    QW_TRY(launch_fill_u64(st.mkey.as<unsigned long long>(), kMapEmpty, st.mcap, s));
    QW_TRY(launch_fill_u64(st.moff.as<unsigned long long>(), ~0ull, st.mcap, s));
    QW_TRY(launch_fill_u64(st.mstamp.as<unsigned long long>(), 0ull, st.mcap, s));
    QW_TRY(launch_fill_u32(st.mneed.as<uint32_t>(), 0u, st.mcap, s));
    QW_TRY(launch_fill_u32(st.dir.as<uint32_t>(), 0xFFFFFFFFu, ix->n, s));
    QW_TRY(launch_fill_u32(st.rstamp.as<uint32_t>(), 0u, ix->n, s));
    QW_TRY(launch_fill_u32(st.rneed.as<uint32_t>(), 0u, ix->n, s));
    QW_TRY(launch_fill_u32(st.owner.as<uint32_t>(), 0xFFFFFFFFu, st.cap_rows, s));
    QW_TRY(launch_fill_u64(st.ctr.as<unsigned long long>(), 0ull, O_WORDS, s));
    st.rows_used = 0;
    st.qbase = 0;
    return QW_OK;
}

qw_status ooc_enable(qw_index *ix, const qw_ooc_opts &o, hipStream_t s)
{
    const int64_t n = ix->n;
    const int elem = ix->dtype == QW_U8 ? 1 : 4;
    const int64_t row_bytes = (int64_t)ix->dp * elem;
    const int64_t ci_bytes = o.cache_bytes / 100 * o.index_percent +
                             (o.cache_bytes % 100) * o.index_percent / 100;
    const int64_t ids_total_raw = ci_bytes / 4;
    const int npools = o.strategy == 1 ? ix->L : 1;
    // a pool never holds more than its layers' n * (L / npools) ids and the
    // data cache never more than n rows, so larger capacities change nothing
    // and are not allocated
    const int64_t cap_pool = std::min<int64_t>(ids_total_raw / npools, n * (ix->L / npools));
    const int64_t cap_rows = std::min<int64_t>((o.cache_bytes - ci_bytes) / row_bytes, n);
    if (npools > kMaxPools) return QW_EUNSUPPORTED;
    if (cap_pool * npools > INT32_MAX || cap_rows > INT32_MAX) return QW_EUNSUPPORTED;

    auto st = std::make_unique<OocState>();
    st->o = o;
    st->npools = npools;
    st->cap_pool = cap_pool;
    st->ids_total = cap_pool * npools;
    st->cap_rows = cap_rows;
    st->row_bytes = row_bytes;
    st->mcap = pow2_ceil(std::max<int64_t>(2 * ix->buckets + 2, 1024));
    if (st->mcap > INT32_MAX) return QW_EUNSUPPORTED;
    const int64_t mcap = st->mcap;
    const int64_t resident_max = std::min<int64_t>(mcap, std::max<int64_t>(st->ids_total, 1));
    st->cand_cap = std::max<int64_t>(std::max<int64_t>(resident_max, cap_rows), 1);
    const int64_t cc = st->cand_cap;
    try {
        QW_TRY(st->arena[0].ensure(sizeof(int32_t) * std::max<int64_t>(st->ids_total, 1)));
        QW_TRY(st->arena[1].ensure(sizeof(int32_t) * std::max<int64_t>(st->ids_total, 1)));
        QW_TRY(st->mkey.ensure(8 * mcap));
        QW_TRY(st->msize.ensure(4 * mcap));
        QW_TRY(st->mstamp.ensure(8 * mcap));
        QW_TRY(st->moff.ensure(8 * mcap));
        QW_TRY(st->mnoff.ensure(8 * mcap));
        QW_TRY(st->mneed.ensure(4 * mcap));
        QW_TRY(st->rows.ensure((size_t)row_bytes * std::max<int64_t>(cap_rows, 1)));
        QW_TRY(st->owner.ensure(4 * std::max<int64_t>(cap_rows, 1)));
        QW_TRY(st->freel.ensure(4 * std::max<int64_t>(cap_rows, 1)));
        QW_TRY(st->dir.ensure(4 * n));
        QW_TRY(st->rstamp.ensure(4 * n));
        QW_TRY(st->rneed.ensure(4 * n));
        QW_TRY(st->missd.ensure(4 * n));
                QW_TRY(st->copyl.ensure(4 * mcap));
        QW_TRY(st->ckeys.ensure(8 * cc));
        QW_TRY(st->ckeys2.ensure(8 * cc));
        QW_TRY(st->cvals.ensure(4 * cc));
        QW_TRY(st->cvals2.ensure(4 * cc));
        QW_TRY(st->csz.ensure(4 * cc));
        QW_TRY(st->cscan.ensure(8 * (cc + 1)));
        QW_TRY(st->sort_hist.ensure(radix_sort_scratch_bytes(cc)));
        QW_TRY(st->scan_tmp.ensure(scan_scratch_bytes(cc)));
        QW_TRY(st->ctr.ensure(sizeof(unsigned long long) * O_WORDS));
        if (ix->ooc) {  // already out of core: keep the host copies
            std::swap(st->host_ids, ix->ooc->host_ids);
            std::swap(st->host_rows, ix->ooc->host_rows);
            st->dev_ids = ix->ooc->dev_ids;
            st->dev_rows = ix->ooc->dev_rows;
            st->host_bytes = ix->ooc->host_bytes;
        } else {
            const size_t ib = ix->ids.bytes, db = ix->data.bytes;
            if (hipHostMalloc(&st->host_ids, ib, hipHostMallocMapped) != hipSuccess) {
                (void)hipGetLastError();
                st->host_ids = nullptr;
                return QW_ENOMEM;
            }
            if (hipHostMalloc(&st->host_rows, db, hipHostMallocMapped) != hipSuccess) {
                (void)hipGetLastError();
                st->host_rows = nullptr;
                return QW_ENOMEM;
            }
            void *dp = nullptr;
            QW_HIP(hipHostGetDevicePointer(&dp, st->host_ids, 0));
            st->dev_ids = dp;
            QW_HIP(hipHostGetDevicePointer(&dp, st->host_rows, 0));
            st->dev_rows = dp;
            st->host_bytes = ib + db;
            QW_HIP(hipMemcpyAsync(st->host_ids, ix->ids.p, ib, hipMemcpyDeviceToHost, s));
            QW_HIP(hipMemcpyAsync(st->host_rows, ix->data.p, db, hipMemcpyDeviceToHost, s));
            QW_HIP(hipStreamSynchronize(s));
        }
    } catch (const std::bad_alloc &) {
        return QW_ENOMEM;
    }
    const bool first = !ix->ooc;
    ix->ooc = std::move(st);
    if (first) {
        ix->ids.release();
        ix->data.release();
    }
    QW_TRY(ooc_reset(ix, s));
    QW_HIP(hipStreamSynchronize(s));
    return QW_OK;
}

qw_status ooc_disable(qw_index *ix, hipStream_t s)
{
    if (!ix->ooc) return QW_OK;
    OocState &st = *ix->ooc;
    const int elem = ix->dtype == QW_U8 ? 1 : 4;
    const size_t ib = sizeof(int32_t) * (size_t)ix->L * ix->n;
    const size_t db = (size_t)elem * ix->n * ix->dp;
    // the caches go first, so the lists and rows have room to come back
    for (DevBuf *b : {&st.arena[0], &st.arena[1], &st.rows, &st.mkey, &st.msize, &st.mstamp,
                      &st.moff, &st.mnoff, &st.mneed, &st.owner, &st.freel, &st.dir, &st.rstamp,
                      &st.rneed, &st.missd, &st.copyl, &st.ckeys, &st.ckeys2,
                      &st.cvals, &st.cvals2, &st.csz, &st.cscan, &st.sort_hist, &st.scan_tmp,
                      &st.bstart2})
        b->release();
    QW_TRY(ix->ids.ensure(ib));
    QW_TRY(ix->data.ensure(db));
    QW_HIP(hipMemcpyAsync(ix->ids.p, st.host_ids, ib, hipMemcpyHostToDevice, s));
    QW_HIP(hipMemcpyAsync(ix->data.p, st.host_rows, db, hipMemcpyHostToDevice, s));
    QW_HIP(hipStreamSynchronize(s));
    ix->ooc.reset();
    return QW_OK;
}

qw_status ooc_answer(qw_index *ix, int64_t Q, const VerifyArgs &tmpl, const void *qrows,
                     int32_t *out_ids, void *out_dist, hipStream_t s, OocIo *io)
{
    OocState &st = *ix->ooc;
    const int32_t L = ix->L;
    const int64_t B = std::min<int64_t>(std::max<int32_t>(st.o.batch, 1), Q);
    QW_TRY(st.bstart2.ensure(2 * sizeof(uint32_t) * (size_t)B * L));  // starts, then sizes
    if (!st.o.keep) QW_TRY(ooc_reset(ix, s));
    const int elem = ix->dtype == QW_U8 ? 1 : 4;
    const int64_t qrow_bytes = (int64_t)ix->dp * elem;
    std::vector<std::pair<int64_t, int64_t>> stack;
    for (int64_t b0 = 0; b0 < Q; b0 += B) {
        stack.clear();
        stack.emplace_back(b0, std::min(Q, b0 + B));
        while (!stack.empty()) {
            const auto r = stack.back();
            stack.pop_back();
            const int64_t lo = r.first, nq = r.second - r.first;
            BatchResult res;
            QW_TRY(run_batch(ix, lo, nq, s, io, &res));
            if (res != B_OK) {
                if (nq == 1) return QW_EUNSUPPORTED;
                ++io->splits;
                const int64_t mid = lo + (nq + 1) / 2;
                stack.emplace_back(mid, r.second);
                stack.emplace_back(lo, mid);
                continue;
            }
            VerifyArgs a = tmpl;
            a.bstart = st.bstart2.as<uint32_t>();
            a.bsize = st.bstart2.as<uint32_t>() + nq * L;
            a.ids = st.arena[st.cur].as<int32_t>();
            a.n = 0;  // list offsets are arena offsets (no layer stride)
            a.data = st.rows.p;
            a.row_slot = st.dir.as<int32_t>();
            a.queries = static_cast<const unsigned char *>(qrows) + lo * qrow_bytes;
            a.out_ids = out_ids + lo * tmpl.K;
            a.out_dist = static_cast<char *>(out_dist) + lo * tmpl.K * 4;
            a.nitems = nq;
            a.counter = nullptr;
            a.ucount_out = tmpl.ucount_out ? tmpl.ucount_out + lo : nullptr;
            QW_TRY(launch_verify(a, (int)nq, s));
            ++io->batches;
        }
    }
    st.qbase += Q;  // with persistent caches, the next call's queries come later
    return QW_OK;
}

}  // namespace qw
