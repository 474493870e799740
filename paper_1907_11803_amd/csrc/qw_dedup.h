// De-duplicated union of one query's bucket id lists (Sections 1.2 and 5.1:
// the candidates are the union of the buckets the query falls in, one per
// layer).  Device code shared by the fused verify kernel and the dedup kernel.
//
// The set is an open-addressing hash table of 2^c slots (kEmpty = free) with
// double hashing; every lane keeps several inserts in flight at once.
#pragma once

#include "qw_internal.h"

namespace qw {

__device__ inline uint32_t hash_id(uint32_t id, int cap_log2)
{
    return (id * 0x9E3779B1u) >> (32 - cap_log2);
}

// odd step: the probe sequence visits every slot of a power-of-two table
__device__ inline uint32_t hash_step(uint32_t id, int cap_log2)
{
    return ((id * 0x85EBCA77u) >> (32 - cap_log2)) | 1u;
}

// Sets that may pass an overflowing query on to a larger set bound the probes
// per id (kShortProbe): at load factor <= 3/4 a longer sequence means the set
// is (nearly) over its limit.  Sets that must hold every id probe every slot.
constexpr uint32_t kShortProbe = 64;

// Inserts the ids id[r] (r < R; bit r of `valid` set, a prefix in r) into the
// set tab (2^cap_log2 slots, cap_log2 >= 1).  Returns the mask of ids that were
// new; sets `full` when some id found no slot within max_probe probes (that id
// is then neither new nor known to be present).
//
// The R ids form S streams (stream s: ids s, s + S, ...); each stream inserts
// its ids one after another, a probe being one compare-and-swap on the slot
// (free: taken, the id: a duplicate, else the next slot of the id's sequence).
// The S streams keep S independent LDS atomics in flight per lane, and the
// work per lane follows the probes its ids need, not the longest sequence of
// the wave times R.
template <int R, int S>
__device__ inline uint32_t insert_streams(uint32_t *tab, int cap_log2, const uint32_t (&id)[R],
                                          uint32_t valid, uint32_t max_probe, bool &full)
{
    static_assert(R % S == 0, "streams split the ids evenly");
    constexpr int E = R / S;
    const uint32_t mask = (1u << cap_log2) - 1u;
    const uint32_t probes = mask < max_probe ? mask + 1 : max_probe;
    // stream s holds its remaining ids in qv[s][0..E) (front = the id being
    // inserted); finishing one shifts the queue, so every index is static
    uint32_t qv[S][E];
    int cur[S], ne[S];
    uint32_t slot[S], np[S];
    uint32_t newm = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        ne[s] = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            qv[s][e] = id[s + e * S];
            ne[s] += (valid >> (s + e * S)) & 1u;
        }
        cur[s] = 0;
        slot[s] = hash_id(qv[s][0], cap_log2);
        np[s] = 0;
    }
    while (true) {
        bool any = false;
#pragma unroll
        for (int s = 0; s < S; ++s) any |= cur[s] < ne[s];
        if (!any) break;
        uint32_t o[S];
#pragma unroll
        for (int s = 0; s < S; ++s)
            o[s] = cur[s] < ne[s] ? atomicCAS(&tab[slot[s]], kEmpty, qv[s][0]) : 0u;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bool act = cur[s] < ne[s];
            const bool is_new = act && o[s] == kEmpty;
            const bool moved = act && o[s] != kEmpty && o[s] != qv[s][0];
            const bool give_up = moved && np[s] + 1 >= probes;
            const bool done = act && (!moved || give_up);
            newm |= is_new ? 1u << (s + cur[s] * S) : 0u;
            full |= give_up;
            np[s] = done ? 0u : np[s] + (moved ? 1u : 0u);
            slot[s] = moved && !give_up ? (slot[s] + hash_step(qv[s][0], cap_log2)) & mask : slot[s];
            if (done) {  // next id of the stream
#pragma unroll
                for (int e = 0; e + 1 < E; ++e) qv[s][e] = qv[s][e + 1];
                ++cur[s];
                slot[s] = hash_id(qv[s][0], cap_log2);
            }
        }
    }
    return newm;
}

// A query's bucket lists: list i of layer layer_of(i).  Without neighbour
// probing every layer has one list (layer = i); with it, each layer has P
// consecutive lists and layer = (i * pmagic) >> 20 with pmagic = ceil(2^20 / P),
// exact for i < kMaxLists.
__device__ inline int layer_of(int i, uint32_t pmagic)
{
    return pmagic ? (int)(((uint32_t)i * pmagic) >> 20) : i;
}

// The lists' id offsets: after a prefix below, lstart[i] maps a position p of
// the concatenated lists that falls in list i to ids[lstart[i] + p]: the
// list's start in its layer plus layer_of(i) * n, minus its prefix (wrapping
// uint32 arithmetic; the index itself is below 2^31 since n * L < 2^31).
__device__ inline uint32_t list_offset(int i, uint32_t start, uint32_t excl, int64_t n, uint32_t pmagic)
{
    return (uint32_t)layer_of(i, pmagic) * (uint32_t)n + start - excl;
}

// Wave 0 only: lpref[1..L] holds the L list sizes and lstart[0..L) their
// starts within their layers; turns lpref[0..L] into the exclusive prefix of
// the sizes and lstart into the list offsets, and returns the total (L <= 64).
__device__ inline uint32_t wave_layer_prefix(uint32_t *lpref, uint32_t *lstart, int L, int64_t n,
                                             uint32_t pmagic)
{
    const int lane = threadIdx.x & 63;
    const uint32_t sz = lane < L ? lpref[lane + 1] : 0u;
    uint32_t v = sz;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)v, off);
        if (lane >= off) v += t;
    }
    if (lane < L) {
        lpref[lane + 1] = v;
        lstart[lane] = list_offset(lane, lstart[lane], v - sz, n, pmagic);
    }
    if (lane == 0) lpref[0] = 0;
    return (uint32_t)__shfl((int)v, 63);
}

// Whole workgroup: lpref[1..nl] holds the nl list sizes and lstart[0..nl)
// their starts (nl <= 4 * kBlock); turns lpref[0..nl] into their exclusive
// prefix and lstart into the list offsets, and returns the total in every
// thread.  tmp: kBlock / 64 words of LDS.  Barriers inside.
__device__ inline uint32_t block_list_prefix(uint32_t *lpref, uint32_t *lstart, int nl, int64_t n,
                                             uint32_t pmagic, uint32_t *tmp)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t v[4], st[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = 4 * tid + i;
        v[i] = e < nl ? lpref[e + 1] : 0u;
        st[i] = e < nl ? lstart[e] : 0u;
        s += v[i];
    }
    uint32_t incl = s;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
        if (lane >= off) incl += t;
    }
    __syncthreads();  // every thread has read its sizes
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    uint32_t run = incl - s, total = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        run += w < wave ? tmp[w] : 0u;
        total += tmp[w];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = 4 * tid + i;
        if (e < nl) {
            lstart[e] = list_offset(e, st[i], run, n, pmagic);
            lpref[e + 1] = run + v[i];
        }
        run += v[i];
    }
    if (tid == 0) lpref[0] = 0;
    __syncthreads();
    return total;
}

// Loads positions base + r * kBlock + threadIdx.x (r < R) of the concatenated
// bucket lists (list i holds positions [lpref[i], lpref[i+1]); lstart holds
// the list offsets of a prefix above) into id[r]; returns the mask of
// positions below T.  The list of a position is found by a binary search
// (TOP = the largest power of two below the list count: 32 for at most 64
// lists), four positions interleaved so their reads and loads are in flight
// together; each group of four positions starts only if some position of the
// workgroup's group lies below T (uniform), so the work follows the query's
// list total rather than R.
template <int R, int TOP = 32>
__device__ inline uint32_t load_ids(const int32_t *__restrict__ ids, int32_t nl,
                                    const uint32_t *lpref, const uint32_t *lstart, uint32_t T,
                                    uint32_t base, uint32_t (&id)[R])
{
    static_assert(R % 4 == 0, "groups of four positions");
    uint32_t valid = 0;
#pragma unroll
    for (int g = 0; g < R / 4; ++g) {
        if (base + (uint32_t)(4 * g * kBlock) < T) {  // uniform
            uint32_t pos[4];
            int lo[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                pos[r] = base + (uint32_t)((4 * g + r) * kBlock) + threadIdx.x;
                lo[r] = 0;
            }
#pragma unroll
            for (int step = TOP; step > 0; step >>= 1)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // largest i < nl with lpref[i] <= pos; lpref[nl] = T > pos stops
                    // the search at the end without a branch around the read
                    const int m = lo[r] + step;
                    const uint32_t v = lpref[m < nl ? m : nl];
                    lo[r] = v <= pos[r] ? m : lo[r];
                }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                id[4 * g + r] = 0;
                if (pos[r] < T) {
                    id[4 * g + r] = (uint32_t)ids[lstart[lo[r]] + pos[r]];
                    valid |= 1u << (4 * g + r);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) id[4 * g + r] = 0;
        }
    }
    return valid;
}

// Whole workgroup (kBlock threads).  Inserts the T ids of the concatenated
// bucket lists (as load_ids reads them) into the cleared set `tab` of
// 2^cap_log2 slots.  The
// unique count goes to *ucount; *ovf is set when it exceeds `limit` or the
// set fills.  Without overflow and with `compact`, the set is then compacted in
// place: tab[0..U) holds the unique ids (unspecified order).  *ucount, *ovf
// and *cpos must be 0 and visible to all threads on entry; returns after a
// barrier.
template <int TOP = 32>
__device__ __attribute__((always_inline)) inline void set_union(const int32_t *__restrict__ ids, int32_t nl,
                                 const uint32_t *lpref, const uint32_t *lstart, uint32_t T,
                                 uint32_t *tab, int cap_log2, uint32_t limit, bool glob,
                                 uint32_t max_probe, bool compact, uint32_t *ucount,
                                 uint32_t *ovf, uint32_t *cpos)
{
    constexpr int R = 8;
    const int tid = threadIdx.x, lane = tid & 63;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    // the next round's ids load while this round's are inserted
    uint32_t idn[R];
    uint32_t pn = load_ids<R, TOP>(ids, nl, lpref, lstart, T, 0u, idn);
    for (uint32_t base = 0; base < T; base += R * kBlock) {
        // every thread reads the flag before any thread of this pass can set
        // it, so the early exit is uniform
        const bool stop = *ovf != 0;
        __syncthreads();
        if (stop) break;
        uint32_t idr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) idr[r] = idn[r];
        const uint32_t pend = pn;
        if (base + R * kBlock < T) pn = load_ids<R, TOP>(ids, nl, lpref, lstart, T, base + R * kBlock, idn);
        bool full = false;
        uint32_t nnew = (uint32_t)__popc(insert_streams<R, 4>(tab, cap_log2, idr, pend, max_probe, full));
        // one LDS atomic per wave for the unique count
        for (int off = 32; off > 0; off >>= 1) nnew += (uint32_t)__shfl_xor((int)nnew, off);
        const bool anyfull = __ballot(full) != 0ull;
        if (lane == 0 && (nnew || anyfull)) {
            const uint32_t tot = atomicAdd(ucount, nnew) + nnew;
            if (tot > limit || anyfull) *ovf = 1;
        }
        if (glob) __threadfence();
        __syncthreads();
    }
    if (!compact || *ovf || *ucount > limit) return;  // uniform: read after the last barrier
    // compact in place: contents move only to lower positions that were read
    // in this or an earlier round
    const uint32_t cap = 1u << cap_log2;
    for (uint32_t base = 0; base < cap; base += kBlock) {
        const uint32_t v = tab[base + tid];
        const bool occ = v != kEmpty;
        if (glob) __threadfence();
        __syncthreads();
        const unsigned long long m = __ballot(occ);
        uint32_t wb = 0;
        if (lane == 0 && m) wb = atomicAdd(cpos, (uint32_t)__popcll(m));
        wb = (uint32_t)__shfl((int)wb, 0);
        if (occ) tab[wb + (uint32_t)__popcll(m & lt_mask)] = v;
    }
    if (glob) __threadfence();
    __syncthreads();
}

}  // namespace qw
