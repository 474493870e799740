// De-duplicated union of one query's bucket id lists (Sections 1.2 and 5.1:
// the candidates are the union of the buckets the query falls in, one per
// layer).  Device code shared by the fused verify kernel and the dedup kernel.
#pragma once

#include "qw_internal.h"

namespace qw {

__device__ inline uint32_t hash_id(uint32_t id, int cap_log2)
{
    return (id * 0x9E3779B1u) >> (32 - cap_log2);
}

enum { INS_NEW = 0, INS_DUP = 1, INS_FULL = 2 };

// Open addressing with linear probing, at most max_probe slots per insert.
// Sets that may pass an overflowing query on to a larger set use a short
// bound (kShortProbe): at load factor <= 3/4 a longer run means the set is
// (nearly) over its limit, and the insert reports INS_FULL instead of scanning
// on.  Sets that must hold every id probe the whole capacity.
constexpr uint32_t kShortProbe = 64;

__device__ inline int set_insert(uint32_t *tab, int cap_log2, uint32_t id, uint32_t max_probe)
{
    const uint32_t mask = (1u << cap_log2) - 1u;
    uint32_t slot = hash_id(id, cap_log2);
    const uint32_t probes = mask < max_probe ? mask + 1 : max_probe;
    for (uint32_t it = 0; it < probes; ++it) {
        uint32_t old = atomicCAS(&tab[slot], kEmpty, id);
        if (old == kEmpty) return INS_NEW;
        if (old == id) return INS_DUP;
        slot = (slot + 1) & mask;
    }
    return INS_FULL;
}

// Whole workgroup (kBlock threads).  Inserts the T ids of the concatenated
// layer lists (layer l holds positions [lpref[l], lpref[l+1]) and starts at
// ids[l*n + lstart[l]]) into the cleared set `tab` of 2^cap_log2 slots.  The
// unique count goes to *ucount; *ovf is set when it exceeds `limit` or the
// set fills.  Without overflow and with `compact`, the set is then compacted in
// place: tab[0..U) holds the unique ids (unspecified order).  *ucount, *ovf
// and *cpos must be 0 and visible to all threads on entry; returns after a
// barrier.
__device__ inline void set_union(const int32_t *__restrict__ ids, int64_t n, int32_t L,
                                 const uint32_t *lpref, const uint32_t *lstart, uint32_t T,
                                 uint32_t *tab, int cap_log2, uint32_t limit, bool glob,
                                 uint32_t max_probe, bool compact, uint32_t *ucount,
                                 uint32_t *ovf, uint32_t *cpos)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (uint32_t base = 0; base < T; base += 4 * kBlock) {
        // every thread reads the flag before any thread of this pass can set
        // it, so the early exit is uniform
        const bool stop = *ovf != 0;
        __syncthreads();
        if (stop) break;
        uint32_t ids4[4];
        bool ok4[4];
        for (int r = 0; r < 4; ++r) {
            const uint32_t pos = base + (uint32_t)(r * kBlock + tid);
            ok4[r] = pos < T;
            ids4[r] = 0;
            if (ok4[r]) {
                int lo = 0, hi = L;  // lpref[lo] <= pos < lpref[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (lpref[mid] <= pos) lo = mid; else hi = mid;
                }
                ids4[r] = (uint32_t)ids[(int64_t)lo * n + lstart[lo] + (pos - lpref[lo])];
            }
        }
        uint32_t nnew = 0;
        bool full = false;
        for (int r = 0; r < 4; ++r) {
            if (!ok4[r]) continue;
            const int res = set_insert(tab, cap_log2, ids4[r], max_probe);
            nnew += res == INS_NEW;
            full |= res == INS_FULL;
        }
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
