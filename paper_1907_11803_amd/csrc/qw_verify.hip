// Candidate union, verification and top-K for one query per workgroup.
//
// For query q the candidates are C(q) = the union over layers l of the bucket
// members ids_l[start_{q,l} .. start_{q,l} + s_{q,l}) (the index accessed to find
// candidates, Sections 1.2 and 5.1).  Each candidate is verified by its exact
// squared Euclidean distance (the false-positive removal of Section 1.2) and the
// K smallest by (distance, id) are returned (the c-k-ANN output, Section 3).
//
// Phase 1 (dedup): the workgroup streams the concatenated bucket id lists
//   (coalesced, four positions per thread in flight) and inserts every id into
//   an open-addressing hash set (LDS, load factor <= 3/4, or global scratch for
//   very large queries).  Wavefront reductions count the new ids with one LDS
//   atomic per wave.  The set is then compacted in place into a dense list with
//   wavefront ballots.
// Phase 2 (verify): groups of G lanes gather candidate rows (16 bytes per lane
//   per load, up to eight candidates in flight per lane) and reduce the distance
//   across the group.  uint8 rows: exact int32 via dot4 (|x|^2 - 2 x.q + |q|^2).
//   float rows: FP32 with a proven relative error bound eps.
// Phase 3 (top-K): group leaders append entries under a threshold to an LDS
//   buffer; a bitonic sort keeps the K best whenever it fills.  For float data
//   every kept entry is first re-ranked by its FP64 index-order distance, and the
//   admission threshold is the K-th FP64 distance times (1 + eps), so no member
//   of the exact top-K is ever rejected.
//
// Work items: a launch serves a segment of the scheduled order plus a queue of
// queries that overflowed a smaller hash set; a query whose unique candidates
// exceed this launch's set is appended to the next launch's queue.
#include "qw_dedup.h"
#include "qw_exact.h"
#include "qw_internal.h"

namespace qw {

struct TopF {  // float data entry
    unsigned long long pri;  // FP32 bits (unranked) or FP64 bits (ranked)
    uint32_t id;
    uint32_t flag;           // 1 = unranked
};

template <int DT> struct TopT;
template <> struct TopT<QW_U8> { using type = unsigned long long; };  // (dist << 32) | id
template <> struct TopT<QW_F32> { using type = TopF; };

enum { S_ITEM = 0, S_UCOUNT, S_OVF, S_BUFCOUNT, S_THR, S_QQ, S_T, S_CAP, S_CPOS, S_TMP = 12,
       S_NSCAL = 16 };

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

struct LdsLayout {
    size_t buf, q, tab, lpref, lstart, scal, total;
};

__host__ __device__ inline LdsLayout lds_layout(int cap_log2, int buf, int global_tab, int nl,
                                                int dp, int dtype)
{
    LdsLayout o;
    const size_t cap = size_t(1) << cap_log2;
    const size_t esz = dtype == QW_U8 ? 8 : 16;
    o.buf = 0;
    o.q = o.buf + align16(size_t(buf) * esz);
    o.tab = o.q + align16(size_t(dp) * (dtype == QW_U8 ? 1 : 4));
    o.lpref = o.tab + (global_tab ? 0 : cap * 4);
    o.lstart = o.lpref + align16(size_t(nl + 1) * 4);
    o.scal = o.lstart + align16(size_t(nl) * 4);
    o.total = o.scal + S_NSCAL * 4;
    return o;
}

size_t verify_lds_bytes(int cap_log2, int buf, int global_tab, int nl, int dp, int dtype)
{
    return lds_layout(cap_log2, buf, global_tab, nl, dp, dtype).total;
}

__device__ inline bool entry_less(unsigned long long a, unsigned long long b) { return a < b; }
__device__ inline bool entry_less(const TopF &a, const TopF &b)
{
    return a.pri < b.pri || (a.pri == b.pri && a.id < b.id);
}
__device__ inline void entry_sentinel(unsigned long long &e) { e = ~0ull; }
__device__ inline void entry_sentinel(TopF &e)
{
    e.pri = ~0ull;
    e.id = 0xFFFFFFFFu;
    e.flag = 0;
}

// Compact the top-K buffer: rank unranked float entries in FP64, sort the live
// entries, keep K, update the admission threshold.  Whole workgroup.
template <int DT>
__device__ void topk_compact(typename TopT<DT>::type *buf, uint32_t *scal, int nbuf, int K,
                             const void *data, int32_t dp, int32_t d, const float *qrow, float eps,
                             const int32_t *slot)
{
    using E = typename TopT<DT>::type;
    __syncthreads();
    const int n_e = (int)scal[S_BUFCOUNT];
    if constexpr (DT == QW_F32) {
        for (int e = threadIdx.x; e < n_e; e += kBlock) {
            if (buf[e].flag) {
                const int64_t r = slot ? (int64_t)slot[buf[e].id] : (int64_t)buf[e].id;
                const float *x = (const float *)data + r * dp;
                const double D = exact_dist_row(x, qrow, dp);
                buf[e].pri = (unsigned long long)__double_as_longlong(D);
                buf[e].flag = 0;
            }
        }
    }
    int nsort = 2;
    while (nsort < n_e) nsort <<= 1;
    if (nsort > nbuf) nsort = nbuf;
    for (int e = n_e + threadIdx.x; e < nsort; e += kBlock) entry_sentinel(buf[e]);
    __syncthreads();
    for (int size = 2; size <= nsort; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < nsort / 2; i += kBlock) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                E a = buf[lo], b = buf[hi];
                if (entry_less(b, a) == asc) {
                    buf[lo] = b;
                    buf[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        const int keep = n_e < K ? n_e : K;
        scal[S_BUFCOUNT] = (uint32_t)keep;
        if (keep == K) {
            if constexpr (DT == QW_U8) {
                scal[S_THR] = (uint32_t)(buf[K - 1] >> 32);
            } else {
                const double DK = __longlong_as_double((long long)buf[K - 1].pri);
                const double t = DK * (1.0 + (double)eps) + (d + 1) * 0x1p-100;
                float f = (float)t;
                if ((double)f < t) f = nextafterf(f, INFINITY);
                scal[S_THR] = __float_as_uint(f);
            }
        }
    }
    __syncthreads();
}

// GLOB: the hash sets live in global scratch (one per workgroup) instead of
// LDS; a compile-time choice so that LDS sets compile to LDS instructions.
// SLOT: rows are read through A.row_slot (the out-of-core data cache).
template <int DT, int UN, int PM, bool GLOB, bool SLOT = false>
__global__ __launch_bounds__(kBlock) void verify_kernel(VerifyArgs A)
{
    using E = typename TopT<DT>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    constexpr int glob = GLOB ? 1 : 0;
    const LdsLayout lay = lds_layout((int)A.cap_log2, (int)A.buf, glob, A.nl, A.dp, A.dtype);
    E *buf = reinterpret_cast<E *>(smem + lay.buf);
    uint32_t *lpref = reinterpret_cast<uint32_t *>(smem + lay.lpref);
    uint32_t *lstart = reinterpret_cast<uint32_t *>(smem + lay.lstart);
    uint32_t *scal = reinterpret_cast<uint32_t *>(smem + lay.scal);
    const size_t gcap = size_t(1) << A.cap_log2;
    uint32_t *tab = GLOB ? A.gscratch + (size_t)blockIdx.x * gcap
                         : reinterpret_cast<uint32_t *>(smem + lay.tab);

    const int elem = DT == QW_U8 ? 1 : 4;
    const int row_bytes = A.dp * elem;
    const int parts = row_bytes / 16;  // 16-byte parts per row
    int G = 1;
    while (G < parts && G < 64) G <<= 1;
    const int P = (parts + G - 1) / G;  // parts per lane
    const int NG = kBlock / G;
    const int per_iter = NG * UN;
    const int grp = tid / G, j = tid % G;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    // relative error bound of the FP32 distance: term rounding (2u), 4P sequential
    // adds per lane, log2(G) <= 6 tree levels; plus the FP64 reference's own error
    const float eps = (float)((4 * P + 16) * 0x1p-24 + (A.d + 2) * 0x1p-52);

    // item space: [0, nseg) from the scheduled order, then [nseg, nseg + nin)
    // from the queue of queries that overflowed a smaller set
    int64_t sbeg = 0, nseg = A.nitems;
    if (A.seg) {
        sbeg = (int64_t)A.seg[0];
        nseg = (int64_t)A.seg[1] - sbeg;
    } else if (A.nitems_dev) {
        nseg = (int64_t)*A.nitems_dev;
    }
    const int64_t nin = A.in_count ? (int64_t)*A.in_count : 0;
    const int64_t nall = nseg + nin;
    int64_t first = A.counter ? -1 : (int64_t)blockIdx.x;

    if (nall == 0) return;  // uniform: an empty queue costs no atomic on the shared counter
    while (true) {
        if (tid == 0) {
            int64_t it = A.counter ? (int64_t)atomicAdd(A.counter, 1u) : first;
            scal[S_ITEM] = it < nall ? (uint32_t)it : 0xFFFFFFFFu;
        }
        __syncthreads();
        if (scal[S_ITEM] == 0xFFFFFFFFu) break;
        const int64_t item = scal[S_ITEM];
        first = nall;  // non-persistent launches serve one item
        int64_t q;
        if (item < nseg) {
            const int64_t o = sbeg + item;
            q = A.order ? (int64_t)A.order[o] : o;
        } else {
            q = (int64_t)A.in_list[item - nseg];
        }

        // ---- per-query setup
        for (int i = tid; i < A.nl; i += kBlock) {
            lstart[i] = A.bstart[q * A.nl + i];
            lpref[i + 1] = A.bsize[q * A.nl + i];
        }
        if (tid == 0) {
            lpref[0] = 0;
            scal[S_UCOUNT] = 0;
            scal[S_OVF] = 0;
            scal[S_BUFCOUNT] = 0;
            scal[S_THR] = DT == QW_U8 ? 0xFFFFFFFFu : __float_as_uint(INFINITY);
            scal[S_QQ] = 0;
            scal[S_CPOS] = 0;
        }
        {  // query row into LDS (+ |q|^2 for uint8)
            const uint4 *src = reinterpret_cast<const uint4 *>((const unsigned char *)A.queries +
                                                               q * (int64_t)row_bytes);
            uint4 *dst = reinterpret_cast<uint4 *>(smem + lay.q);
            uint32_t qq = 0;
            for (int i = tid; i < parts; i += kBlock) {
                uint4 v = src[i];
                dst[i] = v;
                if (DT == QW_U8) {
                    qq = __builtin_amdgcn_udot4(v.x, v.x, qq, false);
                    qq = __builtin_amdgcn_udot4(v.y, v.y, qq, false);
                    qq = __builtin_amdgcn_udot4(v.z, v.z, qq, false);
                    qq = __builtin_amdgcn_udot4(v.w, v.w, qq, false);
                }
            }
            __syncthreads();
            if (DT == QW_U8 && qq) atomicAdd(&scal[S_QQ], qq);
        }
        uint32_t run = 0;
        if (A.nl > 64) run = block_list_prefix(lpref, lstart, A.nl, A.n, A.pmagic, &scal[S_TMP]);  // uniform
        else if (tid < 64) run = wave_layer_prefix(lpref, lstart, A.nl, A.n, A.pmagic);
        if (tid < 64) {
            if (tid == 0) {
                scal[S_T] = run;
                int c = (int)A.cap_log2;
                if (glob) {  // set sized from the exact bound min(sum_l s_{q,l}, n)
                    const uint64_t bound = min((uint64_t)run, (uint64_t)A.n);
                    c = 10;
                    while (c < (int)A.cap_log2 && (3ull << c) < 4 * bound) ++c;
                }
                scal[S_CAP] = (uint32_t)c;
            }
        }
        __syncthreads();
        const int cap_log2 = (int)scal[S_CAP];
        const uint32_t cap = 1u << cap_log2;
        const uint32_t set_limit = (cap >> 2) * 3;  // load factor <= 3/4
        const uint32_t limit = glob ? set_limit : (A.limit < set_limit ? A.limit : set_limit);
        const uint32_t T = A.mode == VM_ALL ? 0u : scal[S_T];
        if (A.mode != VM_ALL)
            for (uint32_t i = tid; i < cap; i += kBlock) tab[i] = kEmpty;
        if (glob) __threadfence();
        __syncthreads();

        // ---- phase 1: de-duplicated union of the bucket lists
        if (A.mode != VM_ALL) {
            const uint32_t mprobe = A.short_probe ? kShortProbe : 0xFFFFFFFFu;
            if (A.nl > 64)  // uniform: neighbour probing, up to kMaxLists lists
                set_union<kMaxLists / 2>(A.ids, A.nl, lpref, lstart, T, tab, cap_log2,
                                         limit, glob != 0, mprobe, true, &scal[S_UCOUNT],
                                         &scal[S_OVF], &scal[S_CPOS]);
            else
                set_union<32>(A.ids, A.nl, lpref, lstart, T, tab, cap_log2, limit,
                              glob != 0, mprobe, true, &scal[S_UCOUNT], &scal[S_OVF],
                              &scal[S_CPOS]);
        }
        const uint32_t U = A.mode == VM_ALL ? (uint32_t)A.n : scal[S_UCOUNT];
        if (A.mode != VM_ALL && (scal[S_OVF] || U > limit)) {
            if (tid == 0) {
                const uint32_t o = atomicAdd(A.ovf_count, 1u);
                A.ovf_list[o] = (int32_t)q;
            }
            __syncthreads();
            continue;
        }
        if (tid == 0 && A.ucount_out && A.mode != VM_ALL) A.ucount_out[q] = U;
        if (A.mode == VM_COUNT) {
            if (tid == 0) A.out_counts[q] = (int32_t)U;
            __syncthreads();
            continue;
        }
        if (A.mode == VM_LIST) {
            const long long o = A.offsets[q];
            for (uint32_t i = tid; i < U; i += kBlock) A.out_ids[o + i] = (int32_t)tab[i];
            __syncthreads();
            continue;
        }

        // ---- phase 2: gather and verify
        const uint32_t qq = scal[S_QQ];
        const unsigned char *qrow_b = smem + lay.q;
        for (uint32_t c0 = 0; c0 < U; c0 += (uint32_t)per_iter) {
            // every thread snapshots the buffer count between two barriers, so
            // the compaction decision is uniform even though leaders append to
            // the buffer later in this iteration
            __syncthreads();
            const int bufcount = (int)scal[S_BUFCOUNT];
            __syncthreads();
            if (bufcount > (int)A.buf - per_iter)
                topk_compact<DT>(buf, scal, (int)A.buf, A.K, A.data, A.dp, A.d,
                                 reinterpret_cast<const float *>(qrow_b), eps,
                                 SLOT ? A.row_slot : nullptr);
            const uint32_t thr = scal[S_THR];
            uint32_t cid[UN];
            bool cv[UN];
            for (int u = 0; u < UN; ++u) {
                const uint32_t c = c0 + grp + (uint32_t)(NG * u);
                cv[u] = c < U;
                cid[u] = cv[u] ? (A.mode == VM_ALL ? c : tab[c]) : 0u;
            }
            uint32_t rid[UN];  // row index of each candidate in A.data
            for (int u = 0; u < UN; ++u) {
                rid[u] = SLOT && cv[u] ? (uint32_t)A.row_slot[cid[u]] : cid[u];
                // every candidate's row is resident before the launch; a row
                // that is not (slot -1) is never read
                if (SLOT && (int32_t)rid[u] < 0) cv[u] = false;
            }
            uint32_t accu[UN];
            float accf[UN];
            for (int u = 0; u < UN; ++u) {
                accu[u] = 0;
                accf[u] = 0.f;
            }
            for (int p0 = 0; p0 < P; p0 += PM) {
                uint4 xv[UN][PM];
                for (int u = 0; u < UN; ++u)
                    for (int pp = 0; pp < PM; ++pp) {
                        const int part = j + G * (p0 + pp);
                        if (cv[u] && p0 + pp < P && part < parts) {
                            const uint4 *row = reinterpret_cast<const uint4 *>(
                                (const unsigned char *)A.data + (int64_t)rid[u] * row_bytes);
                            xv[u][pp] = row[part];
                        } else {
                            xv[u][pp] = make_uint4(0, 0, 0, 0);
                        }
                    }
                for (int pp = 0; pp < PM; ++pp) {
                    const int part = j + G * (p0 + pp);
                    if (p0 + pp >= P || part >= parts) continue;
                    const uint4 qv = reinterpret_cast<const uint4 *>(qrow_b)[part];
                    for (int u = 0; u < UN; ++u) {
                        const uint4 x = xv[u][pp];
                        if (DT == QW_U8) {
                            uint32_t xx = 0, xq = 0;
                            xx = __builtin_amdgcn_udot4(x.x, x.x, xx, false);
                            xx = __builtin_amdgcn_udot4(x.y, x.y, xx, false);
                            xx = __builtin_amdgcn_udot4(x.z, x.z, xx, false);
                            xx = __builtin_amdgcn_udot4(x.w, x.w, xx, false);
                            xq = __builtin_amdgcn_udot4(x.x, qv.x, xq, false);
                            xq = __builtin_amdgcn_udot4(x.y, qv.y, xq, false);
                            xq = __builtin_amdgcn_udot4(x.z, qv.z, xq, false);
                            xq = __builtin_amdgcn_udot4(x.w, qv.w, xq, false);
                            accu[u] += xx - 2u * xq;
                        } else {
                            float d0 = __uint_as_float(x.x) - __uint_as_float(qv.x);
                            float d1 = __uint_as_float(x.y) - __uint_as_float(qv.y);
                            float d2 = __uint_as_float(x.z) - __uint_as_float(qv.z);
                            float d3 = __uint_as_float(x.w) - __uint_as_float(qv.w);
                            float s = accf[u];
                            s = fmaf(d0, d0, s);
                            s = fmaf(d1, d1, s);
                            s = fmaf(d2, d2, s);
                            s = fmaf(d3, d3, s);
                            accf[u] = s;
                        }
                    }
                }
            }
            for (int u = 0; u < UN; ++u) {
                for (int off = G >> 1; off > 0; off >>= 1) {
                    if (DT == QW_U8)
                        accu[u] += (uint32_t)__shfl_xor((int)accu[u], off);
                    else
                        accf[u] += __shfl_xor(accf[u], off);
                }
            }
            if (j == 0) {
                for (int u = 0; u < UN; ++u) {
                    if (!cv[u]) continue;
                    if constexpr (DT == QW_U8) {
                        const uint32_t dist = accu[u] + qq;
                        if (dist <= thr) {
                            const uint32_t e = atomicAdd(&scal[S_BUFCOUNT], 1u);
                            buf[e] = ((unsigned long long)dist << 32) | cid[u];
                        }
                    } else {
                        if (accf[u] <= __uint_as_float(thr)) {
                            const uint32_t e = atomicAdd(&scal[S_BUFCOUNT], 1u);
                            buf[e].pri = __float_as_uint(accf[u]);
                            buf[e].id = cid[u];
                            buf[e].flag = 1;
                        }
                    }
                }
            }
        }
        topk_compact<DT>(buf, scal, (int)A.buf, A.K, A.data, A.dp, A.d,
                         reinterpret_cast<const float *>(qrow_b), eps,
                         SLOT ? A.row_slot : nullptr);
        const int keep = (int)scal[S_BUFCOUNT];
        for (int r = tid; r < A.K; r += kBlock) {
            const int64_t o = q * A.K + r;
            if (r < keep) {
                if constexpr (DT == QW_U8) {
                    A.out_ids[o] = (int32_t)(uint32_t)buf[r];
                    reinterpret_cast<int32_t *>(A.out_dist)[o] = (int32_t)(buf[r] >> 32);
                } else {
                    A.out_ids[o] = (int32_t)buf[r].id;
                    reinterpret_cast<float *>(A.out_dist)[o] =
                        (float)__longlong_as_double((long long)buf[r].pri);
                }
            } else {
                A.out_ids[o] = -1;
                if (DT == QW_U8)
                    reinterpret_cast<int32_t *>(A.out_dist)[o] = INT32_MAX;
                else
                    reinterpret_cast<float *>(A.out_dist)[o] = INFINITY;
            }
        }
        __syncthreads();
    }
}

static bool one_part_per_lane(int dp, int dtype)
{
    return dp * (dtype == QW_U8 ? 1 : 4) / 16 <= 64;
}

int verify_per_iter(int dp, int dtype)
{
    const int parts = dp * (dtype == QW_U8 ? 1 : 4) / 16;
    int G = 1;
    while (G < parts && G < 64) G <<= 1;
    return (kBlock / G) * (one_part_per_lane(dp, dtype) ? 8 : 2);
}

static const void *verify_fn(int dp, int dtype)
{
    const bool small = one_part_per_lane(dp, dtype);
    if (dtype == QW_U8)
        return small ? (const void *)verify_kernel<QW_U8, 8, 1, false>
                     : (const void *)verify_kernel<QW_U8, 2, 4, false>;
    return small ? (const void *)verify_kernel<QW_F32, 8, 1, false>
                 : (const void *)verify_kernel<QW_F32, 2, 4, false>;
}

int verify_blocks_per_cu(int dp, int dtype, size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, verify_fn(dp, dtype), kBlock, lds) !=
        hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb > 0 ? nb : 1;
}

qw_status launch_verify(const VerifyArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    // nl = 0: brute force (no lists)
    if (a.nl < 0 || a.nl > kMaxLists || (a.nl > 64 && !a.pmagic)) return QW_EINVAL;
    const size_t lds = verify_lds_bytes((int)a.cap_log2, (int)a.buf, a.global_tab, a.nl, a.dp,
                                        a.dtype);
    const bool small = one_part_per_lane(a.dp, a.dtype);
    const bool g = a.global_tab != 0;
    if (a.row_slot) {  // out-of-core data cache: LDS sets only
        if (g) return QW_EINVAL;
        if (a.dtype == QW_U8) {
            if (small) verify_kernel<QW_U8, 8, 1, false, true><<<grid, kBlock, lds, s>>>(a);
            else verify_kernel<QW_U8, 2, 4, false, true><<<grid, kBlock, lds, s>>>(a);
        } else {
            if (small) verify_kernel<QW_F32, 8, 1, false, true><<<grid, kBlock, lds, s>>>(a);
            else verify_kernel<QW_F32, 2, 4, false, true><<<grid, kBlock, lds, s>>>(a);
        }
        QW_HIP(hipGetLastError());
        return QW_OK;
    }
    if (a.dtype == QW_U8) {
        if (small && g) verify_kernel<QW_U8, 8, 1, true><<<grid, kBlock, lds, s>>>(a);
        else if (small) verify_kernel<QW_U8, 8, 1, false><<<grid, kBlock, lds, s>>>(a);
        else if (g) verify_kernel<QW_U8, 2, 4, true><<<grid, kBlock, lds, s>>>(a);
        else verify_kernel<QW_U8, 2, 4, false><<<grid, kBlock, lds, s>>>(a);
    } else {
        if (small && g) verify_kernel<QW_F32, 8, 1, true><<<grid, kBlock, lds, s>>>(a);
        else if (small) verify_kernel<QW_F32, 8, 1, false><<<grid, kBlock, lds, s>>>(a);
        else if (g) verify_kernel<QW_F32, 2, 4, true><<<grid, kBlock, lds, s>>>(a);
        else verify_kernel<QW_F32, 2, 4, false><<<grid, kBlock, lds, s>>>(a);
    }
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
