// Flat query pipeline of the fast form: dedup -> gather -> select.
//
// 1. dedup_kernel: one workgroup per query builds C(q) (the union of the
//    query's buckets, Sections 1.2 and 5.1) in an LDS hash set sized by the
//    predicted count, and scatters the unique ids -- each tagged with its query
//    -- into a device-wide pair list through a bump allocator.  Queries whose
//    set overflows move to the next size class.
// 2. gather_kernel: a pure streaming pass over all (query, candidate) pairs:
//    gather the row, compute the exact squared distance (the false-positive
//    removal of Section 1.2), write one (distance, id) key per pair.  The pair
//    list is cut into eight contiguous ranges, one per XCD (workgroup b runs on
//    XCD b % 8); the pairs of a bucket group are adjacent, so their rows are
//    shared through that XCD's L2.  No barriers: every wave keeps loads in
//    flight all the time.
// 3. select_kernel: one workgroup per query selects the K smallest keys of its
//    contiguous pair range by (distance, id) (the c-k-ANN output, Section 3);
//    for float data every key within the proven FP32 error band of the K-th is
//    re-ranked by its FP64 index-order distance.
// Queries that do not fit (list space, band capacity) are flagged and answered
// by the fused per-query kernel afterwards.
#include "qw_dedup.h"
#include "qw_internal.h"

namespace qw {

enum { D_ITEM = 0, D_UCOUNT, D_OVF, D_CPOS, D_T, D_CAP, D_OFF = 6 /* u64 */, D_NSCAL = 8 };

__host__ __device__ inline size_t a16(size_t v) { return (v + 15) & ~size_t(15); }

size_t dedup_lds_bytes(int cap_log2, int global_tab, int L)
{
    return (global_tab ? 0 : (size_t(4) << cap_log2)) + a16(size_t(L + 1) * 4) +
           a16(size_t(L) * 4) + D_NSCAL * 4;
}

__global__ __launch_bounds__(kBlock) void dedup_kernel(DedupArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const bool glob = A.global_tab != 0;
    const size_t tab_bytes = glob ? 0 : (size_t(4) << A.cap_log2);
    uint32_t *lpref = reinterpret_cast<uint32_t *>(smem + tab_bytes);
    uint32_t *lstart = reinterpret_cast<uint32_t *>(smem + tab_bytes + a16(size_t(A.L + 1) * 4));
    uint32_t *scal = reinterpret_cast<uint32_t *>(smem + tab_bytes + a16(size_t(A.L + 1) * 4) +
                                                  a16(size_t(A.L) * 4));
    uint32_t *tab = glob ? A.gscratch + (size_t)blockIdx.x * (size_t(1) << A.cap_log2)
                         : reinterpret_cast<uint32_t *>(smem);
    const int64_t sbeg = (int64_t)A.seg[0];
    const int64_t nseg = (int64_t)A.seg[1] - sbeg;
    const int64_t nin = A.in_count ? (int64_t)*A.in_count : 0;
    const int64_t nall = nseg + nin;

    while (true) {
        if (tid == 0) {
            const int64_t it = (int64_t)atomicAdd(A.counter, 1u);
            scal[D_ITEM] = it < nall ? (uint32_t)it : 0xFFFFFFFFu;
        }
        __syncthreads();
        if (scal[D_ITEM] == 0xFFFFFFFFu) break;
        const int64_t item = scal[D_ITEM];
        const int64_t q = item < nseg ? (int64_t)A.order[sbeg + item]
                                      : (int64_t)A.in_list[item - nseg];
        if (tid < A.L) {
            lstart[tid] = A.bstart[q * A.L + tid];
            lpref[tid + 1] = A.bsize[q * A.L + tid];
        }
        if (tid == 0) {
            scal[D_UCOUNT] = 0;
            scal[D_OVF] = 0;
            scal[D_CPOS] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t run = 0;
            lpref[0] = 0;
            for (int l = 0; l < A.L; ++l) {
                run += lpref[l + 1];
                lpref[l + 1] = run;
            }
            scal[D_T] = run;
            int c = (int)A.cap_log2;
            if (glob) {  // set sized from the exact bound min(sum_l s_{q,l}, n)
                const uint64_t bound = min((uint64_t)run, (uint64_t)A.n);
                c = 10;
                while (c < (int)A.cap_log2 && (3ull << c) < 4 * bound) ++c;
            }
            scal[D_CAP] = (uint32_t)c;
        }
        __syncthreads();
        const int cap_log2 = (int)scal[D_CAP];
        const uint32_t cap = 1u << cap_log2;
        const uint32_t set_limit = (cap >> 2) * 3;
        const uint32_t limit = glob ? set_limit : (A.limit < set_limit ? A.limit : set_limit);
        for (uint32_t i = tid; i < cap; i += kBlock) tab[i] = kEmpty;
        if (glob) __threadfence();
        __syncthreads();
        set_union(A.ids, A.n, A.L, lpref, lstart, scal[D_T], tab, cap_log2, limit, glob,
                  glob ? 0xFFFFFFFFu : kShortProbe, false, &scal[D_UCOUNT], &scal[D_OVF],
                  &scal[D_CPOS]);
        const uint32_t U = scal[D_UCOUNT];
        if (scal[D_OVF] || U > limit) {
            if (tid == 0) {
                const uint32_t o = atomicAdd(A.ovf_count, 1u);
                A.ovf_list[o] = (int32_t)q;
            }
            __syncthreads();
            continue;
        }
        if (A.count_only) {
            if (tid == 0) A.ucount[q] = U;
            __syncthreads();
            continue;
        }
        unsigned long long *soff = reinterpret_cast<unsigned long long *>(&scal[D_OFF]);
        if (tid == 0) {
            unsigned long long off = atomicAdd(A.alloc, (unsigned long long)U);
            if (off + U > A.cand_cap) {  // no list space: answered by the fallback
                A.flag[q] = 1;
                A.ucount[q] = 0;
                off = ~0ull;
            } else {
                A.ucount[q] = U;
                A.coff[q] = off;
                atomicMax(A.valid_end, off + U);
                if (A.unique_total) atomicAdd(A.unique_total, (unsigned long long)U);
            }
            *soff = off;
        }
        __syncthreads();
        const unsigned long long off = *soff;
        if (off != ~0ull) {
            // scatter the set's ids straight from the hashed layout: a wave
            // reserves its run of positions with one LDS atomic per round
            for (uint32_t base = 0; base < cap; base += kBlock) {
                const uint32_t v = tab[base + tid];
                const bool occ = v != kEmpty;
                const unsigned long long m = __ballot(occ);
                uint32_t wb = 0;
                if (lane == 0 && m) wb = atomicAdd(&scal[D_CPOS], (uint32_t)__popcll(m));
                wb = (uint32_t)__shfl((int)wb, 0);
                if (occ) {
                    const unsigned long long e = off + wb + (uint32_t)__popcll(m & lt_mask);
                    A.cand[e] = (int32_t)v;
                    A.candq[e] = (int32_t)q;
                }
            }
        }
        __syncthreads();
    }
}

qw_status launch_dedup(const DedupArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    dedup_kernel<<<grid, kBlock, dedup_lds_bytes((int)a.cap_log2, a.global_tab, a.L), s>>>(a);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

int dedup_blocks_per_cu(size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)dedup_kernel, kBlock, lds) !=
        hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb > 0 ? nb : 1;
}

// ---------------------------------------------------------------- gather

// Every pair e < N: key[e] = (squared distance << 32) | id, uint8 distances
// exact (sum over 16-byte parts of |x|^2 - 2 x.q + |q|^2 by dot4), float
// distances as FP32 bits (non-negative, so the bits order like the values).
template <int DT, int UN, int PM>
__global__ __launch_bounds__(kBlock) void gather_kernel(GatherArgs A)
{
    const int tid = threadIdx.x;
    const int elem = DT == QW_U8 ? 1 : 4;
    const int row_bytes = A.dp * elem;
    const int parts = row_bytes / 16;
    int G = 1;
    while (G < parts && G < 64) G <<= 1;
    const int P = (parts + G - 1) / G;
    const int NG = kBlock / G;
    const int PI = NG * UN;  // pairs per workgroup iteration
    const int grp = tid / G, j = tid % G;
    const unsigned long long N = *A.npairs;
    // XCD-local contiguous range
    const int x = blockIdx.x & 7;
    const int64_t nwg = ((int64_t)gridDim.x - x + 7) / 8;
    const int64_t r = blockIdx.x >> 3;
    const int64_t rb = (int64_t)(N * x / 8), re = (int64_t)(N * (x + 1) / 8);
    for (int64_t base = rb + r * PI; base < re; base += nwg * PI) {
        uint32_t cid[UN], cq[UN];
        bool cv[UN];
        for (int u = 0; u < UN; ++u) {
            const int64_t e = base + grp + (int64_t)NG * u;
            cv[u] = e < re;
            cid[u] = cv[u] ? (uint32_t)A.cand[e] : 0u;
            cq[u] = cv[u] ? (uint32_t)A.candq[e] : 0u;
        }
        uint32_t accu[UN];
        float accf[UN];
        for (int u = 0; u < UN; ++u) {
            accu[u] = 0;
            accf[u] = 0.f;
        }
        for (int p0 = 0; p0 < P; p0 += PM) {
            uint4 xv[UN][PM], qv[UN][PM];
            for (int u = 0; u < UN; ++u)
                for (int pp = 0; pp < PM; ++pp) {
                    const int part = j + G * (p0 + pp);
                    if (cv[u] && p0 + pp < P && part < parts) {
                        xv[u][pp] = reinterpret_cast<const uint4 *>(
                            (const unsigned char *)A.data + (int64_t)cid[u] * row_bytes)[part];
                        qv[u][pp] = reinterpret_cast<const uint4 *>(
                            (const unsigned char *)A.queries + (int64_t)cq[u] * row_bytes)[part];
                    } else {
                        xv[u][pp] = make_uint4(0, 0, 0, 0);
                        qv[u][pp] = make_uint4(0, 0, 0, 0);
                    }
                }
            for (int u = 0; u < UN; ++u)
                for (int pp = 0; pp < PM; ++pp) {
                    const uint4 xw = xv[u][pp], qw = qv[u][pp];
                    if (DT == QW_U8) {
                        uint32_t xx = 0, xq = 0, qq = 0;
                        xx = __builtin_amdgcn_udot4(xw.x, xw.x, xx, false);
                        xx = __builtin_amdgcn_udot4(xw.y, xw.y, xx, false);
                        xx = __builtin_amdgcn_udot4(xw.z, xw.z, xx, false);
                        xx = __builtin_amdgcn_udot4(xw.w, xw.w, xx, false);
                        xq = __builtin_amdgcn_udot4(xw.x, qw.x, xq, false);
                        xq = __builtin_amdgcn_udot4(xw.y, qw.y, xq, false);
                        xq = __builtin_amdgcn_udot4(xw.z, qw.z, xq, false);
                        xq = __builtin_amdgcn_udot4(xw.w, qw.w, xq, false);
                        qq = __builtin_amdgcn_udot4(qw.x, qw.x, qq, false);
                        qq = __builtin_amdgcn_udot4(qw.y, qw.y, qq, false);
                        qq = __builtin_amdgcn_udot4(qw.z, qw.z, qq, false);
                        qq = __builtin_amdgcn_udot4(qw.w, qw.w, qq, false);
                        accu[u] += xx - 2u * xq + qq;
                    } else {
                        const float d0 = __uint_as_float(xw.x) - __uint_as_float(qw.x);
                        const float d1 = __uint_as_float(xw.y) - __uint_as_float(qw.y);
                        const float d2 = __uint_as_float(xw.z) - __uint_as_float(qw.z);
                        const float d3 = __uint_as_float(xw.w) - __uint_as_float(qw.w);
                        float sacc = accf[u];
                        sacc = fmaf(d0, d0, sacc);
                        sacc = fmaf(d1, d1, sacc);
                        sacc = fmaf(d2, d2, sacc);
                        sacc = fmaf(d3, d3, sacc);
                        accf[u] = sacc;
                    }
                }
        }
        for (int u = 0; u < UN; ++u)
            for (int off = G >> 1; off > 0; off >>= 1) {
                if (DT == QW_U8)
                    accu[u] += (uint32_t)__shfl_xor((int)accu[u], off);
                else
                    accf[u] += __shfl_xor(accf[u], off);
            }
        if (j == 0)
            for (int u = 0; u < UN; ++u)
                if (cv[u]) {
                    const uint32_t hi = DT == QW_U8 ? accu[u] : __float_as_uint(accf[u]);
                    A.keys[base + grp + (int64_t)NG * u] = ((unsigned long long)hi << 32) | cid[u];
                }
    }
}

static bool gather_small(int dp, int dtype) { return dp * (dtype == QW_U8 ? 1 : 4) / 16 <= 64; }

static const void *gather_fn(int dp, int dtype)
{
    const bool small = gather_small(dp, dtype);
    if (dtype == QW_U8)
        return small ? (const void *)gather_kernel<QW_U8, 4, 1> : (const void *)gather_kernel<QW_U8, 2, 4>;
    return small ? (const void *)gather_kernel<QW_F32, 4, 1> : (const void *)gather_kernel<QW_F32, 2, 4>;
}

int gather_blocks_per_cu(int dp, int dtype)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gather_fn(dp, dtype), kBlock, 0) !=
        hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb > 0 ? nb : 1;
}

qw_status launch_gather(const GatherArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    const bool small = gather_small(a.dp, a.dtype);
    if (a.dtype == QW_U8) {
        if (small) gather_kernel<QW_U8, 4, 1><<<grid, kBlock, 0, s>>>(a);
        else gather_kernel<QW_U8, 2, 4><<<grid, kBlock, 0, s>>>(a);
    } else {
        if (small) gather_kernel<QW_F32, 4, 1><<<grid, kBlock, 0, s>>>(a);
        else gather_kernel<QW_F32, 2, 4><<<grid, kBlock, 0, s>>>(a);
    }
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// ---------------------------------------------------------------- select

// Bitonic sort of keys[0..n) ascending (the tail up to the next power of two
// is padded with ~0; that power of two must fit the buffer).  Whole workgroup.
__device__ inline void sort_keys(unsigned long long *keys, int n)
{
    int ns = 2;
    while (ns < n) ns <<= 1;
    for (int e = n + threadIdx.x; e < ns; e += kBlock) keys[e] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= ns; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < ns / 2; i += kBlock) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const unsigned long long a = keys[lo], b = keys[hi];
                if ((b < a) == asc) {
                    keys[lo] = b;
                    keys[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Band threshold F_K * (1 + eps) / (1 - eps), rounded up to float: every key
// of the exact top-K has an FP32 distance at most this (see the verify kernel).
__device__ inline float band_threshold(float FK, float eps)
{
    const double t = (double)FK * (1.0 + (double)eps) / (1.0 - (double)eps) + 0x1p-100;
    float f = (float)t;
    if ((double)f < t) f = nextafterf(f, INFINITY);
    return f;
}

struct RankF {
    double D;
    uint32_t id, pad;
};

__device__ __noinline__ double exact_dist_f32_s(const float *__restrict__ x,
                                                const float *__restrict__ q, int32_t d)
{
    double acc = 0.0;
    for (int32_t i = 0; i < d; ++i) {
        const double t = __dsub_rn((double)x[i], (double)q[i]);
        acc = __dadd_rn(acc, __dmul_rn(t, t));
    }
    return acc;
}

// One workgroup per query.  Keys stream through a threshold: a key enters the
// LDS list only if it is at most the current K-th key (uint8: keys are unique
// (distance, id) pairs, so exactly K survive) or within the band of the K-th
// distance (float); when the list passes half its capacity it is sorted and cut
// back to the K best plus the band.
template <int DT>
__global__ __launch_bounds__(kBlock) void select_kernel(SelectArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *lst = reinterpret_cast<unsigned long long *>(smem);
    RankF *rk = reinterpret_cast<RankF *>(smem + size_t(A.LC) * 8);
    __shared__ unsigned long long s_thr;
    __shared__ uint32_t s_cnt, s_bad;
    const int64_t q = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (tid == 0) {
        s_cnt = 0;
        s_thr = ~0ull;
        s_bad = A.flag[q];
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) A.fb_list[atomicAdd(A.fb_count, 1u)] = (int32_t)q;
        return;
    }
    const uint32_t U = A.ucount[q];
    const unsigned long long *keys = A.keys + (U ? A.coff[q] : 0ull);
    // trim: sort the list, keep the K best (uint8) or every key within the band
    // of the K-th (float); the threshold tightens accordingly
    auto trim = [&]() {
        const int n = (int)s_cnt;
        sort_keys(lst, n);
        if (tid == 0 && n >= A.K) {
            const unsigned long long kk = lst[A.K - 1];
            unsigned long long thr = kk;
            int keep = A.K;
            if (DT != QW_U8) {
                const float bt = band_threshold(__uint_as_float((uint32_t)(kk >> 32)), A.eps);
                thr = ((unsigned long long)__float_as_uint(bt) << 32) | 0xFFFFFFFFull;
                while (keep < n && lst[keep] <= thr) ++keep;
            }
            s_cnt = (uint32_t)keep;
            s_thr = thr;
            if (keep > A.LC / 2) s_bad = 1;  // band too wide for the list
        }
        __syncthreads();
    };
    for (uint32_t b0 = 0; b0 < U; b0 += 4 * kBlock) {
        const unsigned long long thr = s_thr;
        for (int i = 0; i < 4; ++i) {
            const uint32_t e = b0 + (uint32_t)(i * kBlock + tid);
            const unsigned long long k = e < U ? keys[e] : ~0ull;
            const bool take = e < U && k <= thr;
            const unsigned long long m = __ballot(take);
            uint32_t wb = 0;
            if (lane == 0 && m) wb = atomicAdd(&s_cnt, (uint32_t)__popcll(m));
            wb = (uint32_t)__shfl((int)wb, 0);
            if (take) lst[wb + (uint32_t)__popcll(m & lt_mask)] = k;
        }
        __syncthreads();
        const bool full = (int)s_cnt > A.LC / 2;
        __syncthreads();  // every thread has read s_cnt before the next pass adds to it
        if (full) trim();
        if (s_bad) break;  // set only inside trim, before its barrier
    }
    if (!s_bad) trim();
    if (s_bad) {
        if (tid == 0) A.fb_list[atomicAdd(A.fb_count, 1u)] = (int32_t)q;
        return;
    }
    const int n = (int)s_cnt;
    if (DT == QW_U8) {
        for (int r = tid; r < A.K; r += kBlock) {
            const int64_t o = q * A.K + r;
            if (r < n) {
                A.out_ids[o] = (int32_t)(uint32_t)lst[r];
                reinterpret_cast<int32_t *>(A.out_dist)[o] = (int32_t)(lst[r] >> 32);
            } else {
                A.out_ids[o] = -1;
                reinterpret_cast<int32_t *>(A.out_dist)[o] = INT32_MAX;
            }
        }
        return;
    }
    // float data: FP64 index-order distances of every key in the band, then
    // the exact (D, id) order
    const float *qrow = (const float *)A.queries + q * (int64_t)A.dp;
    for (int e = tid; e < n; e += kBlock) {
        const uint32_t id = (uint32_t)lst[e];
        rk[e].D = exact_dist_f32_s((const float *)A.data + (int64_t)id * A.dp, qrow, A.d);
        rk[e].id = id;
    }
    int ns = 2;
    while (ns < n) ns <<= 1;
    for (int e = n + tid; e < ns; e += kBlock) {
        rk[e].D = INFINITY;
        rk[e].id = 0xFFFFFFFFu;
    }
    __syncthreads();
    for (int size = 2; size <= ns; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < ns / 2; i += kBlock) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const RankF a = rk[lo], b = rk[hi];
                const bool less = b.D < a.D || (b.D == a.D && b.id < a.id);
                if (less == asc) {
                    rk[lo] = b;
                    rk[hi] = a;
                }
            }
            __syncthreads();
        }
    for (int r = tid; r < A.K; r += kBlock) {
        const int64_t o = q * A.K + r;
        if (r < n) {
            A.out_ids[o] = (int32_t)rk[r].id;
            reinterpret_cast<float *>(A.out_dist)[o] = (float)rk[r].D;
        } else {
            A.out_ids[o] = -1;
            reinterpret_cast<float *>(A.out_dist)[o] = INFINITY;
        }
    }
}

// The key list holds LC entries; the FP64 re-rank of float data needs LC/2
// (a band wider than that goes to the fallback).
size_t select_lds_bytes(int LC, int dtype)
{
    return size_t(LC) * 8 + (dtype == QW_F32 ? size_t(LC / 2) * sizeof(RankF) : 0);
}

qw_status launch_select(const SelectArgs &a, int64_t Q, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    const size_t lds = select_lds_bytes(a.LC, a.dtype);
    if (a.dtype == QW_U8)
        select_kernel<QW_U8><<<(unsigned)Q, kBlock, lds, s>>>(a);
    else
        select_kernel<QW_F32><<<(unsigned)Q, kBlock, lds, s>>>(a);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
