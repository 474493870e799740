// Flat query pipeline of the fast form: dedup -> gather -> select.
//
// 1. dedup_kernel: one workgroup per query builds C(q) (the union of the
//    query's buckets, Sections 1.2 and 5.1) in an LDS hash set sized by the
//    predicted count, and scatters the unique ids -- each tagged with its query
//    -- into a device-wide pair list through a bump allocator.  Queries whose
//    set overflows move to the next size class.
// 2. gather_kernel: a pure streaming pass over all (query, candidate) pairs:
//    gather the row, compute the exact squared distance (the false-positive
//    removal of Section 1.2), write one (distance, id) key per pair.  XCD x
//    (workgroup b runs on XCD b % 8) streams the region of the pair list that
//    the dedup workgroups of XCD x filled.  No barriers: every wave keeps loads
//    in flight all the time.
// 3. select_kernel: one workgroup per query selects the K smallest keys of its
//    contiguous pair range by (distance, id) (the c-k-ANN output, Section 3);
//    for float data every key within the proven FP32 error band of the K-th is
//    re-ranked by its FP64 index-order distance.
// Queries that do not fit (list space, band capacity) are flagged and answered
// by the fused per-query kernel afterwards.
#include "qw_dedup.h"
#include "qw_internal.h"

namespace qw {

enum {
    D_UCOUNT = 0, D_OVF, D_CPOS, D_T, D_CAP, D_OFF = 6 /* u64 */,
    D_WT = 8 /* per-wave counts, kBlock / 64 */, D_NSCAL = 16
};
constexpr int kRegIds = 16;  // ids per thread of the register-resident path

__host__ __device__ inline size_t a16(size_t v) { return (v + 15) & ~size_t(15); }

size_t dedup_lds_bytes(int cap_log2, int global_tab, int L)
{
    return (global_tab ? 0 : (size_t(4) << cap_log2)) + a16(size_t(L + 1) * 4) +
           a16(size_t(L) * 4) + D_NSCAL * 4;
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

// One workgroup per query (persistent: workgroup b takes items b, b + grid,
// ... -- no shared work counter, whose atomics would serialise every
// workgroup on one address).  Queries with at most kRegIds * kBlock
// bucket entries in an LDS set keep their ids in registers from the load to
// the write; larger ones (and the global-memory class, GLOB) go through the
// set and read the unique ids back from it.
template <bool GLOB>
__global__ __launch_bounds__(kBlock) void dedup_kernel(DedupArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    constexpr bool glob = GLOB;
    const size_t tab_bytes = glob ? 0 : (size_t(4) << A.cap_log2);
    uint32_t *lpref = reinterpret_cast<uint32_t *>(smem + tab_bytes);
    uint32_t *lstart = reinterpret_cast<uint32_t *>(smem + tab_bytes + a16(size_t(A.L + 1) * 4));
    uint32_t *scal = reinterpret_cast<uint32_t *>(smem + tab_bytes + a16(size_t(A.L + 1) * 4) +
                                                  a16(size_t(A.L) * 4));
    uint32_t *tab = GLOB ? A.gscratch + (size_t)blockIdx.x * (size_t(1) << A.cap_log2)
                         : reinterpret_cast<uint32_t *>(smem);
    unsigned long long *soff = reinterpret_cast<unsigned long long *>(&scal[D_OFF]);
    const int64_t sbeg = (int64_t)A.seg[0];
    const int64_t nseg = (int64_t)A.seg[1] - sbeg;
    const int64_t nin = A.in_count ? (int64_t)*A.in_count : 0;
    const int64_t nall = nseg + nin;
    const int xcd = blockIdx.x % kXcd;
    const unsigned long long rbase = (unsigned long long)xcd * A.region;

    for (int64_t item = blockIdx.x; item < nall; item += gridDim.x) {
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
        if (tid < 64) {
            const uint32_t run = wave_layer_prefix(lpref, A.L);
            if (tid == 0) {
                scal[D_T] = run;
                int c = (int)A.cap_log2;
                if (glob) {  // set sized from the exact bound min(sum_l s_{q,l}, n)
                    const uint64_t bound = min((uint64_t)run, (uint64_t)A.n);
                    c = 10;
                    while (c < (int)A.cap_log2 && (3ull << c) < 4 * bound) ++c;
                }
                scal[D_CAP] = (uint32_t)c;
            }
        }
        __syncthreads();
        const uint32_t T = scal[D_T];
        const int cap_log2 = (int)scal[D_CAP];
        const uint32_t cap = 1u << cap_log2;
        const uint32_t set_limit = (cap >> 2) * 3;
        const uint32_t limit = glob ? set_limit : (A.limit < set_limit ? A.limit : set_limit);
        const uint32_t max_probe = glob ? 0xFFFFFFFFu : kShortProbe;
        for (uint32_t i = tid; i < cap; i += kBlock) tab[i] = kEmpty;
        if (glob) __threadfence();
        __syncthreads();
        const bool in_regs = !glob && T <= (uint32_t)(kRegIds * kBlock);
        uint32_t idr[kRegIds];
        uint32_t newm = 0;
        uint32_t U = 0, wbase = 0;
        bool ovf = false;
        if (in_regs) {
            const uint32_t pend = load_ids<kRegIds>(A.ids, A.n, A.L, lpref, lstart, T, 0u, idr);
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
            __syncthreads();
            uint32_t tot = 0;
            wbase += wave_base(scal, wave, &tot);
            U = tot;
            ovf = scal[D_OVF] != 0 || U > limit;
        } else {
            set_union(A.ids, A.n, A.L, lpref, lstart, T, tab, cap_log2, limit, glob, max_probe,
                      false, &scal[D_UCOUNT], &scal[D_OVF], &scal[D_CPOS]);
            U = scal[D_UCOUNT];
            ovf = scal[D_OVF] != 0 || U > limit;
        }
        if (ovf) {
            if (tid == 0) {
                const uint32_t o = atomicAdd(A.ovf_count, 1u);
                A.ovf_list[o] = (int32_t)q;
            }
        } else if (A.count_only) {
            if (tid == 0) A.ucount[q] = U;
        } else {
            if (tid == 0) {
                unsigned long long off = atomicAdd(A.alloc + xcd, (unsigned long long)U);
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
                *soff = off;
            }
            __syncthreads();
            const unsigned long long off = *soff;
            if (off != ~0ull && in_regs) {
                unsigned long long e = off + wbase;
#pragma unroll
                for (int r = 0; r < kRegIds; ++r)
                    if ((newm >> r) & 1u) {
                        A.cand[e] = (int32_t)idr[r];
                        A.candq[e] = (int32_t)q;
                        ++e;
                    }
            } else if (off != ~0ull) {
                // read the set back: wave w takes slots [w * cap / 4, (w + 1) * cap / 4)
                const uint32_t seg = cap / (kBlock / 64);
                const uint32_t s0 = (uint32_t)wave * seg;
                uint32_t cnt = 0;
                for (uint32_t i = s0 + lane; i < s0 + seg; i += 64)
                    cnt += (uint32_t)__popcll(__ballot(tab[i] != kEmpty));
                if (lane == 0) scal[D_WT + wave] = cnt;
                __syncthreads();
                uint32_t tot = 0;
                unsigned long long e = off + wave_base(scal, wave, &tot);
                for (uint32_t i = s0 + lane; i < s0 + seg; i += 64) {
                    const uint32_t v = tab[i];
                    const unsigned long long m = __ballot(v != kEmpty);
                    if (v != kEmpty) {
                        const unsigned long long p = e + (uint32_t)__popcll(m & lt_mask);
                        A.cand[p] = (int32_t)v;
                        A.candq[p] = (int32_t)q;
                    }
                    e += (uint32_t)__popcll(m);
                }
            }
        }
        __syncthreads();  // scal is rewritten by the next item
    }
}

qw_status launch_dedup(const DedupArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    const size_t lds = dedup_lds_bytes((int)a.cap_log2, a.global_tab, a.L);
    if (a.global_tab) dedup_kernel<true><<<grid, kBlock, lds, s>>>(a);
    else dedup_kernel<false><<<grid, kBlock, lds, s>>>(a);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

int dedup_blocks_per_cu(size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)dedup_kernel<false>, kBlock, lds) !=
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
    // the XCD's own region of the pair list (filled by the dedup workgroups of
    // the same XCD)
    const int x = blockIdx.x % kXcd;
    const int64_t nwg = ((int64_t)gridDim.x - x + kXcd - 1) / kXcd;
    const int64_t r = blockIdx.x / kXcd;
    unsigned long long used = A.alloc[x];
    const unsigned long long f = A.fail[x];
    if (f && ~f < used) used = ~f;
    const int64_t rb = (int64_t)((unsigned long long)x * A.region);
    const int64_t re = rb + (int64_t)(used < A.region ? used : A.region);
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

// Ascending bitonic sort of one value per lane across a wave.
__device__ inline unsigned long long wave_sort_u64(unsigned long long v)
{
    const int lane = threadIdx.x & 63;
    for (int k = 2; k <= 64; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const unsigned long long o = __shfl_xor(v, j);
            const bool asc = (lane & k) == 0, lower = (lane & j) == 0;
            v = (lower == asc) ? (o < v ? o : v) : (o > v ? o : v);
        }
    return v;
}

// One workgroup per query, over its U keys (unique (distance, id) pairs):
// 1. every lane takes the minimum of its stride-kBlock stream of keys (K > 64:
//    V = ceil(K / kBlock) streams per thread);
// 2. a key t with at least K keys at or below it bounds the K-th key: the K-th
//    smallest minimum of any set of streams is one (K <= 64: per wave, from a
//    shuffle sort of its 64 minima, the smallest over the waves; else the K-th
//    of all minima by rank counting).  Float data widen the bound to the FP32
//    error band of its distance;
// 3. a second pass collects the keys at or below the bound into an LDS list
//    (typically a few K entries);
// 4. uint8: each list entry's rank is counted, ranks below K are the output.
//    float: the K-th key of the list fixes the band, every entry in the band is
//    re-ranked by its FP64 index-order distance (the c-k-ANN output, Section 3).
// A list or band beyond capacity sends the query to the fallback.
template <int DT>
__global__ __launch_bounds__(kBlock) void select_kernel(SelectArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *lst = reinterpret_cast<unsigned long long *>(smem);
    RankF *rk = reinterpret_cast<RankF *>(smem + size_t(A.LC) * 8);
    unsigned long long *s_min = lst;  // the minima (K > 64) are dead before the list fills
    __shared__ unsigned long long s_thr, s_kth;
    __shared__ uint32_t s_cnt, s_nb, s_bad;
    const int64_t q = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (tid == 0) {
        s_cnt = 0;
        s_nb = 0;
        s_thr = ~0ull;
        s_kth = ~0ull;
        s_bad = A.flag[q];
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) A.fb_list[atomicAdd(A.fb_count, 1u)] = (int32_t)q;
        return;
    }
    const uint32_t U = A.ucount[q];
    const int K = A.K;
    const unsigned long long *keys = A.keys + (U ? A.coff[q] : 0ull);
    // ---- 1-2: bound on the K-th key
    if (U > (uint32_t)K) {
        const int V = (K + kBlock - 1) / kBlock;
        unsigned long long thr = ~0ull;
        if (K <= 64) {
            unsigned long long m = ~0ull;
            uint32_t e = tid;
            for (; e + 3 * kBlock < U; e += 4 * kBlock) {
                const unsigned long long k0 = keys[e], k1 = keys[e + kBlock];
                const unsigned long long k2 = keys[e + 2 * kBlock], k3 = keys[e + 3 * kBlock];
                const unsigned long long a = k0 < k1 ? k0 : k1, b = k2 < k3 ? k2 : k3;
                const unsigned long long c = a < b ? a : b;
                m = c < m ? c : m;
            }
            for (; e < U; e += kBlock) m = keys[e] < m ? keys[e] : m;
            // the K-th smallest of this wave's minima; ~0 unless K streams are non-empty
            const unsigned long long t = __shfl(wave_sort_u64(m), K - 1);
            if (lane == 0 && t != ~0ull) atomicMin(&s_thr, t);
        } else {
            for (int v = 0; v < V; ++v) {
                unsigned long long m = ~0ull;
                for (uint32_t e = (uint32_t)(v * kBlock + tid); e < U; e += (uint32_t)(V * kBlock))
                    m = keys[e] < m ? keys[e] : m;
                s_min[v * kBlock + tid] = m;
            }
            __syncthreads();
            const int M = V * kBlock;
            for (int v = 0; v < V; ++v) {
                const unsigned long long m = s_min[v * kBlock + tid];
                if (m == ~0ull) continue;
                int rank = 0;
                for (int i = 0; i < M; ++i) rank += s_min[i] < m;
                if (rank == K - 1) s_thr = m;  // keys are unique: one writer
            }
        }
        __syncthreads();
        thr = s_thr;
        if (DT != QW_U8 && thr != ~0ull) {
            const float bt = band_threshold(__uint_as_float((uint32_t)(thr >> 32)), A.eps);
            thr = ((unsigned long long)__float_as_uint(bt) << 32) | 0xFFFFFFFFull;
        }
        __syncthreads();  // every thread has read s_thr
        if (tid == 0) s_thr = thr;
        __syncthreads();
    }
    // ---- 3: collect the keys at or below the bound
    {
        const unsigned long long thr = s_thr;
        for (uint32_t b0 = 0; b0 < U; b0 += kBlock) {
            const uint32_t e = b0 + tid;
            const unsigned long long k = e < U ? keys[e] : ~0ull;
            const bool take = e < U && k <= thr;
            const unsigned long long m = __ballot(take);
            uint32_t wb = 0;
            if (lane == 0 && m) wb = atomicAdd(&s_cnt, (uint32_t)__popcll(m));
            wb = (uint32_t)__shfl((int)wb, 0);
            const uint32_t pos = wb + (uint32_t)__popcll(m & lt_mask);
            if (take && pos < (uint32_t)A.LC) lst[pos] = k;
        }
    }
    __syncthreads();
    const int c = (int)s_cnt;
    if (c > A.LC) {  // list beyond capacity
        if (tid == 0) A.fb_list[atomicAdd(A.fb_count, 1u)] = (int32_t)q;
        return;
    }
    // ---- 4: ranks within the list (keys are unique)
    if (DT == QW_U8) {
        for (int i = tid; i < c; i += kBlock) {
            const unsigned long long k = lst[i];
            int r = 0;
            for (int j = 0; j < c; ++j) r += lst[j] < k;
            if (r < K) {
                const int64_t o = q * K + r;
                A.out_ids[o] = (int32_t)(uint32_t)k;
                reinterpret_cast<int32_t *>(A.out_dist)[o] = (int32_t)(k >> 32);
            }
        }
        for (int r = c + tid; r < K; r += kBlock) {
            const int64_t o = q * K + r;
            A.out_ids[o] = -1;
            reinterpret_cast<int32_t *>(A.out_dist)[o] = INT32_MAX;
        }
        return;
    }
    // float data: the list's K-th key fixes the band of the exact top K
    if (c >= K)
        for (int i = tid; i < c; i += kBlock) {
            const unsigned long long k = lst[i];
            int r = 0;
            for (int j = 0; j < c; ++j) r += lst[j] < k;
            if (r == K - 1) s_kth = k;
        }
    __syncthreads();
    unsigned long long bthr = ~0ull;
    if (c >= K) {
        const float bt = band_threshold(__uint_as_float((uint32_t)(s_kth >> 32)), A.eps);
        bthr = ((unsigned long long)__float_as_uint(bt) << 32) | 0xFFFFFFFFull;
    }
    const int cap_b = A.LC / 2;
    for (int b0 = 0; b0 < c; b0 += kBlock) {
        const int i = b0 + tid;
        const bool take = i < c && lst[i] <= bthr;
        const unsigned long long m = __ballot(take);
        uint32_t wb = 0;
        if (lane == 0 && m) wb = atomicAdd(&s_nb, (uint32_t)__popcll(m));
        wb = (uint32_t)__shfl((int)wb, 0);
        const uint32_t pos = wb + (uint32_t)__popcll(m & lt_mask);
        if (take && pos < (uint32_t)cap_b) rk[pos].id = (uint32_t)lst[i];
    }
    __syncthreads();
    const int nb = (int)s_nb;
    if (nb > cap_b) {  // band beyond capacity
        if (tid == 0) A.fb_list[atomicAdd(A.fb_count, 1u)] = (int32_t)q;
        return;
    }
    const float *qrow = (const float *)A.queries + q * (int64_t)A.dp;
    for (int i = tid; i < nb; i += kBlock)
        rk[i].D = exact_dist_f32_s((const float *)A.data + (int64_t)rk[i].id * A.dp, qrow, A.d);
    __syncthreads();
    for (int i = tid; i < nb; i += kBlock) {
        const double D = rk[i].D;
        const uint32_t id = rk[i].id;
        int r = 0;
        for (int j = 0; j < nb; ++j) r += rk[j].D < D || (rk[j].D == D && rk[j].id < id);
        if (r < K) {
            const int64_t o = q * K + r;
            A.out_ids[o] = (int32_t)id;
            reinterpret_cast<float *>(A.out_dist)[o] = (float)D;
        }
    }
    for (int r = nb + tid; r < K; r += kBlock) {
        const int64_t o = q * K + r;
        A.out_ids[o] = -1;
        reinterpret_cast<float *>(A.out_dist)[o] = INFINITY;
    }
}

// The key list holds LC >= 4K entries (also room for the ceil(K / kBlock) *
// kBlock minima of K > 64); the FP64 re-rank of float data needs LC/2 (a band
// wider than that goes to the fallback).
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
