// Flat query pipeline of the fast form: dedup -> chunks -> streaming verify ->
// merge.
//
// 1. dedup_kernel: one workgroup per query builds C(q) (the union of the
//    query's buckets, Sections 1.2 and 5.1) in an LDS hash set sized by the
//    predicted count and appends the unique ids to a device-wide list through a
//    bump allocator.  Queries whose set overflows move to the next size class.
// 2. chunk kernels: each query's list is cut into chunks of at most C
//    candidates, emitted in the scheduled (bucket-grouped) query order.
// 3. verify_flat_kernel: persistent workgroups stream the chunks -- gather the
//    rows, exact distances (the false-positive removal of Section 1.2), sort
//    the chunk's keys and keep its K best (plus, for float data, every entry
//    within the proven FP32 error band of the K-th).  Chunks are split into
//    eight contiguous ranges, one per XCD (workgroup b runs on XCD b % 8), so
//    consecutive chunks of a bucket group share that XCD's L2; an XCD that
//    drains its range takes work from the next.
// 4. merge_kernel: per query, the chunk results are combined into the top-K by
//    (distance, id) (the c-k-ANN output, Section 3); float data is re-ranked
//    by the FP64 index-order distance inside the band.
// Queries that do not fit (list space, band or merge capacity) are flagged and
// answered by the fused per-query kernel afterwards.
#include "qw_dedup.h"
#include "qw_internal.h"

namespace qw {

enum { D_ITEM = 0, D_UCOUNT, D_OVF, D_CPOS, D_T, D_CAP, D_NSCAL = 8 };

__host__ __device__ inline size_t a16(size_t v) { return (v + 15) & ~size_t(15); }

size_t dedup_lds_bytes(int cap_log2, int global_tab, int L)
{
    return (global_tab ? 0 : (size_t(4) << cap_log2)) + a16(size_t(L + 1) * 4) +
           a16(size_t(L) * 4) + D_NSCAL * 4;
}

__global__ __launch_bounds__(kBlock) void dedup_kernel(DedupArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
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
                  glob ? 0xFFFFFFFFu : kShortProbe, &scal[D_UCOUNT], &scal[D_OVF],
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
        if (tid == 0) {
            unsigned long long off = atomicAdd(A.alloc, (unsigned long long)U);
            if (off + U > A.cand_cap) {  // no list space: answered by the fallback
                A.flag[q] = 1;
                A.ucount[q] = 0;
                off = ~0ull;
            } else {
                A.ucount[q] = U;
                A.coff[q] = off;
                if (A.unique_total) atomicAdd(A.unique_total, (unsigned long long)U);
            }
            scal[D_T] = (uint32_t)(off == ~0ull ? 0xFFFFFFFFu : 0u);
            reinterpret_cast<unsigned long long *>(lstart)[0] = off;  // broadcast
        }
        __syncthreads();
        if (scal[D_T] == 0u) {
            const unsigned long long off = reinterpret_cast<unsigned long long *>(lstart)[0];
            for (uint32_t i = tid; i < U; i += kBlock) A.cand[off + i] = (int32_t)tab[i];
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

// ---------------------------------------------------------------- chunks

__global__ void nchunks_kernel(const int32_t *__restrict__ order, int64_t Q,
                               const uint32_t *__restrict__ ucount, uint32_t C,
                               uint32_t *__restrict__ nch_item)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Q;
         i += (int64_t)gridDim.x * blockDim.x)
        nch_item[i] = (ucount[order[i]] + C - 1) / C;
}

__global__ void emit_chunks_kernel(const int32_t *__restrict__ order, int64_t Q,
                                   const uint32_t *__restrict__ nch_item,
                                   const unsigned long long *__restrict__ chunk_off, uint32_t C,
                                   unsigned long long *__restrict__ desc,
                                   uint32_t *__restrict__ qcbeg, uint32_t *__restrict__ qnch)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Q;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t q = (uint32_t)order[i];
        const unsigned long long c0 = chunk_off[i];
        const uint32_t nc = nch_item[i];
        qcbeg[q] = (uint32_t)c0;
        qnch[q] = nc;
        for (uint32_t t = 0; t < nc; ++t)
            desc[c0 + t] = ((unsigned long long)q << 32) | (unsigned long long)(t * C);
    }
}

qw_status launch_chunks(const int32_t *order, int64_t Q, const uint32_t *ucount, uint32_t C,
                        uint32_t *nch_item, unsigned long long *chunk_off, DevBuf &scan,
                        unsigned long long *desc, uint32_t *qcbeg, uint32_t *qnch, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    const int g = (int)std::min<int64_t>(4096, ceil_div(Q, kBlock));
    nchunks_kernel<<<g, kBlock, 0, s>>>(order, Q, ucount, C, nch_item);
    QW_HIP(hipGetLastError());
    QW_TRY(launch_scan_u32_to_u64(nch_item, Q, chunk_off, scan, s));
    emit_chunks_kernel<<<g, kBlock, 0, s>>>(order, Q, nch_item, chunk_off, C, desc, qcbeg, qnch);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// ---------------------------------------------------------------- streaming verify

// Bitonic sort of keys[0..n) (n <= cap, cap a power of two) ascending; the
// tail up to the next power of two is padded with ~0.  Whole workgroup.
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

// Relative bound of the FP32 distance (see the verify kernel) and the band
// threshold F_K * (1 + eps) / (1 - eps), rounded up to float.
__device__ inline float band_threshold(float FK, float eps)
{
    const double t = (double)FK * (1.0 + (double)eps) / (1.0 - (double)eps) + 0x1p-100;
    float f = (float)t;
    if ((double)f < t) f = nextafterf(f, INFINITY);
    return f;
}

enum { F_CHUNK = 0, F_QQ, F_NC, F_NSCAL = 8 };

__device__ inline unsigned long long wave_min_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ inline void cswap(unsigned long long &a, unsigned long long &b)
{
    const unsigned long long lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// The R smallest of the 4*64 keys held four per lane, ascending, into out[0..R)
// (lane 0 writes).  Keys are distinct apart from ~0 padding.  One wave.
__device__ inline void wave_extract(unsigned long long e0, unsigned long long e1,
                                    unsigned long long e2, unsigned long long e3, int R,
                                    unsigned long long *out)
{
    cswap(e0, e1);
    cswap(e2, e3);
    cswap(e0, e2);
    cswap(e1, e3);
    cswap(e1, e2);
    int h = 0;
    for (int r = 0; r < R; ++r) {
        const unsigned long long v = h == 0 ? e0 : h == 1 ? e1 : h == 2 ? e2 : h == 3 ? e3 : ~0ull;
        const unsigned long long m = wave_min_u64(v);
        if (v == m && m != ~0ull) ++h;
        if ((threadIdx.x & 63) == 0) out[r] = m;
    }
}

template <int DT, int UN, int PM>
__global__ __launch_bounds__(kBlock) void verify_flat_kernel(FlatArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(smem);
    unsigned char *qrow = smem + size_t(A.C) * 8;
    const int elem = DT == QW_U8 ? 1 : 4;
    const int row_bytes = A.dp * elem;
    uint32_t *scal = reinterpret_cast<uint32_t *>(qrow + a16(row_bytes));
    unsigned long long *wout = reinterpret_cast<unsigned long long *>(
        reinterpret_cast<unsigned char *>(scal) + F_NSCAL * 4 + 16);  // [4][64]
    uint32_t *cids = reinterpret_cast<uint32_t *>(wout + 4 * 64);     // [C] chunk's ids
    const int parts = row_bytes / 16;
    int G = 1;
    while (G < parts && G < 64) G <<= 1;
    const int P = (parts + G - 1) / G;
    const int NG = kBlock / G;
    const int per_iter = NG * UN;
    const int grp = tid / G, j = tid % G;
    const float eps = (float)((4 * P + 16) * 0x1p-24 + (A.d + 2) * 0x1p-52);
    const unsigned long long N = *A.nchunks;
    const int xcd = blockIdx.x & 7;

    while (true) {
        if (tid == 0) {
            unsigned long long pick = ~0ull;
            for (int r = 0; r < 8 && pick == ~0ull; ++r) {
                const int x = (xcd + r) & 7;
                const unsigned long long b = N * x / 8, e = N * (x + 1) / 8;
                if (A.xcd_ctr[x] >= (uint32_t)(e - b)) continue;  // drained (read may be stale)
                const unsigned long long t = b + atomicAdd(&A.xcd_ctr[x], 1u);
                if (t < e) pick = t;
            }
            reinterpret_cast<unsigned long long *>(scal)[0] = pick;
        }
        __syncthreads();
        const unsigned long long chunk = reinterpret_cast<unsigned long long *>(scal)[0];
        if (chunk == ~0ull) break;
        const unsigned long long dsc = A.desc[chunk];
        const int64_t q = (int64_t)(dsc >> 32);
        const uint32_t cb = (uint32_t)dsc;
        const uint32_t U = A.ucount[q];
        const int nc = (int)min((uint32_t)A.C, U - cb);
        const int32_t *list = A.cand + A.coff[q] + cb;
        for (int i = tid; i < nc; i += kBlock) cids[i] = (uint32_t)list[i];
        {  // query row and candidate ids into LDS (+ |q|^2 for uint8)
            const uint4 *src = reinterpret_cast<const uint4 *>((const unsigned char *)A.queries +
                                                               q * (int64_t)row_bytes);
            uint4 *dst = reinterpret_cast<uint4 *>(qrow);
            uint32_t qq = 0;
            for (int i = tid; i < parts; i += kBlock) {
                const uint4 v = src[i];
                dst[i] = v;
                if (DT == QW_U8) {
                    qq = __builtin_amdgcn_udot4(v.x, v.x, qq, false);
                    qq = __builtin_amdgcn_udot4(v.y, v.y, qq, false);
                    qq = __builtin_amdgcn_udot4(v.z, v.z, qq, false);
                    qq = __builtin_amdgcn_udot4(v.w, v.w, qq, false);
                }
            }
            if (tid == 0) scal[2 + F_QQ] = 0;
            __syncthreads();
            if (DT == QW_U8 && qq) atomicAdd(&scal[2 + F_QQ], qq);
            __syncthreads();
        }
        const uint32_t qq = scal[2 + F_QQ];
        for (int c0 = 0; c0 < nc; c0 += per_iter) {
            uint32_t cid[UN];
            bool cv[UN];
            for (int u = 0; u < UN; ++u) {
                const int c = c0 + grp + NG * u;
                cv[u] = c < nc;
                cid[u] = cv[u] ? cids[c] : 0u;
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
                        if (cv[u] && p0 + pp < P && part < parts)
                            xv[u][pp] = reinterpret_cast<const uint4 *>(
                                (const unsigned char *)A.data + (int64_t)cid[u] * row_bytes)[part];
                        else
                            xv[u][pp] = make_uint4(0, 0, 0, 0);
                    }
                for (int pp = 0; pp < PM; ++pp) {
                    const int part = j + G * (p0 + pp);
                    if (p0 + pp >= P || part >= parts) continue;
                    const uint4 qv = reinterpret_cast<const uint4 *>(qrow)[part];
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
                            const float d0 = __uint_as_float(x.x) - __uint_as_float(qv.x);
                            const float d1 = __uint_as_float(x.y) - __uint_as_float(qv.y);
                            const float d2 = __uint_as_float(x.z) - __uint_as_float(qv.z);
                            const float d3 = __uint_as_float(x.w) - __uint_as_float(qv.w);
                            float sacc = accf[u];
                            sacc = fmaf(d0, d0, sacc);
                            sacc = fmaf(d1, d1, sacc);
                            sacc = fmaf(d2, d2, sacc);
                            sacc = fmaf(d3, d3, sacc);
                            accf[u] = sacc;
                        }
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
                for (int u = 0; u < UN; ++u) {
                    if (!cv[u]) continue;
                    const uint32_t hi = DT == QW_U8 ? accu[u] + qq : __float_as_uint(accf[u]);
                    keys[c0 + grp + NG * u] = ((unsigned long long)hi << 32) | cid[u];
                }
        }
        __syncthreads();
        if (A.PS < 64 && A.C == 4 * kBlock) {
            // wave-level selection: each wave extracts the PS+1 smallest of its
            // quarter, then wave 0 extracts the PS+1 smallest of the four lists
            const int wid = tid >> 6, lane = tid & 63, R = A.PS + 1;
            unsigned long long e[4];
            for (int i = 0; i < 4; ++i) {
                const int idx = wid * 256 + lane + 64 * i;
                e[i] = idx < nc ? keys[idx] : ~0ull;
            }
            wave_extract(e[0], e[1], e[2], e[3], R, wout + wid * 64);
            __syncthreads();
            if (wid == 0) {
                for (int i = 0; i < 4; ++i) e[i] = lane < R ? wout[i * 64 + lane] : ~0ull;
                wave_extract(e[0], e[1], e[2], e[3], R, keys);
            }
            __syncthreads();
        } else {
            sort_keys(keys, nc);
        }
        // chunk result: the K best, plus for float data the band around the K-th
        int cnt = nc < A.K ? nc : A.K;
        if (DT == QW_F32 && nc > A.K) {
            const float thr = band_threshold(__uint_as_float((uint32_t)(keys[A.K - 1] >> 32)), eps);
            while (cnt < nc && cnt < A.PS && __uint_as_float((uint32_t)(keys[cnt] >> 32)) <= thr)
                ++cnt;
            if (cnt == A.PS && cnt < nc && __uint_as_float((uint32_t)(keys[cnt] >> 32)) <= thr &&
                tid == 0)
                A.flag[q] = 1;  // band wider than the chunk result: fallback
        }
        for (int t = tid; t < cnt; t += kBlock) A.part[chunk * A.PS + t] = keys[t];
        if (tid == 0) A.pcount[chunk] = (uint32_t)cnt;
        __syncthreads();
    }
}

static bool flat_small(int dp, int dtype) { return dp * (dtype == QW_U8 ? 1 : 4) / 16 <= 64; }

size_t flat_lds_bytes(int C, int dp, int dtype)
{
    return size_t(C) * 8 + a16(size_t(dp) * (dtype == QW_U8 ? 1 : 4)) + F_NSCAL * 4 + 16 +
           4 * 64 * 8 + size_t(C) * 4;
}

static const void *flat_fn(int dp, int dtype)
{
    const bool small = flat_small(dp, dtype);
    if (dtype == QW_U8)
        return small ? (const void *)verify_flat_kernel<QW_U8, 4, 1>
                     : (const void *)verify_flat_kernel<QW_U8, 2, 4>;
    return small ? (const void *)verify_flat_kernel<QW_F32, 4, 1>
                 : (const void *)verify_flat_kernel<QW_F32, 2, 4>;
}

int flat_blocks_per_cu(int C, int dp, int dtype)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, flat_fn(dp, dtype), kBlock,
                                                     flat_lds_bytes(C, dp, dtype)) != hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb > 0 ? nb : 1;
}

qw_status launch_verify_flat(const FlatArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    const size_t lds = flat_lds_bytes(a.C, a.dp, a.dtype);
    const bool small = flat_small(a.dp, a.dtype);
    if (a.dtype == QW_U8) {
        if (small) verify_flat_kernel<QW_U8, 4, 1><<<grid, kBlock, lds, s>>>(a);
        else verify_flat_kernel<QW_U8, 2, 4><<<grid, kBlock, lds, s>>>(a);
    } else {
        if (small) verify_flat_kernel<QW_F32, 4, 1><<<grid, kBlock, lds, s>>>(a);
        else verify_flat_kernel<QW_F32, 2, 4><<<grid, kBlock, lds, s>>>(a);
    }
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// ---------------------------------------------------------------- merge

struct RankF {
    double D;
    uint32_t id, pad;
};

__device__ __noinline__ double exact_dist_f32_m(const float *__restrict__ x,
                                                const float *__restrict__ q, int32_t d)
{
    double acc = 0.0;
    for (int32_t i = 0; i < d; ++i) {
        const double t = __dsub_rn((double)x[i], (double)q[i]);
        acc = __dadd_rn(acc, __dmul_rn(t, t));
    }
    return acc;
}

// One workgroup per query: gather the chunk results, sort, keep K.
template <int DT>
__global__ __launch_bounds__(kBlock) void merge_kernel(MergeArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(smem);
    RankF *rk = reinterpret_cast<RankF *>(smem + size_t(A.MB) * 8);
    __shared__ uint32_t s_total, s_bad;
    const int64_t q = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_total = 0;
        s_bad = A.flag[q];
    }
    __syncthreads();
    const uint32_t nch = A.qnch[q], c0 = A.qcbeg[q];
    if (!s_bad) {
        // chunk results are appended at positions from an LDS counter (order is
        // irrelevant: everything is sorted afterwards)
        for (uint32_t t = tid; t < nch; t += kBlock) {
            const uint32_t cnt = A.pcount[c0 + t];
            const uint32_t pos = atomicAdd(&s_total, cnt);
            if (pos + cnt > (uint32_t)A.MB) {
                s_bad = 1;
                continue;
            }
            for (uint32_t e = 0; e < cnt; ++e) keys[pos + e] = A.part[(size_t)(c0 + t) * A.PS + e];
        }
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) {
            const uint32_t o = atomicAdd(A.fb_count, 1u);
            A.fb_list[o] = (int32_t)q;
        }
        return;
    }
    const int total = (int)s_total;
    sort_keys(keys, total);
    if (DT == QW_U8) {
        for (int r = tid; r < A.K; r += kBlock) {
            const int64_t o = q * A.K + r;
            if (r < total) {
                A.out_ids[o] = (int32_t)(uint32_t)keys[r];
                reinterpret_cast<int32_t *>(A.out_dist)[o] = (int32_t)(keys[r] >> 32);
            } else {
                A.out_ids[o] = -1;
                reinterpret_cast<int32_t *>(A.out_dist)[o] = INT32_MAX;
            }
        }
        return;
    }
    // float data: FP64 index-order distances for every entry within the band of
    // the K-th FP32 distance, then the exact (D, id) order
    int nb = total;
    if (total > A.K) {
        const float thr = band_threshold(__uint_as_float((uint32_t)(keys[A.K - 1] >> 32)), A.eps);
        nb = A.K;
        while (nb < total && __uint_as_float((uint32_t)(keys[nb] >> 32)) <= thr) ++nb;
    }
    const float *qrow = (const float *)A.queries + q * (int64_t)A.dp;
    for (int e = tid; e < nb; e += kBlock) {
        const uint32_t id = (uint32_t)keys[e];
        rk[e].D = exact_dist_f32_m((const float *)A.data + (int64_t)id * A.dp, qrow, A.d);
        rk[e].id = id;
    }
    int ns = 2;
    while (ns < nb) ns <<= 1;
    for (int e = nb + tid; e < ns; e += kBlock) {
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
        if (r < nb) {
            A.out_ids[o] = (int32_t)rk[r].id;
            reinterpret_cast<float *>(A.out_dist)[o] = (float)rk[r].D;
        } else {
            A.out_ids[o] = -1;
            reinterpret_cast<float *>(A.out_dist)[o] = INFINITY;
        }
    }
}

size_t merge_lds_bytes(int MB, int dtype)
{
    return size_t(MB) * 8 + (dtype == QW_F32 ? size_t(MB) * sizeof(RankF) : 0);
}

qw_status launch_merge(const MergeArgs &a, int64_t Q, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    const size_t lds = merge_lds_bytes(a.MB, a.dtype);
    if (a.dtype == QW_U8)
        merge_kernel<QW_U8><<<(unsigned)Q, kBlock, lds, s>>>(a);
    else
        merge_kernel<QW_F32><<<(unsigned)Q, kBlock, lds, s>>>(a);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
