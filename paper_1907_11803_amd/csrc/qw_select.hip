// Select of the fast form: one workgroup per query takes the K smallest keys
// of its contiguous pair range by (distance, id) (the c-k-ANN output,
// Section 3); for float data every key within the proven FP32 error band of
// the K-th is re-ranked by its FP64 index-order distance.  Queries that do not
// fit (list or band capacity) go to the fallback.
#include "qw_exact.h"
#include "qw_internal.h"
#include "qw_wave.h"

namespace qw {

// Band threshold F_K * (1 + eps) / (1 - eps), rounded up to float: every key
// of the exact top-K has an FP32 distance at most this (see the verify kernel).
__device__ inline float band_threshold(float FK, float eps)
{
    const double t = (double)FK * (1.0 + (double)eps) / (1.0 - (double)eps) + 0x1p-100;
    float f = (float)t;
    if ((double)f < t) f = nextafterf(f, INFINITY);
    return f;
}

constexpr int kSelRegs = 8;  // keys per thread held in registers

struct RankF {
    double D;
    uint32_t id, pad;
};

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
    __shared__ uint32_t s_cnt, s_nb;
    const int64_t q = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const unsigned long long lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    // the flag, the count and the range offset load together (uniform)
    const uint32_t bad = A.flag[q];
    const uint32_t U = A.ucount[q];
    const unsigned long long coff = A.coff[q];
    if (bad) {  // uniform
        if (tid == 0) A.fb_list[atomicAdd(A.fb_count, 1u)] = (int32_t)q;
        return;
    }
    const int K = A.K;
    const unsigned long long *keys = A.keys + (U ? coff : 0ull);
    // the first kSelRegs * kBlock keys stay in registers for steps 1 and 3
    unsigned long long kr[kSelRegs];
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r) {
        const uint32_t e = (uint32_t)(tid + r * kBlock);
        kr[r] = e < U ? keys[e] : ~0ull;
    }
    if (tid == 0) {
        s_cnt = 0;
        s_nb = 0;
        s_thr = ~0ull;
        s_kth = ~0ull;
    }
    __syncthreads();
    // ---- 1-2: bound on the K-th key
    if (U > (uint32_t)K) {
        const int V = (K + kBlock - 1) / kBlock;
        unsigned long long thr = ~0ull;
        if (K <= 64) {
            unsigned long long m = ~0ull;
#pragma unroll
            for (int r = 0; r < kSelRegs; ++r) m = kr[r] < m ? kr[r] : m;
            for (uint32_t e = (uint32_t)(tid + kSelRegs * kBlock); e < U; e += kBlock)
                m = keys[e] < m ? keys[e] : m;
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
            const int r = (int)(b0 / kBlock);
            unsigned long long k = ~0ull;
            if (r < kSelRegs) {
#pragma unroll
                for (int i = 0; i < kSelRegs; ++i) k = i == r ? kr[i] : k;
            } else if (e < U) {
                k = keys[e];
            }
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
    if (nb > 0) {  // uniform
        const float *qrow = (const float *)A.queries + q * (int64_t)A.dp;
        float *qs = reinterpret_cast<float *>(smem + size_t(A.LC) * 8 + size_t(A.LC / 2) * sizeof(RankF));
        double *stage = reinterpret_cast<double *>(qs + A.dp);  // dp is a multiple of 4
        for (int i = tid; i < A.dp; i += kBlock) qs[i] = qrow[i];
        __syncthreads();
        exact_dists_staged((const float *)A.data, A.dp, nb, qs, stage,
                           [&](int i) { return rk[i].id; }, [&](int i, double D) { rk[i].D = D; });
    }
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
// kBlock minima of K > 64); the FP64 re-rank of float data needs LC/2 entries
// (a band wider than that goes to the fallback), the query row and the row
// staging area.
size_t select_lds_bytes(int LC, int dtype, int dp)
{
    return size_t(LC) * 8 +
           (dtype == QW_F32 ? size_t(LC / 2) * sizeof(RankF) + size_t(dp) * 4 + kStageBytes : 0);
}

qw_status launch_select(const SelectArgs &a, int64_t Q, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    const size_t lds = select_lds_bytes(a.LC, a.dtype, a.dp);
    if (a.dtype == QW_U8)
        select_kernel<QW_U8><<<(unsigned)Q, kBlock, lds, s>>>(a);
    else
        select_kernel<QW_F32><<<(unsigned)Q, kBlock, lds, s>>>(a);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
