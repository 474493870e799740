// Workload scheduling kernels: hash-set size classes, bucket grouping keys,
// class segments and statistics.
//
// Queries of a workload whose candidate sets overlap are processed back to
// back: the sort key is a min-hash of the candidate set (the minimum over the
// query's buckets of each bucket's minimum id_mix(id), kept in the probe
// table), equal for two queries with probability equal to the Jaccard
// similarity of their sets.  The shared ids and points are then fetched from
// HBM once and served from L2 / the Infinity Cache -- the GPU counterpart of
// keeping reused index files and data objects in the cache (Sections 4 and
// 5.1).
#include "qw_internal.h"
#include "qw_mlp.h"

namespace qw {

__device__ inline uint32_t mix32(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xFF51AFD7ED558CCDull;
    x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

// Size class of a query from its predicted number of unique candidates
// `need`: the smallest c >= cmin with 3/4 * 2^c >= need (hash-set load factor
// <= 3/4).  Classes 0 .. ncls-2 are LDS classes (c = cmin + class), class
// ncls-1 keeps its set in global memory.
// has_pred: pred = the model's log(1 + |C(q)|) prediction.
__device__ inline int class_of(uint64_t tsum, int64_t n, const int32_t *__restrict__ exact, int64_t q,
                               bool has_pred, float pred, float margin, int32_t force_max,
                               int32_t cmin, int32_t cfloor, int32_t cmax, int32_t ncls)
{
    // |C(q)| <= min(sum of the bucket sizes, n): the class of that bound
    // always holds the set; a predicted or exact count may pick a smaller
    // one, but never one below cfloor (no occupancy gained there)
    const uint64_t bound = min(tsum, (uint64_t)n);
    uint64_t need = bound;
    if (exact) {
        need = min(need, (uint64_t)exact[q]);
    } else if (has_pred) {
        const float p = expm1f(pred + margin) + 32.f;
        if (p == p && p < (float)need) need = p > 0.f ? (uint64_t)ceilf(p) : 0;
    }
    int cb = cmin;
    while (cb < 40 && (3ull << cb) < 4 * bound) ++cb;
    int c = cmin;
    while (c < 40 && (3ull << c) < 4 * need) ++c;
    c = max(c, min(cb, cfloor));
    if (force_max && c <= cmax) c = cmax;
    return c <= cmax ? c - cmin : ncls - 1;
}

// Key = class << 16 | 16-bit group of every query, for the radix sort.
__global__ __launch_bounds__(kBlock) void classify_kernel(
    int64_t Q, int32_t L, int64_t n,
    const uint32_t *__restrict__ bmh, const uint32_t *__restrict__ bsize,
    const int32_t *__restrict__ exact, const float *__restrict__ pred_log, float margin,
    int32_t force_max, int32_t cmin, int32_t cfloor, int32_t cmax, int32_t ncls, int32_t group,
    unsigned long long *__restrict__ keys, int32_t *__restrict__ vals,
    unsigned long long *class_count)
{
    __shared__ uint32_t hist[32];
    if (threadIdx.x < 32) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < Q;
         q += (int64_t)gridDim.x * blockDim.x) {
        uint64_t tsum = 0;
        for (int32_t l = 0; l < L; ++l) tsum += bsize[q * L + l];
        const int cls = class_of(tsum, n, exact, q, pred_log != nullptr,
                                 pred_log ? pred_log[q] : 0.f, margin, force_max, cmin, cfloor,
                                 cmax, ncls);
        uint32_t g = 0;
        if (group) {  // min-hash of C(q): misses carry 0xFFFFFFFF
            uint32_t m = 0xFFFFFFFFu;
            for (int32_t l = 0; l < L; ++l) m = min(m, bmh[q * L + l]);
            g = mix32(m) & 0xFFFFu;
        }
        keys[q] = ((unsigned long long)cls << 16) | g;
        vals[q] = (int32_t)q;
        atomicAdd(&hist[cls], 1u);
    }
    __syncthreads();
    if (threadIdx.x < ncls && hist[threadIdx.x])
        atomicAdd(&class_count[threadIdx.x], (unsigned long long)hist[threadIdx.x]);
}

// Without bucket grouping the order within a class is free, so one kernel
// bins the queries: class c's queries go to order[c * Q ..) (any order), a
// workgroup taking one range per class per round of kBlock queries with one
// atomic on the class count.  The last workgroup to finish (its done-counter
// increment sees every other one) writes seg[2c], seg[2c+1] = [c * Q,
// c * Q + count_c).
// mlp_lane (nullable): the count model.  A prediction can only move a query
// whose bound class lies above cfloor (below it the class is the bound's), so
// only those queries are gathered into LDS and run through the MFMA
// inference, 16 at a time.
__global__ __launch_bounds__(kBlock) void classify_bin_kernel(
    int64_t Q, int32_t L, int64_t n, const uint32_t *__restrict__ bsize,
    const int32_t *__restrict__ exact, const uint32_t *__restrict__ mlp_lane, float margin,
    int32_t force_max, int32_t cmin, int32_t cfloor, int32_t cmax, int32_t ncls,
    int32_t *__restrict__ order, unsigned long long *class_count, uint32_t *done,
    unsigned long long *__restrict__ seg)
{
    extern __shared__ __align__(16) uint16_t fsh[];  // mlp: features [kBlock][ld] (bf16)
    __shared__ float pred_sh[kBlock];
    __shared__ uint32_t hist[32];
    __shared__ unsigned long long base[32];
    __shared__ uint32_t last, nmodel;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ksteps = (L + 15) / 16, kp = 16 * ksteps, ld = kp + 4;
    MlpLane m;
    if (mlp_lane) mlp_lane_load_packed(mlp_lane, m);  // in flight with the first sizes
    for (int64_t q0 = (int64_t)blockIdx.x * kBlock; q0 < Q; q0 += (int64_t)gridDim.x * kBlock) {
        const int64_t q = q0 + tid;
        if (tid < 32) hist[tid] = 0;
        if (tid == 0) nmodel = 0;
        // the query's bucket sizes, all loads in flight together (L <= 64)
        uint32_t sz[kMaxL];
#pragma unroll
        for (int32_t l = 0; l < kMaxL; ++l) sz[l] = q < Q && l < L ? bsize[q * L + l] : 0u;
        uint64_t tsum = 0;
#pragma unroll
        for (int32_t l = 0; l < kMaxL; ++l) tsum += sz[l];
        __syncthreads();  // hist and nmodel cleared
        // a slot in the model's list when the bound class exceeds cfloor
        const uint64_t bound = min(tsum, (uint64_t)n);
        const bool use = mlp_lane && q < Q && !exact && (3ull << cfloor) < 4 * bound;
        int slot = -1;
        if (use) {
            slot = (int)atomicAdd(&nmodel, 1u);
            // f_l = log(1 + s_l) by the hardware logarithm (1 + s_l is exact
            // for s_l < 2^24; the feature is rounded to bfloat16 anyway)
#pragma unroll
            for (int32_t l = 0; l < kMaxL; ++l) {
                if (l < L) fsh[slot * ld + l] = bf16_bits(__logf(1.0f + (float)sz[l]));
                else if (l < kp) fsh[slot * ld + l] = 0;
            }
        }
        __syncthreads();
        const int nm = (int)nmodel;
        for (int r0 = wave * 16; r0 < nm; r0 += kBlock / 4) {  // 16 rows per wave step
            // rows past nm hold stale features; their predictions are unused
            const mlp_f4 y = mlp_predict16(fsh + r0 * ld, ld, ksteps, m);
            if ((lane & 15) == 0)
#pragma unroll
                for (int j = 0; j < 4; ++j) pred_sh[r0 + (lane >> 4) * 4 + j] = y[j];
        }
        __syncthreads();  // predictions written
        int cls = 0;
        uint32_t p = 0;
        if (q < Q) {
            cls = class_of(tsum, n, exact, q, use, use ? pred_sh[slot] : 0.f, margin, force_max,
                           cmin, cfloor, cmax, ncls);
            p = atomicAdd(&hist[cls], 1u);
        }
        __syncthreads();
        if (tid < ncls && hist[tid])
            base[tid] = atomicAdd(&class_count[tid], (unsigned long long)hist[tid]);
        __syncthreads();
        if (q < Q) order[(int64_t)cls * Q + (int64_t)(base[cls] + p)] = (int32_t)q;
        __syncthreads();  // hist is cleared for the next round
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(done, 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (last && tid < ncls) {
        __threadfence();
        const unsigned long long cnt = atomicAdd(&class_count[tid], 0ull);  // device-coherent read
        seg[2 * tid] = (unsigned long long)tid * (unsigned long long)Q;
        seg[2 * tid + 1] = (unsigned long long)tid * (unsigned long long)Q + cnt;
    }
}

qw_status launch_classify_bin(int64_t Q, int32_t L, int64_t n, const uint32_t *bsize,
                              const int32_t *exact, const uint32_t *mlp_lane, float margin,
                              int32_t force_max, int32_t cmin, int32_t cfloor, int32_t cmax,
                              int32_t ncls, int32_t *order, unsigned long long *class_count,
                              uint32_t *done, unsigned long long *seg, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    if (ncls > 32 || L > kMaxL) return QW_EINVAL;
    const int g = (int)std::min<int64_t>(1024, ceil_div(Q, kBlock));
    // features of up to kBlock rows (a wave's steps start at multiples of 16)
    const size_t lds = mlp_lane ? sizeof(uint16_t) * (size_t)kBlock * (16 * ((L + 15) / 16) + 4) : 0;
    classify_bin_kernel<<<g, kBlock, lds, s>>>(Q, L, n, bsize, exact, mlp_lane, margin, force_max,
                                               cmin, cfloor, cmax, ncls, order, class_count, done,
                                               seg);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

qw_status launch_classify(int64_t Q, int32_t L, int64_t n,
                          const uint32_t *bmh, const uint32_t *bsize, const int32_t *exact,
                          const float *pred_log, float margin, int32_t force_max, int32_t cmin,
                          int32_t cfloor, int32_t cmax, int32_t ncls, int32_t group,
                          unsigned long long *keys, int32_t *vals,
                          unsigned long long *class_count, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    int g = (int)std::min<int64_t>(1024, ceil_div(Q, kBlock));
    classify_kernel<<<g, kBlock, 0, s>>>(Q, L, n, bmh, bsize, exact, pred_log, margin,
                                         force_max, cmin, cfloor, cmax, ncls, group, keys, vals,
                                         class_count);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// seg[2c], seg[2c+1] = [begin, end) of class c in the class-sorted order.
__global__ void segments_kernel(const unsigned long long *class_count, int32_t ncls,
                                unsigned long long *seg)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long off = 0;
    for (int c = 0; c < ncls; ++c) {
        seg[2 * c] = off;
        off += class_count[c];
        seg[2 * c + 1] = off;
    }
}

qw_status launch_segments(const unsigned long long *class_count, int32_t ncls,
                          unsigned long long *seg, hipStream_t s)
{
    segments_kernel<<<1, 64, 0, s>>>(class_count, ncls, seg);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

__global__ void max_u32_kernel(const uint32_t *__restrict__ v, int64_t count, uint32_t *out)
{
    uint32_t m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, v[i]);
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

qw_status launch_max_u32(const uint32_t *v, int64_t count, uint32_t *out, hipStream_t s)
{
    if (count <= 0) return QW_OK;
    int g = (int)std::min<int64_t>(1024, ceil_div(count, kBlock));
    max_u32_kernel<<<g, kBlock, 0, s>>>(v, count, out);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// max over queries of sum_l s_{q,l} (clamped to 2^32 - 1), one atomic per wave
__global__ __launch_bounds__(kBlock) void max_bucket_sum_kernel(const uint32_t *__restrict__ bsize,
                                                                int64_t Q, int32_t L, uint32_t *out)
{
    uint32_t m = 0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < Q;
         q += (int64_t)gridDim.x * blockDim.x) {
        uint64_t t = 0;
        for (int32_t l = 0; l < L; ++l) t += bsize[q * L + l];
        m = max(m, (uint32_t)min(t, (uint64_t)0xFFFFFFFFu));
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0 && m) atomicMax(out, m);
}

qw_status launch_max_bucket_sum(const uint32_t *bsize, int64_t Q, int32_t L, uint32_t *out,
                                hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    const int g = (int)std::min<int64_t>(64, ceil_div(Q, kBlock));
    max_bucket_sum_kernel<<<g, kBlock, 0, s>>>(bsize, Q, L, out);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// probes that hit a bucket, and the total of the bucket sizes
// Count of non-zero entries and their sum (one atomic pair per workgroup).
__global__ __launch_bounds__(kBlock) void probe_stats_kernel(const uint32_t *__restrict__ v,
                                                             int64_t count,
                                                             unsigned long long *nonzero,
                                                             unsigned long long *total)
{
    __shared__ unsigned long long sh[kBlock / 64], st[kBlock / 64];
    unsigned long long h = 0, t = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = v[i];
        h += x ? 1 : 0;
        t += x;
    }
    for (int off = 32; off > 0; off >>= 1) {
        h += __shfl_xor(h, off);
        t += __shfl_xor(t, off);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = h;
        st[threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            h += sh[w];
            t += st[w];
        }
        atomicAdd(nonzero, h);
        atomicAdd(total, t);
    }
}

qw_status launch_probe_stats(const uint32_t *v, int64_t count, unsigned long long *nonzero,
                             unsigned long long *total, hipStream_t s)
{
    if (count <= 0) return QW_OK;
    int g = (int)std::min<int64_t>(64, ceil_div(count, kBlock));
    probe_stats_kernel<<<g, kBlock, 0, s>>>(v, count, nonzero, total);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// Training minibatch gather and labels.
__global__ void gather_batch_kernel(const float *__restrict__ feats, const float *__restrict__ labels,
                                    const int32_t *__restrict__ perm, int32_t L, int32_t B,
                                    float *__restrict__ fb, float *__restrict__ tb)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B * L; i += gridDim.x * blockDim.x) {
        const int s = i / L, l = i - s * L;
        fb[i] = feats[(int64_t)perm[s] * L + l];
        if (l == 0) tb[s] = labels[perm[s]];
    }
}

qw_status launch_gather_batch(const float *feats, const float *labels, const int32_t *perm,
                              int32_t L, int32_t B, float *fb, float *tb, hipStream_t s)
{
    if (B <= 0) return QW_OK;
    gather_batch_kernel<<<(unsigned)ceil_div((int64_t)B * L, kBlock), kBlock, 0, s>>>(
        feats, labels, perm, L, B, fb, tb);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

__global__ void labels_kernel(const int32_t *__restrict__ counts, int64_t m, float *__restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = log1pf((float)counts[i]);
}

qw_status launch_labels(const int32_t *counts, int64_t m, float *out, hipStream_t s)
{
    if (m <= 0) return QW_OK;
    int g = (int)std::min<int64_t>(4096, ceil_div(m, kBlock));
    labels_kernel<<<g, kBlock, 0, s>>>(counts, m, out);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
