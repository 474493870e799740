// Gather of the fast form: a pure streaming pass over all (query, candidate)
// pairs -- gather the row, compute the exact squared distance (the
// false-positive removal of Section 1.2), write one (distance, id) key per
// pair.
#include "qw_dist.h"
#include "qw_internal.h"

namespace qw {

// Every pair e: key[e] = (squared distance << 32) | id (float distances as
// FP32 bits: non-negative, so the bits order like the values).
//
// XCD x (workgroup b runs on XCD b % 8) streams the region of the pair list
// that the dedup workgroups of XCD x filled; each workgroup takes one
// contiguous chunk of it, in steps of PI pairs.
__device__ inline void gather_chunk(const GatherArgs &A, int PI, int64_t &cb, int64_t &ce)
{
    const int x = blockIdx.x % kXcd;
    const int64_t nwg = ((int64_t)gridDim.x - x + kXcd - 1) / kXcd;
    const int64_t r = blockIdx.x / kXcd;
    unsigned long long used = A.alloc[x];
    const unsigned long long f = A.fail[x];
    if (f && ~f < used) used = ~f;
    if (used > A.region) used = A.region;
    const int64_t rb = (int64_t)((unsigned long long)x * A.region);
    const int64_t steps = ((int64_t)used + PI - 1) / PI;
    cb = rb + (steps * r / nwg) * PI;
    ce = rb + (steps * (r + 1) / nwg) * PI;
    if (ce > rb + (int64_t)used) ce = rb + (int64_t)used;
}

// Rows of at most 64 16-byte parts: a group of G lanes (G >= parts, a power
// of two) holds one row, UN pairs per group per step.  The next step's
// (id, query) pairs are loaded right after the current rows and first used a
// step later; each lane keeps the query part of the last query it saw (the
// pairs of one query are contiguous), so most steps load rows only.  Loads
// other than cache misses are issued without branches (clamped addresses,
// masked results) so that the wait for the rows leaves the next pairs in
// flight.  No barriers.
template <int DT, int UN>
__global__ __launch_bounds__(kBlock) void gather_small_kernel(GatherArgs A)
{
    const int tid = threadIdx.x;
    const int row_bytes = A.dp * (DT == QW_U8 ? 1 : 4);
    const int parts = row_bytes / 16;
    int G = 1;
    while (G < parts) G <<= 1;
    const int NG = kBlock / G;
    const int PI = NG * UN;
    const int grp = tid / G, j = tid % G;
    const int jc = j < parts ? j : parts - 1;
    const bool jin = j < parts;
    int64_t cb, ce;
    gather_chunk(A, PI, cb, ce);
    if (cb >= ce) return;
    const uint4 *qrows = reinterpret_cast<const uint4 *>(A.queries);
    const uint4 *drows = reinterpret_cast<const uint4 *>(A.data);
    uint32_t cached = 0xFFFFFFFFu;
    uint4 qc = make_uint4(0, 0, 0, 0);
    uint32_t nid[UN], nq[UN], nvalid = 0;
    auto load_pairs = [&](int64_t base) {  // uniform base < ce
        const int32_t *pc = A.cand + base, *pq = A.candq + base;
        const uint32_t lim = (uint32_t)min((int64_t)PI, ce - base);
        nvalid = 0;
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const uint32_t o = (uint32_t)(grp + NG * u);
            const uint32_t oc = o < lim ? o : lim - 1;
            nid[u] = (uint32_t)pc[oc];
            nq[u] = (uint32_t)pq[oc];
            nvalid |= (o < lim ? 1u : 0u) << u;
        }
    };
    load_pairs(cb);
    for (int64_t base = cb; base < ce; base += PI) {
        uint32_t cid[UN], cq[UN];
        bool val[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            val[u] = (nvalid >> u) & 1u;
            cid[u] = val[u] ? nid[u] : 0u;
            cq[u] = val[u] ? nq[u] : 0u;
        }
        // query parts that miss the cache (oldest loads), rows, next pairs
        uint4 qv[UN], xv[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            qv[u] = qc;
            if (cq[u] != cached)
                qv[u] = qrows[(int64_t)cq[u] * parts + jc];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) xv[u] = drows[(int64_t)cid[u] * parts + jc];
        load_pairs(base + PI < ce ? base + PI : base);
        __builtin_amdgcn_sched_barrier(0);  // keep every load above ahead of the waits below
        uint32_t accu[UN];
        float accf[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            accu[u] = 0;
            accf[u] = 0.f;
            // computed on whatever was loaded, masked afterwards: a masked
            // operand would let the compiler turn the row load conditional
            const bool in = val[u] && jin;
            part_dist<DT>(xv[u], qv[u], accu[u], accf[u]);
            accu[u] = in ? accu[u] : 0u;
            accf[u] = in ? accf[u] : 0.f;
            const bool upd = val[u] && cq[u] != cached;
            cached = upd ? cq[u] : cached;
            qc.x = upd ? qv[u].x : qc.x;
            qc.y = upd ? qv[u].y : qc.y;
            qc.z = upd ? qv[u].z : qc.z;
            qc.w = upd ? qv[u].w : qc.w;
        }
#pragma unroll
        for (int u = 0; u < UN; ++u)
            for (int off = G >> 1; off > 0; off >>= 1) {
                if (DT == QW_U8)
                    accu[u] += (uint32_t)__shfl_xor((int)accu[u], off);
                else
                    accf[u] += __shfl_xor(accf[u], off);
            }
        unsigned long long *pk = A.keys + base;
        if (j == 0)
#pragma unroll
            for (int u = 0; u < UN; ++u)
                if (val[u]) {
                    const uint32_t hi = DT == QW_U8 ? accu[u] : __float_as_uint(accf[u]);
                    pk[(uint32_t)(grp + NG * u)] = ((unsigned long long)hi << 32) | cid[u];
                }
    }
}

// Wide rows (more than 64 parts): the whole workgroup's groups of 64 lanes,
// P parts per lane, PM at a time.
template <int DT, int UN, int PM>
__global__ __launch_bounds__(kBlock) void gather_kernel(GatherArgs A)
{
    const int tid = threadIdx.x;
    const int row_bytes = A.dp * (DT == QW_U8 ? 1 : 4);
    const int parts = row_bytes / 16;
    const int G = 64;
    const int P = (parts + G - 1) / G;
    const int NG = kBlock / G;
    const int PI = NG * UN;
    const int grp = tid / G, j = tid % G;
    int64_t cb, ce;
    gather_chunk(A, PI, cb, ce);
    for (int64_t base = cb; base < ce; base += PI) {
        uint32_t cid[UN], cq[UN];
        bool cv[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t e = base + grp + (int64_t)NG * u;
            cv[u] = e < ce;
            cid[u] = cv[u] ? (uint32_t)A.cand[e] : 0u;
            cq[u] = cv[u] ? (uint32_t)A.candq[e] : 0u;
        }
        uint32_t accu[UN];
        float accf[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            accu[u] = 0;
            accf[u] = 0.f;
        }
        for (int p0 = 0; p0 < P; p0 += PM) {
            uint4 xv[UN][PM], qv[UN][PM];
#pragma unroll
            for (int u = 0; u < UN; ++u)
#pragma unroll
                for (int pp = 0; pp < PM; ++pp) {
                    const int part = j + G * (p0 + pp);
                    if (cv[u] && part < parts) {
                        xv[u][pp] = reinterpret_cast<const uint4 *>(
                            (const unsigned char *)A.data + (int64_t)cid[u] * row_bytes)[part];
                        qv[u][pp] = reinterpret_cast<const uint4 *>(
                            (const unsigned char *)A.queries + (int64_t)cq[u] * row_bytes)[part];
                    } else {
                        xv[u][pp] = make_uint4(0, 0, 0, 0);
                        qv[u][pp] = make_uint4(0, 0, 0, 0);
                    }
                }
#pragma unroll
            for (int u = 0; u < UN; ++u)
#pragma unroll
                for (int pp = 0; pp < PM; ++pp) part_dist<DT>(xv[u][pp], qv[u][pp], accu[u], accf[u]);
        }
#pragma unroll
        for (int u = 0; u < UN; ++u)
            for (int off = G >> 1; off > 0; off >>= 1) {
                if (DT == QW_U8)
                    accu[u] += (uint32_t)__shfl_xor((int)accu[u], off);
                else
                    accf[u] += __shfl_xor(accf[u], off);
            }
        if (j == 0)
#pragma unroll
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
        return small ? (const void *)gather_small_kernel<QW_U8, 4> : (const void *)gather_kernel<QW_U8, 2, 4>;
    return small ? (const void *)gather_small_kernel<QW_F32, 4> : (const void *)gather_kernel<QW_F32, 2, 4>;
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
        if (small) gather_small_kernel<QW_U8, 4><<<grid, kBlock, 0, s>>>(a);
        else gather_kernel<QW_U8, 2, 4><<<grid, kBlock, 0, s>>>(a);
    } else {
        if (small) gather_small_kernel<QW_F32, 4><<<grid, kBlock, 0, s>>>(a);
        else gather_kernel<QW_F32, 2, 4><<<grid, kBlock, 0, s>>>(a);
    }
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
