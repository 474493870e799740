// FP64 squared distance of float rows, the value the float top K is ranked by
// and reported from (the exact verification of Section 1.2, made reproducible):
// over i in index order, t = x_i - q_i formed in FP64, acc = acc + t * t with the
// product and the sum each rounded (no fused multiply-add; contraction is off
// in every function here).  Rows hold dp elements, zero-padded past d; the
// padding adds exact zeros and leaves the sum unchanged.
#pragma once

#include "qw_internal.h"

namespace qw {

__device__ inline double exact_step(double acc, float x, double q)
{
#pragma clang fp contract(off)
    const double t = (double)x - q;
    const double p = t * t;
    return acc + p;
}

// One row per thread: its 16-byte parts are loaded kExactAhead at a time, the
// next group while the current one is summed.  q: the query row (dp floats).
constexpr int kExactAhead = 8;

__device__ inline double exact_dist_row(const float *__restrict__ x, const float *q, int dp)
{
#pragma clang fp contract(off)
    const float4 *x4 = reinterpret_cast<const float4 *>(x);
    const int n4 = dp >> 2;
    float4 cur[kExactAhead];
#pragma unroll
    for (int i = 0; i < kExactAhead; ++i) cur[i] = x4[i < n4 ? i : n4 - 1];
    double acc = 0.0;
    for (int b = 0; b < n4; b += kExactAhead) {
        float4 nxt[kExactAhead];
#pragma unroll
        for (int i = 0; i < kExactAhead; ++i) {
            const int e = b + kExactAhead + i;
            nxt[i] = x4[e < n4 ? e : n4 - 1];
        }
#pragma unroll
        for (int i = 0; i < kExactAhead; ++i)
            if (b + i < n4) {
                const float *qq = q + 4 * (b + i);
                acc = exact_step(acc, cur[i].x, (double)qq[0]);
                acc = exact_step(acc, cur[i].y, (double)qq[1]);
                acc = exact_step(acc, cur[i].z, (double)qq[2]);
                acc = exact_step(acc, cur[i].w, (double)qq[3]);
            }
#pragma unroll
        for (int i = 0; i < kExactAhead; ++i) cur[i] = nxt[i];
    }
    return acc;
}

// Whole workgroup: the distances of nb rows at once.  Batches of kStageRows
// rows go through LDS in chunks of kStageCols elements: every thread loads
// 16-byte pieces of the rows (coalesced; kStageAhead chunks in flight), forms
// their rounded squares t * t in FP64 and stores them to LDS; the dependent
// sums then run on lanes 0-3 of the four waves (row r on wave r % 4), one add
// per element, so four SIMDs share the chains.
constexpr int kStageRows = 16;
constexpr int kStageCols = 64;
constexpr int kStageAhead = 6;
constexpr int kStageLd = kStageCols + 2;  // row stride (doubles): rows start four banks apart
constexpr size_t kStageBytes = size_t(kStageRows) * kStageLd * 8;

// id(i) -> row id, put(i, D) stores the distance of row i; qs: the query row
// (dp floats, LDS); stage: kStageBytes of LDS.  Ends with a barrier.
template <typename IdOf, typename Put>
__device__ inline void exact_dists_staged(const float *__restrict__ data, int dp, int nb,
                                          const float *qs, double *stage, IdOf id_of, Put put)
{
#pragma clang fp contract(off)
    static_assert(kStageRows <= 4 * 4 && kStageRows % 4 == 0, "rows on lanes 0-3 of 4 waves");
    constexpr int kPer = kStageRows * kStageCols / 4 / kBlock;  // pieces per thread per chunk
    static_assert(kPer * kBlock * 4 == kStageRows * kStageCols, "whole chunks per thread");
    constexpr int kC4 = kStageCols / 4;
    const int tid = threadIdx.x;
    const int my = (tid & 63) * 4 + (tid >> 6);  // chain of row `my` of the batch (lanes 0-3)
    const int nch = (dp + kStageCols - 1) / kStageCols;
    for (int b0 = 0; b0 < nb; b0 += kStageRows) {
        const int nr = nb - b0 < kStageRows ? nb - b0 : kStageRows;
        uint32_t rid[kPer];  // the row ids of this thread's pieces (clamped to the batch)
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int r = (tid + k * kBlock) / kC4;
            rid[k] = id_of(b0 + (r < nr ? r : nr - 1));
        }
        // ring of loaded chunks: ring[0] is the next chunk to store
        float4 ring[kStageAhead][kPer];
        auto load = [&](float4 (&dst)[kPer], int ch) {
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int col = ch * kStageCols + ((tid + k * kBlock) % kC4) * 4;
                const int cc = col < dp ? col : dp - 4;  // in bounds; masked when stored
                dst[k] = *reinterpret_cast<const float4 *>(data + (int64_t)rid[k] * dp + cc);
            }
        };
#pragma unroll
        for (int a = 0; a < kStageAhead; ++a) load(ring[a], a < nch ? a : nch - 1);
        double acc = 0.0;
        for (int ch = 0; ch < nch; ++ch) {
            __syncthreads();  // the previous chunk's chains are done with the stage
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int f = tid + k * kBlock;
                const int r = f / kC4, col = ch * kStageCols + (f % kC4) * 4;
                const bool ok = r < nr && col < dp;
                const float4 v = ring[0][k];
                const float4 u = *reinterpret_cast<const float4 *>(qs + (col < dp ? col : dp - 4));
                double t0 = (double)v.x - (double)u.x, t1 = (double)v.y - (double)u.y;
                double t2 = (double)v.z - (double)u.z, t3 = (double)v.w - (double)u.w;
                double *dst = stage + r * kStageLd + (f % kC4) * 4;
                reinterpret_cast<double2 *>(dst)[0] = double2{ok ? t0 * t0 : 0.0, ok ? t1 * t1 : 0.0};
                reinterpret_cast<double2 *>(dst)[1] = double2{ok ? t2 * t2 : 0.0, ok ? t3 * t3 : 0.0};
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a + 1 < kStageAhead; ++a)
#pragma unroll
                for (int k = 0; k < kPer; ++k) ring[a][k] = ring[a + 1][k];
            {
                const int nx = ch + kStageAhead;
                load(ring[kStageAhead - 1], nx < nch ? nx : nch - 1);
            }
            if (my < nr) {
                // the whole chunk, 16 squares per batch of LDS reads: columns
                // past dp hold +0.0, which leaves the (non-negative) sum unchanged
                const double *srow = stage + my * kStageLd;
#pragma unroll
                for (int e0 = 0; e0 < kStageCols; e0 += 16) {
                    double2 p[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) p[i] = *reinterpret_cast<const double2 *>(srow + e0 + 2 * i);
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        acc = acc + p[i].x;
                        acc = acc + p[i].y;
                    }
                }
            }
        }
        if (my < nr) put(b0 + my, acc);
    }
    __syncthreads();
}

}  // namespace qw
