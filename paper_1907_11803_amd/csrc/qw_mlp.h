// BF16 inference of the candidate-count model y = W2 relu(W1 f + b1) + b2
// (inputs, weights and hidden activations rounded to bfloat16, FP32 sums).
#pragma once

#include <cstring>

#include "qw_internal.h"

namespace qw {

constexpr int kMlpH = QW_MLP_HIDDEN;

// Round-to-nearest-even to bfloat16, returned as the float it represents
// (the same bit operations on the host and the device).
__host__ __device__ inline float bf16_round(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return x;  // inf / nan unchanged
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

__host__ __device__ inline uint16_t bf16_bits(float x)
{
    const float r = bf16_round(x);
    uint32_t u;
    std::memcpy(&u, &r, 4);
    return (uint16_t)(u >> 16);
}

// ---- MFMA inference: the hidden layer of 16 queries at a time is one
// [16 x L] x [L x 64] product (v_mfma_f32_16x16x16bf16_1k: bf16 operands,
// FP32 accumulation), then relu, bf16 rounding, the W2 dot product and b2.
typedef short mlp_s4 __attribute__((ext_vector_type(4)));
typedef float mlp_f4 __attribute__((ext_vector_type(4)));
constexpr int kMlpMaxKs = 4;  // K steps of 16 inputs: L <= 64

// Lane (c = lane % 16, g = lane / 16) holds W1[16 nt + c][16 ks + 4 g + e]
// (e < 4; zero past L) of the four 16-unit column tiles nt, and b1, W2 of its
// four hidden units 16 nt + c.
struct MlpLane {
    mlp_s4 w[4][kMlpMaxKs];
    float b1[4], w2[4], b2;
};

// Whole workgroup (every thread calls it; contains a barrier): the packed
// parameters are staged through LDS (sw: mlp_param_count floats, coalesced
// loads), then every lane takes its registers from there.
__host__ __device__ inline int mlp_param_floats(int L) { return kMlpH * L + 2 * kMlpH + 1; }

__device__ inline void mlp_lane_load(const float *__restrict__ params, int L, float *sw, MlpLane &m)
{
    const int P = mlp_param_floats(L);
    for (int i = threadIdx.x; i < P; i += blockDim.x) sw[i] = params[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
        for (int ks = 0; ks < kMlpMaxKs; ++ks) {
            mlp_s4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = ks * 16 + 4 * g + e;
                v[e] = k < L ? (short)bf16_bits(sw[(nt * 16 + c) * L + k]) : (short)0;
            }
            m.w[nt][ks] = v;
        }
        m.b1[nt] = sw[kMlpH * L + nt * 16 + c];
        m.w2[nt] = bf16_round(sw[kMlpH * L + kMlpH + nt * 16 + c]);
    }
    m.b2 = sw[kMlpH * L + 2 * kMlpH];
}

// The lanes' registers packed in memory: lane l's record is kMlpLaneWords
// words at l * kMlpLaneWords: W1 tiles (nt, ks) as bf16 pairs in words
// 2 (4 nt + ks) .. +1, then b1[4], W2[4] (bf16-rounded) and b2 as floats.
constexpr int kMlpLaneWords = 48;

inline void mlp_pack_lanes(const float *params, int L, uint32_t *out /* 64 * kMlpLaneWords */)
{
    for (int lane = 0; lane < 64; ++lane) {
        uint32_t *r = out + lane * kMlpLaneWords;
        const int c = lane & 15, g = lane >> 4;
        for (int i = 0; i < kMlpLaneWords; ++i) r[i] = 0;
        for (int nt = 0; nt < 4; ++nt) {
            for (int ks = 0; ks < kMlpMaxKs; ++ks)
                for (int e = 0; e < 4; ++e) {
                    const int k = ks * 16 + 4 * g + e;
                    const uint32_t b = k < L ? bf16_bits(params[(nt * 16 + c) * L + k]) : 0u;
                    r[2 * (4 * nt + ks) + e / 2] |= b << (16 * (e & 1));
                }
            const float b1 = params[kMlpH * L + nt * 16 + c];
            const float w2 = bf16_round(params[kMlpH * L + kMlpH + nt * 16 + c]);
            std::memcpy(&r[32 + nt], &b1, 4);
            std::memcpy(&r[36 + nt], &w2, 4);
        }
        std::memcpy(&r[40], &params[kMlpH * L + 2 * kMlpH], 4);
    }
}

__device__ inline void mlp_lane_load_packed(const uint32_t *__restrict__ packed, MlpLane &m)
{
    const uint4 *r = reinterpret_cast<const uint4 *>(packed + (threadIdx.x & 63) * kMlpLaneWords);
    uint4 v[11];
#pragma unroll
    for (int i = 0; i < 11; ++i) v[i] = r[i];  // all loads in flight together
#pragma unroll
    for (int t = 0; t < 16; ++t) {  // tile (nt, ks) = (t / 4, t % 4): words 2 t, 2 t + 1
        const uint32_t w0 = (&v[t / 2].x)[2 * (t & 1)], w1 = (&v[t / 2].x)[2 * (t & 1) + 1];
        m.w[t / 4][t % 4] = mlp_s4{(short)(w0 & 0xFFFFu), (short)(w0 >> 16), (short)(w1 & 0xFFFFu),
                                   (short)(w1 >> 16)};
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        m.b1[nt] = __uint_as_float((&v[8].x)[nt]);
        m.w2[nt] = __uint_as_float((&v[9].x)[nt]);
    }
    m.b2 = __uint_as_float(v[10].x);
}

// Wave: predictions of 16 queries whose features (bf16 bits, zero past L)
// are rows f + r * ld (r < 16, ld halves, 8-byte aligned rows).  Every lane
// of group g (lane / 16) returns the predictions of rows 4 g .. 4 g + 3.
__device__ inline mlp_f4 mlp_predict16(const uint16_t *f, int ld, int ksteps, const MlpLane &m)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    mlp_f4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = mlp_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kMlpMaxKs; ++ks) {
        if (ks >= ksteps) break;
        const mlp_s4 a = *reinterpret_cast<const mlp_s4 *>(f + r * ld + ks * 16 + 4 * g);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, m.w[nt][ks], acc[nt], 0, 0, 0);
    }
    // acc[nt][j] = z of row 4 g + j, hidden unit 16 nt + (lane % 16)
    mlp_f4 y;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float sum = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const float z = acc[nt][j] + m.b1[nt];
            sum += m.w2[nt] * bf16_round(z > 0.f ? z : 0.f);
        }
        y[j] = sum;
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1)
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] += __shfl_xor(y[j], off);
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] += m.b2;
    return y;
}

}  // namespace qw
