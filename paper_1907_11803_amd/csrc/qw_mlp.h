// BF16 inference helpers of the candidate-count model y = W2 relu(W1 f + b1)
// + b2 (inputs, weights and hidden activations rounded to bfloat16, FP32
// sums).
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

// Whole workgroup: packed parameters (W1 [H][L], b1 [H], W2 [H], b2) into LDS
// as W1^T bf16 [L][H], b1 [H], W2 bf16 [H], b2 (mlp_lds_floats(L) floats).
__host__ __device__ inline int mlp_lds_floats(int L) { return kMlpH * L + 2 * kMlpH + 1; }

__device__ inline void mlp_stage(const float *__restrict__ params, int L, float *sw)
{
    const int P = mlp_lds_floats(L);
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const float v = params[i];
        if (i < kMlpH * L) sw[(i % L) * kMlpH + i / L] = bf16_round(v);  // W1[h][l] -> W1^T[l][h]
        else if (i < kMlpH * L + kMlpH || i == P - 1) sw[i] = v;        // biases stay FP32
        else sw[i] = bf16_round(v);                                      // W2
    }
}

}  // namespace qw
