// Exact layer keys: a layer's k hash values packed into 128 bits.
//
// Function j of a layer stores (h_j - hmin_j) in bits [shift_j, shift_j + bits_j)
// where bits_j covers hmax_j - hmin_j over the indexed data.  A field never
// straddles bit 64, so it lives entirely in klo (shift < 64) or khi.  Two
// points share a bucket iff their packed keys are equal (Section 1.1: the
// functions of a layer are combined conjunctively).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qw {

__host__ __device__ inline void key_put(uint64_t &klo, uint64_t &khi, uint64_t v, int32_t shift)
{
    if (shift < 64)
        klo |= v << shift;
    else
        khi |= v << (shift - 64);
}

// 64-bit mix of a 128-bit key (splitmix64 finaliser over a combination).
__host__ __device__ inline uint64_t key_mix(uint64_t lo, uint64_t hi)
{
    uint64_t h = lo * 0x9E3779B97F4A7C15ull ^ (hi + 0x632BE59BD9B4E019ull) * 0xC2B2AE3D27D4EB4Full;
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    return h;
}

// floor(y) as int32, saturating outside the int32 range (such values never
// match a bucket: the index range check rejects them).
__host__ __device__ inline int32_t floor_to_i32(double y)
{
    double f = floor(y);
    if (!(f >= -2147483648.0)) return INT32_MIN;
    if (f > 2147483647.0) return INT32_MAX;
    return (int32_t)f;
}

}  // namespace qw
