// Wave-level helpers shared by the select and the fused dedup kernels.
#pragma once

#include "qw_internal.h"

namespace qw {

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

}  // namespace qw
