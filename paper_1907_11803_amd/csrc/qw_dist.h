// Squared L2 distance pieces of the dedup kernel's verification (the
// false-positive removal of Section 1.2).
#pragma once

#include "qw_internal.h"

namespace qw {

// Squared distance contribution of one 16-byte part: uint8 exact (|x|^2 -
// 2 x.q + |q|^2 by dot4, wrapping uint32 arithmetic, exact in total), float
// FP32 FMAs on the differences.
template <int DT>
__device__ inline void part_dist(const uint4 xw, const uint4 qw, uint32_t &accu, float &accf)
{
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
        accu += xx - 2u * xq + qq;
    } else {
        const float d0 = __uint_as_float(xw.x) - __uint_as_float(qw.x);
        const float d1 = __uint_as_float(xw.y) - __uint_as_float(qw.y);
        const float d2 = __uint_as_float(xw.z) - __uint_as_float(qw.z);
        const float d3 = __uint_as_float(xw.w) - __uint_as_float(qw.w);
        float sacc = accf;
        sacc = fmaf(d0, d0, sacc);
        sacc = fmaf(d1, d1, sacc);
        sacc = fmaf(d2, d2, sacc);
        sacc = fmaf(d3, d3, sacc);
        accf = sacc;
    }
}

// x.q over one 16-byte part of uint8 rows (the cross term of |x|^2 + |q|^2 -
// 2 x.q; the norms come from elsewhere)
__device__ inline uint32_t part_dot_u8(const uint4 xw, const uint4 qw, uint32_t acc)
{
    acc = __builtin_amdgcn_udot4(xw.x, qw.x, acc, false);
    acc = __builtin_amdgcn_udot4(xw.y, qw.y, acc, false);
    acc = __builtin_amdgcn_udot4(xw.z, qw.z, acc, false);
    acc = __builtin_amdgcn_udot4(xw.w, qw.w, acc, false);
    return acc;
}

}  // namespace qw
