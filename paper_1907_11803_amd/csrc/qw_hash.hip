// Projection + hashing h = floor((a.v + b) / w) (Section 3) and per-layer probing.
//
// Exactness: every path first computes an approximate projection, then accepts
// floor(y) only when y lies farther than a rigorous error bound beta from the
// nearest integer; otherwise the value is recomputed in FP64 in index order
// (acc += a_i * v_i, then + b, then / w, each correctly rounded).  The bound
// covers the approximate path's error and the FP64 recomputation's own error,
// so accepted and recomputed values both equal the FP64 index-order result.
#include "qw_internal.h"
#include "qw_keys.h"

namespace qw {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// FP64, index order, correctly rounded steps: the reference sequence.  Rows
// are padded to a multiple of 16 elements, so the inputs are read 16 at a time
// with 16-byte loads; the summation still runs i = 0..d-1 in order.
__device__ inline void load16(const uint8_t *p, float *v)
{
    const uint4 w = *reinterpret_cast<const uint4 *>(p);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = (float)((ws[t >> 2] >> (8 * (t & 3))) & 255u);
}

__device__ inline void load16(const float *p, float *v)
{
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float4 f = reinterpret_cast<const float4 *>(p)[t];
        v[4 * t] = f.x;
        v[4 * t + 1] = f.y;
        v[4 * t + 2] = f.z;
        v[4 * t + 3] = f.w;
    }
}

template <typename T>
__device__ __noinline__ int32_t hash_exact(const T *__restrict__ xrow,
                                           const float *__restrict__ arow, int32_t d, float bf,
                                           double w)
{
    double acc = 0.0;
    for (int32_t i0 = 0; i0 < d; i0 += 16) {
        float xv[16], av[16];
        load16(xrow + i0, xv);
        load16(arow + i0, av);
        const int32_t lim = d - i0 < 16 ? d - i0 : 16;
#pragma unroll
        for (int t = 0; t < 16; ++t)
            if (t < lim) acc = __dadd_rn(acc, __dmul_rn((double)av[t], (double)xv[t]));
    }
    double t = __dadd_rn(acc, (double)bf);
    double y = __ddiv_rn(t, w);
    return floor_to_i32(y);
}

// Accept floor(y) when y is farther than beta from every integer.
__device__ inline bool outside_band(double y, double beta)
{
    double fl = floor(y);
    double fr = y - fl;  // exact for doubles
    double dist = fr < 1.0 - fr ? fr : 1.0 - fr;
    return dist > beta;
}

__device__ inline double band(double coef, double xmax, double w, double y)
{
    return coef * xmax / w + 0x1p-50 * (fabs(y) + 1.0) + 0x1p-40;
}

// ---------------------------------------------------------------- FP32 VALU form
// 64 rows x 64 functions per workgroup; every output accumulates sequentially
// over i = 0..dp-1 with fmaf.  Error <= gamma_{d+2} * sum|a_i v_i|.
template <typename T>
__global__ __launch_bounds__(kBlock) void hash_fp32_kernel(
    const T *__restrict__ x, int64_t m, int32_t dp, int32_t d, const float *__restrict__ a,
    const float *__restrict__ b, int32_t f0, int32_t nfun, double w,
    const double *__restrict__ gbc, int32_t *__restrict__ out, int32_t out_ld,
    unsigned long long *recomputed)
{
    __shared__ float xs[64][33];
    __shared__ float as[64][33];
    __shared__ uint32_t xmax_s[64];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    const int fb0 = f0 + blockIdx.y * 64;
    if (threadIdx.x < 64) xmax_s[threadIdx.x] = 0u;
    float bf[4];  // the epilogue's per-function constants, loaded up front
    double gf[4];
    for (int j = 0; j < 4; ++j) {
        const int f = min(fb0 + tx + 16 * j, f0 + nfun - 1);
        bf[j] = b[f];
        gf[j] = gbc[f];
    }
    float acc[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    for (int kc = 0; kc < dp; kc += 32) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 32; e += kBlock) {
            int r = e >> 5, kk = e & 31;
            int kg = kc + kk;
            int64_t row = row0 + r;
            float xv = 0.f, av = 0.f;
            if (kg < dp) {
                if (row < m) xv = (float)x[row * dp + kg];
                av = a[(int64_t)(fb0 + r) * dp + kg];
            }
            xs[r][kk] = xv;
            as[r][kk] = av;
            atomicMax(&xmax_s[r], __float_as_uint(fabsf(xv)));
        }
        __syncthreads();
        for (int kk = 0; kk < 32; ++kk) {
            float xr[4], ar[4];
            for (int i = 0; i < 4; ++i) xr[i] = xs[ty + 16 * i][kk];
            for (int j = 0; j < 4; ++j) ar[j] = as[tx + 16 * j][kk];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(xr[i], ar[j], acc[i][j]);
        }
    }
    __syncthreads();
    unsigned long long nre = 0;
    for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + ty + 16 * i;
        const double xm = (double)__uint_as_float(xmax_s[ty + 16 * i]);
        for (int j = 0; j < 4; ++j) {
            const int f = fb0 + tx + 16 * j;
            if (row >= m || f >= f0 + nfun) continue;
            double y = ((double)acc[i][j] + (double)bf[j]) / w;
            int32_t h;
            if (outside_band(y, band(gf[j], xm, w, y))) {
                h = floor_to_i32(y);
            } else {
                h = hash_exact<T>(x + row * dp, a + (int64_t)f * dp, d, bf[j], w);
                ++nre;
            }
            out[row * out_ld + (f - f0)] = h;
        }
    }
    if (recomputed && nre) atomicAdd(recomputed, nre);
}

// ---------------------------------------------------------------- FP16 MFMA form (uint8 data)
// a = a_hi + a_lo (+ residual counted in the bound), both FP16; uint8 values are
// exact in FP16; products are exact in FP32.  Each wave computes 16 rows x 64
// functions with v_mfma_f32_16x16x16f16, separately for a_hi and a_lo.
__global__ __launch_bounds__(kBlock) void hash_mfma_f16_kernel(
    const uint8_t *__restrict__ x, int64_t m, int32_t dp, int32_t d,
    const _Float16 *__restrict__ ahi, const _Float16 *__restrict__ alo,
    const float *__restrict__ a32, const float *__restrict__ b, int32_t f0, int32_t nfun,
    double w, const double *__restrict__ gbc, int32_t *__restrict__ out, int32_t out_ld,
    unsigned long long *recomputed)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * 64 + wv * 16;
    const int fbase = f0 + blockIdx.y * 64;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    int64_t xrow = row0 + r;
    if (xrow >= m) xrow = m - 1;
    const uint8_t *xp = x + xrow * dp + kq;
    // the epilogue's per-function constants, loaded up front (clamped to the
    // launch's function range; out-of-range functions are never stored)
    float bf[4];
    double gf[4];
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) {
        const int f = min(fbase + fb * 16 + r, f0 + nfun - 1);
        bf[fb] = b[f];
        gf[fb] = gbc[f];
    }
    floatx4_t acc_hi[4], acc_lo[4];
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) {
        acc_hi[fb] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        acc_lo[fb] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    }
    uint32_t xmax = 0;
    // double-buffered K loop: step kb + 16 is loaded (unconditionally, the
    // last step reloads itself) while step kb feeds the MFMAs
    uint32_t xn;
    half4_t ahn[4], aln[4];
    auto load_step = [&](int kb) {
        xn = *reinterpret_cast<const uint32_t *>(xp + kb);
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
            const int64_t f = fbase + fb * 16 + r;
            ahn[fb] = *reinterpret_cast<const half4_t *>(ahi + f * dp + kb + kq);
            aln[fb] = *reinterpret_cast<const half4_t *>(alo + f * dp + kb + kq);
        }
    };
    load_step(0);
    for (int kb = 0; kb < dp; kb += 16) {
        const uint32_t xv = xn;
        half4_t ah[4], al[4];
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
            ah[fb] = ahn[fb];
            al[fb] = aln[fb];
        }
        load_step(kb + 16 < dp ? kb + 16 : kb);
        const uint32_t b0 = xv & 255u, b1 = (xv >> 8) & 255u, b2 = (xv >> 16) & 255u, b3 = xv >> 24;
        xmax = max(xmax, max(max(b0, b1), max(b2, b3)));
        const half4_t xh = {(_Float16)(float)b0, (_Float16)(float)b1, (_Float16)(float)b2,
                            (_Float16)(float)b3};
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
            acc_hi[fb] = __builtin_amdgcn_mfma_f32_16x16x16f16(xh, ah[fb], acc_hi[fb], 0, 0, 0);
            acc_lo[fb] = __builtin_amdgcn_mfma_f32_16x16x16f16(xh, al[fb], acc_lo[fb], 0, 0, 0);
        }
    }
    xmax = max(xmax, (uint32_t)__shfl_xor((int)xmax, 16));
    xmax = max(xmax, (uint32_t)__shfl_xor((int)xmax, 32));
    double xm[4];
    for (int j = 0; j < 4; ++j) xm[j] = (double)__shfl((int)xmax, (lane >> 4) * 4 + j);
    unsigned long long nre = 0;
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) {
        const int f = fbase + fb * 16 + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = row0 + (lane >> 4) * 4 + j;
            if (row >= m || f >= f0 + nfun) continue;
            const double sum = (double)acc_hi[fb][j] + (double)acc_lo[fb][j];
            const double y = (sum + (double)bf[fb]) / w;
            int32_t h;
            if (outside_band(y, band(gf[fb], xm[j], w, y))) {
                h = floor_to_i32(y);
            } else {
                h = hash_exact<uint8_t>(x + row * dp, a32 + (int64_t)f * dp, d, bf[fb], w);
                ++nre;
            }
            out[row * out_ld + (f - f0)] = h;
        }
    }
    if (recomputed && nre) atomicAdd(recomputed, nre);
}

// ---------------------------------------------------------------- FP32 MFMA form (float data)
// v_mfma_f32_16x16x4f32; each lane loads 4 consecutive k of its row and of its
// function and feeds them to 4 MFMAs, so A and B share one k permutation.
__global__ __launch_bounds__(kBlock) void hash_mfma_f32_kernel(
    const float *__restrict__ x, int64_t m, int32_t dp, int32_t d, const float *__restrict__ a32,
    const float *__restrict__ b, int32_t f0, int32_t nfun, double w,
    const double *__restrict__ gbc, int32_t *__restrict__ out, int32_t out_ld,
    unsigned long long *recomputed)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * 64 + wv * 16;
    const int fbase = f0 + blockIdx.y * 64;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    int64_t xrow = row0 + r;
    if (xrow >= m) xrow = m - 1;
    const float *xp = x + xrow * dp + kq;
    float bf[4];  // the epilogue's per-function constants, loaded up front
    double gf[4];
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) {
        const int f = min(fbase + fb * 16 + r, f0 + nfun - 1);
        bf[fb] = b[f];
        gf[fb] = gbc[f];
    }
    floatx4_t acc[4];
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) acc[fb] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    float xmax = 0.f;
    // double-buffered K loop (the last step reloads itself)
    float4 xn, an[4];
    auto load_step = [&](int kb) {
        xn = *reinterpret_cast<const float4 *>(xp + kb);
#pragma unroll
        for (int fb = 0; fb < 4; ++fb)
            an[fb] = *reinterpret_cast<const float4 *>(a32 + (int64_t)(fbase + fb * 16 + r) * dp + kb + kq);
    };
    load_step(0);
    for (int kb = 0; kb < dp; kb += 16) {
        const float4 xv = xn;
        float4 av[4];
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) av[fb] = an[fb];
        load_step(kb + 16 < dp ? kb + 16 : kb);
        xmax = fmaxf(xmax, fmaxf(fmaxf(fabsf(xv.x), fabsf(xv.y)), fmaxf(fabsf(xv.z), fabsf(xv.w))));
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
            acc[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.x, av[fb].x, acc[fb], 0, 0, 0);
            acc[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.y, av[fb].y, acc[fb], 0, 0, 0);
            acc[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.z, av[fb].z, acc[fb], 0, 0, 0);
            acc[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.w, av[fb].w, acc[fb], 0, 0, 0);
        }
    }
    xmax = fmaxf(xmax, __shfl_xor(xmax, 16));
    xmax = fmaxf(xmax, __shfl_xor(xmax, 32));
    double xm[4];
    for (int j = 0; j < 4; ++j) xm[j] = (double)__shfl(xmax, (lane >> 4) * 4 + j);
    unsigned long long nre = 0;
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) {
        const int f = fbase + fb * 16 + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = row0 + (lane >> 4) * 4 + j;
            if (row >= m || f >= f0 + nfun) continue;
            const double y = ((double)acc[fb][j] + (double)bf[fb]) / w;
            int32_t h;
            if (outside_band(y, band(gf[fb], xm[j], w, y))) {
                h = floor_to_i32(y);
            } else {
                h = hash_exact<float>(x + row * dp, a32 + (int64_t)f * dp, d, bf[fb], w);
                ++nre;
            }
            out[row * out_ld + (f - f0)] = h;
        }
    }
    if (recomputed && nre) atomicAdd(recomputed, nre);
}

qw_status launch_hash(const qw_index *ix, const void *xpad, int64_t m, int32_t f0, int32_t nfun,
                      int32_t form, int32_t *out, int32_t out_ld,
                      unsigned long long *recomputed, hipStream_t s)
{
    if (m <= 0 || nfun <= 0) return QW_OK;
    // nf_pad is a multiple of 64 and zero padded, so 64-function tiles never
    // read past the parameter arrays.
    dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(nfun, 64));
    const double w = (double)ix->w;
    if (form == QW_FORM_PLAIN_FP32) {
        if (ix->dtype == QW_U8)
            hash_fp32_kernel<uint8_t><<<grid, kBlock, 0, s>>>(
                (const uint8_t *)xpad, m, ix->dp, ix->d, ix->a32.as<float>(), ix->b32.as<float>(),
                f0, nfun, w, ix->gb_plain.as<double>(), out, out_ld, recomputed);
        else
            hash_fp32_kernel<float><<<grid, kBlock, 0, s>>>(
                (const float *)xpad, m, ix->dp, ix->d, ix->a32.as<float>(), ix->b32.as<float>(),
                f0, nfun, w, ix->gb_plain.as<double>(), out, out_ld, recomputed);
    } else if (ix->dtype == QW_U8 && ix->fast_f16) {
        hash_mfma_f16_kernel<<<grid, kBlock, 0, s>>>(
            (const uint8_t *)xpad, m, ix->dp, ix->d, ix->a_hi.as<_Float16>(),
            ix->a_lo.as<_Float16>(), ix->a32.as<float>(), ix->b32.as<float>(), f0, nfun, w,
            ix->gb_fast.as<double>(), out, out_ld, recomputed);
    } else if (ix->dtype == QW_F32) {
        hash_mfma_f32_kernel<<<grid, kBlock, 0, s>>>(
            (const float *)xpad, m, ix->dp, ix->d, ix->a32.as<float>(), ix->b32.as<float>(), f0,
            nfun, w, ix->gb_fast.as<double>(), out, out_ld, recomputed);
    } else {
        // uint8 data whose parameters do not fit FP16: FP32 VALU path
        hash_fp32_kernel<uint8_t><<<grid, kBlock, 0, s>>>(
            (const uint8_t *)xpad, m, ix->dp, ix->d, ix->a32.as<float>(), ix->b32.as<float>(),
            f0, nfun, w, ix->gb_plain.as<double>(), out, out_ld, recomputed);
    }
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// ---------------------------------------------------------------- probe
// One thread per (query, layer): pack the layer's k hash values into the exact
// key (values outside the data's range cannot match any bucket: a miss), then
// look the key up in the layer's open-addressing table.
__global__ __launch_bounds__(kBlock) void probe_kernel(
    const int32_t *__restrict__ h, int64_t Q, int32_t L, int32_t k,
    const int32_t *__restrict__ hmin, const int32_t *__restrict__ hmax,
    const int32_t *__restrict__ shift, const TabEntry *__restrict__ tab,
    const long long *__restrict__ tab_off, const uint32_t *__restrict__ tab_mask,
    uint32_t *__restrict__ bstart, uint32_t *__restrict__ bsize, float *__restrict__ feats)
{
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Q * L) return;
    const int64_t q = idx / L;
    const int32_t l = (int32_t)(idx - q * L);
    const int32_t nf = L * k;
    uint64_t klo = 0, khi = 0;
    bool valid = true;
    for (int32_t j = 0; j < k; ++j) {
        const int32_t f = l * k + j;
        const int32_t v = h[q * nf + f];
        if (v < hmin[f] || v > hmax[f]) {
            valid = false;
            break;
        }
        key_put(klo, khi, (uint64_t)((int64_t)v - (int64_t)hmin[f]), shift[f]);
    }
    uint32_t st = 0, sz = 0;
    if (valid) {
        const TabEntry *t = tab + tab_off[l];
        const uint32_t mask = tab_mask[l];
        uint32_t slot = (uint32_t)key_mix(klo, khi) & mask;
        for (uint32_t it = 0; it <= mask; ++it) {
            const TabEntry e = t[slot];
            if (e.size == 0) break;
            if (e.klo == klo && e.khi == khi) {
                st = e.start;
                sz = e.size;
                break;
            }
            slot = (slot + 1) & mask;
        }
    }
    bstart[idx] = st;
    bsize[idx] = sz;
    if (feats) feats[idx] = log1pf((float)sz);  // count-model input, f = log(1 + s)
}

qw_status launch_probe(const qw_index *ix, const int32_t *h, int64_t Q, uint32_t *bstart,
                       uint32_t *bsize, float *feats, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    const int64_t total = Q * ix->L;
    probe_kernel<<<(unsigned)ceil_div(total, kBlock), kBlock, 0, s>>>(
        h, Q, ix->L, ix->k, ix->hmin.as<int32_t>(), ix->hmax.as<int32_t>(),
        ix->shift.as<int32_t>(), ix->tab.as<TabEntry>(), ix->tab_off.as<long long>(),
        ix->tab_mask.as<uint32_t>(), bstart, bsize, feats);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
