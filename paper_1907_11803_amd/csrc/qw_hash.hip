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
// with 16-byte loads; the summation still runs i = 0..d-1 in order.  Each
// product of an FP32 parameter and a uint8 or FP32 input is exact in FP64, so
// a multiply-add the compiler fuses rounds exactly like the separate steps.
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

// Raw 16-element pieces, converted to FP32 values when used.
__device__ inline void piece_load(const uint8_t *p, uint4 (&r)[1]) { r[0] = *reinterpret_cast<const uint4 *>(p); }
__device__ inline void piece_load(const float *p, float4 (&r)[4])
{
#pragma unroll
    for (int t = 0; t < 4; ++t) r[t] = reinterpret_cast<const float4 *>(p)[t];
}
__device__ inline float piece_value(const uint4 (&r)[1], int t)
{
    const uint32_t wd = t < 4 ? r[0].x : t < 8 ? r[0].y : t < 12 ? r[0].z : r[0].w;
    return (float)((wd >> (8 * (t & 3))) & 255u);
}
__device__ inline float piece_value(const float4 (&r)[4], int t)
{
    const float4 v = r[t >> 2];
    return (t & 3) == 0 ? v.x : (t & 3) == 1 ? v.y : (t & 3) == 2 ? v.z : v.w;
}

template <typename T> struct Piece;
template <> struct Piece<uint8_t> { typedef uint4 V[1]; static constexpr int B = 4; };
template <> struct Piece<float> { typedef float4 V[4]; static constexpr int B = 2; };

template <typename T>
__device__ inline int32_t hash_exact(const T *__restrict__ xrow, const float *__restrict__ arow,
                                     int32_t d, float bf, double w)
{
    // B pieces of 16 elements are loaded together (one memory latency per
    // 16 B terms); a piece past the row end re-reads the last piece and
    // contributes nothing
    constexpr int B = Piece<T>::B;
    const int32_t last = (d - 1) & ~15;
    double acc = 0.0;
    for (int32_t i0 = 0; i0 < d; i0 += 16 * B) {
        typename Piece<T>::V xr[B];
        float4 ar[B][4];
#pragma unroll
        for (int p = 0; p < B; ++p) {
            const int32_t o = min(i0 + 16 * p, last);
            piece_load(xrow + o, xr[p]);
            piece_load(arow + o, ar[p]);
        }
        __builtin_amdgcn_sched_barrier(0);  // all loads of the block in flight together
#pragma unroll
        for (int p = 0; p < B; ++p)
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (i0 + 16 * p + t < d)
                    acc = __dadd_rn(acc, __dmul_rn((double)piece_value(ar[p], t),
                                                   (double)piece_value(xr[p], t)));
    }
    double t = __dadd_rn(acc, (double)bf);
    double y = __ddiv_rn(t, w);
    return floor_to_i32(y);
}

// Guard-band test, evaluated in FP32.  s is the approximate projection a.v
// (before + b), bf = b, iw = 1/w rounded to FP32, and cw * xm bounds
// |s - FP64 index-order a.v| / w, plus the reference's own FP64 rounding.
// y = (s + bf) * iw is accepted when its distance to the nearest integer
// exceeds that bound plus the error of evaluating y and the distance in FP32
// (u = 2^-24): the sum s (when it adds two accumulators) and s + bf each
// round once (<= u |s| / w and u |y|), iw and the product add <= 2u |y|, and
// the distances round by at most 2^-24 (they are exact for |y| >= 1).  The
// total is inflated by 2^-20 to cover the rounding of the bound itself.  For
// |y| >= 2^22 the bound exceeds every distance, so nothing out of FP32's
// integer range is accepted.
__device__ inline bool accept_fp32(float s, float bf, float iw, float cwx, int32_t &h)
{
    const float y = (s + bf) * iw;
    const float fl = floorf(y);
    const float dist = fminf(y - fl, (fl + 1.0f) - y);
    const float beta =
        (cwx + 0x1p-22f * (fabsf(y) + fabsf(s) * iw) + 0x1p-23f + 0x1p-40f) * (1.0f + 0x1p-20f);
    h = (int32_t)fl;
    return dist > beta;
}

// Per-function band coefficient scaled by 1/w for accept_fp32 (rounded, then
// inflated past the rounding).
__device__ inline float band_coef(double coef, double w)
{
    return (float)(coef / w) * (1.0f + 0x1p-20f);
}

// Recomputes the outputs a lane marked as inside the guard band.  The lanes
// of a wave recompute their marked outputs side by side, so a wave waits for
// the lane with the most marks rather than once per marked output of any lane.
template <typename T>
__device__ inline void recompute_marked(uint32_t pend, const T *__restrict__ x, int64_t row0,
                                        int32_t rstride, int32_t dp, int32_t d, const float *__restrict__ a32,
                                        const float *__restrict__ b, int fbase, int32_t f0,
                                        double w, int32_t *__restrict__ out, int32_t out_ld,
                                        unsigned long long &nre)
{
    // bit fb * 4 + j: row row0 + j * rstride, function fbase + 16 fb
    while (pend) {
        const int o = __ffs(pend) - 1;
        pend &= pend - 1u;
        const int64_t row = row0 + (int64_t)(o & 3) * rstride;
        const int f = fbase + (o >> 2) * 16;
        out[row * out_ld + (f - f0)] = hash_exact<T>(x + row * dp, a32 + (int64_t)f * dp, d, b[f], w);
        ++nre;
    }
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
    float bf[4], cw[4];  // the epilogue's per-function constants, loaded up front
    for (int j = 0; j < 4; ++j) {
        const int f = min(fb0 + tx + 16 * j, f0 + nfun - 1);
        bf[j] = b[f];
        cw[j] = band_coef(gbc[f], w);
    }
    const float iw = (float)(1.0 / w);
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
    uint32_t pend = 0;  // bit j * 4 + i: output (row0 + ty + 16 i, fb0 + tx + 16 j)
    for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + ty + 16 * i;
        const float xm = __uint_as_float(xmax_s[ty + 16 * i]);
        for (int j = 0; j < 4; ++j) {
            const int f = fb0 + tx + 16 * j;
            if (row >= m || f >= f0 + nfun) continue;
            int32_t h;
            if (accept_fp32(acc[i][j], bf[j], iw, cw[j] * xm, h))
                out[row * out_ld + (f - f0)] = h;
            else
                pend |= 1u << (j * 4 + i);
        }
    }
    unsigned long long nre = 0;
    recompute_marked<T>(pend, x, row0 + ty, 16, dp, d, a, b, fb0 + tx, f0, w, out, out_ld, nre);
    if (recomputed && nre)
        atomicAdd(recomputed + (blockIdx.y * gridDim.x + blockIdx.x) % kRecompSlots, nre);
}

// ---------------------------------------------------------------- MFMA forms
// A workgroup computes 64 rows x 64 functions; wave wv owns rows 16 wv ..
// 16 wv + 15 against all 64 functions (four 16 x 16 output blocks).  The K
// dimension is staged through LDS in chunks: every thread issues its share of
// the chunk's global loads at once, so a chunk costs one memory latency, and
// the next chunk's loads are in flight while the current one is multiplied.
// LDS rows are padded so that the fragment reads of a wave hit distinct banks.
//
// Epilogue: outputs inside the guard band are marked per lane and recomputed
// after the accepted ones are stored.

constexpr int kKcF16 = 128;  // K chunk, FP16 form (uint8 data)
constexpr int kKcF32 = kHashChunkF32;  // K chunk, FP32 form (float data)

// 16 loaded bytes, or zeros (masked per component: a select of the vector
// type would go through memory)
__device__ inline uint4 mask16(uint4 v, bool keep)
{
    const uint32_t mk = keep ? 0xffffffffu : 0u;
    return uint4{v.x & mk, v.y & mk, v.z & mk, v.w & mk};
}

// a = a_hi + a_lo (+ residual counted in the bound), both FP16; uint8 values are
// exact in FP16; products are exact in FP32.  v_mfma_f32_16x16x16f16, once for
// a_hi and once for a_lo.  Three workgroups per CU (registers and LDS), so a
// 10^4-query batch (628 workgroups) runs in one round.
//
// A workgroup takes 64 rows and `bpw` (at most 4) consecutive 64-function
// tiles of them: all of a row's functions up to 256 when the row blocks alone
// fill the GPU twice over.  Each tile's hash values go through LDS (the a_hi
// staging buffer, free once the tile's last MFMA has read it) and leave as
// whole 16-byte pieces of each row's 256-byte run, so a row's runs are written
// together from one workgroup and its cache lines fill in one L2 instead of
// arriving in pieces from workgroups far apart in the launch.  Guard-band
// outputs are marked per lane and recomputed at the end, over the stored
// tile values (inside the tile loop their FP64 registers would spill the
// MFMA loop's).
constexpr int kTileLd = 68;  // ints per staged output row: the four lane groups' rows land on distinct banks

__global__ __launch_bounds__(kBlock, 3) void hash_mfma_f16_kernel(
    const uint8_t *__restrict__ x, int64_t m, int32_t dp, int32_t d,
    const _Float16 *__restrict__ ahi, const _Float16 *__restrict__ alo,
    const float *__restrict__ a32, const float *__restrict__ b, int32_t f0, int32_t nfun,
    int32_t bpw, double w, const double *__restrict__ gbc, int32_t *__restrict__ out,
    int32_t out_ld, unsigned long long *recomputed)
{
    constexpr int KC = kKcF16;
    constexpr int XS = KC + 16;  // bytes per staged row of x
    constexpr int AS = KC + 8;   // halves per staged function row
    __shared__ __align__(16) uint8_t xs[64 * XS];
    __shared__ __align__(16) _Float16 hs[64 * AS];
    __shared__ __align__(16) _Float16 ls[64 * AS];
    static_assert(sizeof(hs) >= sizeof(int32_t) * 64 * kTileLd, "the output tile reuses hs");
    int32_t *tile = reinterpret_cast<int32_t *>(hs);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t rowb = (int64_t)blockIdx.x * 64;
    const int64_t row0 = rowb + wv * 16;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    const int blk0 = (int)blockIdx.y * bpw;
    const int nblk = min((nfun + 63) / 64 - blk0, bpw);
    const int nkc = (dp + KC - 1) / KC;
    const bool vec = (out_ld & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    const float iw = (float)(1.0 / w);
    // staging registers: x = 64 rows x KC bytes (2 x 16 B per thread), a_hi and
    // a_lo = 64 functions x KC halves (4 x 16 B each); rows past m repeat row
    // m - 1; a piece past dp re-reads the row's last piece (every load is in
    // bounds and none waits on a branch) and is stored as zeros.  Step t is
    // chunk t % nkc of tile t / nkc.
    uint4 xr[2], hr[4], lr[4];
    auto load_step = [&](int t) {
        const int kc = (t % nkc) * KC, fbase = f0 + (blk0 + t / nkc) * 64;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + i * kBlock, row = e >> 3, k = kc + (e & 7) * 16;
            const int64_t gr = rowb + row < m ? rowb + row : m - 1;
            xr[i] = *reinterpret_cast<const uint4 *>(x + gr * dp + min(k, dp - 16));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * kBlock, f = e >> 4, k = kc + (e & 15) * 8;
            const int64_t off = (int64_t)(fbase + f) * dp + min(k, dp - 8);
            hr[i] = *reinterpret_cast<const uint4 *>(ahi + off);
            lr[i] = *reinterpret_cast<const uint4 *>(alo + off);
        }
    };
    // masking happens here, not at the load, so the loads of the next chunk
    // stay in flight while the current one is multiplied
    auto store_chunk = [&](int kc) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + i * kBlock;
            *reinterpret_cast<uint4 *>(xs + (e >> 3) * XS + (e & 7) * 16) =
                mask16(xr[i], kc + (e & 7) * 16 < dp);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * kBlock, o = (e >> 4) * AS + (e & 15) * 8;
            const bool keep = kc + (e & 15) * 8 < dp;
            *reinterpret_cast<uint4 *>(hs + o) = mask16(hr[i], keep);
            *reinterpret_cast<uint4 *>(ls + o) = mask16(lr[i], keep);
        }
    };
    unsigned long long marks = 0;  // bit 16 bt + 4 fb + j: output (j, fb) of tile bt in the guard band
    if (nblk > 0) load_step(0);
    for (int bt = 0; bt < nblk; ++bt) {
        const int fbase = f0 + (blk0 + bt) * 64;
        // the tile's epilogue constants (clamped to the launch's function
        // range; functions past it are never stored)
        float bf[4], cw[4];
        floatx4_t acc_hi[4], acc_lo[4];
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
            acc_hi[fb] = floatx4_t{0.f, 0.f, 0.f, 0.f};
            acc_lo[fb] = floatx4_t{0.f, 0.f, 0.f, 0.f};
            const int f = min(fbase + fb * 16 + r, f0 + nfun - 1);
            bf[fb] = b[f];
            cw[fb] = band_coef(gbc[f], w);
        }
        uint32_t xmax = 0;
        for (int c = 0; c < nkc; ++c) {
            const int kc = c * KC;
            __syncthreads();  // the previous chunk's (or tile's) reads are done
            store_chunk(kc);
            __syncthreads();
            // the next chunk (of this tile or the next) flies during this
            // one's MFMAs and the epilogue
            if (c + 1 < nkc || bt + 1 < nblk) load_step(bt * nkc + c + 1);
            const int ns = (dp - kc < KC ? dp - kc : KC) / 16;
#pragma unroll
            for (int st = 0; st < KC / 16; ++st) {
                if (st >= ns) break;
                const uint32_t xv = *reinterpret_cast<const uint32_t *>(xs + (wv * 16 + r) * XS + st * 16 + kq);
                half4_t ah[4], al[4];
#pragma unroll
                for (int fb = 0; fb < 4; ++fb) {
                    const int o = (fb * 16 + r) * AS + st * 16 + kq;
                    ah[fb] = *reinterpret_cast<const half4_t *>(hs + o);
                    al[fb] = *reinterpret_cast<const half4_t *>(ls + o);
                }
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
        }
        // ---- the tile's epilogue
        xmax = max(xmax, (uint32_t)__shfl_xor((int)xmax, 16));
        xmax = max(xmax, (uint32_t)__shfl_xor((int)xmax, 32));
        float xm[4];
        for (int j = 0; j < 4; ++j) xm[j] = (float)__shfl((int)xmax, (lane >> 4) * 4 + j);
        // this lane's outputs: rows rl + j (j < 4), functions fbase + r + 16 fb;
        // tile row tr + j
        const int64_t rl = row0 + (lane >> 4) * 4;
        const int tr = wv * 16 + (lane >> 4) * 4;
        uint32_t pend = 0;
        __syncthreads();  // every wave's MFMAs have read hs
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
            const int f = fbase + fb * 16 + r;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int32_t h = 0;
                if (rl + j < m && f < f0 + nfun &&
                    !accept_fp32(acc_hi[fb][j] + acc_lo[fb][j], bf[fb], iw, cw[fb] * xm[j], h))
                    pend |= 1u << (fb * 4 + j);
                tile[(tr + j) * kTileLd + fb * 16 + r] = h;
            }
        }
        marks |= (unsigned long long)pend << (16 * bt);
        __syncthreads();
        // the tile's rows: 16 pieces of 4 values per row, row-major
        const int nval = min(64, f0 + nfun - fbase);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * kBlock, row = e >> 4, pc = (e & 15) * 4;
            const int64_t gr = rowb + row;
            if (gr >= m || pc >= nval) continue;
            int32_t *dst = out + gr * out_ld + (fbase - f0) + pc;
            const int32_t *src = tile + row * kTileLd + pc;
            if (vec && pc + 4 <= nval) {
                *reinterpret_cast<int4 *>(dst) = *reinterpret_cast<const int4 *>(src);
            } else {
                for (int q = 0; q < 4 && pc + q < nval; ++q) dst[q] = src[q];
            }
        }
    }
    // outputs inside the guard band: the FP64 index-order value, stored over
    // the tile's value.  The workgroup's marks are pooled in LDS (the a_lo
    // staging buffer, free now) and dealt one per thread, so the recomputes
    // of a workgroup take one FP64 sequence's latency rather than one per mark
    // of its busiest lane; when they exceed the pool, each lane recomputes its
    // own.  At the end no other registers are live.  The barriers order every
    // tile store of the workgroup before these; a device-scope fence is not
    // needed and would write back the L2.
    constexpr uint32_t kPool = sizeof(ls) / sizeof(uint32_t);
    uint32_t *pool = reinterpret_cast<uint32_t *>(ls);  // (tile row << 8) | function of the workgroup
    __shared__ uint32_t wtot[kBlock / 64];
    const uint32_t cnt = (uint32_t)__popcll(marks);
    uint32_t incl = cnt;  // this lane's end within its wave's marks
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        const uint32_t t = wtot[i];
        base += i < wv ? t : 0u;
        total += t;
    }
    const bool pooled = total <= kPool;  // the same in every thread
    const int tr = wv * 16 + (lane >> 4) * 4;
    if (pooled) {
        uint32_t e = base + incl - cnt;
        while (marks) {
            const int o = __ffsll(marks) - 1;
            marks &= marks - 1ull;
            pool[e++] = (uint32_t)(tr + (o & 3)) << 8 | (uint32_t)((o >> 4) * 64 + ((o >> 2) & 3) * 16 + r);
        }
    }
    __syncthreads();
    unsigned long long nre = 0;
    const uint32_t np = pooled ? total : 0u;
    for (uint32_t i = tid; i < np; i += kBlock) {
        const uint32_t v = pool[i];
        const int64_t row = rowb + (v >> 8);
        const int f = f0 + blk0 * 64 + (int)(v & 255u);
        out[row * out_ld + (f - f0)] = hash_exact<uint8_t>(x + row * dp, a32 + (int64_t)f * dp, d, b[f], w);
        ++nre;
    }
    const int64_t rl = row0 + (lane >> 4) * 4;
    while (marks) {  // not pooled: more marks than the pool holds
        const int o = __ffsll(marks) - 1;
        marks &= marks - 1ull;
        const int j = o & 3, f = f0 + (blk0 + (o >> 4)) * 64 + ((o >> 2) & 3) * 16 + r;
        out[(rl + j) * out_ld + (f - f0)] =
            hash_exact<uint8_t>(x + (rl + j) * dp, a32 + (int64_t)f * dp, d, b[f], w);
        ++nre;
    }
    if (recomputed && nre)
        atomicAdd(recomputed + (blockIdx.y * gridDim.x + blockIdx.x) % kRecompSlots, nre);
}

// v_mfma_f32_16x16x4f32; each lane reads 4 consecutive k of its row and of its
// function and feeds them to 4 MFMAs, so A and B share one k permutation.
__global__ __launch_bounds__(kBlock) void hash_mfma_f32_kernel(
    const float *__restrict__ x, int64_t m, int32_t dp, int32_t d, const float *__restrict__ a32,
    const float *__restrict__ b, int32_t f0, int32_t nfun, double w,
    const double *__restrict__ gbc, int32_t *__restrict__ out, int32_t out_ld,
    unsigned long long *recomputed)
{
    constexpr int KC = kKcF32;
    constexpr int RS = KC + 4;  // floats per staged row
    __shared__ __align__(16) float xs[64 * RS];
    __shared__ __align__(16) float as[64 * RS];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t rowb = (int64_t)blockIdx.x * 64;
    const int64_t row0 = rowb + wv * 16;
    const int fbase = f0 + blockIdx.y * 64;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    float bf[4], cw[4];  // the epilogue's per-function constants, loaded up front
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) {
        const int f = min(fbase + fb * 16 + r, f0 + nfun - 1);
        bf[fb] = b[f];
        cw[fb] = band_coef(gbc[f], w);
    }
    const float iw = (float)(1.0 / w);
    // staging registers: 64 rows (functions) x KC floats = 4 x 16 B per thread;
    // rows past m repeat row m - 1; a piece past dp re-reads the row's last
    // piece and is stored as zeros
    uint4 xr[4], ar[4];
    auto load_chunk = [&](int kc) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * kBlock, row = e >> 4, k = kc + (e & 15) * 4;
            const int64_t gr = rowb + row < m ? rowb + row : m - 1;
            const int kk = min(k, dp - 4);
            xr[i] = *reinterpret_cast<const uint4 *>(x + gr * dp + kk);
            ar[i] = *reinterpret_cast<const uint4 *>(a32 + (int64_t)(fbase + row) * dp + kk);
        }
    };
    auto store_chunk = [&](int kc) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * kBlock, o = (e >> 4) * RS + (e & 15) * 4;
            const bool keep = kc + (e & 15) * 4 < dp;
            *reinterpret_cast<uint4 *>(xs + o) = mask16(xr[i], keep);
            *reinterpret_cast<uint4 *>(as + o) = mask16(ar[i], keep);
        }
    };
    // each KC-element chunk accumulates in FP32 on the matrix cores and is
    // then added to an FP64 sum, so the FP32 error grows with KC, not d
    floatx4_t acc[4];
    double dacc[4][4];
#pragma unroll
    for (int fb = 0; fb < 4; ++fb)
#pragma unroll
        for (int j = 0; j < 4; ++j) dacc[fb][j] = 0.0;
    float xmax = 0.f;
    load_chunk(0);
    for (int kc = 0; kc < dp; kc += KC) {
        __syncthreads();  // the previous chunk's reads are done
        store_chunk(kc);
        __syncthreads();
        if (kc + KC < dp) load_chunk(kc + KC);
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) acc[fb] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        const int ns = (dp - kc < KC ? dp - kc : KC) / 16;
#pragma unroll
        for (int st = 0; st < KC / 16; ++st) {
            if (st >= ns) break;
            const float4 xv = *reinterpret_cast<const float4 *>(xs + (wv * 16 + r) * RS + st * 16 + kq);
            float4 av[4];
#pragma unroll
            for (int fb = 0; fb < 4; ++fb)
                av[fb] = *reinterpret_cast<const float4 *>(as + (fb * 16 + r) * RS + st * 16 + kq);
            xmax = fmaxf(xmax, fmaxf(fmaxf(fabsf(xv.x), fabsf(xv.y)), fmaxf(fabsf(xv.z), fabsf(xv.w))));
#pragma unroll
            for (int fb = 0; fb < 4; ++fb) {
                acc[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.x, av[fb].x, acc[fb], 0, 0, 0);
                acc[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.y, av[fb].y, acc[fb], 0, 0, 0);
                acc[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.z, av[fb].z, acc[fb], 0, 0, 0);
                acc[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.w, av[fb].w, acc[fb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int fb = 0; fb < 4; ++fb)
#pragma unroll
            for (int j = 0; j < 4; ++j) dacc[fb][j] += (double)acc[fb][j];
    }
    xmax = fmaxf(xmax, __shfl_xor(xmax, 16));
    xmax = fmaxf(xmax, __shfl_xor(xmax, 32));
    float xm[4];
    for (int j = 0; j < 4; ++j) xm[j] = __shfl(xmax, (lane >> 4) * 4 + j);
    const int64_t rl = row0 + (lane >> 4) * 4;
    uint32_t pend = 0;
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) {
        const int f = fbase + fb * 16 + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = rl + j;
            if (row >= m || f >= f0 + nfun) continue;
            int32_t h;
            if (accept_fp32((float)dacc[fb][j], bf[fb], iw, cw[fb] * xm[j], h))
                out[row * out_ld + (f - f0)] = h;
            else
                pend |= 1u << (fb * 4 + j);
        }
    }
    unsigned long long nre = 0;
    recompute_marked<float>(pend, x, rl, 1, dp, d, a32, b, fbase + r, f0, w, out, out_ld, nre);
    if (recomputed && nre)
        atomicAdd(recomputed + (blockIdx.y * gridDim.x + blockIdx.x) % kRecompSlots, nre);
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
        // every function tile of a row block in one workgroup when the row
        // blocks alone give two rounds of the GPU's three workgroups per CU
        const int nblk = (int)ceil_div(nfun, 64);
        const int bpw = grid.x >= 6u * (unsigned)ix->cus ? std::min(nblk, 4) : 1;  // marks: 4 x 16 bits
        const dim3 g16(grid.x, (unsigned)ceil_div(nblk, bpw));
        hash_mfma_f16_kernel<<<g16, kBlock, 0, s>>>(
            (const uint8_t *)xpad, m, ix->dp, ix->d, ix->a_hi.as<_Float16>(),
            ix->a_lo.as<_Float16>(), ix->a32.as<float>(), ix->b32.as<float>(), f0, nfun, bpw, w,
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

// ---------------------------------------------------------------- probe scores
// Query-directed probing: each (query, layer)'s T moves.  The layer's k values
// y_j = (a_j . x + b_j) / w are computed in FP64, index order, one rounding per
// step (a product of a float parameter and a uint8 or float element is exact
// in FP64, so the fused multiply-add rounds as the separate product and sum
// do): the reference's own FP64 values.  Move 2j + s shifts hash value j by
// -1 (s = 0, score f_j * f_j) or +1 (s = 1, score (1 - f_j) * (1 - f_j)),
// f_j = y_j - floor(y_j), every operation rounded in FP64; the probes take the
// smallest (score, move) in order, pass t the smallest above pick t - 1.  The
// floors of the same values are the query's hash values, written too when
// hout is given (the fast form then needs no other hashing of the queries).
//
// One thread per (query, layer); the lanes of a wave take consecutive queries
// of one layer, so the parameters are uniform: scalar loads from a64l, the
// parameters in FP64, [layer][element][function], one layer's values
// contiguous.  Each lane converts a 16-element piece of its row once and
// feeds the k sums; the next piece loads while the current one is used.
// KM: k itself (KEXACT) or a bound on it (functions past k skipped).

template <typename E> struct Piece16;
template <> struct Piece16<uint8_t> {
    typedef uint4 V;
    static __device__ V load(const uint8_t *p) { return *reinterpret_cast<const uint4 *>(p); }
    static __device__ double at(const V &v, int i)
    {
        const uint32_t w = i < 4 ? v.x : i < 8 ? v.y : i < 12 ? v.z : v.w;
        return (double)((w >> (8 * (i & 3))) & 0xFFu);
    }
};
template <> struct Piece16<float> {
    struct V { float4 p[4]; };
    static __device__ V load(const float *p)
    {
        V v;
#pragma unroll
        for (int i = 0; i < 4; ++i) v.p[i] = reinterpret_cast<const float4 *>(p)[i];
        return v;
    }
    static __device__ double at(const V &v, int i)
    {
        const float4 &q = v.p[i >> 2];
        return (double)((i & 3) == 0 ? q.x : (i & 3) == 1 ? q.y : (i & 3) == 2 ? q.z : q.w);
    }
};

template <typename E, int KM, bool KEXACT>
__global__ __launch_bounds__(kBlock) void probe_moves_kernel(
    const E *__restrict__ x, int64_t Q, int32_t dp, const double *__restrict__ a64l,
    const float *__restrict__ b, int32_t L, int32_t k, double w, int32_t T,
    uint8_t *__restrict__ moves, int32_t *__restrict__ hout, uint32_t *__restrict__ clear,
    int32_t nclear)
{
#pragma clang fp contract(off)
    // the pipeline's counters, zeroed here instead of by a launch of their
    // own (this kernel reads none of them; the kernels that do follow it)
    if (clear && blockIdx.x == 0 && blockIdx.y == 0)
        for (int32_t i = threadIdx.x; i < nclear; i += kBlock) clear[i] = 0u;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t l = blockIdx.y;
    const E *xr = x + (q < Q ? q : Q - 1) * dp;  // dp: a multiple of 16 elements, zero padded
    const double *al = a64l + (int64_t)l * dp * k;  // element e, function j: al[e * k + j]
    double acc[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) acc[j] = 0.0;
    typename Piece16<E>::V cur = Piece16<E>::load(xr);
    for (int32_t e0 = 0; e0 < dp; e0 += 16) {
        // the next piece (the last one re-reads itself)
        const typename Piece16<E>::V nxt = Piece16<E>::load(xr + (e0 + 16 < dp ? e0 + 16 : e0));
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const double xv = Piece16<E>::at(cur, u);
            const double *ae = al + (int64_t)(e0 + u) * k;
#pragma unroll
            for (int j = 0; j < KM; ++j)
                if (KEXACT || j < k)  // uniform
                    acc[j] = __builtin_fma(xv, ae[j], acc[j]);
        }
        cur = nxt;
    }
    if (q >= Q) return;
    double fr[KM];
    int32_t hv[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        fr[j] = 0.0;
        hv[j] = 0;
        if (KEXACT || j < k) {
            const double y = __ddiv_rn(__dadd_rn(acc[j], (double)b[l * k + j]), w);
            fr[j] = y - floor(y);
            hv[j] = floor_to_i32(y);  // the reference's own value: its floor is the hash value
        }
    }
    if (hout) {
        int32_t *ho = hout + q * (L * k) + l * k;
        if (KEXACT && KM % 2 == 0) {  // 8-byte aligned: (L k q + k l) is even
#pragma unroll
            for (int j = 0; j < KM; j += 2) *reinterpret_cast<int2 *>(ho + j) = int2{hv[j], hv[j + 1]};
        } else {
#pragma unroll
            for (int j = 0; j < KM; ++j)
                if (j < k) ho[j] = hv[j];
        }
    }
    const int64_t ql = q * L + l;
    double ps = -1.0;
    int32_t pm = -1;
    for (int32_t t = 0; t < T; ++t) {
        double bs = INFINITY;
        int32_t bm = 2 * k;
#pragma unroll
        for (int32_t j = 0; j < KM; ++j) {
            if (!KEXACT && j >= k) continue;
            const double up = 1.0 - fr[j];
            const double s0 = fr[j] * fr[j], s1 = up * up;
            const int32_t m0 = 2 * j, m1 = 2 * j + 1;
            // candidates strictly after the previous pick in (score, move) order
            const bool e0 = s0 > ps || (s0 == ps && m0 > pm);
            const bool e1 = s1 > ps || (s1 == ps && m1 > pm);
            if (e0 && (s0 < bs || (s0 == bs && m0 < bm))) { bs = s0; bm = m0; }
            if (e1 && (s1 < bs || (s1 == bs && m1 < bm))) { bs = s1; bm = m1; }
        }
        moves[ql * T + t] = (uint8_t)bm;
        ps = bs;
        pm = bm;
    }
}

template <typename E>
void launch_probe_moves_t(const qw_index *ix, const E *x, int64_t Q, uint8_t *moves, int32_t *hout,
                          uint32_t *clear, int32_t nclear, hipStream_t s)
{
    const dim3 g((unsigned)ceil_div(Q, kBlock), (unsigned)ix->L);
    const double *a = ix->a64l.as<double>();
    const float *b = ix->b32.as<float>();
    const int32_t T = ix->nprobe - 1;
    const double w = (double)ix->w;
#define QW_PM(KM, EX) probe_moves_kernel<E, KM, EX><<<g, kBlock, 0, s>>>(x, Q, ix->dp, a, b, ix->L, ix->k, w, T, moves, hout, clear, nclear)
    switch (ix->k) {
    case 8: QW_PM(8, true); break;
    case 10: QW_PM(10, true); break;
    case 12: QW_PM(12, true); break;
    case 16: QW_PM(16, true); break;
    default:
        if (ix->k < 8) QW_PM(8, false);
        else if (ix->k < 16) QW_PM(16, false);
        else QW_PM(kMaxK, false);
    }
#undef QW_PM
}

qw_status launch_probe_moves(const qw_index *ix, const void *xpad, int64_t Q, uint8_t *moves,
                             int32_t *hout, hipStream_t s, uint32_t *clear, int32_t nclear)
{
    if (Q <= 0) return clear ? launch_fill_u32(clear, 0u, nclear, s) : QW_OK;
    if (ix->k > kMaxK || ix->nprobe - 1 > 2 * ix->k || !ix->a64l.p || nclear < 0) return QW_EINTERNAL;
    if (ix->dtype == QW_U8)
        launch_probe_moves_t<uint8_t>(ix, (const uint8_t *)xpad, Q, moves, hout, clear, nclear, s);
    else
        launch_probe_moves_t<float>(ix, (const float *)xpad, Q, moves, hout, clear, nclear, s);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// ---------------------------------------------------------------- probe
// One thread per (query, layer), for all of the layer's P probes: probe 0 is
// the query's own bucket; with neighbour probing (P = 2k + 1) probe
// 1 + 2j + s moves hash value j by -1 (s = 0) or +1 (s = 1), the buckets next
// to the query's in one coordinate (the multi-probe variant summarised in
// Section 2); query-directed (moves non-null, P = T + 1) probe 1 + t takes
// the layer's t-th chosen move.  The k values are packed into the exact key
// once; a probe replaces one field.  Values outside the data's range cannot
// match any bucket: such a key is a miss and is never looked up.  Each key is
// looked up in the layer's open-addressing table, kProbeBatch keys with their
// first slots in flight together.  Outputs are [Q][L][P]; bmh (nullable)
// receives the bucket's min-hash (0xFFFFFFFF on a miss).  Per layer [Q][L]
// (each nullable): feats the count-model input log(1 + s) of the layer's size
// s (summed over its probes), lsum s itself and lmh the minimum of its
// probes' min-hashes.  KM: k itself (KEXACT) or a bound on it (functions past
// k skipped).
constexpr int kProbeBatch = 4;
// linear probing, two slots (one 64-byte line) per round trip: at a load
// factor of at most 1/2 most sequences, hits and misses, end within the first
// pair
constexpr uint32_t kProbeRound = 2;

// Looks up the P probes of one (query, layer) and writes their outputs (see
// probe_kernel).  klo/khi: the base key over the fields in range; nbad of
// them out of range, the last badj.  field(j, lo, hi, sh, hj): function j's
// value range, key offset and hash value; move(p): the move of probe p >= 1.
template <class Field, class Move>
__device__ inline void probe_layer(int32_t P, uint64_t klo, uint64_t khi, int32_t nbad,
                                   int32_t badj, const TabEntry *__restrict__ t, uint32_t mask,
                                   Field field, Move move, int64_t ql, uint32_t *__restrict__ bstart,
                                   uint32_t *__restrict__ bsize, uint32_t *__restrict__ bmh,
                                   float *__restrict__ feats, uint32_t *__restrict__ lsum,
                                   uint32_t *__restrict__ lmh)
{
    uint32_t lsz = 0, lm = 0xFFFFFFFFu;  // the layer's size sum and min-hash over its probes
    for (int32_t p0 = 0; p0 < P; p0 += kProbeBatch) {
        uint64_t kl[kProbeBatch], kh[kProbeBatch];
        uint32_t slot[kProbeBatch];
        bool look[kProbeBatch];
#pragma unroll
        for (int b = 0; b < kProbeBatch; ++b) {
            const int32_t p = p0 + b;
            kl[b] = klo;
            kh[b] = khi;
            look[b] = false;
            if (p >= P) continue;
            if (p == 0) {
                look[b] = nbad == 0;
            } else {  // one value moved by one
                const int32_t mv = move(p);
                const int32_t j = mv >> 1;
                int32_t lo, hi, sh, hj32;
                field(j, lo, hi, sh, hj32);
                const int64_t hj = (int64_t)hj32;
                const int64_t nv = hj + (mv & 1 ? 1 : -1);
                const bool in_old = hj >= lo && hj <= hi;
                look[b] = (nbad == 0 || (nbad == 1 && badj == j)) && nv >= lo && nv <= hi;
                if (look[b]) {  // replace field j: the base holds it only when it was in range
                    const uint64_t oldv = in_old ? (uint64_t)(hj - lo) : 0u;
                    const uint64_t newv = (uint64_t)(nv - lo);
                    if (sh < 64) kl[b] = kl[b] - (oldv << sh) + (newv << sh);
                    else kh[b] = kh[b] - (oldv << (sh - 64)) + (newv << (sh - 64));
                }
            }
        }
        TabEntry e[kProbeBatch][kProbeRound];
#pragma unroll
        for (int b = 0; b < kProbeBatch; ++b) {
            slot[b] = (uint32_t)key_mix(kl[b], kh[b]) & mask;
            if (look[b])
#pragma unroll
                for (uint32_t i = 0; i < kProbeRound; ++i) e[b][i] = t[(slot[b] + i) & mask];
        }
#pragma unroll
        for (int b = 0; b < kProbeBatch; ++b) {
            const int32_t p = p0 + b;
            if (p >= P) continue;
            uint32_t st = 0, sz = 0, mh = 0xFFFFFFFFu;
            if (look[b]) {
                bool done = false;
                for (uint32_t it = 0; !done; it += kProbeRound) {
                    if (it > 0) {  // rare: the first pair held other keys
                        if (it > mask) break;
                        slot[b] = (slot[b] + kProbeRound) & mask;
#pragma unroll
                        for (uint32_t i = 0; i < kProbeRound; ++i) e[b][i] = t[(slot[b] + i) & mask];
                    }
#pragma unroll
                    for (uint32_t i = 0; i < kProbeRound; ++i) {
                        if (done) continue;
                        if (e[b][i].size == 0) {
                            done = true;
                        } else if (e[b][i].klo == kl[b] && e[b][i].khi == kh[b]) {
                            st = e[b][i].start;
                            sz = e[b][i].size;
                            mh = e[b][i].mh;
                            done = true;
                        }
                    }
                }
            }
            const int64_t o = ql * P + p;
            bstart[o] = st;
            bsize[o] = sz;
            if (bmh) bmh[o] = mh;
            lsz += sz;
            lm = min(lm, mh);
        }
    }
    if (feats) feats[ql] = log1pf((float)lsz);  // count-model input, f = log(1 + s)
    if (lsum) lsum[ql] = lsz;
    if (lmh) lmh[ql] = lm;
}

template <int KM, bool KEXACT>
__global__ __launch_bounds__(kBlock) void probe_kernel(
    const int32_t *__restrict__ h, int64_t Q, int32_t L, int32_t k, int32_t P,
    const int32_t *__restrict__ hmin, const int32_t *__restrict__ hmax,
    const int32_t *__restrict__ shift, const TabEntry *__restrict__ tab,
    const long long *__restrict__ tab_off, const uint32_t *__restrict__ tab_mask,
    uint32_t *__restrict__ bstart, uint32_t *__restrict__ bsize, float *__restrict__ feats,
    uint32_t *__restrict__ bmh, const uint8_t *__restrict__ moves, uint32_t *__restrict__ lsum,
    uint32_t *__restrict__ lmh)
{
    // per-function constants (value range, bit offset in the key) staged in
    // LDS while the hash values load: one memory latency for both
    extern __shared__ int32_t fconst[];  // [3][nf]: hmin, hmax, shift
    const int32_t nf = L * k;
    for (int32_t f = threadIdx.x; f < nf; f += kBlock) {
        fconst[f] = hmin[f];
        fconst[nf + f] = hmax[f];
        fconst[2 * nf + f] = shift[f];
    }
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = idx < Q * L;
    const int64_t ql = live ? idx : 0;
    const int64_t q = ql / L;
    const int32_t l = (int32_t)(ql - q * L);
    const int32_t *hl = h + q * nf + l * k;
    // the layer's k hash values, all loads issued before any is used
    int32_t hv[KM];
#pragma unroll
    for (int32_t j = 0; j < KM; ++j)
        if (KEXACT || j < k) hv[j] = hl[j];
    const TabEntry *t = tab + tab_off[l];
    const uint32_t mask = tab_mask[l];
    __syncthreads();
    if (!live) return;
    // the base key from the fields in range; nbad fields out of range, the
    // last of them badj
    uint64_t klo = 0, khi = 0;
    int32_t nbad = 0, badj = -1;
#pragma unroll
    for (int32_t j = 0; j < KM; ++j)
        if (KEXACT || j < k) {
            const int32_t f = l * k + j, lo = fconst[f];
            if (hv[j] >= lo && hv[j] <= fconst[nf + f]) {
                key_put(klo, khi, (uint64_t)((int64_t)hv[j] - (int64_t)lo), fconst[2 * nf + f]);
            } else {
                ++nbad;
                badj = j;
            }
        }
    auto field = [&](int32_t j, int32_t &lo, int32_t &hi, int32_t &sh, int32_t &hj) {
        const int32_t f = l * k + j;
        lo = fconst[f];
        hi = fconst[nf + f];
        sh = fconst[2 * nf + f];
        hj = hl[j];
    };
    auto move = [&](int32_t p) { return moves ? (int32_t)moves[ql * (P - 1) + (p - 1)] : p - 1; };
    probe_layer(P, klo, khi, nbad, badj, t, mask, field, move, ql, bstart, bsize, bmh, feats, lsum,
                lmh);
}

qw_status launch_probe(const qw_index *ix, const int32_t *h, int64_t Q, uint32_t *bstart,
                       uint32_t *bsize, float *feats, uint32_t *bmh, const uint8_t *moves,
                       uint32_t *lsum, uint32_t *lmh, hipStream_t s)
{
    if (Q <= 0) return QW_OK;
    if (ix->k > kMaxK) return QW_EINTERNAL;
    const unsigned g = (unsigned)ceil_div(Q * ix->L, kBlock);
    const size_t lds = sizeof(int32_t) * 3 * (size_t)ix->nf;  // nf <= 64 * kMaxK: 24 KiB at most
#define QW_PR(KM, EX)                                                                            \
    probe_kernel<KM, EX><<<g, kBlock, lds, s>>>(                                                  \
        h, Q, ix->L, ix->k, ix->nprobe, ix->hmin.as<int32_t>(), ix->hmax.as<int32_t>(),          \
        ix->shift.as<int32_t>(), ix->tab.as<TabEntry>(), ix->tab_off.as<long long>(),            \
        ix->tab_mask.as<uint32_t>(), bstart, bsize, feats, bmh, moves, lsum, lmh)
    switch (ix->k) {
    case 8: QW_PR(8, true); break;
    case 10: QW_PR(10, true); break;
    case 12: QW_PR(12, true); break;
    case 16: QW_PR(16, true); break;
    default:
        if (ix->k < 8) QW_PR(8, false);
        else if (ix->k < 16) QW_PR(16, false);
        else QW_PR(kMaxK, false);
    }
#undef QW_PR
    QW_HIP(hipGetLastError());
    return QW_OK;
}


}  // namespace qw
