// Device buffers, fills, row padding, prefix scan and a stable LSD radix sort.
#include <cstdio>
#include <cstdlib>
#include <algorithm>

#include "qw_internal.h"

namespace qw {

static thread_local char g_last_error[512];

void note_hip_error(hipError_t e, const char *what, const char *file, int line)
{
    std::snprintf(g_last_error, sizeof(g_last_error), "%s failed: %s (%s:%d)", what,
                  hipGetErrorString(e), file, line);
    if (std::getenv("QWLSH_VERBOSE"))
        std::fprintf(stderr, "qwlsh: %s\n", g_last_error);
}

qw_status DevBuf::ensure(size_t want)
{
    if (want <= bytes && p) return QW_OK;
    if (!owned) return QW_EINTERNAL;  // a view never allocates
    release();
    if (want == 0) want = 16;
    if (want > (SIZE_MAX >> 1)) return QW_ENOMEM;
    want = (want + 255) & ~size_t(255);
    // beyond the device's free memory: refused here, whatever the allocator
    // would do with it
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && want > free_b) return QW_ENOMEM;
    (void)hipGetLastError();
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        bytes = 0;
        return QW_ENOMEM;
    }
    bytes = want;
    return QW_OK;
}

void DevBuf::release()
{
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    owned = true;
}

// ---------------------------------------------------------------- fills

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void iota_kernel(int32_t *p, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

static int grid_for(int64_t count)
{
    int64_t g = ceil_div(count, kBlock);
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

qw_status launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s)
{
    if (count <= 0) return QW_OK;
    fill_u32_kernel<<<grid_for(count), kBlock, 0, s>>>(p, v, count);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

qw_status launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t count,
                          hipStream_t s)
{
    if (count <= 0) return QW_OK;
    fill_u64_kernel<<<grid_for(count), kBlock, 0, s>>>(p, v, count);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

qw_status launch_iota(int32_t *p, int64_t count, hipStream_t s)
{
    if (count <= 0) return QW_OK;
    iota_kernel<<<grid_for(count), kBlock, 0, s>>>(p, count);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// ---------------------------------------------------------------- row padding
// dst rows of dp elements: the first d copied from src rows of d elements, the rest 0.

template <typename T>
__global__ void pad_rows_kernel(const T *__restrict__ src, int64_t m, int32_t d, int32_t dp,
                                T *__restrict__ dst)
{
    const int64_t total = m * (int64_t)dp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i / dp;
        int32_t c = (int32_t)(i - r * dp);
        dst[i] = c < d ? src[r * d + c] : T(0);
    }
}

qw_status launch_pad_rows(const void *src, int64_t m, int32_t d, int32_t dp, int32_t dtype,
                          void *dst, hipStream_t s)
{
    if (m <= 0) return QW_OK;
    int g = grid_for(m * (int64_t)dp);
    if (dtype == QW_U8)
        pad_rows_kernel<uint8_t><<<g, kBlock, 0, s>>>((const uint8_t *)src, m, d, dp,
                                                      (uint8_t *)dst);
    else
        pad_rows_kernel<float><<<g, kBlock, 0, s>>>((const float *)src, m, d, dp, (float *)dst);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// ---------------------------------------------------------------- block scan helpers

// Exclusive scan of one value per thread over a 256-thread block; returns the
// exclusive prefix and writes the block total to *total (all threads).
template <typename T>
__device__ T block_exclusive_scan(T v, T *lds /* >= 4 entries */, T *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    T wave_base = 0, tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        T t = lds[w];
        if (w < wid) wave_base += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return wave_base + x - v;
}

// ---------------------------------------------------------------- device-wide exclusive scan
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void scan_tile_sums(const uint32_t *__restrict__ in,
                                                         int64_t count,
                                                         unsigned long long *__restrict__ sums)
{
    __shared__ unsigned long long lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    unsigned long long acc = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if (i < count) acc += in[i];
    }
    unsigned long long tot;
    (void)block_exclusive_scan<unsigned long long>(acc, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of `count` u64 values in place; writes the
// grand total to sums[count].
__global__ __launch_bounds__(kBlock) void scan_sums_single(unsigned long long *sums, int64_t count)
{
    __shared__ unsigned long long lds[4];
    unsigned long long carry = 0;
    for (int64_t base = 0; base < count; base += kBlock) {
        int64_t i = base + threadIdx.x;
        unsigned long long v = i < count ? sums[i] : 0;
        unsigned long long tot;
        unsigned long long ex = block_exclusive_scan<unsigned long long>(v, lds, &tot);
        if (i < count) sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[count] = carry;
}

__global__ __launch_bounds__(kBlock) void scan_tile_apply(const uint32_t *__restrict__ in,
                                                          int64_t count,
                                                          const unsigned long long *__restrict__ sums,
                                                          unsigned long long *__restrict__ out,
                                                          int64_t ntiles)
{
    __shared__ unsigned long long lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    // each thread owns kScanItems consecutive elements
    uint32_t v[kScanItems];
    unsigned long long loc = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        v[j] = i < count ? in[i] : 0u;
        loc += v[j];
    }
    unsigned long long tot;
    unsigned long long ex = block_exclusive_scan<unsigned long long>(loc, lds, &tot);
    unsigned long long run = sums[blockIdx.x] + ex;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        if (i < count) out[i] = run;
        run += v[j];
    }
    if (blockIdx.x == ntiles - 1 && threadIdx.x == 0) out[count] = sums[ntiles];
}

// Whole scan in one workgroup when count <= kScanTile.
__global__ __launch_bounds__(kBlock) void scan_small_kernel(const uint32_t *__restrict__ in,
                                                            int64_t count,
                                                            unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long lds[4];
    const int64_t base = (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    unsigned long long loc = 0;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        v[j] = i < count ? in[i] : 0u;
        loc += v[j];
    }
    unsigned long long tot;
    unsigned long long run = block_exclusive_scan<unsigned long long>(loc, lds, &tot);
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        if (i < count) out[i] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) out[count] = tot;
}

size_t scan_scratch_bytes(int64_t count)
{
    return sizeof(unsigned long long) * (ceil_div(std::max<int64_t>(count, 1), kScanTile) + 1);
}

qw_status launch_scan_u32_to_u64(const uint32_t *in, int64_t count, unsigned long long *out,
                                 DevBuf &scratch, hipStream_t s)
{
    if (count <= 0) {
        return launch_fill_u64(out, 0ull, 1, s);
    }
    int64_t ntiles = ceil_div(count, kScanTile);
    if (ntiles == 1) {  // one workgroup does it all
        scan_small_kernel<<<1, kBlock, 0, s>>>(in, count, out);
        QW_HIP(hipGetLastError());
        return QW_OK;
    }
    QW_TRY(scratch.ensure(scan_scratch_bytes(count)));
    auto *sums = scratch.as<unsigned long long>();
    scan_tile_sums<<<(unsigned)ntiles, kBlock, 0, s>>>(in, count, sums);
    QW_HIP(hipGetLastError());
    scan_sums_single<<<1, kBlock, 0, s>>>(sums, ntiles);
    QW_HIP(hipGetLastError());
    scan_tile_apply<<<(unsigned)ntiles, kBlock, 0, s>>>(in, count, sums, out, ntiles);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// ---------------------------------------------------------------- stable LSD radix sort
// 8-bit digits.  Per pass: per-tile digit histograms (digit-major), one
// exclusive scan over all (digit, tile) counters, and a scatter that ranks
// equal digits stably inside each tile with wavefront ballots.
constexpr int kRsItems = 16;
constexpr int kRsTile = kBlock * kRsItems;

__global__ __launch_bounds__(kBlock) void rs_hist_kernel(const unsigned long long *__restrict__ keys,
                                                         int64_t count, int shift,
                                                         uint32_t *__restrict__ hist, int64_t ntiles)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int j = 0; j < kRsItems; ++j) {
        int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if (i < count) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void rs_scatter_kernel(
    const unsigned long long *__restrict__ keys, const int32_t *__restrict__ vals, int64_t count,
    int shift, const unsigned long long *__restrict__ offs, int64_t ntiles,
    unsigned long long *__restrict__ kout, int32_t *__restrict__ vout)
{
    __shared__ unsigned long long base[256];
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kBlock / 64][256];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    base[t] = offs[(int64_t)t * ntiles + blockIdx.x];
    running[t] = 0;
    for (int w = 0; w < kBlock / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile = (int64_t)blockIdx.x * kRsTile;
    for (int j = 0; j < kRsItems; ++j) {
        const int64_t i = tile + (int64_t)j * kBlock + t;
        const bool valid = i < count;
        unsigned long long key = valid ? keys[i] : 0ull;
        int32_t val = valid ? vals[i] : 0;
        uint32_t dg = (uint32_t)((key >> shift) & 255u);
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            unsigned long long bal = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[wid][dg] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t before = 0;
            for (int w = 0; w < wid; ++w) before += wcnt[w][dg];
            unsigned long long pos = base[dg] + running[dg] + before + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            add += wcnt[w][t];
            wcnt[w][t] = 0;
        }
        running[t] += add;
        __syncthreads();
    }
}

size_t radix_sort_scratch_bytes(int64_t count)
{
    const int64_t ntiles = ceil_div(std::max<int64_t>(count, 1), kRsTile);
    const int64_t nh = ntiles * 256;
    const size_t off_bytes = ((sizeof(uint32_t) * nh + 255) & ~size_t(255));
    const int64_t scan_tiles = ceil_div(nh, kScanTile);
    return off_bytes + sizeof(unsigned long long) * (nh + 1) +
           sizeof(unsigned long long) * (scan_tiles + 1) + 256;
}

qw_status radix_sort_pairs(unsigned long long *keys, int32_t *vals, int64_t count, int bit_lo,
                           int bits, unsigned long long *keys_alt, int32_t *vals_alt, DevBuf &hist,
                           hipStream_t s, bool *result_in_alt)
{
    *result_in_alt = false;
    if (count <= 1 || bits <= bit_lo) return QW_OK;
    const int64_t ntiles = ceil_div(count, kRsTile);
    const int64_t nh = ntiles * 256;
    // hist: uint32 counters [nh], then uint64 offsets [nh + 1], then scan scratch
    const size_t off_bytes = ((sizeof(uint32_t) * nh + 255) & ~size_t(255));
    const int64_t scan_tiles = ceil_div(nh, kScanTile);
    QW_TRY(hist.ensure(radix_sort_scratch_bytes(count)));
    auto *h32 = hist.as<uint32_t>();
    auto *off64 = reinterpret_cast<unsigned long long *>(hist.as<char>() + off_bytes);
    auto *sums = off64 + nh + 1;
    unsigned long long *kin = keys, *kout = keys_alt;
    int32_t *vin = vals, *vout = vals_alt;
    for (int shift = bit_lo; shift < bits; shift += 8) {
        rs_hist_kernel<<<(unsigned)ntiles, kBlock, 0, s>>>(kin, count, shift, h32, ntiles);
        QW_HIP(hipGetLastError());
        if (scan_tiles == 1) {
            scan_small_kernel<<<1, kBlock, 0, s>>>(h32, nh, off64);
            QW_HIP(hipGetLastError());
        } else {
            scan_tile_sums<<<(unsigned)scan_tiles, kBlock, 0, s>>>(h32, nh, sums);
            QW_HIP(hipGetLastError());
            scan_sums_single<<<1, kBlock, 0, s>>>(sums, scan_tiles);
            QW_HIP(hipGetLastError());
            scan_tile_apply<<<(unsigned)scan_tiles, kBlock, 0, s>>>(h32, nh, sums, off64, scan_tiles);
            QW_HIP(hipGetLastError());
        }
        rs_scatter_kernel<<<(unsigned)ntiles, kBlock, 0, s>>>(kin, vin, count, shift, off64,
                                                              ntiles, kout, vout);
        QW_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
        *result_in_alt = !*result_in_alt;
    }
    return QW_OK;
}

}  // namespace qw
