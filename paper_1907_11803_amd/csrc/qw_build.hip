// Index construction: L layers of k p-stable functions (Sections 1.1 and 3).
//
// Per layer: hash every point (the same exact hashing as the query path), pack
// the k-tuple into an exact key, group equal keys through a temporary
// open-addressing table (one slot per distinct key, claimed by CAS), number the
// occupied slots with a prefix sum (bucket ids), lay the buckets out as CSR id
// lists, and store every bucket in a compact probe table keyed by its packed key.
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "qw_internal.h"
#include "qw_keys.h"

namespace qw {

// ---------------------------------------------------------------- kernels

// The parameters in FP64, layer-major: out[l][e][j] = a[l * k + j][e] (a: the
// zero-padded [nf_pad][dp] rows; L layers of k functions, dp elements).
__global__ void params_f64_kernel(const float *__restrict__ a, int32_t L, int32_t k, int32_t dp,
                                  double *__restrict__ out)
{
    const int64_t total = (int64_t)L * k * dp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = i / dp, e = i - f * dp;  // function f = l * k + j
        const int64_t l = f / k, j = f - l * k;
        out[(l * dp + e) * k + j] = (double)a[i];
    }
}

__global__ void maxabs_f32_kernel(const float *__restrict__ x, int64_t count, uint32_t *out)
{
    float m = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        float v = fabsf(x[i]);
        m = (v > m || v != v) ? v : m;  // NaN propagates (rejected later)
    }
    for (int off = 32; off > 0; off >>= 1) {
        float o = __shfl_xor(m, off);
        m = (o > m || o != o) ? o : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ __launch_bounds__(kBlock) void minmax_kernel(const int32_t *__restrict__ h, int64_t n,
                                                        int32_t ld, int32_t rows_per_block,
                                                        int32_t *hmin, int32_t *hmax)
{
    __shared__ int32_t smin[kBlock / 64], smax[kBlock / 64];
    const int f = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    int32_t mn = INT32_MAX, mx = INT32_MIN;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        int32_t v = h[r * ld + f];
        mn = min(mn, v);
        mx = max(mx, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        mn = min(mn, __shfl_xor(mn, off));
        mx = max(mx, __shfl_xor(mx, off));
    }
    if ((threadIdx.x & 63) == 0) {
        smin[threadIdx.x >> 6] = mn;
        smax[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            mn = min(mn, smin[w]);
            mx = max(mx, smax[w]);
        }
        atomicMin(&hmin[f], mn);
        atomicMax(&hmax[f], mx);
    }
}

// Packed key of layer-local functions [col0, col0+k) of every row.
__global__ void pack_kernel(const int32_t *__restrict__ h, int64_t n, int32_t ld, int32_t col0,
                            int32_t k, const int32_t *__restrict__ hmin,
                            const int32_t *__restrict__ shift, uint64_t *__restrict__ klo,
                            uint64_t *__restrict__ khi)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        uint64_t lo = 0, hi = 0;
        for (int32_t j = 0; j < k; ++j)
            key_put(lo, hi, (uint64_t)((int64_t)h[p * ld + col0 + j] - (int64_t)hmin[j]), shift[j]);
        klo[p] = lo;
        khi[p] = hi;
    }
}

// Temporary table: rep[slot] = first point that claimed the slot, cnt[slot] =
// number of points with that key.  Capacity >= 2n, so probing always ends.
__global__ void tinsert_kernel(const uint64_t *__restrict__ klo, const uint64_t *__restrict__ khi,
                               int64_t n, uint32_t *rep, uint32_t *cnt, uint32_t mask,
                               uint32_t *__restrict__ slot_of)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t lo = klo[p], hi = khi[p];
        uint32_t slot = (uint32_t)key_mix(lo, hi) & mask;
        for (uint32_t it = 0; it <= mask; ++it) {
            uint32_t cur = rep[slot];
            if (cur == kEmpty) {
                uint32_t old = atomicCAS(&rep[slot], kEmpty, (uint32_t)p);
                cur = old == kEmpty ? (uint32_t)p : old;
            }
            if (cur == (uint32_t)p || (klo[cur] == lo && khi[cur] == hi)) {
                atomicAdd(&cnt[slot], 1u);
                slot_of[p] = slot;
                break;
            }
            slot = (slot + 1) & mask;
        }
    }
}

__global__ void occupied_kernel(const uint32_t *__restrict__ rep, int64_t cap, uint32_t *occ)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < cap;
         s += (int64_t)gridDim.x * blockDim.x)
        occ[s] = rep[s] != kEmpty ? 1u : 0u;
}

__global__ void bucket_compact_kernel(const uint32_t *__restrict__ rep,
                                      const uint32_t *__restrict__ cnt, int64_t cap,
                                      const unsigned long long *__restrict__ bidx,
                                      uint32_t *__restrict__ bsize, uint32_t *__restrict__ brep,
                                      uint32_t *maxb)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < cap;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (rep[s] == kEmpty) continue;
        const unsigned long long b = bidx[s];
        bsize[b] = cnt[s];
        brep[b] = rep[s];
        atomicMax(maxb, cnt[s]);
    }
}

// *out += sum over the nb buckets of size^2 (one atomic per workgroup): with
// the layer's n points, sum s^2 / n is the mean size of the bucket a point
// (or a query near the data) falls in
__global__ void sumsq_kernel(const uint32_t *__restrict__ bsize, int64_t nb, unsigned long long *out)
{
    __shared__ unsigned long long part[kBlock / 64];
    unsigned long long acc = 0;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x)
        acc += (unsigned long long)bsize[b] * bsize[b];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        if (t) atomicAdd(out, t);
    }
}

__global__ void bucket_scatter_kernel(const uint32_t *__restrict__ slot_of, int64_t n,
                                      const unsigned long long *__restrict__ bidx,
                                      const unsigned long long *__restrict__ bstart,
                                      uint32_t *cursor, int32_t *__restrict__ ids)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long b = bidx[slot_of[p]];
        const uint32_t pos = atomicAdd(&cursor[b], 1u);
        ids[bstart[b] + pos] = (int32_t)p;
    }
}

__global__ void final_table_kernel(const uint32_t *__restrict__ bsize,
                                   const uint32_t *__restrict__ brep,
                                   const unsigned long long *__restrict__ bstart, int64_t nb,
                                   const uint64_t *__restrict__ klo,
                                   const uint64_t *__restrict__ khi,
                                   const int32_t *__restrict__ ids, TabEntry *tab, uint32_t mask)
{
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t lo = klo[brep[b]], hi = khi[brep[b]];
        const uint32_t st = (uint32_t)bstart[b], sz = bsize[b];
        uint32_t mh = 0xFFFFFFFFu;  // the bucket's min-hash (ids is the layer's CSR)
        for (uint32_t i = 0; i < sz; ++i) mh = min(mh, id_mix((uint32_t)ids[st + i]));
        uint32_t slot = (uint32_t)key_mix(lo, hi) & mask;
        for (uint32_t it = 0; it <= mask; ++it) {
            if (atomicCAS(&tab[slot].size, 0u, sz) == 0u) {
                tab[slot].klo = lo;
                tab[slot].khi = hi;
                tab[slot].mh = mh;
                tab[slot].start = st;
                break;
            }
            slot = (slot + 1) & mask;
        }
    }
}

static int grid_of(int64_t count)
{
    int64_t g = ceil_div(count, kBlock);
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// ---------------------------------------------------------------- host side

static double gamma_n(double n, double u) { return n * u / (1.0 - n * u); }

// Guard-band coefficients and FP16 split (host, FP64).  coef * max|v| bounds
// |approximate projection - FP64 index-order projection|.
static void hash_constants(const std::vector<float> &a, int32_t nf, int32_t d, int32_t dp,
                           bool u8, std::vector<double> &gb_plain, std::vector<double> &gb_fast,
                           std::vector<_Float16> &ahi, std::vector<_Float16> &alo,
                           bool &use_f16, std::vector<double> &anorm)
{
    const double u32 = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
    const double g32 = gamma_n(d + 2, u32), g64 = gamma_n(d + 2, u64);
    // FP32 matrix cores, float data: FP32 within each chunk of kHashChunkF32
    // elements (factor 2: unknown internal order), FP64 over the chunk sums
    const double g32c = gamma_n(kHashChunkF32 + 3, u32);
    const double g64c = gamma_n((dp + kHashChunkF32 - 1) / kHashChunkF32 + 1, u64);
    gb_plain.assign(nf, 0.0);
    gb_fast.assign(nf, 0.0);
    anorm.assign(nf, 0.0);
    float amax = 0.f;
    for (float v : a) amax = std::max(amax, std::fabs(v));
    use_f16 = u8 && amax < 32768.f;
    if (use_f16) {
        ahi.assign((size_t)nf * dp, (_Float16)0.f);
        alo.assign((size_t)nf * dp, (_Float16)0.f);
    }
    for (int32_t f = 0; f < nf; ++f) {
        double an = 0.0, ahn = 0.0, aln = 0.0, rep = 0.0;
        for (int32_t i = 0; i < d; ++i) {
            const float v = a[(size_t)f * d + i];
            an += std::fabs((double)v);
            if (use_f16) {
                _Float16 h = (_Float16)v;
                float r = v - (float)h;  // exact: h is v rounded to 11 bits
                _Float16 l = (_Float16)r;
                if (std::fabs((float)l) < 6.103515625e-05f) l = (_Float16)0.f;  // no FP16 subnormals
                ahi[(size_t)f * dp + i] = h;
                alo[(size_t)f * dp + i] = l;
                ahn += std::fabs((double)(float)h);
                aln += std::fabs((double)(float)l);
                rep += std::fabs((double)v - (double)(float)h - (double)(float)l);
            }
        }
        const double safety = 1.0 + 1e-6;
        an *= safety;
        anorm[f] = an;
        gb_plain[f] = (g32 + g64) * an * safety;
        if (use_f16)
            gb_fast[f] = (rep * safety + 2.0 * g32 * (ahn + aln) * safety + g64 * an) * safety;
        else
            gb_fast[f] = (2.0 * g32c + g64c + g64) * an * safety;
    }
}

qw_status build_index(const void *data, int64_t n, int32_t d, int32_t dtype, const float *a,
                      const float *b, float w, int32_t L, int32_t k, int32_t form,
                      hipStream_t s, qw_index **out)
{
    std::unique_ptr<qw_index> ix(new qw_index());
    QW_HIP(hipGetDevice(&ix->device));
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, ix->device) == hipSuccess && v > 0)
        ix->cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device) == hipSuccess && v > 0)
        ix->lds_max = (size_t)v;
    QW_HIP(hipStreamCreateWithFlags(&ix->side, hipStreamNonBlocking));
    for (auto &e : ix->fork) QW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ix->n = n;
    ix->d = d;
    ix->dp = (int32_t)((d + 15) / 16 * 16);
    ix->dtype = dtype;
    ix->L = L;
    ix->nprobe = 1;
    ix->nl = L;
    ix->pmagic = 0;
    ix->k = k;
    ix->nf = L * k;
    // one extra 64-row tile: function tiles may start at any f0 during the build
    ix->nf_pad = (int32_t)((ix->nf + 63) / 64 * 64 + 64);
    ix->w = w;
    const int32_t nf = ix->nf, dp = ix->dp;

    // parameters to host for the guard-band constants
    std::vector<float> ha((size_t)nf * d), hb(nf);
    QW_HIP(hipMemcpyAsync(ha.data(), a, sizeof(float) * ha.size(), hipMemcpyDeviceToHost, s));
    QW_HIP(hipMemcpyAsync(hb.data(), b, sizeof(float) * hb.size(), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    for (float x : ha)
        if (!std::isfinite(x)) return QW_EINVAL;
    for (float x : hb)
        if (!std::isfinite(x)) return QW_EINVAL;
    std::vector<double> gbp, gbf, anorm;
    std::vector<_Float16> ahi, alo;
    bool use_f16 = false;
    hash_constants(ha, nf, d, dp, dtype == QW_U8, gbp, gbf, ahi, alo, use_f16, anorm);
    ix->fast_f16 = use_f16;

    QW_TRY(ix->a32.ensure(sizeof(float) * (size_t)ix->nf_pad * dp));
    QW_HIP(hipMemsetAsync(ix->a32.p, 0, ix->a32.bytes, s));
    QW_TRY(launch_pad_rows(a, nf, d, dp, QW_F32, ix->a32.p, s));
    QW_TRY(ix->a64l.ensure(sizeof(double) * (size_t)nf * dp));
    params_f64_kernel<<<grid_of((int64_t)nf * dp), kBlock, 0, s>>>(ix->a32.as<float>(), L, k, dp,
                                                                  ix->a64l.as<double>());
    QW_HIP(hipGetLastError());
    QW_TRY(ix->b32.ensure(sizeof(float) * nf));
    QW_HIP(hipMemcpyAsync(ix->b32.p, b, sizeof(float) * nf, hipMemcpyDeviceToDevice, s));
    QW_TRY(ix->gb_plain.ensure(sizeof(double) * nf));
    QW_TRY(ix->gb_fast.ensure(sizeof(double) * nf));
    QW_HIP(hipMemcpyAsync(ix->gb_plain.p, gbp.data(), sizeof(double) * nf, hipMemcpyHostToDevice, s));
    QW_HIP(hipMemcpyAsync(ix->gb_fast.p, gbf.data(), sizeof(double) * nf, hipMemcpyHostToDevice, s));
    if (use_f16) {
        const size_t bytes = sizeof(_Float16) * (size_t)ix->nf_pad * dp;
        QW_TRY(ix->a_hi.ensure(bytes));
        QW_TRY(ix->a_lo.ensure(bytes));
        QW_HIP(hipMemsetAsync(ix->a_hi.p, 0, bytes, s));
        QW_HIP(hipMemsetAsync(ix->a_lo.p, 0, bytes, s));
        QW_HIP(hipMemcpyAsync(ix->a_hi.p, ahi.data(), sizeof(_Float16) * ahi.size(),
                              hipMemcpyHostToDevice, s));
        QW_HIP(hipMemcpyAsync(ix->a_lo.p, alo.data(), sizeof(_Float16) * alo.size(),
                              hipMemcpyHostToDevice, s));
    }

    // data copy with padded rows
    const size_t elem = dtype == QW_U8 ? 1 : 4;
    QW_TRY(ix->data.ensure(elem * (size_t)n * dp));
    QW_TRY(launch_pad_rows(data, n, d, dp, dtype, ix->data.p, s));

    // |a.v + b| / w must stay far inside int32
    double vmax = 255.0;
    DevBuf tmp32;
    if (dtype == QW_F32) {
        QW_TRY(tmp32.ensure(sizeof(uint32_t)));
        QW_TRY(launch_fill_u32(tmp32.as<uint32_t>(), 0u, 1, s));
        maxabs_f32_kernel<<<grid_of(n * (int64_t)dp), kBlock, 0, s>>>(ix->data.as<float>(),
                                                                     n * (int64_t)dp,
                                                                     tmp32.as<uint32_t>());
        QW_HIP(hipGetLastError());
        uint32_t bits = 0;
        QW_HIP(hipMemcpyAsync(&bits, tmp32.p, 4, hipMemcpyDeviceToHost, s));
        QW_HIP(hipStreamSynchronize(s));
        float fm;
        std::memcpy(&fm, &bits, 4);
        if (!std::isfinite(fm)) return QW_EINVAL;
        vmax = fm;
    }
    for (int32_t f = 0; f < nf; ++f)
        if ((anorm[f] * vmax + std::fabs((double)hb[f])) / (double)w + 2.0 >= std::ldexp(1.0, 30))
            return QW_EINVAL;

    // per-function key ranges and shifts
    QW_TRY(ix->hmin.ensure(sizeof(int32_t) * nf));
    QW_TRY(ix->hmax.ensure(sizeof(int32_t) * nf));
    QW_TRY(ix->shift.ensure(sizeof(int32_t) * nf));
    std::vector<int32_t> hmin(nf), hmax(nf), shift(nf, 0);
    ix->key_bits.assign(L, 0);
    QW_TRY(ix->ids.ensure(sizeof(int32_t) * (size_t)L * n));

    // temporaries
    const int64_t chunk_layers = std::max<int64_t>(1, std::min<int64_t>(L, (int64_t(1) << 28) / std::max<int64_t>(1, n * k)));
    DevBuf hbuf, klo, khi, slot_of, trep, tcnt, occ, bidx, bsize, brep, bstart, cursor, scan, maxb, sq;
    int ct_log2 = std::max(10, ceil_log2((uint64_t)(2 * n)));
    const int64_t ct = int64_t(1) << ct_log2;
    QW_TRY(hbuf.ensure(sizeof(int32_t) * (size_t)n * chunk_layers * k));
    QW_TRY(klo.ensure(sizeof(uint64_t) * n));
    QW_TRY(khi.ensure(sizeof(uint64_t) * n));
    QW_TRY(slot_of.ensure(sizeof(uint32_t) * n));
    QW_TRY(trep.ensure(sizeof(uint32_t) * ct));
    QW_TRY(tcnt.ensure(sizeof(uint32_t) * ct));
    QW_TRY(occ.ensure(sizeof(uint32_t) * ct));
    QW_TRY(bidx.ensure(sizeof(unsigned long long) * (ct + 1)));
    QW_TRY(bsize.ensure(sizeof(uint32_t) * (n + 1)));
    QW_TRY(brep.ensure(sizeof(uint32_t) * (n + 1)));
    QW_TRY(bstart.ensure(sizeof(unsigned long long) * (n + 2)));
    QW_TRY(cursor.ensure(sizeof(uint32_t) * (n + 1)));
    QW_TRY(maxb.ensure(sizeof(uint32_t)));
    QW_TRY(launch_fill_u32(maxb.as<uint32_t>(), 0u, 1, s));
    QW_TRY(sq.ensure(sizeof(unsigned long long) * L));  // per layer: sum of bucket size^2
    QW_TRY(launch_fill_u32(sq.as<uint32_t>(), 0u, 2 * (int64_t)L, s));

    std::vector<DevBuf> tabs(L);
    std::vector<uint32_t> masks(L);

    for (int32_t l0 = 0; l0 < L; l0 += (int32_t)chunk_layers) {
        const int32_t nl = (int32_t)std::min<int64_t>(chunk_layers, L - l0);
        const int32_t f0 = l0 * k, nfun = nl * k;
        QW_TRY(launch_hash(ix.get(), ix->data.p, n, f0, nfun, form, hbuf.as<int32_t>(), nfun,
                           nullptr, s));
        QW_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ix->hmin.as<int32_t>() + f0),
                               (uint32_t)INT32_MAX, nfun, s));
        QW_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ix->hmax.as<int32_t>() + f0),
                               (uint32_t)INT32_MIN, nfun, s));
        const int32_t rpb = 8192;
        dim3 mg((unsigned)ceil_div(n, rpb), (unsigned)nfun);
        minmax_kernel<<<mg, kBlock, 0, s>>>(hbuf.as<int32_t>(), n, nfun, rpb,
                                            ix->hmin.as<int32_t>() + f0, ix->hmax.as<int32_t>() + f0);
        QW_HIP(hipGetLastError());
        QW_HIP(hipMemcpyAsync(hmin.data() + f0, ix->hmin.as<int32_t>() + f0, sizeof(int32_t) * nfun,
                              hipMemcpyDeviceToHost, s));
        QW_HIP(hipMemcpyAsync(hmax.data() + f0, ix->hmax.as<int32_t>() + f0, sizeof(int32_t) * nfun,
                              hipMemcpyDeviceToHost, s));
        QW_HIP(hipStreamSynchronize(s));
        for (int32_t l = l0; l < l0 + nl; ++l) {
            int32_t pos = 0;
            for (int32_t j = 0; j < k; ++j) {
                const int32_t f = l * k + j;
                const uint64_t range = (uint64_t)((int64_t)hmax[f] - (int64_t)hmin[f]) + 1;
                const int32_t bits = range <= 1 ? 0 : ceil_log2(range);
                if (pos < 64 && pos + bits > 64) pos = 64;
                shift[f] = pos;
                pos += bits;
            }
            if (pos > 128) return QW_EUNSUPPORTED;
            ix->key_bits[l] = pos;
        }
        QW_HIP(hipMemcpyAsync(ix->shift.as<int32_t>() + f0, shift.data() + f0,
                              sizeof(int32_t) * nfun, hipMemcpyHostToDevice, s));

        for (int32_t l = l0; l < l0 + nl; ++l) {
            const int32_t col0 = (l - l0) * k;
            pack_kernel<<<grid_of(n), kBlock, 0, s>>>(hbuf.as<int32_t>(), n, nfun, col0, k,
                                                      ix->hmin.as<int32_t>() + l * k,
                                                      ix->shift.as<int32_t>() + l * k,
                                                      klo.as<uint64_t>(), khi.as<uint64_t>());
            QW_HIP(hipGetLastError());
            QW_TRY(launch_fill_u32(trep.as<uint32_t>(), kEmpty, ct, s));
            QW_TRY(launch_fill_u32(tcnt.as<uint32_t>(), 0u, ct, s));
            tinsert_kernel<<<grid_of(n), kBlock, 0, s>>>(klo.as<uint64_t>(), khi.as<uint64_t>(), n,
                                                         trep.as<uint32_t>(), tcnt.as<uint32_t>(),
                                                         (uint32_t)(ct - 1), slot_of.as<uint32_t>());
            QW_HIP(hipGetLastError());
            occupied_kernel<<<grid_of(ct), kBlock, 0, s>>>(trep.as<uint32_t>(), ct, occ.as<uint32_t>());
            QW_HIP(hipGetLastError());
            QW_TRY(launch_scan_u32_to_u64(occ.as<uint32_t>(), ct, bidx.as<unsigned long long>(), scan, s));
            unsigned long long nb = 0;
            QW_HIP(hipMemcpyAsync(&nb, bidx.as<unsigned long long>() + ct, sizeof(nb),
                                  hipMemcpyDeviceToHost, s));
            QW_HIP(hipStreamSynchronize(s));
            if ((int64_t)nb > n || nb == 0) return QW_EINTERNAL;
            bucket_compact_kernel<<<grid_of(ct), kBlock, 0, s>>>(
                trep.as<uint32_t>(), tcnt.as<uint32_t>(), ct, bidx.as<unsigned long long>(),
                bsize.as<uint32_t>(), brep.as<uint32_t>(), maxb.as<uint32_t>());
            QW_HIP(hipGetLastError());
            sumsq_kernel<<<grid_of((int64_t)nb), kBlock, 0, s>>>(bsize.as<uint32_t>(), (int64_t)nb,
                                                               sq.as<unsigned long long>() + l);
            QW_HIP(hipGetLastError());
            QW_TRY(launch_scan_u32_to_u64(bsize.as<uint32_t>(), (int64_t)nb,
                                          bstart.as<unsigned long long>(), scan, s));
            QW_TRY(launch_fill_u32(cursor.as<uint32_t>(), 0u, (int64_t)nb, s));
            bucket_scatter_kernel<<<grid_of(n), kBlock, 0, s>>>(
                slot_of.as<uint32_t>(), n, bidx.as<unsigned long long>(),
                bstart.as<unsigned long long>(), cursor.as<uint32_t>(),
                ix->ids.as<int32_t>() + (int64_t)l * n);
            QW_HIP(hipGetLastError());
            const int fl = std::max(6, ceil_log2(2 * nb));
            const int64_t fc = int64_t(1) << fl;
            QW_TRY(tabs[l].ensure(sizeof(TabEntry) * fc));
            QW_TRY(launch_fill_u32(tabs[l].as<uint32_t>(), 0u, (int64_t)(sizeof(TabEntry) / 4) * fc, s));
            final_table_kernel<<<grid_of((int64_t)nb), kBlock, 0, s>>>(
                bsize.as<uint32_t>(), brep.as<uint32_t>(), bstart.as<unsigned long long>(),
                (int64_t)nb, klo.as<uint64_t>(), khi.as<uint64_t>(),
                ix->ids.as<int32_t>() + (int64_t)l * n, tabs[l].as<TabEntry>(),
                (uint32_t)(fc - 1));
            QW_HIP(hipGetLastError());
            masks[l] = (uint32_t)(fc - 1);
            ix->buckets += (int64_t)nb;
        }
    }
    // concatenate the probe tables
    std::vector<long long> off(L);
    int64_t total = 0;
    for (int32_t l = 0; l < L; ++l) {
        off[l] = total;
        total += (int64_t)masks[l] + 1;
    }
    QW_TRY(ix->tab.ensure(sizeof(TabEntry) * total));
    for (int32_t l = 0; l < L; ++l)
        QW_HIP(hipMemcpyAsync(ix->tab.as<TabEntry>() + off[l], tabs[l].p,
                              sizeof(TabEntry) * ((int64_t)masks[l] + 1), hipMemcpyDeviceToDevice, s));
    QW_TRY(ix->tab_off.ensure(sizeof(long long) * L));
    QW_TRY(ix->tab_mask.ensure(sizeof(uint32_t) * L));
    QW_HIP(hipMemcpyAsync(ix->tab_off.p, off.data(), sizeof(long long) * L, hipMemcpyHostToDevice, s));
    QW_HIP(hipMemcpyAsync(ix->tab_mask.p, masks.data(), sizeof(uint32_t) * L, hipMemcpyHostToDevice, s));
    uint32_t mb = 0;
    std::vector<unsigned long long> sqh(L);
    QW_HIP(hipMemcpyAsync(&mb, maxb.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    QW_HIP(hipMemcpyAsync(sqh.data(), sq.p, sizeof(unsigned long long) * L, hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    ix->max_bucket = mb;
    double sb = 0.0;
    for (int32_t l = 0; l < L; ++l) sb += (double)sqh[l] / (double)n;
    ix->mean_hit_bucket = sb / L;
    for (auto &t : tabs) t.release();
    *out = ix.release();
    return QW_OK;
}

}  // namespace qw
