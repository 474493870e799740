// Staged candidate kernel: the GPU form of the paper's split of a fixed cache
// between index files and data objects (Sections 4 and 5: C = C_I + C_D, the
// split chosen from the data's cardinality and dimensionality).  A workgroup
// takes runs of consecutive queries of the schedule's order (with bucket
// grouping, neighbouring queries share buckets) and keeps two caches in its
// LDS across them: bucket id lists (the index part, C_I) and candidate rows
// (the data part, C_D), their sizes set by the split.  A list or row found in
// its cache is read from LDS instead of the memory hierarchy.  Each query's
// unique candidates are verified and written as (distance, id) keys for the
// select kernel; queries that do not fit (a list total beyond the set, or no
// key space) are flagged for the fallback.  Caching changes no result.
#include "qw_dedup.h"
#include "qw_dist.h"
#include "qw_internal.h"

namespace qw {
namespace {

constexpr int kStageSetLog2 = 13;
constexpr uint32_t kStageSet = 1u << kStageSetLog2;   // set slots (32 KiB)
constexpr uint32_t kStageLimit = kStageSet / 4 * 3;   // list total at most (load <= 3/4)
constexpr uint32_t kNoTag = 0xFFFFFFFFu;
constexpr uint32_t kMissBit = 0x80000000u;            // ids are below 2^31
enum { S_T = 0, S_U, S_OVF, S_KP, S_CHUNK, S_OFF = 8 /* 2 words */, kScal = 16 };

// LDS layout in 32-bit words: the set, list prefix (65 -> 80 words), list
// offsets (64), miss flags of the lists (64), scalars (16), the query row
// (4 words per part), then the index cache (tags, then kStageIps ids per
// slot) and the data cache (tags, then the rows, 16-byte aligned).
struct StageLayout {
    uint32_t lpref, lstart, lmiss, scal, qrow, itag, icache, dtag, dcache, words;
};
__host__ __device__ inline uint32_t w4(uint32_t v) { return (v + 3u) & ~3u; }
__host__ __device__ inline StageLayout stage_layout(int parts, uint32_t icn, uint32_t dcn)
{
    StageLayout l;
    l.lpref = kStageSet;
    l.lstart = l.lpref + 80;
    l.lmiss = l.lstart + 64;
    l.scal = l.lmiss + 64;
    l.qrow = l.scal + kScal;
    l.itag = l.qrow + 4u * (uint32_t)parts;
    l.icache = l.itag + w4(icn);
    l.dtag = l.icache + icn * kStageIps;
    l.dcache = l.dtag + w4(dcn);
    l.words = l.dcache + dcn * 4u * (uint32_t)parts;
    return l;
}

template <int DT>
__global__ __launch_bounds__(kBlock) void stage_kernel(StageArgs A)
{
    extern __shared__ __align__(16) uint32_t sm[];
    const int tid = threadIdx.x;
    const int parts = A.dp * (DT == QW_U8 ? 1 : 4) / 16;
    const StageLayout ly = stage_layout(parts, A.icn, A.dcn);
    uint32_t *tab = sm;
    uint32_t *lpref = sm + ly.lpref, *lstart = sm + ly.lstart, *lmiss = sm + ly.lmiss;
    uint32_t *scal = sm + ly.scal;
    uint4 *qrow = reinterpret_cast<uint4 *>(sm + ly.qrow);
    uint32_t *itag = sm + ly.itag, *icache = sm + ly.icache, *dtag = sm + ly.dtag;
    uint4 *dcache = reinterpret_cast<uint4 *>(sm + ly.dcache);
    const uint4 *drows = reinterpret_cast<const uint4 *>(A.data);
    const int xcd = blockIdx.x % kXcd;
    const unsigned long long rbase = (unsigned long long)xcd * A.region;
    for (uint32_t i = tid; i < A.icn; i += kBlock) itag[i] = kNoTag;
    for (uint32_t i = tid; i < A.dcn; i += kBlock) dtag[i] = kNoTag;
    int64_t nall = 0;
    for (int c = 0; c < A.ncls; ++c) nall += (int64_t)(A.seg[2 * c + 1] - A.seg[2 * c]);
    // item -> query: the classes largest first, each segment in order
    auto query_of = [&](int64_t it) -> int64_t {
        for (int c = A.ncls - 1; c > 0; --c) {
            const int64_t len = (int64_t)(A.seg[2 * c + 1] - A.seg[2 * c]);
            if (it < len) return (int64_t)A.order[A.seg[2 * c] + it];
            it -= len;
        }
        return (int64_t)A.order[A.seg[0] + it];
    };
    // list of position p (lpref[nl] = T > p ends the search)
    auto list_of = [&](uint32_t p) -> int {
        int lo = 0;
        for (int step = 32; step > 0; step >>= 1) {
            const int m = lo + step;
            if (m < A.nl && lpref[m] <= p) lo = m;
        }
        return lo;
    };
    for (;;) {
        __syncthreads();  // the previous run is done with scal
        if (tid == 0) scal[S_CHUNK] = atomicAdd(A.counter, 1u);
        __syncthreads();
        const int64_t it0 = (int64_t)scal[S_CHUNK] * A.chunk;
        if (it0 >= nall) break;  // uniform
        const int64_t it1 = it0 + A.chunk < nall ? it0 + A.chunk : nall;
        for (int64_t it = it0; it < it1; ++it) {
            const int64_t q = query_of(it);
            // ---- the query's lists and row
            if (tid < A.nl) {
                lstart[tid] = A.bstart[q * A.nl + tid];
                lpref[tid + 1] = A.bsize[q * A.nl + tid];
            }
            for (int i = tid; i < parts; i += kBlock)
                qrow[i] = reinterpret_cast<const uint4 *>(A.queries)[q * parts + i];
            if (tid == 0) {
                scal[S_U] = 0;
                scal[S_OVF] = 0;
                scal[S_KP] = 0;
            }
            __syncthreads();
            if (tid < 64) {
                const uint32_t T = wave_layer_prefix(lpref, lstart, A.nl, A.n, A.pmagic);
                if (tid == 0) scal[S_T] = T;
            }
            __syncthreads();
            const uint32_t T = scal[S_T];
            bool bad = T > kStageLimit;  // uniform
            // a list is a cache miss when it is short enough to cache and not there
            if (!bad && tid < A.nl) {
                const uint32_t sz = lpref[tid + 1] - lpref[tid];
                const uint32_t g0 = lstart[tid] + lpref[tid];  // the list's first id index
                lmiss[tid] = A.icn && sz > 0 && sz <= (uint32_t)kStageIps &&
                             itag[id_mix(g0) % A.icn] != g0;
            }
            if (!bad)
                for (uint32_t i = 4u * tid; i < kStageSet; i += 4u * kBlock)
                    *reinterpret_cast<uint4 *>(tab + i) = uint4{kEmpty, kEmpty, kEmpty, kEmpty};
            __syncthreads();
            // ---- union: ids from the index cache or memory into the set
            if (!bad) {
                uint32_t nnew = 0;
                bool full = false;
                for (uint32_t p = tid; p < T; p += kBlock) {
                    const int i = list_of(p);
                    const uint32_t sz = lpref[i + 1] - lpref[i];
                    const uint32_t g0 = lstart[i] + lpref[i];
                    uint32_t id;
                    const uint32_t slot = A.icn ? id_mix(g0) % A.icn : 0u;
                    if (A.icn && sz <= (uint32_t)kStageIps && itag[slot] == g0)
                        id = icache[slot * kStageIps + (p - lpref[i])];
                    else
                        id = (uint32_t)A.ids[lstart[i] + p];
                    uint32_t h = hash_id(id, kStageSetLog2);
                    const uint32_t st = hash_step(id, kStageSetLog2);
                    for (uint32_t probe = 0;; ++probe) {
                        if (probe >= kShortProbe) {
                            full = true;
                            break;
                        }
                        const uint32_t o = atomicCAS(&tab[h], kEmpty, id);
                        if (o == kEmpty) {
                            ++nnew;
                            break;
                        }
                        if (o == id) break;
                        h = (h + st) & (kStageSet - 1u);
                    }
                }
                for (int off = 32; off > 0; off >>= 1) nnew += (uint32_t)__shfl_xor((int)nnew, off);
                const bool anyfull = __ballot(full) != 0ull;
                if ((tid & 63) == 0) {
                    if (nnew) atomicAdd(&scal[S_U], nnew);
                    if (anyfull) scal[S_OVF] = 1;
                }
            }
            __syncthreads();
            bad = bad || scal[S_OVF] != 0;  // uniform
            const uint32_t U = scal[S_U];
            unsigned long long *soff = reinterpret_cast<unsigned long long *>(&scal[S_OFF]);
            if (tid == 0) {
                unsigned long long off = ~0ull;
                if (!bad) {
                    off = atomicAdd(A.alloc + xcd, (unsigned long long)U);
                    if (off + U > A.region) {  // no list space
                        atomicMax(A.fail + xcd, ~off);
                        off = ~0ull;
                    }
                }
                if (off == ~0ull) {  // answered by the fallback
                    A.flag[q] = 1;
                    A.ucount[q] = 0;
                } else {
                    off += rbase;
                    A.ucount[q] = U;
                    A.coff[q] = off;
                }
                *soff = off;
            }
            __syncthreads();
            const unsigned long long off = *soff;
            if (off == ~0ull) continue;  // uniform; the next item starts with a barrier-free write
                                         // of lists the previous reads are done with (below)
            // ---- verification: rows from the data cache or memory
            for (uint32_t sl = tid; sl < kStageSet; sl += kBlock) {
                const uint32_t id = tab[sl];
                if (id == kEmpty) continue;
                const uint32_t ds = A.dcn ? id_mix(id) % A.dcn : 0u;
                const bool hit = A.dcn && dtag[ds] == id;
                const uint4 *row = hit ? dcache + (size_t)ds * parts : drows + (int64_t)id * parts;
                uint32_t hi;
                if (DT == QW_U8) {
                    uint32_t xx = 0, xq = 0, qq = 0;
                    for (int c = 0; c < parts; ++c) {
                        const uint4 xv = row[c], qv = qrow[c];
                        xx = part_dot_u8(xv, xv, xx);
                        xq = part_dot_u8(xv, qv, xq);
                        qq = part_dot_u8(qv, qv, qq);
                    }
                    hi = xx - 2u * xq + qq;  // the exact squared distance
                } else {
                    double acc = 0.0;
                    for (int c = 0; c < parts; ++c) {
                        const float4 xv = reinterpret_cast<const float4 *>(row)[c];
                        const float4 qv = reinterpret_cast<const float4 *>(qrow)[c];
                        const double d0 = (double)xv.x - (double)qv.x, d1 = (double)xv.y - (double)qv.y;
                        const double d2 = (double)xv.z - (double)qv.z, d3 = (double)xv.w - (double)qv.w;
                        acc += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
                    }
                    hi = __float_as_uint((float)acc);  // within half an FP32 ulp
                }
                const uint32_t k = atomicAdd(&scal[S_KP], 1u);
                A.keys[off + k] = ((unsigned long long)hi << 32) | id;
                if (A.dcn && !hit) tab[sl] = id | kMissBit;  // to be cached
            }
            __syncthreads();
            // ---- cache fills: claim the slots, then copy (no reader until the next query)
            if (tid < A.nl && lmiss[tid]) {
                const uint32_t g0 = lstart[tid] + lpref[tid];
                itag[id_mix(g0) % A.icn] = g0;
            }
            for (uint32_t sl = tid; sl < kStageSet; sl += kBlock) {
                const uint32_t v = tab[sl];
                if (v != kEmpty && (v & kMissBit)) dtag[id_mix(v & ~kMissBit) % A.dcn] = v & ~kMissBit;
            }
            __syncthreads();
            for (uint32_t p = tid; p < T; p += kBlock) {
                const int i = list_of(p);
                if (!lmiss[i]) continue;
                const uint32_t g0 = lstart[i] + lpref[i];
                const uint32_t slot = id_mix(g0) % A.icn;
                if (itag[slot] == g0) icache[slot * kStageIps + (p - lpref[i])] = (uint32_t)A.ids[lstart[i] + p];
            }
            for (uint32_t sl = tid; sl < kStageSet; sl += kBlock) {
                const uint32_t v = tab[sl];
                if (v == kEmpty || !(v & kMissBit)) continue;
                const uint32_t id = v & ~kMissBit, ds = id_mix(id) % A.dcn;
                if (dtag[ds] == id)
                    for (int c = 0; c < parts; ++c) dcache[(size_t)ds * parts + c] = drows[(int64_t)id * parts + c];
            }
            __syncthreads();
        }
    }
}

}  // namespace

size_t stage_lds_bytes(int row_bytes, int32_t split, uint32_t *icn, uint32_t *dcn)
{
    const int parts = row_bytes / 16;
    const StageLayout base = stage_layout(parts, 0, 0);
    const size_t fixed = sizeof(uint32_t) * base.words + 64;  // tag padding
    const size_t avail = kStageLdsBytes > fixed ? kStageLdsBytes - fixed : 0;
    const size_t ib = avail * (size_t)split / 100, db = avail - ib;
    *icn = (uint32_t)(ib / (sizeof(uint32_t) * (1 + kStageIps)));
    *dcn = (uint32_t)(db / (sizeof(uint32_t) + (size_t)row_bytes));
    return sizeof(uint32_t) * stage_layout(parts, *icn, *dcn).words;
}

qw_status launch_stage(const StageArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0) return QW_OK;
    const int rb = a.dp * (a.dtype == QW_U8 ? 1 : 4);
    if (a.nl < 1 || a.nl > 64 || rb % 16 || rb > kStageMaxRow || a.chunk < 1 || a.ncls < 1 ||
        a.ncls > 16)
        return QW_EINVAL;
    const size_t lds = sizeof(uint32_t) * stage_layout(rb / 16, a.icn, a.dcn).words;
    if (lds > kStageLdsBytes) return QW_EINVAL;
    if (a.dtype == QW_U8)
        stage_kernel<QW_U8><<<grid, kBlock, lds, s>>>(a);
    else
        stage_kernel<QW_F32><<<grid, kBlock, lds, s>>>(a);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
