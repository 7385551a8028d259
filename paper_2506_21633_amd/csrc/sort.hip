// Binning of (Gaussian, tile) pairs and the device radix sort that builds
// the depth-indexed per-tile Gaussian lists (paper Sec. II-A: the scattering
// intensity is computed along depth-indexed Gaussian lists; the third radar
// coordinate serves as the sorting depth).
//
//   1. records are sorted by (view, fl32 depth, index) with a stable LSD
//      radix sort of 64-bit keys (index order is the initial order);
//   2. their pair counts are scanned in that order and every record emits
//      (tile bucket, record) pairs -- computation-plane pairs in depth order,
//      imaging-plane pairs in index order;
//   3. a stable LSD radix sort of the pairs on the bucket id yields, per
//      tile, the Gaussians in depth order (computation plane) or in index
//      order (imaging plane, where the order only fixes the FP32 summation
//      order);
//   4. tile ranges [start, end) are read off the sorted bucket ids.
//
// All kernels work on 4096-element blocks (256 threads x 16 items).
#include "common.hpp"

#include <algorithm>
#include <cstring>

namespace sdgr {
namespace {

constexpr int SB = 256;          // threads per sort/scan block
constexpr int SI = 16;           // items per thread
constexpr int SN = SB * SI;      // items per block
constexpr int MAX_RADIX = 1 << 10;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + SN - 1) / SN); }

__global__ void __launch_bounds__(256) k_fill(uint32_t* p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Exclusive scan of one 4096-element block; the block total goes to sums.
__global__ void __launch_bounds__(SB)
k_scan_block(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums)
{
    __shared__ uint32_t buf[SN + SN / 32];   // padded: index k -> k + k/32
    __shared__ uint32_t wtot[SB / WAVE];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SN;
    auto pad = [](int k) { return k + (k >> 5); };
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        int64_t idx = base + k * SB + tid;
        buf[pad(k * SB + tid)] = idx < n ? in[idx] : 0u;
    }
    __syncthreads();
    uint32_t v[SI];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        v[k] = buf[pad(tid * SI + k)];
        sum += v[k];
    }
    // inclusive wave scan of the per-thread sums
    const int lane = tid & (WAVE - 1), w = tid / WAVE;
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t t = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += t;
    }
    if (lane == WAVE - 1) wtot[w] = inc;
    __syncthreads();
    uint32_t woff = 0, total = 0;
#pragma unroll
    for (int k = 0; k < SB / WAVE; ++k) {
        if (k < w) woff += wtot[k];
        total += wtot[k];
    }
    uint32_t run = woff + inc - sum;
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        buf[pad(tid * SI + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        int64_t idx = base + k * SB + tid;
        if (idx < n) out[idx] = buf[pad(k * SB + tid)];
    }
    if (tid == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(256) k_scan_add(uint32_t* out, int64_t n, const uint32_t* sums)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += sums[i / SN];
}

// Digit width of a sort: the fewest passes of at most 10 bits, then the
// narrowest digit (8 to 10 bits) that covers the key in that many passes.
inline int digit_bits(int bits)
{
    const int passes = (bits + 9) / 10;
    const int d = (bits + passes - 1) / passes;
    return d < 8 ? 8 : d;
}

template <class K, int BITS>
__global__ void __launch_bounds__(SB)
k_radix_hist(const K* __restrict__ keys, const uint32_t* __restrict__ n_dev, int shift,
             uint32_t* __restrict__ hist, unsigned nb)
{
    constexpr int R = 1 << BITS;
    __shared__ uint32_t h[R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int d = tid; d < R; d += SB) h[d] = 0;
    __syncthreads();
    const int64_t n = *n_dev;
    const int64_t base = (int64_t)blockIdx.x * SN;
#pragma unroll 4
    for (int k = 0; k < SI; ++k) {
        int64_t idx = base + k * SB + tid;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & (R - 1)], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int d = tid; d < R; d += SB) hist[(int64_t)d * nb + blockIdx.x] = h[d];
}

// Stable scatter: items are taken in index order in rounds of 256; within a
// round the rank of an item among equal digits is its lane order inside the
// wave (ballot match over the digit bits) plus the counts of the lower waves.
template <class K, int BITS>
__global__ void __launch_bounds__(SB)
k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                K* __restrict__ kout, uint32_t* __restrict__ vout,
                const uint32_t* __restrict__ n_dev, int shift,
                const uint32_t* __restrict__ offs, unsigned nb)
{
    constexpr int R = 1 << BITS;
    __shared__ uint32_t base[R];
    __shared__ uint32_t wc[SB / WAVE][R];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int64_t n = *n_dev;
    const int64_t blk = (int64_t)blockIdx.x * SN;
    if (blk >= n) return;
#pragma unroll
    for (int d = tid; d < R; d += SB) {
        base[d] = offs[(int64_t)d * nb + blockIdx.x];
#pragma unroll
        for (int k = 0; k < SB / WAVE; ++k) wc[k][d] = 0;
    }
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    for (int round = 0; round < SI; ++round) {
        const int64_t idx = blk + round * SB + tid;
        const bool valid = idx < n;
        K key = valid ? kin[idx] : (K)0;
        uint32_t val = valid ? vin[idx] : 0u;
        uint32_t d = (uint32_t)(key >> shift) & (R - 1);
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            uint64_t bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(m & below);
        if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(m);
        __syncthreads();
#pragma unroll
        for (int dd = tid; dd < R; dd += SB) {
            uint32_t b0 = base[dd];
            uint32_t c0 = wc[0][dd], c1 = wc[1][dd], c2 = wc[2][dd], c3 = wc[3][dd];
            wc[0][dd] = b0;
            wc[1][dd] = b0 + c0;
            wc[2][dd] = b0 + c0 + c1;
            wc[3][dd] = b0 + c0 + c1 + c2;
            base[dd] = b0 + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = wc[w][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
#pragma unroll
        for (int dd = tid; dd < R; dd += SB) {
#pragma unroll
            for (int k = 0; k < SB / WAVE; ++k) wc[k][dd] = 0;
        }
        __syncthreads();
    }
}

template <class K, int BITS>
hipError_t radix_passes(K* keys[2], uint32_t* vals[2], int64_t cap, const uint32_t* n_dev,
                        int bits, uint32_t* hist, uint32_t* scan_tmp, int* cur, hipStream_t s)
{
    constexpr int R = 1 << BITS;
    const unsigned nb = nblocks(cap);
    const int64_t hn = (int64_t)R * nb;
    for (int shift = 0; shift < bits; shift += BITS) {
        hipLaunchKernelGGL((k_radix_hist<K, BITS>), dim3(nb), dim3(SB), 0, s, keys[*cur], n_dev,
                           shift, hist, nb);
        hipError_t e = launch_exclusive_scan(hist, hist, hn, scan_tmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_radix_scatter<K, BITS>), dim3(nb), dim3(SB), 0, s, keys[*cur],
                           vals[*cur], keys[*cur ^ 1], vals[*cur ^ 1], n_dev, shift, hist, nb);
        *cur ^= 1;
    }
    return hipGetLastError();
}

template <class K>
hipError_t radix_sort(K* keys[2], uint32_t* vals[2], int64_t cap, const uint32_t* n_dev,
                      int bits, uint32_t* hist, uint32_t* scan_tmp, int* which, hipStream_t s)
{
    int cur = 0;
    *which = 0;
    if (cap <= 0 || bits <= 0) return hipSuccess;
    hipError_t e;
    switch (digit_bits(bits)) {
    case 8: e = radix_passes<K, 8>(keys, vals, cap, n_dev, bits, hist, scan_tmp, &cur, s); break;
    case 9: e = radix_passes<K, 9>(keys, vals, cap, n_dev, bits, hist, scan_tmp, &cur, s); break;
    default: e = radix_passes<K, 10>(keys, vals, cap, n_dev, bits, hist, scan_tmp, &cur, s); break;
    }
    *which = cur;
    return e;
}

__global__ void __launch_bounds__(256)
k_gather(const uint32_t* __restrict__ order, const uint32_t* __restrict__ cnt, int64_t n,
         uint32_t* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = cnt[order[i]];
}

// status[ST_PAIRS_*] from the u64 totals of the projection (kept in
// status[8..11] as two u64); flags overflow against the capacities.
__global__ void k_pair_totals(int64_t cap_c, int64_t cap_i, uint32_t* status)
{
    const unsigned long long* tot = (const unsigned long long*)(status + ST_COUNT);
    unsigned long long kc = tot[0], ki = tot[1];
    bool over = kc > (unsigned long long)cap_c || ki > (unsigned long long)cap_i;
    status[ST_OVERFLOW] |= over ? 1u : 0u;
    status[ST_PAIRS_C] = over ? 0u : (uint32_t)kc;
    status[ST_PAIRS_I] = over ? 0u : (uint32_t)ki;
    status[ST_PAIRS_ALL] = over ? 0u : (uint32_t)(kc + ki);
}

__global__ void __launch_bounds__(256)
k_emit(const DevView* __restrict__ views, int nv, int64_t records,
       const uint64_t* __restrict__ dkey, const uint32_t* __restrict__ dval,
       const uint2* __restrict__ rect_c, const uint2* __restrict__ rect_i,
       const uint32_t* __restrict__ off_c, const uint32_t* __restrict__ off_i,
       int64_t cap_c, int64_t cap_i, const uint32_t* __restrict__ status,
       uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= records) return;
    const uint32_t kc = status[ST_PAIRS_C], ki = status[ST_PAIRS_I];
    if (status[ST_OVERFLOW]) return;
    {   // computation plane, depth-sorted position p
        const uint32_t r = dval[p];
        const int v = (int)(dkey[p] >> 32);
        const DevView& V = views[v];
        const uint2 rc = rect_c[r];
        const uint32_t tx0 = rc.x & 0xFFFF, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFF,
                       ty1 = rc.y >> 16;
        uint64_t o = off_c[p];
        for (uint32_t ty = ty0; ty < ty1; ++ty)
            for (uint32_t tx = tx0; tx < tx1; ++tx, ++o)
                if (o < kc && o < (uint64_t)cap_c) {
                    pkey[o] = (uint32_t)V.tile_c + ty * (uint32_t)V.txc + tx;
                    pval[o] = r;
                }
    }
    {   // imaging plane, record p
        const int v = find_view(nv, p, [&](int k) { return views[k].rec_off; });
        const DevView& V = views[v];
        const uint2 ri = rect_i[p];
        const uint32_t tx0 = ri.x & 0xFFFF, tx1 = ri.x >> 16, ty0 = ri.y & 0xFFFF,
                       ty1 = ri.y >> 16;
        uint64_t o = off_i[p];
        for (uint32_t ty = ty0; ty < ty1; ++ty)
            for (uint32_t tx = tx0; tx < tx1; ++tx, ++o)
                if (o < ki && o < (uint64_t)cap_i) {
                    pkey[kc + o] = (uint32_t)V.tile_i + ty * (uint32_t)V.txi + tx;
                    pval[kc + o] = (uint32_t)p;
                }
    }
}

__global__ void __launch_bounds__(256)
k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev, int64_t buckets,
         uint2* __restrict__ ranges)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = *n_dev;
    if (p >= n) return;
    const uint32_t k = keys[p];
    if (k >= buckets) return;
    if (p == 0 || keys[p - 1] != k) ranges[k].x = (uint32_t)p;
    if (p == n - 1 || keys[p + 1] != k) ranges[k].y = (uint32_t)(p + 1);
}

inline unsigned grid256(int64_t n) { return (unsigned)((n + 255) / 256); }

// Host-to-device copy of small tables through kernel arguments: the runtime
// copies the argument block at launch, so the host buffer may be released
// as soon as the launch returns and the copy stays stream-ordered.
constexpr int UPLOAD_CHUNK = 3072;
struct UploadChunk {
    unsigned char bytes[UPLOAD_CHUNK];
};

__global__ void __launch_bounds__(256) k_upload(unsigned char* dst, UploadChunk c, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.bytes[i];
}

}  // namespace

hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const unsigned char* p = static_cast<const unsigned char*>(src);
    unsigned char* d = static_cast<unsigned char*>(dst);
    for (size_t off = 0; off < bytes; off += UPLOAD_CHUNK) {
        UploadChunk c;
        int n = (int)std::min<size_t>(UPLOAD_CHUNK, bytes - off);
        memcpy(c.bytes, p + off, (size_t)n);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, d + off, c, n);
    }
    return hipGetLastError();
}

size_t scan_tmp_words(int64_t n)
{
    size_t words = 0;
    while (n > 1) {
        int64_t nb = (n + SN - 1) / SN;
        words += (size_t)((nb + 63) / 64 * 64);
        n = nb;
    }
    return words + 64;
}

hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                                 hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + SN - 1) / SN;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SB), 0, s, in, out, n, tmp);
    if (nb > 1) {
        uint32_t* next = tmp + (nb + 63) / 64 * 64;
        hipError_t e = launch_exclusive_scan(tmp, tmp, nb, next, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scan_add, dim3(grid256(n)), dim3(256), 0, s, out, n, tmp);
    }
    return hipGetLastError();
}

size_t radix_hist_words(int64_t cap) { return (size_t)MAX_RADIX * nblocks(cap > 0 ? cap : 1); }

int radix_passes_for(int bits)
{
    if (bits <= 0) return 0;
    const int d = digit_bits(bits);
    return (bits + d - 1) / d;
}

hipError_t launch_radix_sort_u64(uint64_t* keys[2], uint32_t* vals[2], int64_t cap,
                                 const uint32_t* n_dev, int bits, uint32_t* hist,
                                 uint32_t* scan_tmp, int* which, hipStream_t s)
{
    return radix_sort<uint64_t>(keys, vals, cap, n_dev, bits, hist, scan_tmp, which, s);
}

hipError_t launch_radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], int64_t cap,
                                 const uint32_t* n_dev, int bits, uint32_t* hist,
                                 uint32_t* scan_tmp, int* which, hipStream_t s)
{
    return radix_sort<uint32_t>(keys, vals, cap, n_dev, bits, hist, scan_tmp, which, s);
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid256(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_gather_counts(const uint32_t* order, const uint32_t* cnt, int64_t n,
                                uint32_t* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid256(n)), dim3(256), 0, s, order, cnt, n, out);
    return hipGetLastError();
}

hipError_t launch_pair_totals(int64_t cap_c, int64_t cap_i, uint32_t* status, hipStream_t s)
{
    hipLaunchKernelGGL(k_pair_totals, dim3(1), dim3(1), 0, s, cap_c, cap_i, status);
    return hipGetLastError();
}

hipError_t launch_emit_pairs(const DevView* views, int nv, int64_t records,
                             const uint64_t* dkey_sorted, const uint32_t* dval_sorted,
                             const uint2* rect_c, const uint2* rect_i, const uint32_t* off_c,
                             const uint32_t* off_i, int64_t cap_c, int64_t cap_i,
                             const uint32_t* status, uint32_t* pkey, uint32_t* pval,
                             hipStream_t s)
{
    if (records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit, dim3(grid256(records)), dim3(256), 0, s, views, nv, records,
                       dkey_sorted, dval_sorted, rect_c, rect_i, off_c, off_i, cap_c, cap_i,
                       status, pkey, pval);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t* keys, int64_t cap, const uint32_t* n_dev,
                              int64_t buckets, uint2* ranges, hipStream_t s)
{
    hipError_t e = launch_fill_u32((uint32_t*)ranges, 0u, 2 * buckets, s);
    if (e != hipSuccess || cap <= 0) return e;
    hipLaunchKernelGGL(k_ranges, dim3(grid256(cap)), dim3(256), 0, s, keys, n_dev, buckets,
                       ranges);
    return hipGetLastError();
}

}  // namespace sdgr
