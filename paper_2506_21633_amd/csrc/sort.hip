// Binning of (Gaussian, tile) pairs and the device radix sort that builds
// the depth-indexed per-tile Gaussian lists (paper Sec. II-A: the scattering
// intensity is computed along depth-indexed Gaussian lists; the third radar
// coordinate serves as the sorting depth).
//
//   1. records are sorted by (fl32 depth, index) with a stable LSD radix
//      sort of 32-bit keys (index order is the initial order, the first
//      pass generates the indices); with up to SEG_MAX views each view's
//      records are sorted among themselves (a segmented sort), so the order
//      is view-major and the reads by record index that follow stay inside
//      one view at a time; with more views they are sorted together;
//   2. their computation-plane pair counts are scanned in that order and
//      every record emits (tile bucket, record) pairs in depth order;
//   3. a stable LSD radix sort of the pairs on the bucket id yields, per
//      tile, the Gaussians in depth order (segmented by view when the
//      records were: only the tile bits within a view are sorted);
//   4. tile ranges [start, end) are read off the sorted bucket ids;
//   5. after pass A, records with a nonzero intensity emit their
//      imaging-plane pairs in index order (after the computation-plane
//      ones) and the same sort groups them by tile, the order only fixing
//      the FP32 summation order of pass B.
//
// Sort blocks work on runs of 4096-element tiles (256 threads x 16 items).
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


// Digit width of a sort: the fewest passes of at most 10 bits, then the
// narrowest digit (8 to 10 bits) that covers the key in that many passes.
inline int digit_bits(int bits)
{
    const int passes = (bits + 9) / 10;
    const int d = (bits + passes - 1) / passes;
    return d < 8 ? 8 : d;
}

// Sort grids have at most max_blocks blocks; each takes a contiguous
// run of 4096-item tiles of the actual item count, so the per-block digit
// counts (digit-major, R x nb words) and their scan stay small however long
// the array is.
inline unsigned sort_grid(int64_t cap, unsigned max_blocks)
{
    return std::min(nblocks(cap), max_blocks);
}

struct SortSpan {
    int64_t n;      // items
    uint32_t nb;    // blocks with items
    uint32_t tpb;   // tiles per block
};

__device__ __forceinline__ SortSpan sort_span(const uint32_t* n_dev, uint32_t grid)
{
    SortSpan sp;
    sp.n = *n_dev;
    const uint32_t tiles = (uint32_t)((sp.n + SN - 1) / SN);
    sp.tpb = max(1u, (tiles + grid - 1) / grid);
    sp.nb = (tiles + sp.tpb - 1) / sp.tpb;
    return sp;
}

// Items of one sort block: a run of tiles of the whole array, or (segmented
// sorts) a run of tiles of one segment. Digits are taken from key - kb; slot is
// the block's column in the digit-major count matrix of stride columns.
struct BlockItems {
    int64_t first, end;
    uint32_t tiles, stride, kb;
    int s;
};

__device__ __forceinline__ bool span_items(const uint32_t* n_dev, BlockItems& bi)
{
    const SortSpan sp = sort_span(n_dev, gridDim.x);
    if (blockIdx.x >= sp.nb) return false;
    bi.first = (int64_t)blockIdx.x * sp.tpb * SN;
    bi.end = sp.n;
    bi.tiles = sp.tpb;
    bi.stride = sp.nb;
    bi.kb = 0u;
    bi.s = 0;
    return true;
}

// Segment of block b: the last s with tp[s] <= b (empty segments own no
// block, so the block lands in the non-empty one that follows them).
__device__ __forceinline__ bool seg_items(const SegTable* t, int S, uint32_t* s_tp, BlockItems& bi)
{
    for (int k = threadIdx.x; k <= S; k += blockDim.x) s_tp[k] = t->tp[k];
    __syncthreads();
    const uint32_t T = s_tp[S], b = blockIdx.x;
    if (b >= T) return false;
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_tp[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const uint32_t tpb = t->tpb;
    bi.s = lo;
    bi.first = (int64_t)t->seg[lo] + (int64_t)(b - s_tp[lo]) * tpb * SN;
    bi.end = min(bi.first + (int64_t)tpb * SN, (int64_t)t->seg[lo + 1]);
    bi.tiles = tpb;
    bi.stride = T;
    bi.kb = t->kb[lo];
    return true;
}

// Segment table of a segmented sort: item offsets (views' records, or the
// computation-plane pair offsets the emission wrote for the first record of
// each view), key bases, and the block offsets of every segment, with as
// many tiles per block as keep the blocks near MAX_SORT_BLOCKS.
__global__ void __launch_bounds__(SEG_MAX)
k_seg_setup(const DevView* __restrict__ views, int nv, int64_t records,
            const uint32_t* __restrict__ n_dev, int pairs, uint32_t max_blocks,
            SegTable* __restrict__ t)
{
    __shared__ uint32_t s_seg[SEG_MAX + 1];
    __shared__ uint8_t s_empty[SEG_MAX];
    __shared__ uint32_t s_w[SEG_MAX / WAVE];
    const int tid = threadIdx.x;
    const uint32_t n = *n_dev;
    if (tid < nv) {
        const int64_t r0 = views[tid].rec_off;
        const int64_t r1 = tid + 1 < nv ? views[tid + 1].rec_off : records;
        s_empty[tid] = r1 <= r0;
        s_seg[tid] = pairs ? t->seg[tid] : (uint32_t)r0;
    }
    __syncthreads();
    if (tid == 0) {
        // empty segments start where the next one does; all clamped to n
        // (0 after a pair overflow)
        uint32_t next = n;
        for (int v = nv - 1; v >= 0; --v) {
            const uint32_t o = s_empty[v] ? next : min(s_seg[v], next);
            s_seg[v] = o;
            next = o;
        }
        s_seg[nv] = n;
    }
    __syncthreads();
    const uint32_t len = tid < nv ? s_seg[tid + 1] - s_seg[tid] : 0u;
    const uint32_t tiles = (len + SN - 1) / SN;
    uint32_t all_tiles, total;
    (void)block_excl_scan_256(tiles, s_w, all_tiles);
    const uint32_t tpb = max(1u, (all_tiles + max_blocks - 1) / max_blocks);
    __syncthreads();   // s_w is reused by the second scan
    const uint32_t tp = block_excl_scan_256((tiles + tpb - 1) / tpb, s_w, total);
    if (tid < nv) {
        t->seg[tid] = s_seg[tid];
        t->tp[tid] = tp;
        t->kb[tid] = pairs ? (uint32_t)views[tid].tile_c : 0u;
    }
    if (tid == 0) {
        t->seg[nv] = n;
        t->tp[nv] = total;
        t->tpb = tpb;
    }
}

// Block digit histogram over the block's tiles, one LDS atomic per item.
// (Grouping a wave's lanes by digit first, with a ballot match over the
// digit bits, was slower for every key set here, the pair keys of a few busy
// tiles included.)
template <int BITS, bool SEG>
__global__ void __launch_bounds__(SB)
k_radix_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev, int shift,
             uint32_t* __restrict__ hist, const SegTable* __restrict__ segt, int S)
{
    constexpr int R = 1 << BITS;
    __shared__ uint32_t h[R];
    __shared__ uint32_t s_tp[SEG ? SEG_MAX + 1 : 1];
    BlockItems bi;
    if constexpr (SEG) {
        if (!seg_items(segt, S, s_tp, bi)) return;
    } else {
        if (!span_items(n_dev, bi)) return;
    }
    const int tid = threadIdx.x;
#pragma unroll
    for (int d = tid; d < R; d += SB) h[d] = 0;
    __syncthreads();
    const int64_t n = bi.end;
    for (uint32_t t = 0; t < bi.tiles; ++t) {
        const int64_t base = bi.first + (int64_t)t * SN;
        if (base >= n) break;
        uint32_t key[SI];
#pragma unroll
        for (int k = 0; k < SI; ++k) {
            const int64_t idx = base + k * SB + tid;
            key[k] = idx < n ? keys[idx] : 0u;
        }
#pragma unroll
        for (int k = 0; k < SI; ++k) {
            const int64_t idx = base + k * SB + tid;
            if (idx < n) atomicAdd(&h[((key[k] - bi.kb) >> shift) & (R - 1)], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int d = tid; d < R; d += SB) hist[(int64_t)d * bi.stride + blockIdx.x] = h[d];
}

// Spine of one pass: block d turns row d of the digit-major block counts
// into its exclusive prefix over blocks, in place, and writes the digit's
// total to tot[d] (the scatter adds the prefix over digits).
__global__ void __launch_bounds__(SB)
k_radix_spine(uint32_t* __restrict__ hist, uint32_t* __restrict__ tot,
              const uint32_t* __restrict__ n_dev, unsigned grid, const SegTable* __restrict__ segt,
              int S)
{
    constexpr int PER = MAX_SORT_BLOCKS / SB;
    __shared__ uint32_t wtot[SB / WAVE];
    // a segmented sort's blocks (one tile each) may exceed MAX_SORT_BLOCKS:
    // the row is taken MAX_SORT_BLOCKS at a time with a running carry
    const uint32_t nb = segt ? segt->tp[S] : sort_span(n_dev, grid).nb;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    uint32_t* row = hist + (int64_t)blockIdx.x * nb;
    uint32_t carry = 0u;
    for (uint32_t base = 0; base < nb; base += MAX_SORT_BLOCKS) {
        uint32_t v[PER], sum = 0u;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint32_t b = base + (uint32_t)(tid * PER + k);
            v[k] = b < nb ? row[b] : 0u;
            sum += v[k];
        }
        uint32_t inc = sum;
#pragma unroll
        for (int dd = 1; dd < WAVE; dd <<= 1) {
            const uint32_t c = __shfl_up(inc, dd, WAVE);
            if (lane >= dd) inc += c;
        }
        if (lane == WAVE - 1) wtot[w] = inc;
        __syncthreads();
        uint32_t run = carry + inc - sum, all = 0u;
#pragma unroll
        for (int ww = 0; ww < SB / WAVE; ++ww) {
            if (ww < w) run += wtot[ww];
            all += wtot[ww];
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint32_t b = base + (uint32_t)(tid * PER + k);
            if (b < nb) row[b] = run;
            run += v[k];
        }
        carry += all;
        __syncthreads();   // wtot is rewritten by the next chunk
    }
    if (tid == 0) tot[blockIdx.x] = carry;
}

// Stable scatter, one 4096-item tile at a time over the block's tiles. Each
// wave ranks its own 1024 consecutive items in 16 rounds of 64 (ballot
// match over the digit bits, per-wave digit counters in LDS, no block
// barrier); the block then turns the per-wave counts into digit-major local
// offsets, places the items in LDS in digit order and writes them out so
// that the items of one digit leave as a contiguous run. The block's next
// position per digit carries over from tile to tile. With vin null the
// values are the items' input positions. V2 moves a second value array
// along (vin2 null: the input positions).
template <int BITS, bool SEG, bool V2>
__global__ void __launch_bounds__(SB)
k_radix_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                const uint32_t* __restrict__ n_dev, int shift,
                const uint32_t* __restrict__ offs, const uint32_t* __restrict__ tot,
                const SegTable* __restrict__ segt, int S,
                const uint32_t* __restrict__ vin2, uint32_t* __restrict__ vout2)
{
    constexpr int R = 1 << BITS;
    constexpr int NW = SB / WAVE;
    constexpr int DPT = R / SB;                  // digits per thread
    __shared__ uint32_t wc[NW][R];              // per-wave digit counters, then offsets
    __shared__ uint32_t gbase[R];               // global position minus local offset
    __shared__ uint32_t wsum[NW];
    __shared__ uint32_t s_key[SN];
    __shared__ uint32_t s_val[SN];
    __shared__ uint32_t s_val2[V2 ? SN : 1];
    __shared__ uint32_t s_tp[SEG ? SEG_MAX + 1 : 1];
    BlockItems bi;
    if constexpr (SEG) {
        if (!seg_items(segt, S, s_tp, bi)) return;
    } else {
        if (!span_items(n_dev, bi)) return;
    }
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int64_t n = bi.end;
    uint32_t run[DPT];   // next output position of my digits
    {
        // items of all smaller digits (exclusive scan of the digit totals;
        // segmented: of the segment's digit totals, from the segment start)
        uint32_t t[DPT], pb[DPT], sum = 0u, seg0 = 0u;
        const int64_t col = blockIdx.x;
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            const int64_t row = (int64_t)(tid * DPT + k) * bi.stride;
            if constexpr (SEG) {
                const uint32_t b0 = s_tp[bi.s], b1 = s_tp[bi.s + 1];
                const uint32_t p0 = offs[row + b0];
                const uint32_t p1 = b1 < bi.stride ? offs[row + b1] : tot[tid * DPT + k];
                t[k] = p1 - p0;
                pb[k] = offs[row + col] - p0;
            } else {
                t[k] = tot[tid * DPT + k];
                pb[k] = offs[row + col];
            }
            sum += t[k];
        }
        if constexpr (SEG) seg0 = segt->seg[bi.s];
        uint32_t inc = sum;
#pragma unroll
        for (int dd = 1; dd < WAVE; dd <<= 1) {
            const uint32_t c = __shfl_up(inc, dd, WAVE);
            if (lane >= dd) inc += c;
        }
        if (lane == WAVE - 1) wsum[w] = inc;
        __syncthreads();
        uint32_t base = inc - sum;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww)
            if (ww < w) base += wsum[ww];
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            run[k] = seg0 + base + pb[k];
            base += t[k];
        }
        __syncthreads();   // wsum is reused per tile
    }
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    uint32_t key[SI], val[SI], rank[SI], val2[V2 ? SI : 1];
    auto load_tile = [&](int64_t blk) {
#pragma unroll
        for (int k = 0; k < SI; ++k) {
            const int64_t idx = blk + (int64_t)w * (SI * WAVE) + k * WAVE + lane;
            const bool valid = idx < n;
            key[k] = valid ? kin[idx] : 0u;
            val[k] = valid ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
            if constexpr (V2) val2[k] = valid ? (vin2 ? vin2[idx] : (uint32_t)idx) : 0u;
        }
    };
    const int64_t first = bi.first;
    load_tile(first);
    for (uint32_t t = 0; t < bi.tiles; ++t) {
        const int64_t blk = first + (int64_t)t * SN;
        if (blk >= n) break;
        const uint32_t cnt_blk = (uint32_t)min((int64_t)SN, n - blk);
#pragma unroll
        for (int k = 0; k < DPT; ++k)
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) wc[ww][tid * DPT + k] = 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SI; ++k) {
            const int64_t idx = blk + (int64_t)w * (SI * WAVE) + k * WAVE + lane;
            const bool valid = idx < n;
            const uint32_t d = ((key[k] - bi.kb) >> shift) & (R - 1);
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < BITS; ++b) {
                const uint64_t bb = __ballot((d >> b) & 1u);
                m &= ((d >> b) & 1u) ? bb : ~bb;
            }
            const uint32_t before = valid ? wc[w][d] : 0u;
            rank[k] = before + (uint32_t)__popcll(m & below);
            __builtin_amdgcn_wave_barrier();
            if (valid && (m & below) == 0ull) wc[w][d] = before + (uint32_t)__popcll(m);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
        // digit totals of the tile, exclusive scan over digits (digit-major)
        uint32_t tot[DPT], sum = 0u;
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            uint32_t c = 0u;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) c += wc[ww][tid * DPT + k];
            tot[k] = c;
            sum += c;
        }
        uint32_t inc = sum;
#pragma unroll
        for (int dd = 1; dd < WAVE; dd <<= 1) {
            const uint32_t c = __shfl_up(inc, dd, WAVE);
            if (lane >= dd) inc += c;
        }
        if (lane == WAVE - 1) wsum[w] = inc;
        __syncthreads();
        uint32_t lofs = inc - sum;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww)
            if (ww < w) lofs += wsum[ww];
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            const int d = tid * DPT + k;
            gbase[d] = run[k] - lofs;
            run[k] += tot[k];
            uint32_t o = lofs;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t c = wc[ww][d];
                wc[ww][d] = o;
                o += c;
            }
            lofs += tot[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SI; ++k) {
            const int64_t idx = blk + (int64_t)w * (SI * WAVE) + k * WAVE + lane;
            if (idx < n) {
                const uint32_t d = ((key[k] - bi.kb) >> shift) & (R - 1);
                const uint32_t pos = wc[w][d] + rank[k];
                s_key[pos] = key[k];
                s_val[pos] = val[k];
                if constexpr (V2) s_val2[pos] = val2[k];
            }
        }
        // the next tile's items load while this one is written out
        if (t + 1 < bi.tiles && blk + SN < n) load_tile(blk + SN);
        __syncthreads();
#pragma unroll 4
        for (uint32_t i = tid; i < cnt_blk; i += SB) {
            const uint32_t k = s_key[i];
            const uint32_t g = gbase[((k - bi.kb) >> shift) & (R - 1)] + i;
            if (kout) kout[g] = k;
            vout[g] = s_val[i];
            if constexpr (V2) vout2[g] = s_val2[i];
        }
    }
}

// Grid of a sort pass: a segmented sort's blocks take a run of tiles of
// their segment, and every segment may end in a shorter block.
inline unsigned pass_grid(int64_t cap, int S, bool seg, unsigned max_blocks)
{
    return seg ? sort_grid(cap, max_blocks) + (unsigned)S : sort_grid(cap, max_blocks);
}

template <int BITS, bool SEG>
hipError_t radix_passes(uint32_t* keys[2], uint32_t* vals[2], int64_t cap, const uint32_t* n_dev,
                        int bits, bool iota_vals, uint32_t* hist, int* cur, hipStream_t s,
                        int shift0, const SegTable* segt, int S, bool keys_out,
                        uint32_t* const* vals2, unsigned max_blocks)
{
    constexpr int R = 1 << BITS;
    const unsigned grid = pass_grid(cap, S, SEG, max_blocks);
    uint32_t* tot = hist + (int64_t)MAX_RADIX * grid;   // digit totals after the counts
    for (int shift = shift0; shift < shift0 + bits; shift += BITS) {
        hipLaunchKernelGGL((k_radix_hist<BITS, SEG>), dim3(grid), dim3(SB), 0, s, keys[*cur],
                           n_dev, shift, hist, segt, S);
        hipLaunchKernelGGL(k_radix_spine, dim3(R), dim3(SB), 0, s, hist, tot, n_dev, grid,
                           SEG ? segt : nullptr, S);
        const uint32_t* vin = (iota_vals && shift == shift0) ? nullptr : vals[*cur];
        // the last pass writes no keys when the caller needs only the values
        uint32_t* kout = (keys_out || shift + BITS < shift0 + bits) ? keys[*cur ^ 1] : nullptr;
        if (vals2) {
            const uint32_t* vin2 = shift == shift0 ? nullptr : vals2[*cur];
            hipLaunchKernelGGL((k_radix_scatter<BITS, SEG, true>), dim3(grid), dim3(SB), 0, s,
                               keys[*cur], vin, kout, vals[*cur ^ 1], n_dev, shift, hist, tot,
                               segt, S, vin2, vals2[*cur ^ 1]);
        } else {
            hipLaunchKernelGGL((k_radix_scatter<BITS, SEG, false>), dim3(grid), dim3(SB), 0, s,
                               keys[*cur], vin, kout, vals[*cur ^ 1], n_dev, shift, hist, tot,
                               segt, S, nullptr, nullptr);
        }
        *cur ^= 1;
    }
    return hipGetLastError();
}

template <bool SEG>
hipError_t radix_sort_t(uint32_t* keys[2], uint32_t* vals[2], int64_t cap, const uint32_t* n_dev,
                        int bits, bool iota_vals, uint32_t* hist, int* cur, hipStream_t s,
                        int shift0, const SegTable* segt, int S, bool keys_out,
                        uint32_t* const* vals2, unsigned max_blocks)
{
    switch (digit_bits(bits)) {
    case 8:
        return radix_passes<8, SEG>(keys, vals, cap, n_dev, bits, iota_vals, hist, cur, s, shift0,
                                    segt, S, keys_out, vals2, max_blocks);
    case 9:
        return radix_passes<9, SEG>(keys, vals, cap, n_dev, bits, iota_vals, hist, cur, s, shift0,
                                    segt, S, keys_out, vals2, max_blocks);
    default:
        return radix_passes<10, SEG>(keys, vals, cap, n_dev, bits, iota_vals, hist, cur, s,
                                     shift0, segt, S, keys_out, vals2, max_blocks);
    }
}

hipError_t radix_sort(uint32_t* keys[2], uint32_t* vals[2], int64_t cap, const uint32_t* n_dev,
                      int bits, bool iota_vals, uint32_t* hist, int* which, hipStream_t s,
                      int shift0, const SegTable* segt, int S, bool keys_out,
                      uint32_t* const* vals2, unsigned max_blocks)
{
    int cur = 0;
    *which = 0;
    if (cap <= 0 || bits <= 0) return hipSuccess;
    if (segt && (S < 1 || S > SEG_MAX)) return hipErrorInvalidValue;
    const hipError_t e =
        segt ? radix_sort_t<true>(keys, vals, cap, n_dev, bits, iota_vals, hist, &cur, s, shift0,
                                  segt, S, keys_out, vals2, max_blocks)
             : radix_sort_t<false>(keys, vals, cap, n_dev, bits, iota_vals, hist, &cur, s, shift0,
                                   nullptr, 0, keys_out, vals2, max_blocks);
    *which = cur;
    return e;
}

// Tile rectangles of the records in depth order, and the computation-plane
// pair count of each block of 256 (the emission scans within the block). A
// workgroup takes four blocks of 256, so each lane has four gathers in
// flight.
constexpr int GATHER_BLOCKS = 4;

__global__ void __launch_bounds__(256)
k_gather_rects(const uint32_t* __restrict__ order, const uint2* __restrict__ rect, int64_t n,
               uint2* __restrict__ rect_sorted, uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t s_w[GATHER_BLOCKS][4];
    // each XCD walks a contiguous part of the order: in view-major order its
    // reads stay inside a view or two, which its L2 holds
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    uint32_t o[GATHER_BLOCKS];
#pragma unroll
    for (int k = 0; k < GATHER_BLOCKS; ++k) {
        const int64_t i = ((int64_t)blk * GATHER_BLOCKS + k) * 256 + threadIdx.x;
        o[k] = i < n ? order[i] : 0u;
    }
    uint2 rc[GATHER_BLOCKS];
#pragma unroll
    for (int k = 0; k < GATHER_BLOCKS; ++k) {
        const int64_t i = ((int64_t)blk * GATHER_BLOCKS + k) * 256 + threadIdx.x;
        rc[k] = i < n ? rect[o[k]] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < GATHER_BLOCKS; ++k) {
        const int64_t b0 = ((int64_t)blk * GATHER_BLOCKS + k) * 256;
        const int64_t i = b0 + threadIdx.x;
        if (i < n) rect_sorted[i] = rc[k];
        const uint32_t c = ((rc[k].x >> 16) - (rc[k].x & 0xFFFF)) *
                           ((rc[k].y >> 16) - (rc[k].y & 0xFFFF));
        uint32_t tot;
        (void)block_excl_scan_256(c, s_w[k], tot);
        if (threadIdx.x == 0 && b0 < n) bsum[blk * GATHER_BLOCKS + k] = tot;
    }
}

// Exclusive scan in place of the per-block counts, one workgroup walking
// them 8192 at a time with a running carry (coalesced loads and stores
// through LDS, each thread scanning 8 consecutive counts, the next 8192
// loading meanwhile); the total
// optionally becomes a pair count in status (0 and the overflow flag when
// above the capacity).
__global__ void __launch_bounds__(1024)
k_scan_blocks(uint32_t* __restrict__ a, int64_t n, int64_t cap, uint32_t* __restrict__ status,
              int slot)
{
    constexpr int ITEMS = 8, NT = 1024, NWV = NT / WAVE, CH = NT * ITEMS;
    __shared__ uint32_t s_v[CH + CH / 32];   // padded: index k -> k + k / 32
    __shared__ uint32_t s_w[NWV];
    __shared__ unsigned long long s_carry;
    auto pad = [](int k) { return k + (k >> 5); };
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    if (tid == 0) s_carry = 0ull;
    // the next chunk's counts load while this one is scanned and written
    uint32_t nx[ITEMS];
    auto load = [&](int64_t base) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int64_t idx = base + k * NT + tid;
            nx[k] = idx < n ? a[idx] : 0u;
        }
    };
    load(0);
    for (int64_t base = 0; base < n; base += CH) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) s_v[pad(k * NT + tid)] = nx[k];
        __syncthreads();
        if (base + CH < n) load(base + CH);
        uint32_t v[ITEMS], sum = 0u;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            v[k] = s_v[pad(tid * ITEMS + k)];
            sum += v[k];
        }
        uint32_t inc = sum;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const uint32_t t = __shfl_up(inc, d, WAVE);
            if (lane >= d) inc += t;
        }
        if (lane == WAVE - 1) s_w[w] = inc;
        __syncthreads();
        uint32_t off = 0u, total = 0u;
#pragma unroll
        for (int k = 0; k < NWV; ++k) {
            if (k < w) off += s_w[k];
            total += s_w[k];
        }
        uint32_t run = (uint32_t)s_carry + off + inc - sum;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            s_v[pad(tid * ITEMS + k)] = run;
            run += v[k];
        }
        __syncthreads();   // everyone has read s_carry and s_w; s_v holds the prefixes
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int64_t idx = base + k * NT + tid;
            if (idx < n) a[idx] = s_v[pad(k * NT + tid)];
        }
        if (tid == 0) s_carry += total;
        __syncthreads();
    }
    if (tid == 0 && slot >= 0) {
        const unsigned long long tot = s_carry;
        const bool over = tot > (unsigned long long)cap;
        status[ST_OVERFLOW] |= over ? 1u : 0u;
        status[slot] = over ? 0u : (uint32_t)tot;
    }
}

// status[ST_PAIRS_C] from the u64 total of the projection (status + 8);
// flags overflow against the capacity.
__global__ void k_pair_total_c(int64_t cap_c, uint32_t* status)
{
    const unsigned long long* tot = (const unsigned long long*)(status + ST_COUNT);
    const unsigned long long kc = tot[0];
    const bool over = kc > (unsigned long long)cap_c;
    status[ST_OVERFLOW] |= over ? 1u : 0u;
    status[ST_PAIRS_C] = over ? 0u : (uint32_t)kc;
}


// View of a record through a copy of the view offsets in LDS (records in
// depth order come from all views at random unless the depth sort was
// segmented by view).
constexpr int LDS_VIEWS = 512;

// Pair writes of one wave's records (imaging plane: few records have pairs,
// and a loop per record would leave most lanes idle). Record (lane) l
// owns the wave's pairs [ex[l], ex[l] + cnt_l) in row-major order over its
// tile rectangle (width w, first tile local0, tile row stride txn); the key
// is kadd + local, or (local << 8) | kadd for view-major imaging keys. The
// lanes take the wave's pairs 64 at a time, each finding its pair's record
// by binary search over the offsets (the largest l with ex[l] <= j owns j:
// records without pairs share their offset with the next record), so each
// store writes 64 consecutive entries whatever the spread of the counts.
struct EmitWaves {
    uint32_t ex[4][WAVE];
    uint32_t local0[4][WAVE];
    uint32_t w[4][WAVE];
    uint32_t txn[4][WAVE];
    uint32_t kadd[4][WAVE];
    uint32_t val[4][WAVE];
};

__device__ __forceinline__ void emit_wave_pairs(const EmitWaves& L, int w, uint32_t lane,
                                                uint64_t o0, uint32_t total, uint64_t lim,
                                                bool vm, uint32_t* __restrict__ pkey,
                                                uint32_t* __restrict__ pval)
{
    for (uint32_t j = lane; j < total; j += WAVE) {
        uint32_t l = 0;
#pragma unroll
        for (uint32_t step = WAVE / 2; step > 0; step >>= 1)
            if (L.ex[w][l + step] <= j) l += step;
        const uint32_t t = j - L.ex[w][l], rw = L.w[w][l];
        const uint32_t row = t / rw, col = t - row * rw;
        const uint32_t local = L.local0[w][l] + row * L.txn[w][l] + col;
        const uint64_t o = o0 + j;
        if (o < lim) {
            pkey[o] = ikey_encode(vm, (int)L.kadd[w][l], L.kadd[w][l], local);
            pval[o] = L.val[w][l];
        }
    }
}

// Offsets of a wave's records relative to the wave (ex: block-relative
// exclusive offsets), stored with the records' emission data; returns the
// wave's pair count and its first offset in *ex0.
__device__ __forceinline__ uint32_t stage_wave_records(EmitWaves& L, int w, uint32_t lane,
                                                       uint32_t ex, uint32_t cnt, uint2 rc,
                                                       uint32_t txn, uint32_t kadd, uint32_t val,
                                                       uint32_t* ex0)
{
    const uint32_t first = __shfl(ex, 0, WAVE);
    const uint32_t total = __shfl(ex + cnt, WAVE - 1, WAVE) - first;
    const uint32_t tx0 = rc.x & 0xFFFF, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFF;
    L.ex[w][lane] = ex - first;
    L.local0[w][lane] = ty0 * txn + tx0;
    L.w[w][lane] = tx1 - tx0;
    L.txn[w][lane] = txn;
    L.kadd[w][lane] = kadd;
    L.val[w][lane] = val;
    *ex0 = first;
    return total;
}

// Computation-plane pairs, one thread per record in depth order: the
// record emits (tile bucket, record) for every tile of its rectangle at its
// scanned offset, so each tile's pairs leave in depth order.
__global__ void __launch_bounds__(256)
k_emit_c(const DevView* __restrict__ views, int nv, int64_t records,
         const uint32_t* __restrict__ dval, const uint2* __restrict__ rect_sorted,
         const uint32_t* __restrict__ bscan, int64_t cap_c, const uint32_t* __restrict__ status,
         uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval, uint32_t* __restrict__ seg,
         uint32_t* __restrict__ dord, uint32_t* __restrict__ poff)
{
    __shared__ uint32_t s_w[4];
    __shared__ int64_t s_off[LDS_VIEWS];
    __shared__ int32_t s_tile[LDS_VIEWS], s_tx[LDS_VIEWS];
    const bool cached = nv <= LDS_VIEWS;
    if (cached)
        for (int k = threadIdx.x; k < nv; k += blockDim.x) {
            s_off[k] = views[k].rec_off;
            s_tile[k] = views[k].tile_c;
            s_tx[k] = views[k].txc;
        }
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint2 rc = p < records ? rect_sorted[p] : make_uint2(0u, 0u);
    const uint32_t tx0 = rc.x & 0xFFFF, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFF, ty1 = rc.y >> 16;
    // offset: the block's prefix plus the counts of the block's records before
    uint32_t tot;
    const uint32_t ex = block_excl_scan_256((tx1 - tx0) * (ty1 - ty0), s_w, tot);
    if (p >= records) return;
    // the first pair of this depth rank's record and the record
    // (deterministic mode)
    if (poff) poff[p] = bscan[blockIdx.x] + ex;
    if (dord) dord[p] = dval[p];
    int vp = -1;   // the view of position p, when the order is view-major
    if (seg && cached) {
        // view-major order (segmented depth sort): the first record of each
        // view marks where the view's pairs start
        int lo = 0, hi = nv - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= p) lo = mid; else hi = mid - 1;
        }
        if (s_off[lo] == p) seg[lo] = bscan[blockIdx.x] + ex;
        vp = lo;
    }
    const uint32_t kc = status[ST_PAIRS_C];
    if (status[ST_OVERFLOW]) return;
    if (tx0 >= tx1 || ty0 >= ty1) return;
    const uint32_t r = dval[p];
    uint32_t tile0, txc;
    if (vp >= 0) {   // the record at p is one of that view's
        tile0 = (uint32_t)s_tile[vp];
        txc = (uint32_t)s_tx[vp];
    } else if (cached) {
        int lo = 0, hi = nv - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= (int64_t)r) lo = mid; else hi = mid - 1;
        }
        tile0 = (uint32_t)s_tile[lo];
        txc = (uint32_t)s_tx[lo];
    } else {
        const int v = find_view(nv, (int64_t)r, [&](int k) { return views[k].rec_off; });
        tile0 = (uint32_t)views[v].tile_c;
        txc = (uint32_t)views[v].txc;
    }
    uint64_t o = (uint64_t)bscan[blockIdx.x] + ex;
    for (uint32_t ty = ty0; ty < ty1; ++ty)
        for (uint32_t tx = tx0; tx < tx1; ++tx, ++o)
            if (o < kc && o < (uint64_t)cap_c) {
                pkey[o] = tile0 + ty * txc + tx;
                pval[o] = r;
            }
}

// Deterministic sums over the computation-plane pairs: thread = depth rank
// p, its record's pairs are [poff[p], next) before the pair sort (one
// record's tiles, row by row); their partials are added in that order.
// After a pair overflow the lists are empty and no partial was written:
// nothing is summed (the call's results are void anyway).
__global__ void __launch_bounds__(256)
k_reduce_pairs(const uint32_t* __restrict__ dord, const uint32_t* __restrict__ poff,
               int64_t records, const uint32_t* __restrict__ status,
               const float* __restrict__ part, int ncomp, int64_t part_stride,
               float* __restrict__ out, int64_t out_comp, int64_t out_rec)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= records || status[ST_OVERFLOW]) return;
    const uint32_t kc = status[ST_PAIRS_C];
    const uint32_t lo = min(poff[p], kc);
    const uint32_t hi = p + 1 < records ? min(poff[p + 1], kc) : kc;
    const uint32_t r = dord[p];
    for (int k = 0; k < ncomp; ++k) {
        const float* src = part + (int64_t)k * part_stride;
        float acc = 0.0f;
        for (uint32_t i = lo; i < hi; ++i) acc += src[i];
        out[(int64_t)k * out_comp + (int64_t)r * out_rec] = acc;
    }
}

// The stored-hit pass A backward's per-pair partials, summed per record.
// A wave takes RT_ROUNDS x 256 consecutive pair positions (pre-sort order,
// where each record's pairs are contiguous); per round each lane reads the
// touched marks and rows of four consecutive positions, coalesced. The
// rows name their record, and runs of equal record over the touched rows
// are summed: in the lane first, where a run with a run of another record
// on both sides is complete and stored at once; then across the lanes, by
// a segmented scan of each lane's last run (a lane's first run closes with
// the sum carried from the lanes below), the run still open after the last
// lane carrying into the next round. A run with a run of another record
// before and after it inside the wave has every pair in the wave, and its
// sums are stored (this runs before the tiles whose hits are re-derived add
// theirs with atomics). The wave's first and last runs may go on in the
// neighbouring waves and are added with atomics, which is why the rows of
// the records pass A visits start at zero (the image backward clears them).
// Skipped after a pair overflow.
constexpr int RT_ROUNDS = 4;
constexpr int RT_LANE = 4;   // consecutive positions per lane and round
constexpr int RT_WAVE = RT_ROUNDS * WAVE * RT_LANE;

// Six segmented inclusive lane sums that share their segment flags (the
// DPP steps of seg_incl_scan).
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_sum6_step(float (&x)[6], int& f)
{
    const int fl = dpp_from<CTRL, ROWS>(f);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float xl = __int_as_float(dpp_from<CTRL, ROWS>(__float_as_int(x[k])));
        x[k] = f ? x[k] : xl + x[k];
    }
    f |= fl;
}

__device__ __forceinline__ void seg_incl_scan6(float (&x)[6], bool head)
{
    int f = head ? 1 : 0;
    seg_sum6_step<0x111, 0xF>(x, f);
    seg_sum6_step<0x112, 0xF>(x, f);
    seg_sum6_step<0x114, 0xF>(x, f);
    seg_sum6_step<0x118, 0xF>(x, f);
    seg_sum6_step<0x142, 0xA>(x, f);
    seg_sum6_step<0x143, 0xC>(x, f);
}

__global__ void __launch_bounds__(256)
k_reduce_touched(int64_t cap, int64_t records, const uint32_t* __restrict__ status,
                 const unsigned char* __restrict__ touched, const float* __restrict__ part,
                 float* __restrict__ grad_c)
{
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    const int lane = lane_id();
    const int64_t base = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE) * RT_WAVE;
    if (status[ST_OVERFLOW]) return;
    const int64_t kc = min((int64_t)status[ST_PAIRS_C], cap);
    if (base >= kc) return;   // wave-uniform
    // touched marks of the lane's four positions per round, one word each
    // (the marks array has four bytes of slack past the capacity)
    uint32_t tw[RT_ROUNDS];
#pragma unroll
    for (int r = 0; r < RT_ROUNDS; ++r) {
        const int64_t i = base + (int64_t)(r * WAVE + lane) * RT_LANE;
        uint32_t w = 0u;
        if (i < kc) {
            w = *reinterpret_cast<const uint32_t*>(touched + i);
            const int64_t left = kc - i;   // marks past the pair count are not read
            if (left < RT_LANE) w &= (1u << (8 * left)) - 1u;
        }
        tw[r] = w;
    }
    auto put = [&](uint32_t rec, const float (&v)[6], bool add) {
        if ((int64_t)rec >= records) return;
        float* g = grad_c + (int64_t)rec * GC_STRIDE;
        if (add) {
#pragma unroll
            for (int k = 0; k < 6; ++k) unsafeAtomicAdd(&g[k], v[k]);
        } else {
            reinterpret_cast<float4*>(g)[0] = make_float4(v[0], v[1], v[2], v[3]);
            reinterpret_cast<float2*>(g)[2] = make_float2(v[4], v[5]);
        }
    };
    uint32_t ckey = NONE;      // record of the run open after the last lane (wave-uniform)
    float cs[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};   // its sums so far
    bool first = true;         // no run of the wave has closed yet
#pragma unroll
    for (int r = 0; r < RT_ROUNDS; ++r) {
        const int64_t i0 = base + (int64_t)(r * WAVE + lane) * RT_LANE;
        float4 ra[RT_LANE], rb[RT_LANE];
#pragma unroll
        for (int j = 0; j < RT_LANE; ++j) {
            ra[j] = rb[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if ((tw[r] >> (8 * j)) & 0xFFu) {
                const float4* src = reinterpret_cast<const float4*>(
                    part + (uint64_t)(i0 + j) * HIT_PART_STRIDE);
                ra[j] = src[0];
                rb[j] = src[1];
            }
        }
        // the lane's runs: the first one's sums, the last (open) one's sums
        int nr = 0;
        uint32_t fkey = NONE, lkey = NONE;
        float fs[6], ls[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) fs[k] = ls[k] = 0.0f;
#pragma unroll
        for (int j = 0; j < RT_LANE; ++j) {
            if (!((tw[r] >> (8 * j)) & 0xFFu)) continue;
            const uint32_t key = __float_as_uint(rb[j].z);
            const float v[6] = {ra[j].x, ra[j].y, ra[j].z, ra[j].w, rb[j].x, rb[j].y};
            if (nr > 0 && key == lkey) {
#pragma unroll
                for (int k = 0; k < 6; ++k) ls[k] += v[k];
                continue;
            }
            if (nr == 1) {
#pragma unroll
                for (int k = 0; k < 6; ++k) fs[k] = ls[k];   // the first run ends
            } else if (nr > 1) {
                put(lkey, ls, false);   // a run between two others in the lane
            }
            if (nr == 0) fkey = key;
            ++nr;
            lkey = key;
#pragma unroll
            for (int k = 0; k < 6; ++k) ls[k] = v[k];
        }
        const uint64_t m = __ballot(nr > 0);
        if (m) {
            // the open run ends where this round's first touched row names
            // another record
            const uint32_t fk = (uint32_t)__builtin_amdgcn_readlane((int)fkey,
                                                                    __ffsll((long long)m) - 1);
            if (ckey != NONE && fk != ckey) {
                if (lane == 0) put(ckey, cs, first);
                first = false;
                ckey = NONE;
#pragma unroll
                for (int k = 0; k < 6; ++k) cs[k] = 0.0f;
            }
        }
        const uint64_t below = m & ((1ull << lane) - 1ull);
        const uint64_t above = lane == WAVE - 1 ? 0ull : m & ~((2ull << lane) - 1ull);
        // the open record at the nearest lane with rows below, and the first
        // record of the nearest one above (every lane takes part)
        const int lb = below ? 63 - __clzll((long long)below) : lane;
        const int la = above ? __ffsll((long long)above) - 1 : lane;
        const uint32_t pk_ = (uint32_t)__shfl((int)lkey, lb, WAVE);
        const uint32_t nk = (uint32_t)__shfl((int)fkey, la, WAVE);
        const uint32_t prev = below ? pk_ : ckey;
        const bool head = nr > 1 || (nr == 1 && fkey != prev);
        float x[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) x[k] = ls[k] + (lane == 0 && !head ? cs[k] : 0.0f);
        seg_incl_scan6(x, head || lane == 0);
        // the sums carried into the lane: the open run after the lane below
        float cin[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float xb = __int_as_float(from_lane_below(__float_as_int(x[k])));
            cin[k] = lane == 0 ? cs[k] : xb;
        }
        // closings: a lane's first run when a second one starts in it, and
        // its last run when the next lane with rows starts another record
        const bool close_first = nr > 1;
        const bool close_last = nr > 0 && above && nk != lkey;
        const uint64_t cm = __ballot(close_first || close_last);
        const bool lead = first && cm && lane == __ffsll((long long)cm) - 1;
        if (close_first) {
            float t[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) t[k] = fs[k] + (prev == fkey ? cin[k] : 0.0f);
            put(fkey, t, lead);
        }
        if (close_last) put(lkey, x, lead && !close_first);
        if (cm) first = false;
        if (m) ckey = (uint32_t)__builtin_amdgcn_readlane((int)lkey, 63 - __clzll((long long)m));
#pragma unroll
        for (int k = 0; k < 6; ++k)
            cs[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[k]), WAVE - 1));
    }
    if (ckey != NONE && lane == 0) put(ckey, cs, true);
}

// Imaging-plane tile ranges (deterministic pass B): runs of equal keys in
// the sorted imaging-plane keys, indexed by the tile's imaging bucket minus
// tiles_c (keys (tile within the view << 8) | view when vm).
__global__ void __launch_bounds__(256)
k_ranges_i(const DevView* __restrict__ views, const uint32_t* __restrict__ keys,
           const uint32_t* __restrict__ status, int64_t cap_i, int64_t tiles_c, int64_t tiles_i,
           int vm, uint2* __restrict__ ranges)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = min((int64_t)status[ST_PAIRS_I], cap_i);
    if (p >= n) return;
    const uint32_t k = keys[p];
    const int64_t t = vm ? (int64_t)views[k & 0xFFu].tile_i - tiles_c + (k >> 8)
                         : (int64_t)k - tiles_c;
    if (t < 0 || t >= tiles_i) return;
    if (p == 0 || keys[p - 1] != k) ranges[t].x = (uint32_t)p;
    if (p == n - 1 || keys[p + 1] != k) ranges[t].y = (uint32_t)(p + 1);
}

// Imaging-plane pairs of the records in index order, only for the records
// whose intensity is nonzero (cnt_i = 0 otherwise); written after the
// first cap_c entries of the pair arrays.
__global__ void __launch_bounds__(256)
k_emit_i(const DevView* __restrict__ views, int nv, int64_t records,
         const uint2* __restrict__ rect_i, const uint32_t* __restrict__ cnt_i,
         const uint32_t* __restrict__ bscan, int64_t cap_c, int64_t cap_i, int vm,
         const uint32_t* __restrict__ status, uint32_t* __restrict__ pkey,
         uint32_t* __restrict__ pval)
{
    __shared__ uint32_t s_w[4];
    __shared__ EmitWaves L;
    const uint32_t lane = lane_id();
    const int w = threadIdx.x / WAVE;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t cnt = p < records ? cnt_i[p] : 0u;
    // offset: the block's prefix plus the counts of the block's records before
    uint32_t tot;
    const uint32_t ex = block_excl_scan_256(cnt, s_w, tot);
    if (status[ST_OVERFLOW]) return;
    const uint64_t lim = min((uint64_t)status[ST_PAIRS_I], (uint64_t)cap_i);
    uint2 ri = make_uint2(0u, 0u);
    uint32_t kadd = 0u, txi = 1u;
    if (cnt) {
        const int v = find_view(nv, p, [&](int k) { return views[k].rec_off; });
        const DevView& V = views[v];
        ri = rect_i[p];
        txi = (uint32_t)V.txi;
        kadd = vm ? (uint32_t)v : (uint32_t)V.tile_i;
    }
    uint32_t ex0;
    const uint32_t total =
        stage_wave_records(L, w, lane, ex, cnt, ri, txi, kadd, (uint32_t)p, &ex0);
    __syncthreads();
    emit_wave_pairs(L, w, lane, (uint64_t)bscan[blockIdx.x] + ex0, total, lim, vm != 0,
                    pkey + cap_c, pval + cap_c);
}

// Tile ranges from the sorted bucket ids, four keys per thread (one 16-byte
// load when the four are in range) and the neighbours of the first and last.
__global__ void __launch_bounds__(256)
k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev, int64_t buckets,
         uint2* __restrict__ ranges)
{
    const int64_t p0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    const int64_t n = *n_dev;
    if (p0 >= n) return;
    uint32_t k[4];
    if (p0 + 4 <= n) {
        const uint4 q = *reinterpret_cast<const uint4*>(keys + p0);
        k[0] = q.x; k[1] = q.y; k[2] = q.z; k[3] = q.w;
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) k[i] = p0 + i < n ? keys[p0 + i] : 0xFFFFFFFFu;
    }
    const uint32_t before = p0 > 0 ? keys[p0 - 1] : 0xFFFFFFFFu;
    const uint32_t after = p0 + 4 < n ? keys[p0 + 4] : 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t p = p0 + i;
        if (p >= n || k[i] >= buckets) continue;
        const uint32_t prev = i == 0 ? before : k[i - 1];
        const uint32_t next = i == 3 ? after : k[i + 1];
        if (p == 0 || prev != k[i]) ranges[k[i]].x = (uint32_t)p;
        if (p == n - 1 || next != k[i]) ranges[k[i]].y = (uint32_t)(p + 1);
    }
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



size_t radix_hist_words(int64_t cap)
{
    // counts (up to one block per tile and a partial tile per segment),
    // digit totals
    return (size_t)MAX_RADIX * (pass_grid(cap > 0 ? cap : 1, SEG_MAX, true, MAX_SORT_BLOCKS) + 1);
}

int radix_passes_for(int bits)
{
    if (bits <= 0) return 0;
    const int d = digit_bits(bits);
    return (bits + d - 1) / d;
}

hipError_t launch_radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], int64_t cap,
                                 const uint32_t* n_dev, int bits, bool iota_vals, uint32_t* hist,
                                 int* which, hipStream_t s, int shift0, const SegTable* segt,
                                 int S, bool keys_out, uint32_t* const* vals2,
                                 unsigned max_blocks)
{
    if (max_blocks < SB || max_blocks > MAX_SORT_BLOCKS) return hipErrorInvalidValue;
    return radix_sort(keys, vals, cap, n_dev, bits, iota_vals, hist, which, s, shift0, segt, S,
                      keys_out, vals2, max_blocks);
}

hipError_t launch_seg_setup(const DevView* views, int nv, int64_t records, const uint32_t* n_dev,
                            bool pairs, SegTable* segt, hipStream_t s, unsigned max_blocks)
{
    if (nv < 1 || nv > SEG_MAX) return hipErrorInvalidValue;
    if (max_blocks < SB || max_blocks > MAX_SORT_BLOCKS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_seg_setup, dim3(1), dim3(SEG_MAX), 0, s, views, nv, records, n_dev,
                       pairs ? 1 : 0, (uint32_t)max_blocks, segt);
    return hipGetLastError();
}

namespace {
// dst |= src[0] (one word; for accumulating a status flag on the device)
__global__ void k_or_word(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst)
{
    if (threadIdx.x == 0) {
        const uint32_t v = src[0];
        if (v) dst[0] |= v;
    }
}
}  // namespace

hipError_t launch_or_word(const uint32_t* src, uint32_t* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_or_word, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid256(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_gather_rects(const uint32_t* order, const uint2* rect, int64_t n,
                               uint2* rect_sorted, uint32_t* bsum, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((n + 256 * GATHER_BLOCKS - 1) / (256 * GATHER_BLOCKS));
    hipLaunchKernelGGL(k_gather_rects, dim3(grid), dim3(256), 0, s, order, rect, n, rect_sorted,
                       bsum);
    return hipGetLastError();
}

hipError_t launch_scan_blocks(uint32_t* bsum, int64_t n, int64_t cap, uint32_t* status,
                              int status_slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, bsum, n, cap, status,
                       status_slot);
    return hipGetLastError();
}

hipError_t launch_pair_total_c(int64_t cap_c, uint32_t* status, hipStream_t s)
{
    hipLaunchKernelGGL(k_pair_total_c, dim3(1), dim3(1), 0, s, cap_c, status);
    return hipGetLastError();
}

hipError_t launch_emit_pairs_c(const DevView* views, int nv, int64_t records,
                               const uint32_t* dval_sorted, const uint2* rect_sorted,
                               const uint32_t* bscan_c, int64_t cap_c, const uint32_t* status,
                               uint32_t* pkey, uint32_t* pval, uint32_t* seg, uint32_t* dord,
                               uint32_t* poff, hipStream_t s)
{
    if (records <= 0) return hipSuccess;
    if (seg && nv > LDS_VIEWS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_emit_c, dim3(grid256(records)), dim3(256), 0, s, views, nv, records,
                       dval_sorted, rect_sorted, bscan_c, cap_c, status, pkey, pval, seg, dord,
                       poff);
    return hipGetLastError();
}

hipError_t launch_reduce_pairs(const uint32_t* dord, const uint32_t* poff, int64_t records,
                               const uint32_t* status, const float* part, int ncomp,
                               int64_t part_stride, float* out, int64_t out_comp,
                               int64_t out_rec, hipStream_t s)
{
    if (records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_pairs, dim3(grid256(records)), dim3(256), 0, s, dord, poff,
                       records, status, part, ncomp, part_stride, out, out_comp, out_rec);
    return hipGetLastError();
}

hipError_t launch_reduce_touched(int64_t cap, int64_t records, const uint32_t* status,
                                 const unsigned char* touched, const float* part, float* grad_c,
                                 hipStream_t s)
{
    if (records <= 0 || cap <= 0) return hipSuccess;
    constexpr int64_t per_block = 4 * (int64_t)RT_WAVE;   // four waves of 256 threads
    const int64_t grid = (cap + per_block - 1) / per_block;
    if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce_touched, dim3((unsigned)grid), dim3(256), 0, s, cap, records,
                       status, touched, part, grad_c);
    return hipGetLastError();
}

hipError_t launch_ranges_i(const DevView* views, const uint32_t* keys, const uint32_t* status,
                           int64_t cap_i, int64_t tiles_c, int64_t tiles_i, bool vm,
                           uint2* ranges, hipStream_t s)
{
    hipError_t e = launch_fill_u32((uint32_t*)ranges, 0u, 2 * tiles_i, s);
    if (e != hipSuccess || cap_i <= 0) return e;
    hipLaunchKernelGGL(k_ranges_i, dim3(grid256(cap_i)), dim3(256), 0, s, views, keys, status,
                       cap_i, tiles_c, tiles_i, vm ? 1 : 0, ranges);
    return hipGetLastError();
}

hipError_t launch_emit_pairs_i(const DevView* views, int nv, int64_t records,
                               const uint2* rect_i, const uint32_t* cnt_i,
                               const uint32_t* bscan_i, int64_t cap_c, int64_t cap_i, bool vm,
                               const uint32_t* status, uint32_t* pkey, uint32_t* pval,
                               hipStream_t s)
{
    if (records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit_i, dim3(grid256(records)), dim3(256), 0, s, views, nv, records,
                       rect_i, cnt_i, bscan_i, cap_c, cap_i, vm ? 1 : 0, status, pkey, pval);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t* keys, int64_t cap, const uint32_t* n_dev,
                              int64_t buckets, uint2* ranges, hipStream_t s)
{
    hipError_t e = launch_fill_u32((uint32_t*)ranges, 0u, 2 * buckets, s);
    if (e != hipSuccess || cap <= 0) return e;
    hipLaunchKernelGGL(k_ranges, dim3(grid256((cap + 3) / 4)), dim3(256), 0, s, keys, n_dev,
                       buckets, ranges);
    return hipGetLastError();
}

}  // namespace sdgr
