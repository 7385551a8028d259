// Shared device-side definitions of the SDGR HIP implementation (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdgr {

// One 8x8 tile of rays (computation plane) or pixels (imaging plane) is one
// wave64: lane l handles cell (l % 8, l / 8) of its tile.
constexpr int TILE = 8;
constexpr int WAVE = 64;
constexpr int RASTER_WAVES = 4;            // independent waves per workgroup
constexpr int RASTER_THREADS = RASTER_WAVES * WAVE;

// Per-view constants, built on the host in FP64 (glibc sin/cos/tan) and
// copied to the device once per call.
struct DevView {
    double ex[3], ey[3], ez[3];   // rows of the world-to-radar rotation
    double dA, dR, dAc, dEc;      // image and computation-plane spacings
    double iA, iR, iAc, iEc;      // their reciprocals
    double hW, hH, hWc, hHc;      // half sizes (centre of each grid)
    int64_t rec_off;              // first record (view, Gaussian) of the view
    int64_t img_off;              // float offset of the image
    int64_t ray_off;              // first computation-plane cell
    int64_t pix_off;              // first pixel in the concatenation of all images
    double range;                 // radar's slant distance from the origin (0: plane wave)
    double pscale;                // factor on P: the cell area dAc dEc, or 1
    int32_t W, H, Wc, Hc;
    int32_t txc, tyc, txi, tyi;   // tiles per axis on each plane
    int32_t tile_c, tile_i;       // first bucket id on each plane
    int32_t scene, n;
};

struct DevScene {
    const float* means;
    const float* scales;
    const float* quats;
    const float* amp;
    const float* ext;
    const float* ext_back;   // or null: ext is the total extinction
    const float* sh;         // [n, shc] phase-function SH coefficients, or null
    float* d_means;
    float* d_scales;
    float* d_quats;
    float* d_amp;            // may be null with sh
    float* d_ext;
    float* d_ext_back;
    float* d_sh;
    int64_t n;
    int64_t item_off;   // first Gaussian of this scene in the flat item space
    int32_t shc;        // SH coefficients per Gaussian, (degree + 1)^2, 0 without sh
    int32_t sh_stride;  // floats between consecutive rows of sh and d_sh
};

// Computation-plane record of one (view, Gaussian), gathered whole by the
// footprint masks and both pass A kernels (one 32-byte piece instead of one
// line per field): centre and conic (cx, cy, a, b), then the conic's c, the
// extinction kappa, the record's tile count and, once the image backward has
// run, the record's c = P dL/dI that pass A's backward needs per hit (0 from
// the projection), so that it comes with the same gather.
struct alignas(32) CRec {
    float4 q;   // cx, cy, a, b
    float4 w;   // c, kappa, the record's tile count (bits of a uint32), P dL/dI
};

struct RasterParams {
    float q_max;       // footprint cutoff
    float eps;         // exp(-q_max / 2)
    float inv1meps;    // 1 / (1 - eps)
    float tau_max;     // early-termination optical depth (huge = off)
    int32_t shadowing;
    float dilation;
    // work counters (null = off): [0..3] footprint hits of pass A forward,
    // pass A backward, pass B forward, pass B backward; [4..6] list entries
    // evaluated by all 64 lanes in pass A forward, pass A backward, pass B
    // forward; [7] summed list prefix the tiles of pass A used; [8], [9]
    // most chunk batches one tile read in pass A forward, backward; [10],
    // [11] hit groups beyond the first of a batch (batches whose hits
    // overflow the compaction buffer) in pass A forward, backward; [12] rays
    // stopped at tau_max; [13] longest list prefix one tile used; [14], [15]
    // tiles the pass A backward ran as long and as short lists; [16], [17]
    // tiles the pass A backward read from stored hits and re-derived from
    // the footprint masks
    unsigned long long* work = nullptr;
    // deterministic mode (null = off): every computation-plane pair's
    // position before the pair sort; pass A writes its per-(tile, record)
    // sums there, in `part` (component k at k * part_stride), instead of
    // adding them into the records' sums with float atomics
    const uint32_t* ppos = nullptr;
    float* part = nullptr;
    int64_t part_stride = 0;
    // stored hits (null = off): pass A's forward keeps the hits each tile's
    // rays processed, hit group by hit group, in `hits` (hit_cap 16-byte
    // units, taken in blocks through the counter at status[ST_HIT_TOP]) as a
    // chain of records whose last one is hit_tail[tile]; the backward walks
    // each chain back to front instead of re-deriving the hits from the
    // footprint masks. A record is three header units (the previous record
    // or HIT_NONE and the hit count; the list positions / 64 of the batch's
    // eight chunks) and then one 8-byte word per hit in processing order
    // (ray-major, each ray front to back): the record id in bits 0..31, the
    // ray (cell of the tile) in bits 32..37, the entry's slot in the batch
    // (chunk * 64 + entry) in bits 40..48.
    uint4* hits = nullptr;
    uint32_t* hit_tail = nullptr;
    unsigned long long* hit_top = nullptr;
    uint32_t hit_cap = 0;
    // the stored-hit backward's output: per list entry it touched, its six
    // sums and its record (plain stores of a row of HIT_PART_STRIDE floats
    // at the pair's position before the pair sort, hit_ppos) and a mark in
    // hit_touched, added per record afterwards (launch_reduce_touched), so
    // that no float atomics are needed
    const uint32_t* hit_ppos = nullptr;
    float* hit_part = nullptr;
    unsigned char* hit_touched = nullptr;
};

constexpr uint32_t HIT_NONE = 0xFFFFFFFFu;       // chain end / a tile with no hits
constexpr uint32_t HIT_OVERFLOW = 0xFFFFFFFEu;   // the stream was full: backward re-derives
constexpr uint32_t HIT_HEADER_UNITS = 3;
constexpr int GC_STRIDE = 8;   // floats per record in grad_c and grad_i
constexpr int HIT_PART_STRIDE = 8;   // floats per pair partial: six sums, the record, spare

// The calling thread's error message of the C ABI (sdgr_last_error): set
// with a code to return, or cleared at the start of a call.
int report_error(int code, const char* msg);
void clear_error();

constexpr int WORK_WORD = 16;    // work counters live at status + 16
// the tile worklist's bins follow the status words: bins[0..32] tile counts
// by the bit length of the list length, bins[33..65] (after placement) the
// number of tiles whose list has at least that bit length
constexpr int WL_BINS_WORD = 64;
constexpr int WORK_COUNTERS = 18;   // u64 each: status words 16 .. 51

// Device-side scalars kept at the start of the state buffer.
enum StatusSlot : int {
    ST_OVERFLOW = 0,   // nonzero if pairs exceeded the planned capacity
    ST_PAIRS_C = 1,    // computation-plane pairs of the last projection (sort length)
    ST_PAIRS_I = 2,    // imaging-plane pairs of records with nonzero intensity
    ST_WORK_TILES = 4, // non-empty computation-plane tiles in the worklist
    ST_ACTIVE = 5,     // records pass A used (backward list length)
    ST_HIT_TOP = 6,    // u64 (words 6, 7): 16-byte units of the hit stream taken so far
    ST_COUNT = 8       // u64 pair totals of the projection at status + 8
};

// Index of the view a global record / bucket belongs to: the last v with
// off(v) <= x, for offsets non-decreasing in v. The lanes of a wave almost
// always fall in one view, so the search runs once for the first active
// lane on wave-uniform values (scalar loads); only lanes outside that view
// search on their own.
template <class F>
__device__ __forceinline__ int find_view(int nv, int64_t x, F off)
{
    const uint32_t xlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t xhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    const int64_t x0 = (int64_t)(((uint64_t)xhi << 32) | xlo);
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off(mid) <= x0) lo = mid; else hi = mid - 1;
    }
    if (off(lo) <= x && (lo + 1 >= nv || x < off(lo + 1))) return lo;
    lo = 0;
    hi = nv - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off(mid) <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Orderable bits of a float: unsigned compare of the result matches the
// float order (with -0 mapped to +0 beforehand).
__device__ __forceinline__ uint32_t float_order_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ---- wave64 helpers ------------------------------------------------------

// Sum of v over the 64 lanes of the wave (all lanes must be active);
// result is wave-uniform.
__device__ __forceinline__ float wave_sum(float v)
{
    // quad sums
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
    // 8-lane sums (row_half_mirror), then 16-lane row sums (row_mirror)
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, false));
    float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Value of the lane a DPP row shift or row broadcast names, 0 where there
// is none (bound control) or the row is masked off.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_from(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}

__device__ __forceinline__ int from_lane_below(int v) { return dpp_from<0x138, 0xF>(v); }  // lane - 1
__device__ __forceinline__ int from_lane_above(int v) { return dpp_from<0x130, 0xF>(v); }  // lane + 1

// Scans over the 64 lanes in lane order: shifts by 1, 2, 4, 8 within rows
// of 16 lanes, then the last lane of a row into the next row (row_bcast 15)
// and of the first two rows into the last two (row_bcast 31).
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_sum_step(float& x, int& f)
{
    const float xl = __int_as_float(dpp_from<CTRL, ROWS>(__float_as_int(x)));
    const int fl = dpp_from<CTRL, ROWS>(f);
    x = f ? x : xl + x;
    f |= fl;
}

// Segmented inclusive prefix sum: `head` marks the first lane of a segment
// (lane 0 must be one); each lane gets the sum over its segment up to itself.
__device__ __forceinline__ float seg_incl_scan(float x, bool head)
{
    int f = head ? 1 : 0;
    seg_sum_step<0x111, 0xF>(x, f);
    seg_sum_step<0x112, 0xF>(x, f);
    seg_sum_step<0x114, 0xF>(x, f);
    seg_sum_step<0x118, 0xF>(x, f);
    seg_sum_step<0x142, 0xA>(x, f);
    seg_sum_step<0x143, 0xC>(x, f);
    return x;
}

// Workgroups go to the eight XCDs (each with its own L2) round-robin by id.
// For a grid whose first n workgroups have work, this renumbering hands each
// XCD one contiguous range of [0, n), so workgroups that read the same
// records (neighbouring list entries) share an L2; ids >= n stay as they are.
constexpr uint32_t XCDS = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t pid, uint32_t n)
{
    if (pid >= n) return pid;
    const uint32_t x = pid % XCDS, q = n / XCDS, r = n % XCDS;
    return x * q + min(x, r) + pid / XCDS;
}

__device__ __forceinline__ float quadform(float4 g, float c, float dx, float dy)
{
    return g.z * dx * dx + 2.0f * g.w * dx * dy + c * dy * dy;
}

// Imaging-plane bucket keys. With at most IKEY_VIEWS views a key is
// (tile within the view << 8) | view: pairs are emitted view by view, so a
// stable sort on the tile bits alone groups every (view, tile); otherwise
// the key is the global bucket id (views' imaging tiles after all
// computation-plane ones).
constexpr int IKEY_VIEWS = 256;
__device__ __forceinline__ uint32_t ikey_encode(bool vm, int v, uint32_t tile_i, uint32_t local)
{
    return vm ? ((local << 8) | (uint32_t)v) : tile_i + local;
}

// Segmented sorts (at most SEG_MAX segments, one per view): segment s holds
// items [seg[s], seg[s+1]), its keys minus kb[s] are sorted, and it owns the
// sort blocks tp[s] .. tp[s+1] - 1 (tp[S] = all blocks), each a run of tpb
// 4096-item tiles of the segment (the last one shorter).
constexpr int SEG_MAX = 256;
struct SegTable {
    uint32_t seg[SEG_MAX + 1];
    uint32_t kb[SEG_MAX];
    uint32_t tp[SEG_MAX + 1];
    uint32_t tpb;
};

// Exclusive prefix of one value per thread over a 256-thread block, and the
// block total (s_w: four LDS words; every thread of the block must call).
__device__ inline uint32_t block_excl_scan_256(uint32_t v, uint32_t* s_w, uint32_t& total)
{
    const int lane = lane_id(), w = (int)threadIdx.x / WAVE;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += t;
    }
    if (lane == WAVE - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t off = 0u;
    total = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < w) off += s_w[k];
        total += s_w[k];
    }
    return off + inc - v;
}

// Cells of tile (tx, ty) inside the ellipse q < q_max of a Gaussian with
// centre (cx, cy) and conic (a, b, c): per row the column span from the
// quadratic, widened by a slack that covers the rounding of the hardware
// reciprocal and square root, so the mask holds every cell whose FP32 q is
// below q_max (callers test q itself). Bit 8 * row + col.
__device__ inline uint64_t footprint_mask(float cx, float cy, float a, float b, float c, float qm,
                                   int tx, int ty)
{
    const float det = a * c - b * b;
    if (!(det > 0.0f) || !(a > 0.0f)) return 0ull;
    const float slack = 1e-3f;
    const float ia = __builtin_amdgcn_rcpf(a);
    const float aq = a * qm, dmin = -1e-4f * aq;
    // rows 0-3 and 4-7 in two 32-bit words, each row's cells j0..j1 as 8
    // bits without a branch (none when the row is out of reach)
    uint32_t m[2] = {0u, 0u};
    const float x0 = (float)(tx * TILE) + 0.5f;
#pragma unroll
    for (int k = 0; k < TILE; ++k) {
        const float dy = (float)(ty * TILE + k) + 0.5f - cy;
        const float D = aq - det * dy * dy;
        const float half = __builtin_amdgcn_sqrtf(fmaxf(D, 0.0f)) * ia + slack;
        const float xc = cx - b * ia * dy;
        // local columns j with |x0 + j - xc| <= half
        const float lo = fmaxf(ceilf(xc - half - x0), 0.0f);
        const float hi = fminf(floorf(xc + half - x0), (float)(TILE - 1));
        const bool reach = !(D < dmin) && lo <= hi;
        const uint32_t j0 = reach ? (uint32_t)lo : 8u, j1 = reach ? (uint32_t)hi : 0u;
        const uint32_t row = (0xFFu << j0) & (0xFFu >> (7u - j1)) & 0xFFu;
        m[k >> 2] |= row << (TILE * (k & 3));
    }
    return ((uint64_t)m[1] << 32) | m[0];
}


}  // namespace sdgr

// ---- host-side launchers (defined in the .hip files) ----------------------
namespace sdgr {


// Pair totals of the projection are accumulated in 2 x TOTAL_SLOTS u64
// slots (spread atomics) and summed into totals[0..1].
constexpr int TOTAL_SLOTS = 1024;
hipError_t launch_preprocess(const DevView* views, const DevScene* scenes, int nv, int nscenes,
                             int64_t items, const RasterParams& rp,
                             bool write_records, CRec* crec, float4* iq,
                             float2* iw, uint2* rect_c, uint2* rect_i, uint32_t* dkey,
                             float* A_zero, float* prec, unsigned long long* slots,
                             unsigned long long* totals, hipStream_t s);

hipError_t launch_set_intensity(const DevView* views, const DevScene* scenes, int nv,
                                int64_t records, const float* A, const float* prec,
                                float2* iw, const uint2* rect_i, uint32_t* cnt_i,
                                uint32_t* bsum_i, uint32_t* status, uint32_t* active,
                                hipStream_t s);

// Per-record gradient buffers: grad_c = (dcx, dcy, da, db, dc, dkappa) on
// the computation plane and grad_i = (dcx, dcy, da, db, dc, dI) on the
// imaging plane, both record-major (component k of record r at
// [r * GC_STRIDE + k]), so that the sums of one record share one 32-byte
// sector: the six pass A adds per list entry, and the image backward's
// single write of each used record's.
hipError_t launch_params_backward(const DevView* views, const DevScene* scenes, int nv,
                                  int nscenes, int64_t scene_items,
                                  const RasterParams& rp, const float* A,
                                  const float* grad_c, const float* grad_i,
                                  int64_t records, int sh_coeffs, float* part,
                                  hipStream_t s);
// Scratch floats of the per-view-group gradient parts (0: one group);
// sh_coeffs: the most SH coefficients of any scene.
size_t params_part_floats(int nv, int64_t items, int sh_coeffs);

// Sort grids have at most max_blocks blocks (each takes a contiguous run of
// 4096-item tiles), between 256 and MAX_SORT_BLOCKS. Fewer, longer blocks
// write longer runs per digit; more blocks hide more latency. Measured on
// the 72-view vehicle: the depth sorts (four 8-bit passes) are fastest at
// 2048, the pair sorts (one pass with wider digits) at 1024.
constexpr unsigned MAX_SORT_BLOCKS = 2048;
constexpr unsigned PAIR_SORT_BLOCKS = 1024;
// stable LSD radix sort of (key, value) pairs on the low `bits` key bits.
// n_dev points at the device-side element count (<= cap). Buffers [0] hold
// the input; returns in *which the index of the buffer holding the output.
size_t radix_hist_words(int64_t cap);
int radix_passes_for(int bits);   // passes a sort of `bits` key bits takes
// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits,
// n_dev items (at most cap); iota_vals: the input values are the positions
// 0..n-1 and vals[0] is not read. *which: the buffer holding the result
// (with keys_out false only the values are valid there). vals2 (optional,
// two buffers): a second value array that ends up holding every item's
// input position (vals2[*which] after the sort).
hipError_t launch_radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], int64_t cap,
                                 const uint32_t* n_dev, int bits, bool iota_vals, uint32_t* hist,
                                 int* which, hipStream_t s, int shift0 = 0,
                                 const SegTable* segt = nullptr, int S = 0,
                                 bool keys_out = true, uint32_t* const* vals2 = nullptr,
                                 unsigned max_blocks = MAX_SORT_BLOCKS);
// Segment table of a segmented sort over the views: records (pairs = false)
// or computation-plane pairs (pairs = true; seg[] as the emission wrote it),
// n_dev items in all.
hipError_t launch_seg_setup(const DevView* views, int nv, int64_t records, const uint32_t* n_dev,
                            bool pairs, SegTable* segt, hipStream_t s,
                            unsigned max_blocks = MAX_SORT_BLOCKS);

// Tile rectangles of the records in depth order, and the computation-plane
// pair count of every 256 of them (bsum).
hipError_t launch_gather_rects(const uint32_t* order, const uint2* rect, int64_t n,
                               uint2* rect_sorted, uint32_t* bsum, hipStream_t s);
// Exclusive scan in place of n per-block counts (one workgroup); with
// status_slot >= 0 the total goes to status[status_slot], flagged against
// cap as an overflow.
hipError_t launch_scan_blocks(uint32_t* bsum, int64_t n, int64_t cap, uint32_t* status,
                              int status_slot, hipStream_t s);
// overflow check and actual pair counts from the projection's u64 totals
hipError_t launch_pair_total_c(int64_t cap_c, uint32_t* status, hipStream_t s);
// (dord, poff optional: the record at each depth rank and its first pair)
hipError_t launch_emit_pairs_c(const DevView* views, int nv, int64_t records,
                               const uint32_t* dval_sorted, const uint2* rect_sorted,
                               const uint32_t* bscan_c, int64_t cap_c, const uint32_t* status,
                               uint32_t* pkey, uint32_t* pval, uint32_t* seg, uint32_t* dord,
                               uint32_t* poff, hipStream_t s);
// out[k * out_comp + dord[p] * out_rec] = sum of part[k * part_stride + i]
// over the pairs i in [poff[p], poff[p + 1]) in order (the last record's end
// is status[ST_PAIRS_C]), for every depth rank p < records and k < ncomp.
hipError_t launch_reduce_pairs(const uint32_t* dord, const uint32_t* poff, int64_t records,
                               const uint32_t* status, const float* part, int ncomp,
                               int64_t part_stride, float* out, int64_t out_comp,
                               int64_t out_rec, hipStream_t s);
// Sums of the per-pair partials the stored-hit pass A backward wrote: the
// rows part[i * HIT_PART_STRIDE ..] of the pair positions i < min(cap,
// status[ST_PAIRS_C]) marked in `touched`, summed per record (the record a
// row names; each record's positions are contiguous) into its six sums in
// grad_c. Records whose rows all fall in one wave's positions are stored;
// the others are added, so the rows of every record that can have touched
// pairs must start at zero. Records with no touched pair are left alone.
hipError_t launch_reduce_touched(int64_t cap, int64_t records, const uint32_t* status,
                                 const unsigned char* touched, const float* part, float* grad_c,
                                 hipStream_t s);
hipError_t launch_emit_pairs_i(const DevView* views, int nv, int64_t records,
                               const uint2* rect_i, const uint32_t* cnt_i,
                               const uint32_t* bscan_i, int64_t cap_c, int64_t cap_i, bool vm,
                               const uint32_t* status, uint32_t* pkey, uint32_t* pval,
                               hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t* keys, int64_t cap, const uint32_t* n_dev,
                              int64_t buckets, uint2* ranges, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_or_word(const uint32_t* src, uint32_t* dst, hipStream_t s);
hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s);

hipError_t launch_pair_masks(const DevView* views, int nv, int64_t cap_c, const RasterParams& rp,
                             const uint32_t* status, const uint32_t* pkey,
                             const uint32_t* pvals, const CRec* crec,
                             uint64_t* pmask, uint64_t* psum, hipStream_t s);
hipError_t launch_tile_worklist(const uint2* ranges, int64_t tiles_c, uint32_t* worklist,
                                uint32_t* bins, uint32_t* status, hipStream_t s);
hipError_t launch_raster_a_fwd(const DevView* views, int nv, int64_t tiles_c,
                               const RasterParams& rp, const uint32_t* status,
                               const uint32_t* worklist, const uint2* ranges,
                               const uint32_t* pvals, const uint64_t* pmask,
                               const uint64_t* psum, const CRec* crec,
                               float* A, float* tau, uint32_t* nlast, hipStream_t s);
hipError_t launch_raster_b_fwd(const DevView* views, int nv, int64_t pixels, int64_t cap_c,
                               int64_t cap_i, const RasterParams& rp, const uint32_t* status,
                               const uint32_t* pkey, const uint32_t* pvals, const float4* iq,
                               const float2* iw, float* images, bool vm, hipStream_t s);
hipError_t launch_ranges_i(const DevView* views, const uint32_t* keys, const uint32_t* status,
                           int64_t cap_i, int64_t tiles_c, int64_t tiles_i, bool vm,
                           uint2* ranges, hipStream_t s);
// Deterministic pass B: one wave per imaging tile over its whole list (in
// list order per pixel), from the imaging-plane tile ranges it builds.
hipError_t launch_raster_b_tiles(const DevView* views, int nv, int64_t pixels, int64_t cap_c,
                                 int64_t cap_i, int64_t tiles_c, int64_t tiles_i,
                                 const RasterParams& rp, const uint32_t* status,
                                 const uint32_t* pkey, const uint32_t* pvals, const float4* iq,
                                 const float2* iw, uint2* ranges_i, float* images, bool vm,
                                 hipStream_t s);
hipError_t launch_image_bwd(const DevView* views, const DevScene* scenes, int nv,
                            int64_t records, const RasterParams& rp, const uint32_t* status,
                            const uint32_t* active, const float4* iq, const float2* iw,
                            const float* prec, const float* dimg, float* grad_i, CRec* crec,
                            float* grad_c, hipStream_t s);
// the tiles with stored hits (rp.hits): per-pair partials, and the sums of
// records with one tile
hipError_t launch_raster_a_bwd_hits(const DevView* views, int nv, int64_t tiles_c,
                                    const RasterParams& rp, const uint32_t* status,
                                    const uint32_t* worklist, const CRec* crec,
                                    const float* tau, float* grad_c, int64_t stride,
                                    hipStream_t s);
// the other tiles (all without stored hits), adding into grad_c with atomics
hipError_t launch_raster_a_bwd(const DevView* views, int nv, int64_t tiles_c,
                               const RasterParams& rp, const uint32_t* status,
                               const uint32_t* worklist, const uint2* ranges,
                               const uint32_t* pvals, const uint64_t* pmask,
                               const uint64_t* psum, const CRec* crec,
                               const float* tau, const uint32_t* nlast, float* grad_c,
                               int64_t stride, hipStream_t s);

}  // namespace sdgr
