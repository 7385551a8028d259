// Rasterizers of the SAR Gaussian splatting renderer (paper Sec. II-A,
// scattering intensity and imaging; Sec. II-B, their gradients).
//
// Computation plane (order matters: front-to-back along each ray)
//   One wave64 (a workgroup of its own) owns one 8x8 tile: lane l handles ray
//   (l % 8, l / 8); only non-empty tiles run, longest lists first. Every
//   (tile, Gaussian) pair carries a 64-bit mask of the tile cells inside the
//   footprint ellipse, and every 64 consecutive pairs of the sorted array (a
//   chunk) the OR of their masks (k_pair_masks). The tile's depth-sorted list
//   is walked chunk by chunk: chunks whose summary misses every ray still in
//   play are skipped unread, the next chunk's masks are prefetched, and in a
//   chunk that is read the 64 masks are bit-transposed so that each lane
//   iterates only over the entries covering its own cell.
//   pass A forward : alpha = 1 - exp(-kappa f), A_i += alpha T, T *= exp(-kappa f);
//                    per-entry sums in LDS (float atomics), one global atomic
//                    per (tile, Gaussian); a ray leaves after its optical
//                    depth reaches tau_max.
//   pass A backward: back to front from each ray's last contributing entry:
//                    tau -= kappa f, T = exp(-tau), dL/dalpha = T (c - U),
//                    U <- c alpha + (1 - alpha) U (division-free), c = P dL/dI.
// Imaging plane (order-free additive layover)
//   pass B forward : fixed 128-entry segments of the sorted (tile, Gaussian)
//                    pair array, one wave each (balanced however long a
//                    tile's list is); footprint masks computed on the fly
//                    and bit-transposed, so lane = pixel sums only the
//                    entries covering it; partial pixel sums are added to
//                    the image at tile boundaries.
//   pass B backward: one thread per record walks its footprint ellipse and
//                    gathers dL/dS (no atomics).
#include <cfloat>
#include <type_traits>

#include "common.hpp"

namespace sdgr {
namespace {

constexpr uint32_t B_SEGMENT = 128;    // pair entries per pass-B forward wave

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, WAVE));
    return v;
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---- wave64 data movement without the LDS crossbar --------------------
// Lane i reads lane i ^ S: S = 32 and 16 through the gfx950 permlane swaps,
// S = 8 by a DPP row rotation, S = 4 by DPP row shifts, S = 2 and 1 by DPP
// quad permutes.
template <int S>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v)
{
    const int lane = lane_id();
    if constexpr (S == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return lane < 32 ? r[1] : r[0];
    } else if constexpr (S == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else if constexpr (S == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);
    } else if constexpr (S == 4) {
        const uint32_t from_below = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
        const uint32_t from_above = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x104, 0xF, 0xF, false);
        return (lane & 4) ? from_below : from_above;
    } else if constexpr (S == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    } else {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    }
}

template <int S>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v)
{
    return ((uint64_t)xor_lane<S>((uint32_t)(v >> 32)) << 32) | xor_lane<S>((uint32_t)v);
}

// Lanes with bit S clear keep their own LO blocks and take the partner's LO
// blocks moved up; the others keep their high blocks and take the partner's
// high blocks moved down. Both results are formed and one is picked by a
// lane mask, so the step has no branch (a select between the two shifted
// forms compiles to divergent half-wave paths).
template <int S, uint64_t LO>
__device__ __forceinline__ uint64_t transpose_step(uint64_t v)
{
    const uint64_t p = xor_lane64<S>(v);
    const uint64_t lo = (v & LO) | ((p & LO) << S);
    const uint64_t hi = (v & ~LO) | ((p & ~LO) >> S);
    const uint64_t up = (lane_id() & S) ? ~0ull : 0ull;
    return (lo & ~up) | (hi & up);
}

// 64x64 bit-matrix transpose across the wave: on return, bit j of lane i is
// bit i of lane j's input. Recursive block swap: at step s, lanes i and
// i ^ s exchange the s-wide bit blocks that sit off the diagonal.
__device__ __forceinline__ uint64_t transpose64(uint64_t v)
{
    v = transpose_step<32, 0x00000000FFFFFFFFull>(v);
    v = transpose_step<16, 0x0000FFFF0000FFFFull>(v);
    v = transpose_step<8, 0x00FF00FF00FF00FFull>(v);
    v = transpose_step<4, 0x0F0F0F0F0F0F0F0Full>(v);
    v = transpose_step<2, 0x3333333333333333ull>(v);
    v = transpose_step<1, 0x5555555555555555ull>(v);
    return v;
}

// N independent transposes, step by step over all of them, so that their
// cross-lane moves and bit operations interleave (one transpose after the
// other is a chain of dependent instructions).
template <int N>
__device__ __forceinline__ void transpose64_n(uint64_t (&v)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = transpose_step<32, 0x00000000FFFFFFFFull>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = transpose_step<16, 0x0000FFFF0000FFFFull>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = transpose_step<8, 0x00FF00FF00FF00FFull>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = transpose_step<4, 0x0F0F0F0F0F0F0F0Full>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = transpose_step<2, 0x3333333333333333ull>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = transpose_step<1, 0x5555555555555555ull>(v[i]);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    v += xor_lane64<1>(v);
    v += xor_lane64<2>(v);
    v += xor_lane64<4>(v);
    v += xor_lane64<8>(v);
    v += xor_lane64<16>(v);
    v += xor_lane64<32>(v);
    return v;
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v)
{
    v |= xor_lane64<1>(v);
    v |= xor_lane64<2>(v);
    v |= xor_lane64<4>(v);
    v |= xor_lane64<8>(v);
    v |= xor_lane64<16>(v);
    v |= xor_lane64<32>(v);
    return v;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_affine_step(float& a, float& b, int& f)
{
    // lanes without a source see the identity map (a = 1, b = 0)
    const float al = __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(1.0f), __float_as_int(a), CTRL, ROWS, 0xF, false));
    const float bl = __int_as_float(dpp_from<CTRL, ROWS>(__float_as_int(b)));
    const int fl = dpp_from<CTRL, ROWS>(f);
    if (!f) {
        b = a * bl + b;
        a = a * al;
    }
    f |= fl;
}

// Segmented inclusive composition of the affine maps U -> a U + b held by
// the lanes, earlier lanes applied first: lane l gets f_l o ... o f_head.
__device__ __forceinline__ void seg_incl_affine(float& a, float& b, bool head)
{
    int f = head ? 1 : 0;
    seg_affine_step<0x111, 0xF>(a, b, f);
    seg_affine_step<0x112, 0xF>(a, b, f);
    seg_affine_step<0x114, 0xF>(a, b, f);
    seg_affine_step<0x118, 0xF>(a, b, f);
    seg_affine_step<0x142, 0xA>(a, b, f);
    seg_affine_step<0x143, 0xC>(a, b, f);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void sum_step_u32(uint32_t& x)
{
    x += (uint32_t)dpp_from<CTRL, ROWS>((int)x);
}

// Wave totals of N values at once (inclusive scans, step by step over all
// of them, read at the last lane).
template <int N>
__device__ __forceinline__ void wave_total_u32_n(uint32_t (&x)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) sum_step_u32<0x111, 0xF>(x[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) sum_step_u32<0x112, 0xF>(x[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) sum_step_u32<0x114, 0xF>(x[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) sum_step_u32<0x118, 0xF>(x[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) sum_step_u32<0x142, 0xA>(x[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) sum_step_u32<0x143, 0xC>(x[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = (uint32_t)__builtin_amdgcn_readlane((int)x[i], WAVE - 1);
}

// Exclusive prefix sum of small unsigned counts over the 64 lanes.
__device__ __forceinline__ uint32_t wave_excl_scan_u32(uint32_t v)
{
    uint32_t x = v;
    sum_step_u32<0x111, 0xF>(x);
    sum_step_u32<0x112, 0xF>(x);
    sum_step_u32<0x114, 0xF>(x);
    sum_step_u32<0x118, 0xF>(x);
    sum_step_u32<0x142, 0xA>(x);
    sum_step_u32<0x143, 0xC>(x);
    return x - v;
}

// Direct global-to-LDS loads (gfx950): every lane's 16 (or 4) bytes land
// at dst + lane * 16 (or 4) without passing through registers, so a batch's
// gathers all stay in flight until one wait.
__device__ __forceinline__ void load16_to_lds(const void* src, void* dst_wave_base)
{
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)src,
                                     (void __attribute__((address_space(3)))*)dst_wave_base,
                                     16, 0, 0);
}

__device__ __forceinline__ void load4_to_lds(const void* src, void* dst_wave_base)
{
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)src,
                                     (void __attribute__((address_space(3)))*)dst_wave_base,
                                     4, 0, 0);
}

__device__ __forceinline__ void wait_all_memory()
{
    __builtin_amdgcn_s_waitcnt(0);
}

struct TileCell {
    int v;
    int tx, ty;
    int col, row;
    bool inside;
};

// Tile coordinates of a bucket id (computation-plane ids first, then
// imaging-plane ids), and this lane's cell.
__device__ __forceinline__ TileCell tile_cell(const DevView* views, int nv, int64_t bucket,
                                              bool comp_plane)
{
    TileCell t;
    if (comp_plane)
        t.v = find_view(nv, bucket, [&](int k) { return (int64_t)views[k].tile_c; });
    else
        t.v = find_view(nv, bucket, [&](int k) { return (int64_t)views[k].tile_i; });
    const DevView& V = views[t.v];
    const int64_t local = bucket - (comp_plane ? V.tile_c : V.tile_i);
    const int tx_n = comp_plane ? V.txc : V.txi;
    t.tx = (int)(local % tx_n);
    t.ty = (int)(local / tx_n);
    const int lane = lane_id();
    t.col = t.tx * TILE + (lane & (TILE - 1));
    t.row = t.ty * TILE + (lane / TILE);
    t.inside = comp_plane ? (t.col < V.Wc && t.row < V.Hc) : (t.col < V.W && t.row < V.H);
    return t;
}

// Tile coordinates and this lane's pixel of an imaging-plane key (view-major
// when vm, else a global bucket id).
__device__ __forceinline__ TileCell tile_cell_i(const DevView* views, int nv, uint32_t key, bool vm)
{
    if (!vm) return tile_cell(views, nv, (int64_t)key, false);
    TileCell t;
    t.v = (int)(key & 0xFFu);
    const DevView& V = views[t.v];
    const uint32_t local = key >> 8;
    t.tx = (int)(local % (uint32_t)V.txi);
    t.ty = (int)(local / (uint32_t)V.txi);
    const int lane = lane_id();
    t.col = t.tx * TILE + (lane & (TILE - 1));
    t.row = t.ty * TILE + (lane / TILE);
    t.inside = t.col < V.W && t.row < V.H;
    return t;
}

// Footprint mask of every computation-plane pair (bit 8 * row + col for
// the tile cells inside the ellipse q < q_max), and per 64-pair chunk of
// the sorted array (aligned to the array, so a chunk may span two tiles)
// the OR of its masks. A block takes PM_ITEMS runs of 256 pairs, each wave
// one chunk of every run, so that each lane has PM_ITEMS independent record
// reads in flight.
constexpr int PM_ITEMS = 4;

__global__ void __launch_bounds__(256)
k_pair_masks(const DevView* __restrict__ views, int nv, int64_t cap, RasterParams rp,
             const uint32_t* __restrict__ status, const uint32_t* __restrict__ pkey,
             const uint32_t* __restrict__ pvals, const CRec* __restrict__ crec,
             uint64_t* __restrict__ pmask, uint64_t* __restrict__ psum)
{
    constexpr int BP = 256 * PM_ITEMS;
    const int64_t kc = min(cap, (int64_t)status[ST_PAIRS_C]);
    const uint32_t nblk = (uint32_t)((kc + BP - 1) / BP);
    const int64_t base = (int64_t)xcd_block(blockIdx.x, nblk) * BP + threadIdx.x;
    if (base - lane_id() >= kc) return;   // whole wave past the end
    uint32_t bucket[PM_ITEMS], r[PM_ITEMS];
#pragma unroll
    for (int k = 0; k < PM_ITEMS; ++k) {
        const int64_t p = base + k * 256;
        bucket[k] = p < kc ? pkey[p] : 0u;
        r[k] = p < kc ? pvals[p] : 0u;
    }
    float4 g[PM_ITEMS], g2[PM_ITEMS];
#pragma unroll
    for (int k = 0; k < PM_ITEMS; ++k) {
        if (base + k * 256 < kc) {
            g[k] = crec[r[k]].q;
            g2[k] = crec[r[k]].w;
        }
    }
#pragma unroll
    for (int k = 0; k < PM_ITEMS; ++k) {
        const int64_t p = base + k * 256;
        if (p - lane_id() >= kc) break;   // this and later chunks of the wave are past the end
        uint64_t m = 0ull;
        if (p < kc) {
            const int v = find_view(nv, (int64_t)bucket[k],
                                    [&](int j) { return (int64_t)views[j].tile_c; });
            const DevView& V = views[v];
            const int local = (int)(bucket[k] - (uint32_t)V.tile_c);
            m = footprint_mask(g[k].x, g[k].y, g[k].z, g[k].w, g2[k].x, rp.q_max, local % V.txc,
                               local / V.txc);
            pmask[p] = m;
        }
        m = wave_or_u64(m);
        if (lane_id() == 0) psum[p / WAVE] = m;
    }
}

// Pass A forward, one wave per non-empty 8x8 tile; the wave's rays are the
// tile's 64 cells. The list is walked in 64-entry chunks aligned to the
// global pair array; a chunk whose footprint summary misses every ray still
// in play is skipped without reading its entries. Chunks that are read are
// taken A_BATCH at a time: their masks are loaded together, then the
// records of the entries any live ray needs are gathered together, so a
// batch pays two memory latencies. Inside a chunk the 64x64 bit matrix of
// footprint masks is transposed (lane = ray: which entries cover my cell),
// the (ray, entry) hits are compacted ray-major into LDS, and the wave
// takes them 64 at a time, lane = hit: each ray's optical depth in front of
// each of its hits is a segmented prefix sum, so a round costs the same
// however the hits are spread over the rays. Per-entry sums collect in LDS
// and leave with one global atomic per (tile, entry).
constexpr int A_BATCH = 4;

// DET: deterministic mode (per-pair partials at their pre-sort positions)
template <bool DET>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_raster_a_fwd(const DevView* __restrict__ views, int nv, RasterParams rp,
               const uint32_t* __restrict__ status, const uint32_t* __restrict__ worklist,
               const uint2* __restrict__ ranges, const uint32_t* __restrict__ pvals,
               const uint64_t* __restrict__ pmask, const uint64_t* __restrict__ psum,
               const CRec* __restrict__ crec,
               float* __restrict__ A, float* __restrict__ tau, uint32_t* __restrict__ nlast)
{
    constexpr int NB = 2 * A_BATCH;   // the forward keeps less per chunk in LDS
    constexpr int HKB = NB <= 8 ? 3 : 4;   // bits of a hit's chunk index
    constexpr int HRS = 6 + HKB;           // shift of a hit's ray index
    static_assert(NB <= 16, "hits are packed in 16 bits");
    static_assert(NB == 8, "stored-hit records carry eight chunk ids");
    __shared__ float4 s_q[NB][WAVE];
    __shared__ float s_wc[NB][WAVE], s_wk[NB][WAVE];   // conic c and extinction
    // per-entry sums in GC copies picked by ray (as in the backward; one
    // atomic per hit conflicts little enough that one copy is fastest here)
    constexpr int GC = 1;
    __shared__ float s_A[GC][NB][WAVE + 1];
    __shared__ uint64_t s_m[NB][WAVE];
    __shared__ uint32_t s_r[NB][WAVE];        // record of each entry (stored hits)
    __shared__ uint32_t s_chk[NB];
    __shared__ uint16_t s_hit[WAVE * WAVE];   // (ray, chunk, entry) packed, ray-major
    // per ray during a chunk: first hit in s_hit, optical depth, transmittance,
    // last list position used (one 16-byte read per hit)
    struct alignas(16) RayF { uint32_t o; float t, T; uint32_t last; };
    __shared__ RayF s_ray[WAVE];
    const int lane = threadIdx.x;
    if (blockIdx.x >= status[ST_WORK_TILES]) return;
    const int64_t bucket = worklist[blockIdx.x];
    const TileCell tc = tile_cell(views, nv, bucket, true);
    const DevView& V = views[tc.v];
    const float x0 = (float)(tc.tx * TILE) + 0.5f, y0 = (float)(tc.ty * TILE) + 0.5f;
    const uint2 rg = ranges[bucket];
#pragma unroll
    for (int g = 0; g < GC; ++g)
#pragma unroll
        for (int k = 0; k < NB; ++k) s_A[g][k][lane] = 0.0f;
    float T = 1.0f, t = 0.0f;
    bool alive = tc.inside;
    uint32_t last = 0;
    unsigned long long n_iter = 0, n_hits = 0;   // work counters
    unsigned long long n_batch = 0, n_group = 0;
    uint64_t live = __ballot(alive);
    // per-entry sums of the last processed batch leave with one atomic each;
    // they are sent once the next batch's loads have landed, so the wait for
    // those loads never waits for the atomics
    uint32_t r_prev[NB], r_cur[NB];   // record of my entry in each chunk
    uint32_t d_prev[NB], d_cur[NB];   // deterministic mode: its pair's position before the sort
    // stored hits: this tile's chain of batch records (h_on while the stream
    // has room; h_prev becomes HIT_OVERFLOW when it runs out), the block of
    // the stream the tile writes into [h_top, h_end) and the block size it
    // takes next, the current record and its hit count
    bool h_on = !DET && rp.hits != nullptr;
    uint32_t h_top = 0u, h_end = 0u, h_blk = 256u, h_prev = HIT_NONE, h_rec = 0u, h_kept = 0u;
    // (a nonzero sum means a live ray hit the entry, so its record was
    // gathered and r_prev holds it: all eight sums are read at once, without
    // a branch per chunk)
    auto flush = [&]() {
        float a[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            a[k] = 0.0f;
#pragma unroll
            for (int g = 0; g < GC; ++g) a[k] += s_A[g][k][lane];
        }
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
            for (int g = 0; g < GC; ++g) s_A[g][k][lane] = 0.0f;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (a[k] != 0.0f) {
                if constexpr (DET) rp.part[d_prev[k]] = a[k];
                else unsafeAtomicAdd(&A[r_prev[k]], a[k]);
            }
        }
    };
    const uint32_t c_first = rg.x / WAVE, c_end = (rg.y + WAVE - 1) / WAVE;
    for (uint32_t g0 = c_first; g0 < c_end && live != 0ull; g0 += WAVE) {
        const uint64_t sm = g0 + lane < c_end ? psum[g0 + lane] : 0ull;
        uint64_t todo = __ballot((sm & live) != 0ull);   // chunks to read, in order
        // up to NB chunks per batch: their masks and values are fetched one
        // batch ahead (in flight while the current batch's hits are
        // processed), then the records the live rays need
        uint32_t chk_n[NB], r_n[NB], d_n[NB];
        uint64_t m_n[NB];
        int nb_n = 0;
        auto fetch = [&]() {
            nb_n = 0;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                chk_n[k] = 0u;
                if (todo != 0ull) {
                    chk_n[k] = g0 + (uint32_t)__builtin_ctzll(todo);
                    todo &= todo - 1ull;
                    nb_n = k + 1;
                }
            }
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const uint32_t e = chk_n[k] * WAVE + lane;
                const bool in = k < nb_n && e >= rg.x && e < rg.y;
                m_n[k] = in ? pmask[e] : 0ull;
                r_n[k] = in ? pvals[e] : 0u;
                if constexpr (DET) d_n[k] = in ? rp.ppos[e] : 0u;
            }
        };
        fetch();
        while (nb_n > 0 && live != 0ull) {
            ++n_batch;
            const int nb = nb_n;
            {
                uint32_t chk[NB];
                uint64_t m[NB];
                uint32_t* r = r_cur;
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    chk[k] = chk_n[k];
                    m[k] = m_n[k];
                    r[k] = r_n[k];
                    if constexpr (DET) d_cur[k] = d_n[k];
                }
                // records straight into LDS, all in flight together (entries
                // no live ray needs read record 0, one shared line)
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const bool need = (m[k] & live) != 0ull;
                    const uint32_t rk = need ? r[k] : 0u;
                    const float* w = reinterpret_cast<const float*>(&crec[rk].w);
                    load16_to_lds(&crec[rk].q, &s_q[k][0]);
                    load4_to_lds(w, &s_wc[k][0]);
                    load4_to_lds(w + 1, &s_wk[k][0]);
                }
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    s_m[k][lane] = m[k];
                    if (h_on) s_r[k][lane] = r[k];
                    if (lane == k) s_chk[k] = chk[k];
                }
            }
            wait_all_memory();
            wave_lds_sync();
            fetch();   // the next batch's masks and values
            flush();
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                r_prev[k] = r_cur[k];
                if constexpr (DET) d_prev[k] = d_cur[k];
            }
            // the batch's chunks, transposed: bit j of col[k] is entry j of
            // chunk k covering my cell (rays already out of play keep none)
            uint64_t col[NB];
            uint32_t hk[NB];   // hits of each chunk over the wave
            // every chunk slot is transposed (the unused ones' stale masks are
            // dropped), all eight together; the chunks' hit totals (at most
            // 4096 each) are summed two to a word
#pragma unroll
            for (int k = 0; k < NB; ++k) col[k] = s_m[k][lane];
            transpose64_n(col);
#pragma unroll
            for (int k = 0; k < NB; ++k) col[k] = (k < nb && alive) ? col[k] : 0ull;
            {
                uint32_t tot[NB / 2];
#pragma unroll
                for (int i = 0; i < NB / 2; ++i)
                    tot[i] = (uint32_t)__popcll(col[2 * i]) |
                             ((uint32_t)__popcll(col[2 * i + 1]) << 16);
                wave_total_u32_n(tot);
#pragma unroll
                for (int i = 0; i < NB / 2; ++i) {
                    hk[2 * i] = tot[i] & 0xFFFFu;
                    hk[2 * i + 1] = tot[i] >> 16;
                }
            }
            if (h_on) {
                // room for the batch's records, one per hit group (so that no
                // ray's hits interleave with another group's in a record):
                // their headers and at most every hit; a new block when the
                // tile's is short (sizes doubling up to 64 KB, so short tiles
                // waste little and long ones seldom ask)
                uint32_t H = 0u;
#pragma unroll
                for (int k = 0; k < NB; ++k) H += hk[k];
                const uint32_t units = NB * (HIT_HEADER_UNITS + 1u) + (H + 1u) / 2u;
                if (h_end - h_top < units) {
                    const uint32_t take = max(units, h_blk);
                    h_blk = min(2u * h_blk, 4096u);
                    unsigned long long base = 0ull;
                    if (lane == 0) base = atomicAdd(rp.hit_top, (unsigned long long)take);
                    base = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane(
                                (int)(uint32_t)(base >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
                    if (base + take > (unsigned long long)rp.hit_cap) {
                        h_on = false;
                        h_prev = HIT_OVERFLOW;
                    } else {
                        h_top = (uint32_t)base;
                        h_end = h_top + take;
                    }
                }
            }
            // groups of consecutive chunks whose hits fit s_hit; each group's
            // hits are compacted ray-major (chunk by chunk, front to back) and
            // taken 64 per round
            for (int g0 = 0; g0 < nb && live != 0ull;) {
                ++n_group;
                h_rec = h_top;
                h_kept = 0u;
                int g1 = g0;
                uint32_t H = 0;
                bool open = true;
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    if (k < g0 || k >= nb || !open) continue;
                    if (H + hk[k] <= (uint32_t)(WAVE * WAVE)) {
                        H += hk[k];
                        g1 = k + 1;
                    } else {
                        open = false;
                    }
                }
                uint32_t nr = 0;
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (k >= g0 && k < g1) nr += (uint32_t)__popcll(col[k]);
                const uint32_t o = wave_excl_scan_u32(nr);
                if (H > 0u) {
                    uint32_t w = o;
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        if (k < g0 || k >= g1) continue;
                        uint64_t c = col[k];
                        while (c != 0ull) {
                            const int j = __builtin_ctzll(c);
                            c &= c - 1ull;
                            s_hit[w++] = (uint16_t)((lane << HRS) | (k << 6) | j);
                        }
                    }
                    s_ray[lane] = RayF{o, t, T, last};
                    wave_lds_sync();
                    for (uint32_t base = 0; base < H; base += WAVE) {
                        ++n_iter;
                        const uint32_t L = base + lane;
                        const bool valid = L < H;
                        const uint32_t hv = valid ? (uint32_t)s_hit[L] : 0u;
                        const int rr = (int)(hv >> HRS), k = (int)((hv >> 6) & ((1u << HKB) - 1u)),
                                  j = (int)(hv & 63u);
                        // ray state and entry record, read together (lanes past
                        // the last hit read entry 0 of ray 0 and ignore it)
                        const RayF rs = s_ray[rr];
                        const float4 g = s_q[k][j];
                        const float gc = s_wc[k][j], gk = s_wk[k][j];
                        const uint32_t pos = s_chk[k] * WAVE + (uint32_t)j - rg.x;   // list position
                        const int seg0 = valid ? max((int)rs.o - (int)base, 0) : lane;
                        bool real = false;
                        float x = 0.0f, E = 1.0f;
                        if (valid) {
                            const float dx = x0 + (float)(rr & (TILE - 1)) - g.x;
                            const float dy = y0 + (float)(rr / TILE) - g.y;
                            const float q = quadform(g, gc, dx, dy);
                            if (q < rp.q_max) {
                                real = true;
                                x = gk * ((__expf(-0.5f * q) - rp.eps) * rp.inv1meps);
                                E = __expf(-x);
                            }
                        }
                        const float incl = seg_incl_scan(x, lane == seg0);
                        const float excl = incl - x;
                        const float tr = valid ? rs.t : 0.0f;
                        const float Tr = valid ? rs.T : 1.0f;
                        // a ray's hits are processed up to the first one reached
                        // with an optical depth of tau_max (a prefix of its segment)
                        const uint64_t stop =
                            __ballot(valid && rp.shadowing && !(tr + excl < rp.tau_max));
                        const uint64_t after = stop & (~0ull << seg0);
                        const bool proc = valid && (after == 0ull || lane < __builtin_ctzll(after));
                        if (h_on) {
                            // the processed hits, in processing order: record,
                            // ray and the entry's slot in the batch
                            const uint64_t kb = __ballot(proc);
                            if (proc)
                                reinterpret_cast<unsigned long long*>(
                                    rp.hits + h_rec + HIT_HEADER_UNITS)[h_kept + lanes_below(kb)] =
                                    (unsigned long long)s_r[k][j] | ((unsigned long long)rr << 32) |
                                    ((unsigned long long)(k * WAVE + j) << 40);
                            h_kept += (uint32_t)__popcll(kb);
                        }
                        if (proc && real) {
                            // at least FLT_MIN, so that A > 0 marks exactly the
                            // records some ray used (the exact alpha T is > 0
                            // for every footprint hit)
                            const float a = fmaxf(
                                (1.0f - E) * (rp.shadowing ? Tr * __expf(-excl) : 1.0f), FLT_MIN);
                            atomicAdd(&s_A[(rr + (rr >> 3)) & (GC - 1)][k][j], a);
                        }
                        const uint64_t hb = __ballot(proc && real);
                        if (lane == 0) n_hits += (unsigned long long)__popcll(hb);
                        // the last processed hit of each ray in this round updates the ray
                        const int nxt = from_lane_above(proc ? (int)hv : -1);
                        const bool endseg = proc && (lane == WAVE - 1 || (nxt >> HRS) != rr);
                        wave_lds_sync();
                        if (endseg)
                            s_ray[rr] = RayF{rs.o, tr + incl, rp.shadowing ? Tr * __expf(-incl) : Tr,
                                             pos + 1u};
                        wave_lds_sync();
                    }
                    {
                        const RayF rs = s_ray[lane];
                        t = rs.t;
                        T = rs.T;
                        last = rs.last;
                    }
                    if (rp.shadowing && t >= rp.tau_max) alive = false;
                    live = __ballot(alive);
                    wave_lds_sync();
                }
                if (h_on && h_kept > 0u) {   // the group's record
                    if (lane == 0) rp.hits[h_rec] = make_uint4(h_prev, h_kept, 0u, 0u);
                    if (lane == 1)
                        rp.hits[h_rec + 1] = make_uint4(s_chk[0], s_chk[1], s_chk[2], s_chk[3]);
                    if (lane == 2)
                        rp.hits[h_rec + 2] = make_uint4(s_chk[4], s_chk[5], s_chk[6], s_chk[7]);
                    h_prev = h_rec;
                    h_top = h_rec + HIT_HEADER_UNITS + (h_kept + 1u) / 2u;
                }
                g0 = g1;
            }
            wave_lds_sync();
        }
    }
    flush();
    if (!DET && rp.hits != nullptr && lane == 0) rp.hit_tail[bucket] = h_prev;
    if (rp.work) {
        n_hits = wave_sum_u64(n_hits);
        const uint32_t used = wave_max_u32(last);   // list prefix any ray used
        const uint64_t stopped = __ballot(tc.inside && rp.shadowing && t >= rp.tau_max);
        if (lane == 0) {
            atomicAdd(&rp.work[4], n_iter);
            atomicAdd(&rp.work[0], n_hits);
            atomicAdd(&rp.work[7], (unsigned long long)used);
            atomicMax(&rp.work[8], n_batch);
            atomicAdd(&rp.work[10], n_group - n_batch);
            atomicAdd(&rp.work[12], (unsigned long long)__popcll(stopped));
            atomicMax(&rp.work[13], (unsigned long long)used);
        }
    }
    if (tc.inside) {
        const int64_t ray = V.ray_off + (int64_t)tc.row * V.Wc + tc.col;
        tau[ray] = t;
        nlast[ray] = last;
    }
}

// Zero every view's image before the segmented accumulation.
__global__ void __launch_bounds__(256)
k_zero_images(const DevView* __restrict__ views, int nv, int64_t pixels, float* __restrict__ images)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pixels) return;
    const int v = find_view(nv, p, [&](int k) { return views[k].pix_off; });
    images[views[v].img_off + (p - views[v].pix_off)] = 0.0f;
}

// Pass B forward over fixed B_SEGMENT-entry segments of the sorted imaging-plane
// pair array (one wave each, balanced however long a tile's list is).
// Lane = entry: gather the record, compute its footprint mask on the
// entry's tile; then, per run of entries of one tile, the masks are
// bit-transposed and lane = pixel sums only the entries covering it. The
// partial pixel sums are added to the image when the tile changes.
__global__ void __launch_bounds__(RASTER_THREADS)
k_raster_b_fwd(const DevView* __restrict__ views, int nv, RasterParams rp, int64_t cap_c,
               const uint32_t* __restrict__ status, const uint32_t* __restrict__ pkey,
               const uint32_t* __restrict__ pvals, const float4* __restrict__ iq,
               const float2* __restrict__ iw, float* __restrict__ images, int vm)
{
    __shared__ float4 s_q[RASTER_WAVES][WAVE];
    __shared__ float2 s_w[RASTER_WAVES][WAVE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const uint32_t ki = status[ST_PAIRS_I];
    const uint32_t nblk = (uint32_t)(((uint64_t)ki + (uint64_t)B_SEGMENT * RASTER_WAVES - 1) /
                                     ((uint64_t)B_SEGMENT * RASTER_WAVES));
    const uint64_t seg = (uint64_t)xcd_block(blockIdx.x, nblk) * RASTER_WAVES + w;
    const uint64_t p0 = (uint64_t)cap_c + seg * B_SEGMENT;
    const uint64_t pend = (uint64_t)cap_c + ki;
    if (p0 >= pend) return;
    const uint32_t p1 = (uint32_t)min(pend, p0 + B_SEGMENT);
    uint32_t cur = 0xFFFFFFFFu;
    float acc = 0.0f, px = 0.0f, py = 0.0f;
    int64_t pix = -1;
    unsigned long long n_iter = 0, n_hits = 0;   // work counters
    // software pipeline over the 64-entry steps: the records of step s + 1
    // and the keys and record ids of step s + 2 load while step s runs
    const uint32_t e0 = (uint32_t)p0 + lane;
    uint32_t key_n = e0 < p1 ? pkey[e0] : 0xFFFFFFFFu;
    uint32_t r_n = e0 < p1 ? pvals[e0] : 0u;
    float4 g_n = iq[r_n];
    float2 g2_n = iw[r_n];
    uint32_t key_nn = e0 + WAVE < p1 ? pkey[e0 + WAVE] : 0xFFFFFFFFu;
    uint32_t r_nn = e0 + WAVE < p1 ? pvals[e0 + WAVE] : 0u;
    for (uint32_t b0 = (uint32_t)p0; b0 < p1; b0 += WAVE) {
        const uint32_t e = b0 + lane;
        const bool in = e < p1;
        const uint32_t key = key_n;
        const float4 g = g_n;
        const float2 g2 = g2_n;
        key_n = key_nn;
        g_n = iq[r_nn];
        g2_n = iw[r_nn];
        key_nn = e + 2 * WAVE < p1 ? pkey[e + 2 * WAVE] : 0xFFFFFFFFu;
        r_nn = e + 2 * WAVE < p1 ? pvals[e + 2 * WAVE] : 0u;
        uint64_t m = 0ull;
        if (in) {
            s_q[w][lane] = g;
            s_w[w][lane] = g2;
            const TileCell tk = tile_cell_i(views, nv, key, vm != 0);
            if (g2.y != 0.0f)   // zero intensity adds nothing
                m = footprint_mask(g.x, g.y, g.z, g.w, g2.x, rp.q_max, tk.tx, tk.ty);
        }
        wave_lds_sync();
        uint64_t rest = __ballot(in);
        while (rest != 0ull) {
            // the run of entries of the first remaining tile (keys are sorted)
            const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key,
                                                                  __builtin_ctzll(rest));
            const uint64_t sel = __ballot(in && key == k) & rest;
            rest &= ~sel;
            if (k != cur) {   // tile change: flush the partial sums
                if (pix >= 0 && acc != 0.0f) unsafeAtomicAdd(&images[pix], acc);
                const TileCell tc = tile_cell_i(views, nv, k, vm != 0);
                const DevView& V = views[tc.v];
                px = tc.col + 0.5f;
                py = tc.row + 0.5f;
                pix = tc.inside ? V.img_off + (int64_t)tc.row * V.W + tc.col : -1;
                acc = 0.0f;
                cur = k;
            }
            uint64_t col = transpose64(((sel >> lane) & 1ull) ? m : 0ull);
            if (pix < 0) col = 0ull;
            for (;;) {
                if (__ballot(col != 0ull) == 0ull) break;
                ++n_iter;
                if (col != 0ull) {
                    const int j = __builtin_ctzll(col);
                    col &= col - 1ull;
                    const float4 g = s_q[w][j];
                    const float2 g2 = s_w[w][j];
                    const float dx = px - g.x, dy = py - g.y;
                    const float q = quadform(g, g2.x, dx, dy);
                    if (q < rp.q_max) {
                        ++n_hits;
                        acc += (__expf(-0.5f * q) - rp.eps) * rp.inv1meps * g2.y;
                    }
                }
            }
        }
        wave_lds_sync();
    }
    if (pix >= 0 && acc != 0.0f) unsafeAtomicAdd(&images[pix], acc);
    if (rp.work) {
        n_hits = wave_sum_u64(n_hits);
        if (lane == 0) {
            atomicAdd(&rp.work[6], n_iter);
            atomicAdd(&rp.work[2], n_hits);
        }
    }
}

// Deterministic pass B: one wave per imaging tile (bucket tiles_c + t) walks
// its whole list, 64 entries at a time: lane = entry while the records load
// and the footprint masks form, then lane = pixel adding the entries that
// cover it in list order. Every pixel is written once, by a plain store on
// the zeroed image, so repeated runs agree bit for bit.
__global__ void __launch_bounds__(RASTER_THREADS)
k_raster_b_tile(const DevView* __restrict__ views, int nv, RasterParams rp, int64_t cap_c,
                int64_t tiles_c, int64_t tiles_i, const uint2* __restrict__ ranges_i,
                const uint32_t* __restrict__ pvals, const float4* __restrict__ iq,
                const float2* __restrict__ iw, float* __restrict__ images)
{
    __shared__ float4 s_q[RASTER_WAVES][WAVE];
    __shared__ float2 s_w[RASTER_WAVES][WAVE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t t = (int64_t)blockIdx.x * RASTER_WAVES + w;
    if (t >= tiles_i) return;
    const uint2 rg = ranges_i[t];
    if (rg.y <= rg.x) return;
    const TileCell tc = tile_cell(views, nv, tiles_c + t, false);
    const DevView& V = views[tc.v];
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    float acc = 0.0f;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += WAVE) {
        const uint32_t e = b0 + lane;
        uint64_t m = 0ull;
        if (e < rg.y) {
            const uint32_t r = pvals[cap_c + e];
            const float4 g = iq[r];
            const float2 g2 = iw[r];
            s_q[w][lane] = g;
            s_w[w][lane] = g2;
            if (g2.y != 0.0f)   // zero intensity adds nothing
                m = footprint_mask(g.x, g.y, g.z, g.w, g2.x, rp.q_max, tc.tx, tc.ty);
        }
        wave_lds_sync();
        // the transpose exchanges bits between lanes: every lane takes part,
        // pixels outside the image drop their column afterwards
        uint64_t col = transpose64(m);
        if (!tc.inside) col = 0ull;
        while (col != 0ull) {
            const int j = __builtin_ctzll(col);
            col &= col - 1ull;
            const float4 g = s_q[w][j];
            const float2 g2 = s_w[w][j];
            const float q = quadform(g, g2.x, px - g.x, py - g.y);
            if (q < rp.q_max) acc += (__expf(-0.5f * q) - rp.eps) * rp.inv1meps * g2.y;
        }
        wave_lds_sync();
    }
    if (tc.inside) images[V.img_off + (int64_t)tc.row * V.W + tc.col] = acc;
}

// Imaging-plane backward, one thread per used record (view, Gaussian): the
// additive image formation has no order, so each thread walks its own
// footprint ellipse q < q_max row by row (exact column span from the conic,
// widened by one pixel), gathers dL/dS there and keeps dL/dI and the centre
// and conic gradients in registers -- no atomics, no tile list. It also
// clears the record's computation-plane gradient sums for pass A.
__global__ void __launch_bounds__(256)
k_image_bwd(const DevView* __restrict__ views, const DevScene* __restrict__ scenes, int nv,
            int64_t records, RasterParams rp, const uint32_t* __restrict__ status,
            const uint32_t* __restrict__ active, const float4* __restrict__ iq,
            const float2* __restrict__ iw, const float* __restrict__ prec,
            const float* __restrict__ dimg, float* __restrict__ grad_i,
            CRec* __restrict__ crec, float* __restrict__ grad_c)
{
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((int64_t)blockIdx.x * blockDim.x >= (int64_t)status[ST_ACTIVE]) return;
    unsigned long long hits = 0;
    if (t0 < (int64_t)status[ST_ACTIVE]) {
    const int64_t r = active[t0];
    const int v = find_view(nv, r, [&](int k) { return views[k].rec_off; });
    const DevView& V = views[v];
    const float4 g = iq[r];
    const float2 g2 = iw[r];
    const float a = g.z, b = g.w, c = g2.x, I = g2.y;
    const float det = a * c - b * b;
    float dI = 0.f, dcx = 0.f, dcy = 0.f, da = 0.f, db = 0.f, dc = 0.f;
    if (det > 0.0f && a > 0.0f) {
        const float qm = rp.q_max;
        const float ry = sqrtf(qm * a / det);
        const int W = V.W;
        // clamp in float before converting (far-away centres stay in range)
        const int row0 = (int)fmaxf(0.0f, ceilf(g.y - ry - 0.5f) - 1.0f);
        const int row1 = (int)fminf((float)(V.H - 1), floorf(g.y + ry - 0.5f) + 1.0f);
        // the column span only bounds the pixels tested (one pixel of slack
        // each side; q < q_max decides), so 1/a by one reciprocal is enough
        const float inv_a = 1.0f / a;
        const float* G = dimg + V.img_off;
        for (int row = row0; row <= row1; ++row) {
            const float dy = row + 0.5f - g.y;
            const float D = a * qm - det * dy * dy;
            if (D < -1e-4f * a * qm) continue;   // rows an FP32 q < q_max can still reach
            const float half = sqrtf(fmaxf(D, 0.0f)) * inv_a;
            const float xc = g.x - b * dy * inv_a;
            const int col0 = (int)fmaxf(0.0f, ceilf(xc - half - 0.5f) - 1.0f);
            const int col1 = (int)fminf((float)(W - 1), floorf(xc + half - 0.5f) + 1.0f);
            const float* Grow = G + (int64_t)row * W;
            // four columns' cotangents load together (a load per pixel, each
            // waited for, left every pixel a full memory latency)
            for (int c0 = col0; c0 <= col1; c0 += 4) {
                float Gq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) Gq[u] = c0 + u <= col1 ? Grow[c0 + u] : 0.0f;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int col = c0 + u;
                    if (col > col1) break;
                    const float dx = col + 0.5f - g.x;
                    const float q = quadform(g, c, dx, dy);
                    if (!(q < qm)) continue;
                    ++hits;
                    const float Gp = Gq[u];
                    const float e = __expf(-0.5f * q);
                    dI += Gp * (e - rp.eps) * rp.inv1meps;
                    const float dq = Gp * I * (-0.5f * e * rp.inv1meps);
                    dcx += -2.0f * dq * (a * dx + b * dy);
                    dcy += -2.0f * dq * (b * dx + c * dy);
                    da += dq * dx * dx;
                    db += 2.0f * dq * dx * dy;
                    dc += dq * dy * dy;
                }
            }
        }
    }
    float4* gi = reinterpret_cast<float4*>(grad_i + r * GC_STRIDE);
    gi[0] = make_float4(dcx, dcy, da, db);
    gi[1] = make_float4(dc, dI, 0.0f, 0.0f);
    // c = P dL/dI for pass A (P the record's phase factor), in the record
    // pass A's backward gathers per hit
    reinterpret_cast<float*>(&crec[r].w)[3] =
        (prec ? prec[r] : scenes[V.scene].amp[r - V.rec_off] * (float)V.pscale) * dI;
    // pass A backward adds into the record's computation-plane sums
    float4* gc = reinterpret_cast<float4*>(grad_c + r * GC_STRIDE);
    gc[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    gc[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    if (rp.work) {   // one atomic per wave
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1)
            hits += (unsigned long long)__shfl_xor((long long)hits, d, WAVE);
        if (lane_id() == 0 && hits) atomicAdd(&rp.work[3], hits);
    }
}

// Pass A backward, same tiling, chunk batches and hit compaction as the
// forward, but back to front from each ray's last contributing entry:
// tau -= kappa f, dL/dalpha = exp(-tau) (c - U), U <- c alpha + (1 - alpha) U,
// with c = P dL/dI. A ray takes part in a chunk only if it used an entry at
// or past the chunk's start in the forward, so the chunks behind the point
// where most rays saturated are skipped as in the forward. Within a round
// (lane = hit, hits of a ray back to front) the optical depth is a
// segmented prefix sum and U a segmented prefix composition of the affine
// maps U -> (1 - alpha) U + c alpha. The six per-entry gradient sums collect
// in LDS and leave with one global atomic each per (tile, entry).
// Two variants, by list length (the worklist holds the long lists first;
// when long lists are the majority the first variant runs every tile):
//   FLUSHER (lists of at least 2^(LONG_LIST_BITS - 1) entries): a second wave
//     of the workgroup sends each batch's atomics while the first goes on,
//     so a long chain of batches never waits on them; two sum buffers and
//     two copies picked by ray (fewer same-address LDS atomics);
//   short lists: one wave sends its own atomics, one buffer and one copy:
//     less than half the LDS, so more tiles run per CU.
constexpr int LONG_LIST_BITS = 12;

template <bool FLUSHER, bool DET>
__global__ void __launch_bounds__(FLUSHER ? 2 * WAVE : WAVE) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_raster_a_bwd(const DevView* __restrict__ views, int nv,
               RasterParams rp, const uint32_t* __restrict__ status,
               const uint32_t* __restrict__ worklist, const uint2* __restrict__ ranges,
               const uint32_t* __restrict__ pvals, const uint64_t* __restrict__ pmask,
               const uint64_t* __restrict__ psum, const CRec* __restrict__ crec,
               const float* __restrict__ tau, const uint32_t* __restrict__ nlast,
               float* __restrict__ grad_c, int64_t stride)
{
    constexpr int NB = 2 * A_BATCH;
    constexpr int HKB = NB <= 8 ? 3 : 4;   // bits of a hit's chunk index
    constexpr int HRS = 6 + HKB;           // shift of a hit's ray index
    static_assert(NB <= 16, "hits are packed in 16 bits");
    __shared__ float4 s_q[NB][WAVE];
    __shared__ float s_wc[NB][WAVE], s_wk[NB][WAVE];   // conic c and extinction
    __shared__ float s_c[NB][WAVE];                    // c = P dL/dI of the entry
    // per-entry gradient sums in GC copies, picked by ray so that the hits
    // of one entry from neighbouring rays in a round add to different
    // addresses (rows padded by one word: copies and rows differ in bank)
    constexpr int GC = FLUSHER ? 2 : 1;
    // two buffers with the flusher: the second wave of the workgroup sends
    // one batch's sums with atomics while the first accumulates the next
    // batch in the other
    constexpr int GB = FLUSHER ? 2 : 1;
    __shared__ float s_G[GB][GC][NB][6][WAVE + 1];
    __shared__ uint32_t s_rf[GB][FLUSHER ? NB : 1][WAVE];   // records of the handed-off entries
    __shared__ uint32_t s_cmd[GB][WAVE];      // per entry lane: chunks gathered (bits), last flag
    __shared__ uint32_t s_chk[NB];
    __shared__ uint16_t s_hit[WAVE * WAVE];   // (ray, chunk, entry) packed, ray-major, back to front
    // per ray during a chunk: first hit in s_hit, optical depth, U
    struct alignas(16) RayB { uint32_t o; float t, U, pad; };
    __shared__ RayB s_ray[WAVE];
    // worklist entries [0, nlong) hold the long lists; when they are the
    // majority the run is bound by their chains and the flusher variant
    // takes every tile (short ones then fill its gaps)
    const uint32_t ntiles = status[ST_WORK_TILES];
    uint32_t nlong = status[WL_BINS_WORD + 33 + LONG_LIST_BITS];
    if (2u * nlong >= ntiles) nlong = ntiles;
    const uint32_t wi = FLUSHER ? blockIdx.x : nlong + blockIdx.x;
    if (wi >= (FLUSHER ? nlong : ntiles)) return;
    // tiles whose hits the forward stored run in k_raster_a_bwd_hits
    if (!DET && rp.hits != nullptr && rp.hit_tail[worklist[wi]] != HIT_OVERFLOW) return;
    constexpr uint32_t LAST = 1u << 31;
    if (FLUSHER && threadIdx.x >= WAVE) {
        // the flusher: per hand-off, the six sums of every handed-off entry
        // leave with one atomic each, and the buffer is cleared for reuse
        const int fl = threadIdx.x - WAVE;
        for (int hb = 0;; hb ^= 1) {
            __syncthreads();
            const uint32_t cmd = s_cmd[hb][fl];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (!(cmd & (1u << k))) continue;
                const uint32_t rk = s_rf[hb][k][fl];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    float v = 0.0f;
#pragma unroll
                    for (int g = 0; g < GC; ++g) {
                        v += s_G[hb][g][k][c][fl];
                        s_G[hb][g][k][c][fl] = 0.0f;
                    }
                    if (v == 0.0f) continue;
                    if constexpr (DET) rp.part[c * rp.part_stride + rk] = v;
                    else unsafeAtomicAdd(&grad_c[(int64_t)rk * GC_STRIDE + c], v);
                }
            }
            if (cmd & LAST) return;
        }
    }
    const int lane = threadIdx.x;
    const int64_t bucket = worklist[wi];
    const TileCell tc = tile_cell(views, nv, bucket, true);
    const DevView& V = views[tc.v];
    const float x0 = (float)(tc.tx * TILE) + 0.5f, y0 = (float)(tc.ty * TILE) + 0.5f;
    const uint2 rg = ranges[bucket];
    const int64_t ray = V.ray_off + (int64_t)tc.row * V.Wc + tc.col;
    const uint32_t n_mine = tc.inside ? nlast[ray] : 0u;   // entries [0, n_mine) were used
    float t = tc.inside ? tau[ray] : 0.0f;
    float U = 0.0f;
#pragma unroll
    for (int b = 0; b < GB; ++b)
#pragma unroll
        for (int g = 0; g < GC; ++g)
#pragma unroll
            for (int k = 0; k < NB; ++k)
#pragma unroll
                for (int c = 0; c < 6; ++c) s_G[b][g][k][c][lane] = 0.0f;
    unsigned long long n_iter = 0, n_hits = 0;   // work counters
    unsigned long long n_batch = 0, n_group = 0;
    const uint32_t n_max = wave_max_u32(n_mine);
    const uint32_t e_end = rg.x + n_max;           // exclusive end of the used entries
    // the six per-entry sums of the last processed batch leave once the next
    // batch's loads have landed: handed to the flusher wave (the barrier also
    // returns the buffer it emptied last), or sent by this wave before the
    // next batch accumulates into the same buffer
    uint32_t got_prev = 0u;
    // where each entry's sums go: its record, or in deterministic mode its
    // pair's position before the sort
    uint32_t r_prev[NB], r_cur[NB];
    int hb = 0;                        // buffer the current batch accumulates in
    auto flush = [&](bool last) {
        if constexpr (FLUSHER) {
#pragma unroll
            for (int k = 0; k < NB; ++k) s_rf[hb][k][lane] = r_prev[k];
            s_cmd[hb][lane] = got_prev | (last ? LAST : 0u);
            __syncthreads();
            hb ^= 1;
        } else {
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (!(got_prev & (1u << k))) continue;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const float v = s_G[0][0][k][c][lane];
                    s_G[0][0][k][c][lane] = 0.0f;
                    if (v == 0.0f) continue;
                    if constexpr (DET) rp.part[c * rp.part_stride + r_prev[k]] = v;
                    else unsafeAtomicAdd(&grad_c[(int64_t)r_prev[k] * GC_STRIDE + c], v);
                }
            }
            wave_lds_sync();
        }
        got_prev = 0u;
    };
    // One round of up to 64 hits, lane = hit (each ray's hits contiguous,
    // back to front; `head` marks a ray's first hit in the round, rs is its
    // state before the round): optical depths and U by segmented scans, the
    // per-entry gradient sums into LDS, each ray's state after its last hit
    // back to s_ray.
    auto hit_round = [&](const uint32_t hv, const bool valid, const bool head, const RayB rs) {
        const int rr = (int)(hv >> HRS), k = (int)((hv >> 6) & ((1u << HKB) - 1u)),
                  j = (int)(hv & 63u);
        const float4 g = s_q[k][j];
        const float2 g2 = make_float2(s_wc[k][j], s_wk[k][j]);
        const float cj = s_c[k][j];
        bool real = false;
        float x = 0.0f, E = 1.0f, ex = 0.0f, f = 0.0f, dx = 0.0f, dy = 0.0f;
        float c = 0.0f;
        if (valid) {
            dx = x0 + (float)(rr & (TILE - 1)) - g.x;
            dy = y0 + (float)(rr / TILE) - g.y;
            const float q = quadform(g, g2.x, dx, dy);
            if (q < rp.q_max) {
                real = true;
                c = cj;
                ex = __expf(-0.5f * q);
                f = (ex - rp.eps) * rp.inv1meps;
                x = g2.y * f;
                E = __expf(-x);
            }
        }
        const float sx = seg_incl_scan(x, head);   // this and the later hits
        float sa = E, sb = real ? c * (1.0f - E) : 0.0f;
        seg_incl_affine(sa, sb, head);
        float ea = __int_as_float(from_lane_below(__float_as_int(sa)));
        float eb = __int_as_float(from_lane_below(__float_as_int(sb)));
        if (head) {
            ea = 1.0f;
            eb = 0.0f;
        }
        const float tr = valid ? rs.t : 0.0f;
        const float Ur = valid ? rs.U : 0.0f;
        if (real) {
            float dalpha;
            if (rp.shadowing) {
                const float Tn = __expf(-fmaxf(tr - sx, 0.0f));
                dalpha = Tn * (c - (ea * Ur + eb));
            } else {
                dalpha = c;
            }
            const float dxx = dalpha * E;   // d alpha / d x = exp(-x)
            const float dq = dxx * g2.y * (-0.5f * ex * rp.inv1meps);
            const int gc = (rr + (rr >> 3)) & (GC - 1);
            atomicAdd(&s_G[hb][gc][k][0][j], -2.0f * dq * (g.z * dx + g.w * dy));
            atomicAdd(&s_G[hb][gc][k][1][j], -2.0f * dq * (g.w * dx + g2.x * dy));
            atomicAdd(&s_G[hb][gc][k][2][j], dq * dx * dx);
            atomicAdd(&s_G[hb][gc][k][3][j], 2.0f * dq * dx * dy);
            atomicAdd(&s_G[hb][gc][k][4][j], dq * dy * dy);
            atomicAdd(&s_G[hb][gc][k][5][j], dxx * f);
        }
        const uint64_t hbits = __ballot(real);
        if (lane == 0) n_hits += (unsigned long long)__popcll(hbits);
        const int nxt = from_lane_above(valid ? (int)hv : -1);
        const bool endseg = valid && (lane == WAVE - 1 || (nxt >> HRS) != rr);
        wave_lds_sync();
        if (endseg && rp.shadowing) s_ray[rr] = RayB{rs.o, tr - sx, sa * Ur + sb, 0.0f};
        wave_lds_sync();
    };
    const int64_t c_first = rg.x / WAVE, c_end = (int64_t)(e_end + WAVE - 1) / WAVE;
    for (int64_t g1 = c_end; g1 > c_first && n_max > 0u; g1 -= WAVE) {
        const int64_t g0 = max(c_first, g1 - (int64_t)WAVE);
        // lane = chunk g0 + lane: the rays that used an entry at or past its start
        const int64_t cpos = (g0 + lane) * WAVE - (int64_t)rg.x;
        uint64_t live_c = 0ull;
        for (int rr = 0; rr < WAVE; ++rr) {
            const uint32_t nm = (uint32_t)__builtin_amdgcn_readlane((int)n_mine, rr);
            if ((int64_t)nm > cpos) live_c |= 1ull << rr;
        }
        const uint64_t sm = g0 + lane < g1 ? psum[g0 + lane] : 0ull;
        uint64_t todo = __ballot((sm & live_c) != 0ull);   // chunks to read, back to front
        // up to NB chunks per batch: their masks and values are fetched one
        // batch ahead (in flight while the current batch's hits are
        // processed), then the records the rays need
        uint32_t chk_n[NB], rec_n[NB], r_n[NB];
        uint64_t lv_n[NB], m_n[NB];
        int nb_n = 0;
        auto fetch = [&]() {
            nb_n = 0;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                chk_n[k] = 0u;
                lv_n[k] = 0ull;
                if (todo != 0ull) {
                    const int hi = 63 - __builtin_clzll(todo);
                    todo &= ~(1ull << hi);
                    chk_n[k] = (uint32_t)g0 + (uint32_t)hi;
                    const uint32_t l0 =
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)live_c, hi);
                    const uint32_t l1 =
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(live_c >> 32), hi);
                    lv_n[k] = ((uint64_t)l1 << 32) | l0;
                    nb_n = k + 1;
                }
            }
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const uint32_t e = chk_n[k] * WAVE + lane;
                const bool in = k < nb_n && e >= rg.x && e < e_end;
                m_n[k] = in ? pmask[e] : 0ull;
                rec_n[k] = in ? pvals[e] : 0u;
                if constexpr (DET) r_n[k] = in ? rp.ppos[e] : 0u;
                else r_n[k] = rec_n[k];
            }
        };
        fetch();
        while (nb_n > 0) {
            ++n_batch;
            uint32_t got = 0u;
            const int nb = nb_n;
            uint64_t m[NB];   // lane = entry: the cells it covers
            {
                uint32_t chk[NB];
                uint64_t lv[NB];
                uint32_t* r = r_cur;
                uint32_t rec[NB];
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    chk[k] = chk_n[k];
                    lv[k] = lv_n[k];
                    m[k] = m_n[k];
                    rec[k] = rec_n[k];
                    r[k] = r_n[k];
                }
                // records straight into LDS, all in flight together (entries
                // no ray needs read record 0 of the view, one shared line)
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const bool need = (m[k] & lv[k]) != 0ull;
                    got |= need ? 1u << k : 0u;
                    const uint32_t rk = need ? rec[k] : (uint32_t)V.rec_off;
                    const float* w = reinterpret_cast<const float*>(&crec[rk].w);
                    load16_to_lds(&crec[rk].q, &s_q[k][0]);
                    load4_to_lds(w, &s_wc[k][0]);
                    load4_to_lds(w + 1, &s_wk[k][0]);
                    load4_to_lds(w + 3, &s_c[k][0]);
                }
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (lane == k) s_chk[k] = chk[k];
            }
            wait_all_memory();
            wave_lds_sync();
            fetch();   // the next batch's masks and values
            flush(false);
            got_prev = got;
#pragma unroll
            for (int k = 0; k < NB; ++k) r_prev[k] = r_cur[k];
            // the batch's chunks, transposed: bit j of col[k] is entry j of
            // chunk k covering my cell that my ray used in the forward
            // (all eight transposed together, as in the forward; the hit
            // totals summed two to a word)
            static_assert(NB % 2 == 0, "hit totals are summed in pairs");
            uint64_t col[NB];
            uint32_t hk[NB];   // hits of each chunk over the wave
#pragma unroll
            for (int k = 0; k < NB; ++k) col[k] = m[k];
            transpose64_n(col);
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                uint64_t used = 0ull;
                if (k < nb) {
                    const int64_t pos0 = (int64_t)s_chk[k] * WAVE - rg.x;
                    const int64_t nu = (int64_t)n_mine - pos0;   // used: positions < n_mine
                    used = nu >= WAVE ? ~0ull : (nu <= 0 ? 0ull : ((1ull << nu) - 1ull));
                }
                col[k] &= used;
            }
            {
                uint32_t tot[NB / 2];
#pragma unroll
                for (int i = 0; i < NB / 2; ++i)
                    tot[i] = (uint32_t)__popcll(col[2 * i]) |
                             ((uint32_t)__popcll(col[2 * i + 1]) << 16);
                wave_total_u32_n(tot);
#pragma unroll
                for (int i = 0; i < NB / 2; ++i) {
                    hk[2 * i] = tot[i] & 0xFFFFu;
                    hk[2 * i + 1] = tot[i] >> 16;
                }
            }
            // groups of consecutive chunks whose hits fit s_hit; each group's
            // hits are compacted ray-major, back to front (the batch's chunks
            // come back to front), and taken 64 per round
            for (int g0 = 0; g0 < nb;) {
                ++n_group;
                int g1 = g0;
                uint32_t H = 0;
                bool open = true;
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    if (k < g0 || k >= nb || !open) continue;
                    if (H + hk[k] <= (uint32_t)(WAVE * WAVE)) {
                        H += hk[k];
                        g1 = k + 1;
                    } else {
                        open = false;
                    }
                }
                uint32_t nr = 0;
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (k >= g0 && k < g1) nr += (uint32_t)__popcll(col[k]);
                const uint32_t o = wave_excl_scan_u32(nr);
                if (H > 0u) {
                    uint32_t w = o;
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        if (k < g0 || k >= g1) continue;
                        uint64_t c = col[k];
                        while (c != 0ull) {
                            const int j = 63 - __builtin_clzll(c);
                            c &= ~(1ull << j);
                            s_hit[w++] = (uint16_t)((lane << HRS) | (k << 6) | j);
                        }
                    }
                    s_ray[lane] = RayB{o, t, U, 0.0f};
                    wave_lds_sync();
                    for (uint32_t base = 0; base < H; base += WAVE) {
                        ++n_iter;
                        const uint32_t L = base + lane;
                        const bool valid = L < H;
                        const uint32_t hv = valid ? (uint32_t)s_hit[L] : 0u;
                        // ray state (lanes past the last hit read ray 0 and ignore it)
                        const RayB rs = s_ray[hv >> HRS];
                        const int seg0 = valid ? max((int)rs.o - (int)base, 0) : lane;
                        hit_round(hv, valid, lane == seg0, rs);
                    }
                    {
                        const RayB rs = s_ray[lane];
                        t = rs.t;
                        U = rs.U;
                    }
                    wave_lds_sync();
                }
                g0 = g1;
            }
            wave_lds_sync();
        }
    }
    flush(true);
    if (rp.work) {
        n_hits = wave_sum_u64(n_hits);
        if (lane == 0) {
            atomicAdd(&rp.work[5], n_iter);
            atomicAdd(&rp.work[1], n_hits);
            atomicMax(&rp.work[9], n_batch);
            atomicAdd(&rp.work[11], n_group - n_batch);
            atomicAdd(&rp.work[FLUSHER ? 14 : 15], 1ull);
            atomicAdd(&rp.work[17], 1ull);
        }
    }
}

// Pass A backward over the hits the forward stored (RasterParams::hits).
// The tile's records are walked back to front, 64 hits a round, each round
// from the back of one record (one hit group of the forward, so each ray's
// hits are contiguous and back to front, as the segmented scans need). A
// hit gathers its list entry's record into registers; loads run ahead of
// the arithmetic (hit words HB_HIT_AHEAD rounds, records HB_REC_AHEAD
// rounds). The six gradient terms collect per entry slot of the record in
// LDS; once per record a second wave, while the first goes on, stores each
// touched entry's six sums with plain stores at its pair's position before
// the pair sort and marks it, and launch_reduce_touched adds them per
// record (float atomics, one per sum, would cost several times the whole
// pass); an entry whose record has no other tile stores its sums as the
// record's directly. Only these sums and the rays' state live in LDS, so many tiles
// run per CU. Records that do not fit the stream, links that do not go
// back in it, record ids past the record count and list positions past the
// pair count end the walk or are skipped, so a stream that holds anything
// else cannot send the kernel out of bounds.
constexpr int HB_HIT_AHEAD = 4, HB_REC_AHEAD = 2;
constexpr int HB_SLOTS = 8 * WAVE;   // entry slots of a record (chunks x entries)

__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

__global__ void __launch_bounds__(2 * WAVE)
k_raster_a_bwd_hits(const DevView* __restrict__ views, int nv, RasterParams rp,
                    const uint32_t* __restrict__ status, const uint32_t* __restrict__ worklist,
                    const CRec* __restrict__ crec, const float* __restrict__ tau,
                    float* __restrict__ grad_c, int64_t stride)
{
    // two buffers of per-slot sums and the record of each touched slot
    // (HIT_NONE: untouched); the flusher empties one while the main wave
    // fills the other
    __shared__ float s_G[2][6][HB_SLOTS];
    __shared__ uint32_t s_rec[2][HB_SLOTS];
    __shared__ unsigned char s_one[2][HB_SLOTS];   // the record has only this tile
    __shared__ uint32_t s_last[2], s_hrec[2];   // per hand-off: last one?, the stream record
    __shared__ float2 s_ray[WAVE];   // per ray: optical depth, U
    if (blockIdx.x >= status[ST_WORK_TILES]) return;
    const int64_t bucket = worklist[blockIdx.x];
    const uint32_t tail = rp.hit_tail[bucket];
    if (tail == HIT_OVERFLOW) return;   // k_raster_a_bwd re-derives this tile's hits
    for (int i = threadIdx.x; i < 2 * HB_SLOTS; i += 2 * WAVE) {
        (&s_rec[0][0])[i] = HIT_NONE;
#pragma unroll
        for (int c = 0; c < 6; ++c) s_G[i / HB_SLOTS][c][i % HB_SLOTS] = 0.0f;
    }
    __syncthreads();
    if (threadIdx.x >= WAVE) {
        // the flusher: per hand-off, each touched slot's sums to its pair's
        // partial (slot = chunk * 64 + entry; the record's header holds the
        // chunks' list positions), and the buffer cleared for reuse
        const int fl = threadIdx.x - WAVE;
        const uint32_t kc = status[ST_PAIRS_C];
        const uint32_t* hw32 = reinterpret_cast<const uint32_t*>(rp.hits);
        constexpr int NBLK = HB_SLOTS / WAVE;
        for (int fb = 0;; fb ^= 1) {
            __syncthreads();
            const uint32_t hr = s_hrec[fb];
            const uint32_t chw = hr != HIT_NONE && fl < 8 ? hw32[((uint64_t)hr + 1) * 4 + fl] : 0u;
            // every slot's pair position in flight together (one latency),
            // the sums read and cleared, then all the stores (no store waits
            // on another)
            uint32_t rk[NBLK], pp[NBLK];
            bool one[NBLK];
#pragma unroll
            for (int i = 0; i < NBLK; ++i) {
                const int sl = i * WAVE + fl;
                rk[i] = s_rec[fb][sl];
                one[i] = s_one[fb][sl] != 0;
                const uint32_t pos = (uint32_t)__builtin_amdgcn_readlane((int)chw, i) * WAVE + fl;
                pp[i] = rk[i] != HIT_NONE && !one[i] && pos < kc ? rp.hit_ppos[pos] : kc;
            }
            float v[NBLK][6];
#pragma unroll
            for (int i = 0; i < NBLK; ++i) {
                const int sl = i * WAVE + fl;
#pragma unroll
                for (int c = 0; c < 6; ++c) v[i][c] = 0.0f;
                if (rk[i] == HIT_NONE) continue;
                s_rec[fb][sl] = HIT_NONE;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    v[i][c] = s_G[fb][c][sl];
                    s_G[fb][c][sl] = 0.0f;
                }
            }
            // one store path: a record with no other tile takes its sums
            // directly (its eight floats: six sums and two spare), any other
            // entry its pair's partial row (six sums, the record, a spare);
            // the mark of a direct store lands in the spare byte at the pair
            // count, which the reduction never reads
#pragma unroll
            for (int i = 0; i < NBLK; ++i) {
                if (rk[i] == HIT_NONE || (!one[i] && pp[i] >= kc)) continue;
                float4* dst = reinterpret_cast<float4*>(
                    one[i] ? grad_c + (int64_t)rk[i] * GC_STRIDE
                           : rp.hit_part + (uint64_t)pp[i] * HIT_PART_STRIDE);
                dst[0] = make_float4(v[i][0], v[i][1], v[i][2], v[i][3]);
                dst[1] = make_float4(v[i][4], v[i][5], __uint_as_float(rk[i]), 0.0f);
                rp.hit_touched[one[i] ? kc : pp[i]] = 1;
            }
            if (s_last[fb]) return;
        }
    }
    const int lane = threadIdx.x;
    const TileCell tc = tile_cell(views, nv, bucket, true);
    const DevView& V = views[tc.v];
    const uint32_t rec0 = (uint32_t)V.rec_off;   // read by lanes without a hit
    const float x0 = (float)(tc.tx * TILE) + 0.5f, y0 = (float)(tc.ty * TILE) + 0.5f;
    const int64_t ray = V.ray_off + (int64_t)tc.row * V.Wc + tc.col;
    s_ray[lane] = make_float2(tc.inside ? tau[ray] : 0.0f, 0.0f);
    const unsigned long long* hw = reinterpret_cast<const unsigned long long*>(rp.hits);
    const uint64_t cap = rp.hit_cap;
    unsigned long long n_iter = 0, n_hits = 0, n_batch = 0;   // work counters

    // the cursor (wave-uniform): the record rounds are taken from, its hits
    // not yet taken, the record before it and that one's header, loaded
    // when the cursor enters a record
    uint32_t cur = HIT_NONE, left = 0u, prev = HIT_NONE;
    unsigned long long pend = 0ull;
    auto enter = [&](uint32_t r, unsigned long long h) {
        const uint32_t kept = (uint32_t)(h >> 32), pv = (uint32_t)h;
        if (kept == 0u || (uint64_t)r + HIT_HEADER_UNITS + (kept + 1u) / 2u > cap) {
            cur = HIT_NONE;
            return;
        }
        ++n_batch;
        cur = r;
        left = kept;
        prev = pv < r ? pv : HIT_NONE;
        if (prev != HIT_NONE) pend = hw[(uint64_t)prev * 2];
    };
    // the next round: index of its first hit word in the stream, its hit
    // count (0 once the chain is done; lane i takes word base + n - 1 - i),
    // whether it ends its record and the record
    auto next = [&](uint64_t& base, uint32_t& n, bool& last, uint32_t& rec) {
        if (cur != HIT_NONE && left == 0u) {
            if (prev == HIT_NONE) cur = HIT_NONE;
            else enter(prev, uniform_u64(pend));
        }
        rec = cur;
        if (cur == HIT_NONE) {
            base = 0;
            n = 0u;
            last = true;
            return;
        }
        n = min(left, (uint32_t)WAVE);
        left -= n;
        base = ((uint64_t)cur + HIT_HEADER_UNITS) * 2 + left;
        last = left == 0u;
    };
    if ((uint64_t)tail + HIT_HEADER_UNITS <= cap) enter(tail, uniform_u64(hw[(uint64_t)tail * 2]));

    struct Rec { float4 q; float2 w; float c; bool one; };
    auto load_hit = [&](uint64_t base, uint32_t n) {
        return (uint32_t)lane < n ? hw[base + n - 1u - (uint32_t)lane] : 0ull;
    };
    auto gather = [&](unsigned long long h, uint32_t n) {
        const uint32_t id = (uint32_t)h;
        const uint32_t rk = ((uint32_t)lane < n && (int64_t)id < stride) ? id : rec0;
        Rec g;
        g.q = crec[rk].q;
        const float4 w = crec[rk].w;
        g.w = make_float2(w.x, w.y);
        g.one = __float_as_uint(w.z) == 1u;
        g.c = w.w;
        return g;
    };
    uint64_t b[HB_HIT_AHEAD + 1];
    uint32_t nn[HB_HIT_AHEAD + 1];
    bool ends[HB_HIT_AHEAD + 1];
    uint32_t rc[HB_HIT_AHEAD + 1];
    unsigned long long h[HB_HIT_AHEAD + 1];
    Rec g[HB_REC_AHEAD + 1];
#pragma unroll
    for (int i = 0; i <= HB_HIT_AHEAD; ++i) {
        next(b[i], nn[i], ends[i], rc[i]);
        h[i] = load_hit(b[i], nn[i]);
    }
#pragma unroll
    for (int i = 0; i < HB_REC_AHEAD; ++i) g[i] = gather(h[i], nn[i]);
    wave_lds_sync();
    int hb = 0;   // buffer the current record's sums go to
    while (nn[0] > 0u) {
        ++n_iter;
        g[HB_REC_AHEAD] = gather(h[HB_REC_AHEAD], nn[HB_REC_AHEAD]);
        // the round: lane = hit, each ray's hits back to front
        const bool valid = (uint32_t)lane < nn[0];
        const uint32_t id = (uint32_t)h[0];
        const int rr = valid ? (int)((h[0] >> 32) & (uint64_t)(WAVE - 1)) : 0;
        const int sl = (int)((h[0] >> 40) & (uint64_t)(HB_SLOTS - 1));
        const float2 rs = s_ray[rr];
        // the neighbours' rays, read by every lane (a cross-lane read inside
        // a condition would see the lanes it skips as zero)
        const int key = valid ? rr : -1;
        const int below = from_lane_below(key), above = from_lane_above(key);
        const bool head = !valid || lane == 0 || below != rr;
        const float4 q = g[0].q;
        const float2 w = g[0].w;   // conic c, extinction
        bool real = false;
        float x = 0.0f, E = 1.0f, ex = 0.0f, f = 0.0f, dx = 0.0f, dy = 0.0f, c = 0.0f;
        if (valid && (int64_t)id < stride) {
            dx = x0 + (float)(rr & (TILE - 1)) - q.x;
            dy = y0 + (float)(rr / TILE) - q.y;
            const float qf = quadform(q, w.x, dx, dy);
            if (qf < rp.q_max) {
                real = true;
                c = g[0].c;
                ex = __expf(-0.5f * qf);
                f = (ex - rp.eps) * rp.inv1meps;
                x = w.y * f;
                E = __expf(-x);
            }
        }
        const float sx = seg_incl_scan(x, head);   // this and the later hits
        float sa = E, sb = real ? c * (1.0f - E) : 0.0f;
        seg_incl_affine(sa, sb, head);
        float ea = __int_as_float(from_lane_below(__float_as_int(sa)));
        float eb = __int_as_float(from_lane_below(__float_as_int(sb)));
        if (head) {
            ea = 1.0f;
            eb = 0.0f;
        }
        const float tr = valid ? rs.x : 0.0f;
        const float Ur = valid ? rs.y : 0.0f;
        if (real) {
            float dalpha;
            if (rp.shadowing) {
                const float Tn = __expf(-fmaxf(tr - sx, 0.0f));
                dalpha = Tn * (c - (ea * Ur + eb));
            } else {
                dalpha = c;
            }
            const float dxx = dalpha * E;   // d alpha / d x = exp(-x)
            const float dq = dxx * w.y * (-0.5f * ex * rp.inv1meps);
            s_rec[hb][sl] = id;
            s_one[hb][sl] = g[0].one ? 1 : 0;
            atomicAdd(&s_G[hb][0][sl], -2.0f * dq * (q.z * dx + q.w * dy));
            atomicAdd(&s_G[hb][1][sl], -2.0f * dq * (q.w * dx + w.x * dy));
            atomicAdd(&s_G[hb][2][sl], dq * dx * dx);
            atomicAdd(&s_G[hb][3][sl], 2.0f * dq * dx * dy);
            atomicAdd(&s_G[hb][4][sl], dq * dy * dy);
            atomicAdd(&s_G[hb][5][sl], dxx * f);
        }
        const uint64_t hbits = __ballot(real);
        if (lane == 0) n_hits += (unsigned long long)__popcll(hbits);
        const bool endseg = valid && (lane == WAVE - 1 || above != rr);
        wave_lds_sync();
        if (endseg && rp.shadowing) s_ray[rr] = make_float2(tr - sx, sa * Ur + sb);
        wave_lds_sync();
        if (ends[0]) {
            // the record's sums to the flusher (the barrier also returns the
            // buffer it emptied last)
            if (lane == 0) {
                s_last[hb] = nn[1] == 0u ? 1u : 0u;
                s_hrec[hb] = rc[0];
            }
            __syncthreads();
            hb ^= 1;
        }
#pragma unroll
        for (int i = 0; i < HB_HIT_AHEAD; ++i) {
            b[i] = b[i + 1];
            nn[i] = nn[i + 1];
            ends[i] = ends[i + 1];
            rc[i] = rc[i + 1];
            h[i] = h[i + 1];
        }
#pragma unroll
        for (int i = 0; i < HB_REC_AHEAD; ++i) g[i] = g[i + 1];
        next(b[HB_HIT_AHEAD], nn[HB_HIT_AHEAD], ends[HB_HIT_AHEAD], rc[HB_HIT_AHEAD]);
        h[HB_HIT_AHEAD] = load_hit(b[HB_HIT_AHEAD], nn[HB_HIT_AHEAD]);
    }
    if (n_iter == 0) {   // no round: release the flusher
        if (lane == 0) {
            s_last[hb] = 1u;
            s_hrec[hb] = HIT_NONE;
        }
        __syncthreads();
    }
    if (rp.work && lane == 0) {
        atomicAdd(&rp.work[5], n_iter);
        atomicAdd(&rp.work[1], n_hits);
        atomicMax(&rp.work[9], n_batch);
        atomicAdd(&rp.work[16], 1ull);
    }
}

// Non-empty computation-plane tiles, longest lists first (binned by the
// bit length of the list size), so the heaviest tiles start earliest. Three
// steps over global bins (bins[0..32] counts, bins[33..65] cursors): count
// per bin, turn the counts into starts (one workgroup; the tile count goes
// to status[ST_WORK_TILES]), place each tile at its bin's cursor.
__global__ void __launch_bounds__(256)
k_worklist_count(const uint2* __restrict__ ranges, int64_t tiles_c, uint32_t* __restrict__ bins)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles_c) return;
    const uint2 rg = ranges[t];
    const uint32_t len = rg.y > rg.x ? rg.y - rg.x : 0u;
    if (len) atomicAdd(&bins[32 - __clz(len)], 1u);
}

__global__ void k_worklist_starts(uint32_t* __restrict__ bins, uint32_t* __restrict__ status)
{
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int lvl = 32; lvl >= 1; --lvl) {
        bins[33 + lvl] = acc;
        acc += bins[lvl];
    }
    status[ST_WORK_TILES] = acc;
}

__global__ void __launch_bounds__(256)
k_worklist_place(const uint2* __restrict__ ranges, int64_t tiles_c, uint32_t* __restrict__ bins,
                 uint32_t* __restrict__ worklist)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles_c) return;
    const uint2 rg = ranges[t];
    const uint32_t len = rg.y > rg.x ? rg.y - rg.x : 0u;
    if (len) worklist[atomicAdd(&bins[33 + 32 - __clz(len)], 1u)] = (uint32_t)t;
}

inline unsigned raster_grid(int64_t waves)
{
    return (unsigned)((waves + RASTER_WAVES - 1) / RASTER_WAVES);
}

inline unsigned grid256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_pair_masks(const DevView* views, int nv, int64_t cap_c, const RasterParams& rp,
                             const uint32_t* status, const uint32_t* pkey,
                             const uint32_t* pvals, const CRec* crec,
                             uint64_t* pmask, uint64_t* psum, hipStream_t s)
{
    if (cap_c <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((cap_c + 256 * PM_ITEMS - 1) / (256 * PM_ITEMS));
    hipLaunchKernelGGL(k_pair_masks, dim3(grid), dim3(256), 0, s, views, nv, cap_c, rp, status,
                       pkey, pvals, crec, pmask, psum);
    return hipGetLastError();
}

hipError_t launch_tile_worklist(const uint2* ranges, int64_t tiles_c, uint32_t* worklist,
                                uint32_t* bins, uint32_t* status, hipStream_t s)
{
    hipError_t e = launch_fill_u32(bins, 0u, 66, s);
    if (e != hipSuccess) return e;
    if (tiles_c > 0)
        hipLaunchKernelGGL(k_worklist_count, dim3(grid256(tiles_c)), dim3(256), 0, s, ranges,
                           tiles_c, bins);
    hipLaunchKernelGGL(k_worklist_starts, dim3(1), dim3(64), 0, s, bins, status);
    if (tiles_c > 0)
        hipLaunchKernelGGL(k_worklist_place, dim3(grid256(tiles_c)), dim3(256), 0, s, ranges,
                           tiles_c, bins, worklist);
    return hipGetLastError();
}

hipError_t launch_raster_a_fwd(const DevView* views, int nv, int64_t tiles_c,
                               const RasterParams& rp, const uint32_t* status,
                               const uint32_t* worklist, const uint2* ranges,
                               const uint32_t* pvals, const uint64_t* pmask,
                               const uint64_t* psum, const CRec* crec,
                               float* A, float* tau, uint32_t* nlast, hipStream_t s)
{
    if (tiles_c <= 0) return hipSuccess;
    if (rp.ppos)
        hipLaunchKernelGGL(k_raster_a_fwd<true>, dim3((unsigned)tiles_c), dim3(WAVE), 0, s, views,
                           nv, rp, status, worklist, ranges, pvals, pmask, psum, crec, A, tau,
                           nlast);
    else
        hipLaunchKernelGGL(k_raster_a_fwd<false>, dim3((unsigned)tiles_c), dim3(WAVE), 0, s, views,
                           nv, rp, status, worklist, ranges, pvals, pmask, psum, crec, A, tau,
                           nlast);
    return hipGetLastError();
}

hipError_t launch_raster_b_fwd(const DevView* views, int nv, int64_t pixels, int64_t cap_c,
                               int64_t cap_i, const RasterParams& rp, const uint32_t* status,
                               const uint32_t* pkey, const uint32_t* pvals, const float4* iq,
                               const float2* iw, float* images, bool vm, hipStream_t s)
{
    if (pixels <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_images, dim3(grid256(pixels)), dim3(256), 0, s, views, nv, pixels,
                       images);
    if (cap_i <= 0) return hipGetLastError();
    const int64_t segs = (cap_i + B_SEGMENT - 1) / B_SEGMENT;
    hipLaunchKernelGGL(k_raster_b_fwd, dim3(raster_grid(segs)), dim3(RASTER_THREADS), 0, s, views,
                       nv, rp, cap_c, status, pkey, pvals, iq, iw, images, vm ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_raster_b_tiles(const DevView* views, int nv, int64_t pixels, int64_t cap_c,
                                 int64_t cap_i, int64_t tiles_c, int64_t tiles_i,
                                 const RasterParams& rp, const uint32_t* status,
                                 const uint32_t* pkey, const uint32_t* pvals, const float4* iq,
                                 const float2* iw, uint2* ranges_i, float* images, bool vm,
                                 hipStream_t s)
{
    if (pixels <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_images, dim3(grid256(pixels)), dim3(256), 0, s, views, nv, pixels,
                       images);
    if (cap_i <= 0 || tiles_i <= 0) return hipGetLastError();
    hipError_t e = launch_ranges_i(views, pkey + cap_c, status, cap_i, tiles_c, tiles_i, vm,
                                   ranges_i, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_raster_b_tile, dim3(raster_grid(tiles_i)), dim3(RASTER_THREADS), 0, s,
                       views, nv, rp, cap_c, tiles_c, tiles_i, ranges_i, pvals, iq, iw, images);
    return hipGetLastError();
}

hipError_t launch_image_bwd(const DevView* views, const DevScene* scenes, int nv,
                            int64_t records, const RasterParams& rp, const uint32_t* status,
                            const uint32_t* active, const float4* iq, const float2* iw,
                            const float* prec, const float* dimg, float* grad_i, CRec* crec,
                            float* grad_c, hipStream_t s)
{
    if (records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_image_bwd, dim3(grid256(records)), dim3(256), 0, s, views, scenes, nv,
                       records, rp, status, active, iq, iw, prec, dimg, grad_i, crec, grad_c);
    return hipGetLastError();
}

hipError_t launch_raster_a_bwd_hits(const DevView* views, int nv, int64_t tiles_c,
                                    const RasterParams& rp, const uint32_t* status,
                                    const uint32_t* worklist, const CRec* crec,
                                    const float* tau, float* grad_c, int64_t stride,
                                    hipStream_t s)
{
    if (tiles_c <= 0 || !rp.hits || rp.ppos) return hipSuccess;
    hipLaunchKernelGGL(k_raster_a_bwd_hits, dim3((unsigned)tiles_c), dim3(2 * WAVE), 0, s, views,
                       nv, rp, status, worklist, crec, tau, grad_c, stride);
    return hipGetLastError();
}

hipError_t launch_raster_a_bwd(const DevView* views, int nv, int64_t tiles_c,
                               const RasterParams& rp, const uint32_t* status,
                               const uint32_t* worklist, const uint2* ranges,
                               const uint32_t* pvals, const uint64_t* pmask,
                               const uint64_t* psum, const CRec* crec,
                               const float* tau, const uint32_t* nlast, float* grad_c,
                               int64_t stride, hipStream_t s)
{
    if (tiles_c <= 0) return hipSuccess;
    // long lists (the front of the worklist), then the short ones
    auto two = [&](auto det) {
        constexpr bool D = decltype(det)::value;
        hipLaunchKernelGGL((k_raster_a_bwd<true, D>), dim3((unsigned)tiles_c), dim3(2 * WAVE), 0,
                           s, views, nv, rp, status, worklist, ranges, pvals, pmask, psum, crec,
                           tau, nlast, grad_c, stride);
        hipLaunchKernelGGL((k_raster_a_bwd<false, D>), dim3((unsigned)tiles_c), dim3(WAVE), 0, s,
                           views, nv, rp, status, worklist, ranges, pvals, pmask, psum, crec,
                           tau, nlast, grad_c, stride);
    };
    if (rp.ppos)
        two(std::true_type{});
    else
        two(std::false_type{});
    return hipGetLastError();
}

}  // namespace sdgr
