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
//   pass B forward : fixed 2048-entry segments of the sorted (tile, Gaussian)
//                    pair array, one wave each (balanced however long a
//                    tile's list is); footprint masks computed on the fly
//                    and bit-transposed, so lane = pixel sums only the
//                    entries covering it; partial pixel sums are added to
//                    the image at tile boundaries.
//   pass B backward: one thread per record walks its footprint ellipse and
//                    gathers dL/dS (no atomics).
#include "common.hpp"

namespace sdgr {
namespace {

constexpr uint32_t B_SEGMENT = 2048;   // pair entries per pass-B forward wave

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

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int d)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d, WAVE);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

// 64x64 bit-matrix transpose across the wave: on return, bit j of lane i is
// bit i of lane j's input. Recursive block swap: at step s, lanes i and
// i ^ s exchange the s-wide bit blocks that sit off the diagonal.
__device__ __forceinline__ uint64_t transpose64(uint64_t v)
{
    const int lane = lane_id();
    constexpr uint64_t LO[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull,
                                0x00FF00FF00FF00FFull, 0x0F0F0F0F0F0F0F0Full,
                                0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int s = 32 >> k;
        const uint64_t lo = LO[k];
        const uint64_t p = shfl_xor_u64(v, s);
        v = (lane & s) ? ((v & ~lo) | ((p & ~lo) >> s)) : ((v & lo) | ((p & lo) << s));
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) v += shfl_xor_u64(v, d);
    return v;
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) v |= shfl_xor_u64(v, d);
    return v;
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

__device__ __forceinline__ float quadform(float4 g, float c, float dx, float dy)
{
    return g.z * dx * dx + 2.0f * g.w * dx * dy + c * dy * dy;
}

// Cells of tile (tx, ty) inside the ellipse q < q_max of a Gaussian with
// centre (cx, cy) and conic (a, b, c): per row the exact column span from
// the quadratic, widened by a small slack. Bit 8 * row + col.
__device__ uint64_t footprint_mask(float cx, float cy, float a, float b, float c, float qm,
                                   int tx, int ty)
{
    const float det = a * c - b * b;
    if (!(det > 0.0f) || !(a > 0.0f)) return 0ull;
    const float slack = 1e-3f;
    uint64_t m = 0ull;
    const float x0 = (float)(tx * TILE);
#pragma unroll
    for (int k = 0; k < TILE; ++k) {
        const float dy = (float)(ty * TILE + k) + 0.5f - cy;
        const float D = a * qm - det * dy * dy;
        if (D < 0.0f) continue;
        const float half = sqrtf(D) / a + slack;
        const float xc = cx - b * dy / a;
        // local columns j with |x0 + j + 1/2 - xc| <= half
        const float lo = fmaxf(ceilf(xc - half - 0.5f - x0), 0.0f);
        const float hi = fminf(floorf(xc + half - 0.5f - x0), (float)(TILE - 1));
        if (lo > hi) continue;
        const uint32_t j0 = (uint32_t)lo, j1 = (uint32_t)hi;
        const uint64_t row_bits = ((1ull << (j1 - j0 + 1)) - 1ull) << j0;
        m |= row_bits << (TILE * k);
    }
    return m;
}

// Footprint mask of every computation-plane pair, and per 64-pair chunk of
// the sorted array (aligned to the array, so a chunk may span two tiles)
// the OR of its masks. Blocks are whole waves, so a wave is a chunk.
__global__ void __launch_bounds__(256)
k_pair_masks(const DevView* __restrict__ views, int nv, int64_t cap, RasterParams rp,
             const uint32_t* __restrict__ status, const uint32_t* __restrict__ pkey,
             const uint32_t* __restrict__ pvals, const float4* __restrict__ cq,
             const float2* __restrict__ cw, uint64_t* __restrict__ pmask,
             uint64_t* __restrict__ psum)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t kc = min(cap, (int64_t)status[ST_PAIRS_C]);
    if (p - lane_id() >= kc) return;   // whole wave past the end
    uint64_t m = 0ull;
    if (p < kc) {
        const uint32_t bucket = pkey[p];
        const int v = find_view(nv, (int64_t)bucket,
                                [&](int k) { return (int64_t)views[k].tile_c; });
        const DevView& V = views[v];
        const int local = (int)(bucket - (uint32_t)V.tile_c);
        const uint32_t r = pvals[p];
        const float4 g = cq[r];
        const float2 g2 = cw[r];
        m = footprint_mask(g.x, g.y, g.z, g.w, g2.x, rp.q_max, local % V.txc, local / V.txc);
        pmask[p] = m;
    }
    m = wave_or_u64(m);
    if (lane_id() == 0) psum[p / WAVE] = m;
}

// Pass A forward, one wave per non-empty 8x8 tile, lane = ray. The list
// is walked in 64-entry chunks aligned to the global pair array; a chunk
// whose footprint summary misses every ray still in play is skipped
// without reading its entries (rays at a silhouette rarely saturate, and
// the lists run to ~5e4 entries). Chunks that are read are taken AF_BATCH
// at a time: their masks are loaded together, then the records of the
// entries any live ray needs are gathered together, so one batch pays two
// memory latencies. In each chunk the 64x64 bit matrix of footprint masks
// is transposed so that each lane walks only the entries covering its own
// cell, front to back; per-entry sums go into LDS with float atomics and
// leave with one global atomic per (tile, entry).
constexpr int AF_BATCH = 8;

__global__ void __launch_bounds__(WAVE)
k_raster_a_fwd(const DevView* __restrict__ views, int nv, RasterParams rp,
               const uint32_t* __restrict__ status, const uint32_t* __restrict__ worklist,
               const uint2* __restrict__ ranges, const uint32_t* __restrict__ pvals,
               const uint64_t* __restrict__ pmask, const uint64_t* __restrict__ psum,
               const float4* __restrict__ cq, const float2* __restrict__ cw,
               float* __restrict__ A, float* __restrict__ tau, uint32_t* __restrict__ nlast)
{
    constexpr int NB = AF_BATCH;
    __shared__ float4 s_q[NB][WAVE];
    __shared__ float2 s_w[NB][WAVE];
    __shared__ float s_A[NB][WAVE];
    const int lane = threadIdx.x;
    if (blockIdx.x >= status[ST_WORK_TILES]) return;
    const int64_t bucket = worklist[blockIdx.x];
    const TileCell tc = tile_cell(views, nv, bucket, true);
    const DevView& V = views[tc.v];
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    const uint2 rg = ranges[bucket];
#pragma unroll
    for (int k = 0; k < NB; ++k) s_A[k][lane] = 0.0f;
    float T = 1.0f, t = 0.0f;
    bool alive = tc.inside;
    uint32_t last = 0;
    unsigned long long n_iter = 0, n_hits = 0;   // work counters
    uint64_t live = __ballot(alive);
    const uint32_t c_first = rg.x / WAVE, c_end = (rg.y + WAVE - 1) / WAVE;
    for (uint32_t g0 = c_first; g0 < c_end && live != 0ull; g0 += WAVE) {
        const uint64_t sm = g0 + lane < c_end ? psum[g0 + lane] : 0ull;
        uint64_t todo = __ballot((sm & live) != 0ull);   // chunks to read, in order
        while (todo != 0ull && live != 0ull) {
            uint32_t chk[NB];
            uint64_t m[NB];
            uint32_t r[NB];
            int nb = 0;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                chk[k] = 0u;
                if (todo != 0ull) {
                    chk[k] = g0 + (uint32_t)__builtin_ctzll(todo);
                    todo &= todo - 1ull;
                    nb = k + 1;
                }
            }
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const uint32_t e = chk[k] * WAVE + lane;
                const bool in = k < nb && e >= rg.x && e < rg.y;
                m[k] = in ? pmask[e] : 0ull;
                r[k] = in ? pvals[e] : 0u;
            }
            uint32_t got = 0u;   // bit k: this lane's entry of chunk k was gathered
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if ((m[k] & live) != 0ull) {
                    s_q[k][lane] = cq[r[k]];
                    s_w[k][lane] = cw[r[k]];
                    got |= 1u << k;
                }
            }
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (k >= nb || live == 0ull) break;
                if (__ballot((m[k] & live) != 0ull) == 0ull) continue;
                uint64_t col = transpose64(m[k]);   // entries covering my cell (all lanes)
                if (!alive) col = 0ull;
                const uint32_t pos0 = chk[k] * WAVE - rg.x;   // list position of entry 0
                for (;;) {
                    const bool act = alive && col != 0ull;
                    if (__ballot(act) == 0ull) break;
                    ++n_iter;
                    if (act) {
                        const int j = __builtin_ctzll(col);
                        col &= col - 1ull;
                        const float4 g = s_q[k][j];
                        const float2 g2 = s_w[k][j];
                        const float dx = px - g.x, dy = py - g.y;
                        const float q = quadform(g, g2.x, dx, dy);
                        if (q < rp.q_max) {
                            ++n_hits;
                            const float f = (__expf(-0.5f * q) - rp.eps) * rp.inv1meps;
                            const float x = g2.y * f;
                            const float E = __expf(-x);
                            atomicAdd(&s_A[k][j], (1.0f - E) * T);
                            if (rp.shadowing) T *= E;
                            t += x;
                            last = pos0 + (uint32_t)j + 1u;
                            if (rp.shadowing && t >= rp.tau_max) alive = false;
                        }
                    }
                }
                live = __ballot(alive);
            }
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (got & (1u << k)) {
                    const float a = s_A[k][lane];
                    if (a != 0.0f) unsafeAtomicAdd(&A[r[k]], a);
                    s_A[k][lane] = 0.0f;
                }
            }
            wave_lds_sync();
        }
    }
    if (rp.work) {
        n_hits = wave_sum_u64(n_hits);
        if (lane == 0) {
            atomicAdd(&rp.work[4], n_iter);
            atomicAdd(&rp.work[0], n_hits);
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

// Pass B forward over fixed 2048-entry segments of the sorted imaging-plane
// pair array (one wave each, balanced however long a tile's list is).
// Lane = entry: gather the record, compute its footprint mask on the
// entry's tile; then, per run of entries of one tile, the masks are
// bit-transposed and lane = pixel sums only the entries covering it. The
// partial pixel sums are added to the image when the tile changes.
__global__ void __launch_bounds__(RASTER_THREADS)
k_raster_b_fwd(const DevView* __restrict__ views, int nv, RasterParams rp,
               const uint32_t* __restrict__ status, const uint32_t* __restrict__ pkey,
               const uint32_t* __restrict__ pvals, const float4* __restrict__ iq,
               const float2* __restrict__ iw, float* __restrict__ images)
{
    __shared__ float4 s_q[RASTER_WAVES][WAVE];
    __shared__ float2 s_w[RASTER_WAVES][WAVE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const uint32_t kc = status[ST_PAIRS_C], ki = status[ST_PAIRS_I];
    const uint64_t seg = (uint64_t)blockIdx.x * RASTER_WAVES + w;
    const uint64_t p0 = (uint64_t)kc + seg * B_SEGMENT;
    const uint64_t pend = (uint64_t)kc + ki;
    if (p0 >= pend) return;
    const uint32_t p1 = (uint32_t)min(pend, p0 + B_SEGMENT);
    uint32_t cur = 0xFFFFFFFFu;
    float acc = 0.0f, px = 0.0f, py = 0.0f;
    int64_t pix = -1;
    unsigned long long n_iter = 0, n_hits = 0;   // work counters
    for (uint32_t b0 = (uint32_t)p0; b0 < p1; b0 += WAVE) {
        const uint32_t e = b0 + lane;
        const bool in = e < p1;
        const uint32_t key = in ? pkey[e] : 0xFFFFFFFFu;
        uint64_t m = 0ull;
        if (in) {
            const uint32_t r = pvals[e];
            const float4 g = iq[r];
            const float2 g2 = iw[r];
            s_q[w][lane] = g;
            s_w[w][lane] = g2;
            const int v = find_view(nv, (int64_t)key,
                                    [&](int k) { return (int64_t)views[k].tile_i; });
            const int local = (int)(key - (uint32_t)views[v].tile_i);
            const int txi = views[v].txi;
            if (g2.y != 0.0f)   // zero intensity adds nothing
                m = footprint_mask(g.x, g.y, g.z, g.w, g2.x, rp.q_max, local % txi, local / txi);
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
                const TileCell tc = tile_cell(views, nv, (int64_t)k, false);
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

// Imaging-plane backward, one thread per record (view, Gaussian): the
// additive image formation has no order, so each thread walks its own
// footprint ellipse q < q_max row by row (exact column span from the conic,
// widened by one pixel), gathers dL/dS there and keeps dL/dI and the centre
// and conic gradients in registers -- no atomics, no tile list.
__global__ void __launch_bounds__(256)
k_image_bwd(const DevView* __restrict__ views, int nv, int64_t records, RasterParams rp,
            const float4* __restrict__ iq, const float2* __restrict__ iw,
            const float* __restrict__ dimg, float* __restrict__ grad_i)
{
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long hits = 0;
    if (r0 < records) {
    const int64_t r = r0;
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
        // clamp in float before converting (far-away centres stay in range)
        const int row0 = (int)fmaxf(0.0f, ceilf(g.y - ry - 0.5f) - 1.0f);
        const int row1 = (int)fminf((float)(V.H - 1), floorf(g.y + ry - 0.5f) + 1.0f);
        const float* G = dimg + V.img_off;
        for (int row = row0; row <= row1; ++row) {
            const float dy = row + 0.5f - g.y;
            const float D = a * qm - det * dy * dy;
            if (D < 0.0f) continue;
            const float half = sqrtf(D) / a;
            const float xc = g.x - b * dy / a;
            const int col0 = (int)fmaxf(0.0f, ceilf(xc - half - 0.5f) - 1.0f);
            const int col1 = (int)fminf((float)(V.W - 1), floorf(xc + half - 0.5f) + 1.0f);
            for (int col = col0; col <= col1; ++col) {
                const float dx = col + 0.5f - g.x;
                const float q = quadform(g, c, dx, dy);
                if (!(q < qm)) continue;
                ++hits;
                const float Gp = G[(int64_t)row * V.W + col];
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
    grad_i[r] = dcx;
    grad_i[records + r] = dcy;
    grad_i[2 * records + r] = da;
    grad_i[3 * records + r] = db;
    grad_i[4 * records + r] = dc;
    grad_i[5 * records + r] = dI;
    }
    if (rp.work) {   // one atomic per wave
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1)
            hits += (unsigned long long)__shfl_xor((long long)hits, d, WAVE);
        if (lane_id() == 0 && hits) atomicAdd(&rp.work[3], hits);
    }
}

// Pass A backward, same tiling and batched chunk walk as the forward but
// back to front from each ray's last contributing entry: tau -= kappa f,
// dL/dalpha = exp(-tau) (c - U), U <- c alpha + (1 - alpha) U, with
// c = P dL/dI. A ray takes part in a chunk only if it used an entry at or
// past the chunk's start in the forward, so the chunks behind the point
// where most rays saturated are skipped as in the forward. The six
// per-entry gradient sums go into LDS with float atomics and leave with one
// global atomic each per (tile, entry).
constexpr int AB_BATCH = 4;

__global__ void __launch_bounds__(WAVE)
k_raster_a_bwd(const DevView* __restrict__ views, const DevScene* __restrict__ scenes, int nv,
               RasterParams rp, const uint32_t* __restrict__ status,
               const uint32_t* __restrict__ worklist, const uint2* __restrict__ ranges,
               const uint32_t* __restrict__ pvals, const uint64_t* __restrict__ pmask,
               const uint64_t* __restrict__ psum, const float4* __restrict__ cq,
               const float2* __restrict__ cw, const float* __restrict__ tau,
               const uint32_t* __restrict__ nlast, const float* __restrict__ grad_i,
               float* __restrict__ grad_c, int64_t stride)
{
    constexpr int NB = AB_BATCH;
    __shared__ float4 s_q[NB][WAVE];
    __shared__ float2 s_w[NB][WAVE];
    __shared__ float s_c[NB][WAVE];
    __shared__ float s_G[NB][6][WAVE];
    const int lane = threadIdx.x;
    if (blockIdx.x >= status[ST_WORK_TILES]) return;
    const int64_t bucket = worklist[blockIdx.x];
    const TileCell tc = tile_cell(views, nv, bucket, true);
    const DevView& V = views[tc.v];
    const float* amp = scenes[V.scene].amp;
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    const uint2 rg = ranges[bucket];
    const int64_t ray = V.ray_off + (int64_t)tc.row * V.Wc + tc.col;
    const uint32_t n_mine = tc.inside ? nlast[ray] : 0u;   // entries [0, n_mine) were used
    float t = tc.inside ? tau[ray] : 0.0f;
    float U = 0.0f;
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int c = 0; c < 6; ++c) s_G[k][c][lane] = 0.0f;
    unsigned long long n_iter = 0, n_hits = 0;   // work counters
    const uint32_t n_max = wave_max_u32(n_mine);
    const uint32_t e_end = rg.x + n_max;           // exclusive end of the used entries
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
        while (todo != 0ull) {
            uint32_t chk[NB];
            uint64_t lv[NB];
            int nb = 0;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                chk[k] = 0u;
                lv[k] = 0ull;
                if (todo != 0ull) {
                    const int hi = 63 - __builtin_clzll(todo);
                    todo &= ~(1ull << hi);
                    chk[k] = (uint32_t)g0 + (uint32_t)hi;
                    const uint32_t l0 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)live_c, hi);
                    const uint32_t l1 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(live_c >> 32), hi);
                    lv[k] = ((uint64_t)l1 << 32) | l0;
                    nb = k + 1;
                }
            }
            uint64_t m[NB];
            uint32_t r[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const uint32_t e = chk[k] * WAVE + lane;
                const bool in = k < nb && e >= rg.x && e < e_end;
                m[k] = in ? pmask[e] : 0ull;
                r[k] = in ? pvals[e] : 0u;
            }
            uint32_t got = 0u;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if ((m[k] & lv[k]) != 0ull) {
                    s_q[k][lane] = cq[r[k]];
                    s_w[k][lane] = cw[r[k]];
                    s_c[k][lane] = amp[r[k] - V.rec_off] * grad_i[5 * stride + r[k]];
                    got |= 1u << k;
                }
            }
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (k >= nb) break;
                // entries of this chunk my ray used in the forward: positions < n_mine
                const int64_t pos0 = (int64_t)chk[k] * WAVE - rg.x;
                const int64_t nu = (int64_t)n_mine - pos0;
                const uint64_t used =
                    nu >= WAVE ? ~0ull : (nu <= 0 ? 0ull : ((1ull << nu) - 1ull));
                uint64_t col = transpose64(m[k]) & used;
                for (;;) {
                    const bool act = col != 0ull;
                    if (__ballot(act) == 0ull) break;
                    ++n_iter;
                    if (act) {
                        const int j = 63 - __builtin_clzll(col);
                        col &= ~(1ull << j);
                        const float4 g = s_q[k][j];
                        const float2 g2 = s_w[k][j];
                        const float dx = px - g.x, dy = py - g.y;
                        const float q = quadform(g, g2.x, dx, dy);
                        if (q < rp.q_max) {
                            ++n_hits;
                            const float ex = __expf(-0.5f * q);
                            const float f = (ex - rp.eps) * rp.inv1meps;
                            const float kappa = g2.y;
                            const float x = kappa * f;
                            const float E = __expf(-x);
                            const float c = s_c[k][j];
                            float dalpha;
                            if (rp.shadowing) {
                                t -= x;
                                const float Tn = __expf(-fmaxf(t, 0.0f));
                                dalpha = Tn * (c - U);
                                U = c * (1.0f - E) + E * U;
                            } else {
                                dalpha = c;
                            }
                            const float dxx = dalpha * E;   // d alpha / d x = exp(-x)
                            const float dq = dxx * kappa * (-0.5f * ex * rp.inv1meps);
                            atomicAdd(&s_G[k][0][j], -2.0f * dq * (g.z * dx + g.w * dy));
                            atomicAdd(&s_G[k][1][j], -2.0f * dq * (g.w * dx + g2.x * dy));
                            atomicAdd(&s_G[k][2][j], dq * dx * dx);
                            atomicAdd(&s_G[k][3][j], 2.0f * dq * dx * dy);
                            atomicAdd(&s_G[k][4][j], dq * dy * dy);
                            atomicAdd(&s_G[k][5][j], dxx * f);
                        }
                    }
                }
            }
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (got & (1u << k)) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        const float v = s_G[k][c][lane];
                        if (v != 0.0f) unsafeAtomicAdd(&grad_c[c * stride + r[k]], v);
                        s_G[k][c][lane] = 0.0f;
                    }
                }
            }
            wave_lds_sync();
        }
    }
    if (rp.work) {
        n_hits = wave_sum_u64(n_hits);
        if (lane == 0) {
            atomicAdd(&rp.work[5], n_iter);
            atomicAdd(&rp.work[1], n_hits);
        }
    }
}

// Non-empty computation-plane tiles, longest lists first (binned by the
// bit length of the list size), so the heaviest tiles start earliest. One
// workgroup; the count goes to status[ST_WORK_TILES].
__global__ void __launch_bounds__(1024)
k_tile_worklist(const uint2* __restrict__ ranges, int64_t tiles_c, uint32_t* __restrict__ worklist,
                uint32_t* __restrict__ status)
{
    __shared__ uint32_t cnt[33], base[33];
    const int tid = threadIdx.x;
    if (tid < 33) cnt[tid] = 0;
    __syncthreads();
    for (int64_t t = tid; t < tiles_c; t += blockDim.x) {
        const uint2 rg = ranges[t];
        const uint32_t len = rg.y > rg.x ? rg.y - rg.x : 0u;
        if (len) atomicAdd(&cnt[32 - __clz(len)], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int lvl = 32; lvl >= 1; --lvl) {
            base[lvl] = acc;
            acc += cnt[lvl];
        }
        status[ST_WORK_TILES] = acc;
    }
    __syncthreads();
    for (int64_t t = tid; t < tiles_c; t += blockDim.x) {
        const uint2 rg = ranges[t];
        const uint32_t len = rg.y > rg.x ? rg.y - rg.x : 0u;
        if (len) worklist[atomicAdd(&base[32 - __clz(len)], 1u)] = (uint32_t)t;
    }
}

inline unsigned raster_grid(int64_t waves)
{
    return (unsigned)((waves + RASTER_WAVES - 1) / RASTER_WAVES);
}

inline unsigned grid256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_pair_masks(const DevView* views, int nv, int64_t cap_c, const RasterParams& rp,
                             const uint32_t* status, const uint32_t* pkey,
                             const uint32_t* pvals, const float4* cq, const float2* cw,
                             uint64_t* pmask, uint64_t* psum, hipStream_t s)
{
    if (cap_c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_masks, dim3(grid256(cap_c)), dim3(256), 0, s, views, nv, cap_c, rp,
                       status, pkey, pvals, cq, cw, pmask, psum);
    return hipGetLastError();
}

hipError_t launch_tile_worklist(const uint2* ranges, int64_t tiles_c, uint32_t* worklist,
                                uint32_t* status, hipStream_t s)
{
    hipLaunchKernelGGL(k_tile_worklist, dim3(1), dim3(1024), 0, s, ranges, tiles_c, worklist,
                       status);
    return hipGetLastError();
}

hipError_t launch_raster_a_fwd(const DevView* views, int nv, int64_t tiles_c,
                               const RasterParams& rp, const uint32_t* status,
                               const uint32_t* worklist, const uint2* ranges,
                               const uint32_t* pvals, const uint64_t* pmask,
                               const uint64_t* psum, const float4* cq, const float2* cw,
                               float* A, float* tau, uint32_t* nlast, hipStream_t s)
{
    if (tiles_c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_a_fwd, dim3((unsigned)tiles_c), dim3(WAVE), 0, s, views, nv, rp,
                       status, worklist, ranges, pvals, pmask, psum, cq, cw, A, tau, nlast);
    return hipGetLastError();
}

hipError_t launch_raster_b_fwd(const DevView* views, int nv, int64_t pixels, int64_t cap_i,
                               const RasterParams& rp, const uint32_t* status,
                               const uint32_t* pkey, const uint32_t* pvals, const float4* iq,
                               const float2* iw, float* images, hipStream_t s)
{
    if (pixels <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_images, dim3(grid256(pixels)), dim3(256), 0, s, views, nv, pixels,
                       images);
    if (cap_i <= 0) return hipGetLastError();
    const int64_t segs = (cap_i + B_SEGMENT - 1) / B_SEGMENT;
    hipLaunchKernelGGL(k_raster_b_fwd, dim3(raster_grid(segs)), dim3(RASTER_THREADS), 0, s, views,
                       nv, rp, status, pkey, pvals, iq, iw, images);
    return hipGetLastError();
}

hipError_t launch_image_bwd(const DevView* views, int nv, int64_t records,
                            const RasterParams& rp, const float4* iq, const float2* iw,
                            const float* dimg, float* grad_i, hipStream_t s)
{
    if (records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_image_bwd, dim3(grid256(records)), dim3(256), 0, s, views, nv, records,
                       rp, iq, iw, dimg, grad_i);
    return hipGetLastError();
}

hipError_t launch_raster_a_bwd(const DevView* views, const DevScene* scenes, int nv,
                               int64_t tiles_c, const RasterParams& rp, const uint32_t* status,
                               const uint32_t* worklist, const uint2* ranges,
                               const uint32_t* pvals, const uint64_t* pmask,
                               const uint64_t* psum, const float4* cq, const float2* cw,
                               const float* tau, const uint32_t* nlast, const float* grad_i,
                               float* grad_c, int64_t stride, hipStream_t s)
{
    if (tiles_c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_a_bwd, dim3((unsigned)tiles_c), dim3(WAVE), 0, s, views, scenes,
                       nv, rp, status, worklist, ranges, pvals, pmask, psum, cq, cw, tau, nlast,
                       grad_i, grad_c, stride);
    return hipGetLastError();
}

}  // namespace sdgr
