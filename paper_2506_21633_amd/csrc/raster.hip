// Rasterizers of the SAR Gaussian splatting renderer (paper Sec. II-A,
// scattering intensity and imaging; Sec. II-B, their gradients).
//
// Computation plane (order matters: front-to-back along each ray)
//   One wave64 (a workgroup of its own) owns one 8x8 tile: lane l handles ray
//   (l % 8, l / 8); only non-empty tiles run, longest lists first. Every
//   (tile, Gaussian) pair carries a 64-bit mask of the tile cells inside the
//   footprint ellipse (k_pair_masks). The tile's depth-sorted list is walked
//   in batches of 64 entries: the masks are read coalesced, entries whose mask
//   misses every ray still in play are dropped, and only the survivors are
//   gathered into LDS (in order) and swept by all lanes as a broadcast.
//   pass A forward : alpha = 1 - exp(-kappa f), A_i += alpha T, T *= exp(-kappa f);
//                    per-Gaussian sums over the wave's rays by a transposed
//                    LDS reduction (GroupReduce), one float atomic per
//                    (tile, Gaussian); a ray leaves after its optical depth
//                    reaches tau_max.
//   pass A backward: back to front from each ray's last contributing entry:
//                    tau -= kappa f, T = exp(-tau), dL/dalpha = T (c - U),
//                    U <- c alpha + (1 - alpha) U (division-free), c = P dL/dI.
// Imaging plane (order-free additive layover)
//   pass B forward : fixed 2048-entry segments of the sorted (tile, Gaussian)
//                    pair array, one wave each (balanced however long a
//                    tile's list is); lane = pixel; partial pixel sums are
//                    added to the image at tile boundaries.
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

// Transposed reduction of per-lane values over the 64 lanes of a wave for a
// group of list entries: each lane writes its values of the group's entries
// into its own LDS row; at a flush, lane c sums column c over the 64 rows and
// adds the total to the Gaussian that column belongs to with one atomic.
// About 20 instructions per entry for six values instead of six 64-lane DPP
// reductions. Rows have an even stride so 8-byte writes stay aligned.
template <int VALS, int GROUP>
struct GroupReduce {
    static constexpr int STRIDE = VALS * GROUP + ((VALS * GROUP) % 2 == 0 ? 2 : 1);
    float row[WAVE][STRIDE];
    uint32_t rec[GROUP];
};

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

__global__ void __launch_bounds__(256)
k_pair_masks(const DevView* __restrict__ views, int nv, int64_t cap, RasterParams rp,
             const uint32_t* __restrict__ status, const uint32_t* __restrict__ pkey,
             const uint32_t* __restrict__ pvals, const float4* __restrict__ cq,
             const float2* __restrict__ cw, uint64_t* __restrict__ pmask)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= cap || p >= (int64_t)status[ST_PAIRS_C]) return;
    const uint32_t bucket = pkey[p];
    const int v = find_view(nv, (int64_t)bucket, [&](int k) { return (int64_t)views[k].tile_c; });
    const DevView& V = views[v];
    const int local = (int)(bucket - (uint32_t)V.tile_c);
    const uint32_t r = pvals[p];
    const float4 g = cq[r];
    const float2 g2 = cw[r];
    pmask[p] = footprint_mask(g.x, g.y, g.z, g.w, g2.x, rp.q_max, local % V.txc, local / V.txc);
}

__global__ void __launch_bounds__(WAVE)
k_raster_a_fwd(const DevView* __restrict__ views, int nv, RasterParams rp,
               const uint32_t* __restrict__ status, const uint32_t* __restrict__ worklist,
               const uint2* __restrict__ ranges, const uint32_t* __restrict__ pvals,
               const uint64_t* __restrict__ pmask, const float4* __restrict__ cq,
               const float2* __restrict__ cw, float* __restrict__ A, float* __restrict__ tau,
               uint32_t* __restrict__ nlast)
{
    constexpr int w = 0;   // one wave per workgroup: heavy tiles schedule one by one
    __shared__ float4 s_q[1][WAVE];
    __shared__ float2 s_w[1][WAVE];
    __shared__ uint64_t s_m[1][WAVE];
    __shared__ uint32_t s_r[1][WAVE];
    __shared__ uint32_t s_e[1][WAVE];
    constexpr int GA = 32;
    __shared__ GroupReduce<1, GA> s_red[1];
    const int lane = threadIdx.x;
    if (blockIdx.x >= status[ST_WORK_TILES]) return;
    const int64_t bucket = worklist[blockIdx.x];
    const TileCell tc = tile_cell(views, nv, bucket, true);
    const DevView& V = views[tc.v];
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    const uint2 rg = ranges[bucket];
    GroupReduce<1, GA>& red = s_red[w];
    int group = 0;
    auto flush = [&]() {
        wave_lds_sync();
        if (lane < group) {
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll 4
            for (int k = 0; k < WAVE; k += 4) {
                s0 += red.row[k][lane];
                s1 += red.row[k + 1][lane];
                s2 += red.row[k + 2][lane];
                s3 += red.row[k + 3][lane];
            }
            const float sum = (s0 + s1) + (s2 + s3);
            if (sum != 0.0f) unsafeAtomicAdd(&A[red.rec[lane]], sum);
        }
        wave_lds_sync();
        group = 0;
    };
    float T = 1.0f, t = 0.0f;
    bool alive = tc.inside;
    uint32_t last = 0;
    unsigned long long n_entries = 0, n_hits = 0;   // work counters (wave-uniform)
    uint64_t live = __ballot(alive);
    for (uint32_t b0 = rg.x; b0 < rg.y && live != 0ull; b0 += WAVE) {
        const uint32_t e = b0 + lane;
        const uint64_t m = e < rg.y ? pmask[e] : 0ull;
        const bool need = (m & live) != 0ull;
        const uint64_t nb = __ballot(need);
        if (nb == 0ull) continue;
        if (need) {
            const uint32_t slot = lanes_below(nb);
            const uint32_t r = pvals[e];
            s_q[w][slot] = cq[r];
            s_w[w][slot] = cw[r];
            s_m[w][slot] = m;
            s_r[w][slot] = r;
            s_e[w][slot] = e - rg.x;
        }
        wave_lds_sync();
        const uint32_t cnt = (uint32_t)__popcll(nb);
        for (uint32_t j = 0; j < cnt; ++j) {
            const uint64_t mj = s_m[w][j];
            if ((mj & live) == 0ull) continue;
            const float4 g = s_q[w][j];
            const float2 g2 = s_w[w][j];
            const float dx = px - g.x, dy = py - g.y;
            const float q = quadform(g, g2.x, dx, dy);
            const bool hit = alive && ((mj >> lane) & 1ull) && q < rp.q_max;
            const uint64_t hb = __ballot(hit);
            n_entries += 1;
            n_hits += (unsigned long long)__popcll(hb);
            if (hb == 0ull) continue;
            float contrib = 0.0f, x = 0.0f, E = 1.0f;
            if (hit) {
                const float f = (__expf(-0.5f * q) - rp.eps) * rp.inv1meps;
                x = g2.y * f;
                E = __expf(-x);
                contrib = (1.0f - E) * T;
            }
            red.row[lane][group] = contrib;
            if (lane == 0) red.rec[group] = s_r[w][j];
            if (++group == GA) flush();
            if (hit) {
                if (rp.shadowing) T *= E;
                t += x;
                last = s_e[w][j] + 1;
                if (rp.shadowing && t >= rp.tau_max) alive = false;
            }
            live = __ballot(alive);
        }
        wave_lds_sync();
    }
    if (group > 0) flush();
    if (rp.work && lane == 0) {
        atomicAdd(&rp.work[4], n_entries);
        atomicAdd(&rp.work[0], n_hits);
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

__global__ void __launch_bounds__(RASTER_THREADS)
k_raster_b_fwd(const DevView* __restrict__ views, int nv, RasterParams rp,
               const uint32_t* __restrict__ status, const uint32_t* __restrict__ pkey,
               const uint32_t* __restrict__ pvals, const float4* __restrict__ iq,
               const float2* __restrict__ iw, float* __restrict__ images)
{
    __shared__ float4 s_q[RASTER_WAVES][WAVE];
    __shared__ float2 s_w[RASTER_WAVES][WAVE];
    __shared__ uint32_t s_k[RASTER_WAVES][WAVE];
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
    unsigned long long n_entries = 0, n_hits = 0;   // work counters (wave-uniform)
    for (uint32_t b0 = (uint32_t)p0; b0 < p1; b0 += WAVE) {
        const uint32_t cnt = min((uint32_t)WAVE, p1 - b0);
        if (lane < cnt) {
            const uint32_t r = pvals[b0 + lane];
            s_q[w][lane] = iq[r];
            s_w[w][lane] = iw[r];
            s_k[w][lane] = pkey[b0 + lane];
        }
        wave_lds_sync();
        for (uint32_t j = 0; j < cnt; ++j) {
            const uint32_t k = s_k[w][j];
            if (k != cur) {   // tile boundary: flush the partial sums
                if (pix >= 0) unsafeAtomicAdd(&images[pix], acc);
                const TileCell tc = tile_cell(views, nv, (int64_t)k, false);
                const DevView& V = views[tc.v];
                px = tc.col + 0.5f;
                py = tc.row + 0.5f;
                pix = tc.inside ? V.img_off + (int64_t)tc.row * V.W + tc.col : -1;
                acc = 0.0f;
                cur = k;
            }
            const float4 g = s_q[w][j];
            const float2 g2 = s_w[w][j];
            const float dx = px - g.x, dy = py - g.y;
            const float q = quadform(g, g2.x, dx, dy);
            if (q < rp.q_max) acc += (__expf(-0.5f * q) - rp.eps) * rp.inv1meps * g2.y;
            if (rp.work) {
                n_entries += 1;
                n_hits += (unsigned long long)__popcll(__ballot(q < rp.q_max && pix >= 0));
            }
        }
        wave_lds_sync();
    }
    if (pix >= 0) unsafeAtomicAdd(&images[pix], acc);
    if (rp.work && lane == 0) {
        atomicAdd(&rp.work[6], n_entries);
        atomicAdd(&rp.work[2], n_hits);
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

__global__ void __launch_bounds__(WAVE)
k_raster_a_bwd(const DevView* __restrict__ views, const DevScene* __restrict__ scenes, int nv,
               RasterParams rp, const uint32_t* __restrict__ status,
               const uint32_t* __restrict__ worklist, const uint2* __restrict__ ranges,
               const uint32_t* __restrict__ pvals, const uint64_t* __restrict__ pmask,
               const float4* __restrict__ cq, const float2* __restrict__ cw,
               const float* __restrict__ tau, const uint32_t* __restrict__ nlast,
               const float* __restrict__ grad_i, float* __restrict__ grad_c, int64_t stride)
{
    constexpr int w = 0;   // one wave per workgroup: heavy tiles schedule one by one
    __shared__ float4 s_q[1][WAVE];
    __shared__ float2 s_w[1][WAVE];
    __shared__ uint64_t s_m[1][WAVE];
    __shared__ float s_c[1][WAVE];
    __shared__ uint32_t s_r[1][WAVE];
    __shared__ uint32_t s_e[1][WAVE];
    constexpr int GB = 8;
    __shared__ GroupReduce<6, GB> s_red[1];
    const int lane = threadIdx.x;
    if (blockIdx.x >= status[ST_WORK_TILES]) return;
    const int64_t bucket = worklist[blockIdx.x];
    const TileCell tc = tile_cell(views, nv, bucket, true);
    const DevView& V = views[tc.v];
    const float* amp = scenes[V.scene].amp;
    GroupReduce<6, GB>& red = s_red[w];
    int group = 0;
    auto flush = [&]() {
        wave_lds_sync();
        if (lane < 6 * group) {
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll 4
            for (int k = 0; k < WAVE; k += 4) {
                s0 += red.row[k][lane];
                s1 += red.row[k + 1][lane];
                s2 += red.row[k + 2][lane];
                s3 += red.row[k + 3][lane];
            }
            const float sum = (s0 + s1) + (s2 + s3);
            const int slot = lane / 6, comp = lane - 6 * slot;
            if (sum != 0.0f) unsafeAtomicAdd(&grad_c[comp * stride + red.rec[slot]], sum);
        }
        wave_lds_sync();
        group = 0;
    };
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    const uint2 rg = ranges[bucket];
    const int64_t ray = V.ray_off + (int64_t)tc.row * V.Wc + tc.col;
    const uint32_t n_mine = tc.inside ? nlast[ray] : 0u;
    float t = tc.inside ? tau[ray] : 0.0f;
    float U = 0.0f;
    unsigned long long n_entries = 0, n_hits = 0;   // work counters (wave-uniform)
    const uint32_t n_max = wave_max_u32(n_mine);
    // batches back to front over list entries [0, n_max)
    for (int64_t be = n_max; be > 0; be -= WAVE) {
        const uint32_t bs = (uint32_t)max((int64_t)0, be - WAVE);
        const uint32_t e = bs + lane;
        // rays that processed some entry >= bs in the forward
        const uint64_t live = __ballot(n_mine > bs);
        const uint64_t m = e < (uint32_t)be ? pmask[rg.x + e] : 0ull;
        const bool need = (m & live) != 0ull;
        const uint64_t nb = __ballot(need);
        if (nb == 0ull) continue;
        if (need) {
            const uint32_t slot = lanes_below(nb);
            const uint32_t r = pvals[rg.x + e];
            s_q[w][slot] = cq[r];
            s_w[w][slot] = cw[r];
            s_m[w][slot] = m;
            s_c[w][slot] = amp[r - V.rec_off] * grad_i[5 * stride + r];
            s_r[w][slot] = r;
            s_e[w][slot] = e;
        }
        wave_lds_sync();
        const int cnt = __popcll(nb);
        for (int j = cnt - 1; j >= 0; --j) {
            const uint32_t ej = s_e[w][j];
            const uint64_t mj = s_m[w][j];
            const float4 g = s_q[w][j];
            const float2 g2 = s_w[w][j];
            const float dx = px - g.x, dy = py - g.y;
            const float q = quadform(g, g2.x, dx, dy);
            const bool hit = ej < n_mine && ((mj >> lane) & 1ull) && q < rp.q_max;
            const uint64_t hb = __ballot(hit);
            n_entries += 1;
            n_hits += (unsigned long long)__popcll(hb);
            if (hb == 0ull) continue;
            float dcx = 0.f, dcy = 0.f, da = 0.f, db = 0.f, dc = 0.f, dk = 0.f;
            if (hit) {
                const float ex = __expf(-0.5f * q);
                const float f = (ex - rp.eps) * rp.inv1meps;
                const float kappa = g2.y;
                const float x = kappa * f;
                const float E = __expf(-x);
                const float c = s_c[w][j];
                float dalpha;
                if (rp.shadowing) {
                    t -= x;
                    const float T = __expf(-fmaxf(t, 0.0f));
                    dalpha = T * (c - U);
                    U = c * (1.0f - E) + E * U;
                } else {
                    dalpha = c;
                }
                const float dx_ = dalpha * E;          // d alpha / d x = exp(-x)
                dk = dx_ * f;
                const float dq = dx_ * kappa * (-0.5f * ex * rp.inv1meps);
                dcx = -2.0f * dq * (g.z * dx + g.w * dy);
                dcy = -2.0f * dq * (g.w * dx + g2.x * dy);
                da = dq * dx * dx;
                db = 2.0f * dq * dx * dy;
                dc = dq * dy * dy;
            }
            float2* dst = reinterpret_cast<float2*>(&red.row[lane][6 * group]);
            dst[0] = make_float2(dcx, dcy);
            dst[1] = make_float2(da, db);
            dst[2] = make_float2(dc, dk);
            if (lane == 0) red.rec[group] = s_r[w][j];
            if (++group == GB) flush();
        }
        wave_lds_sync();
    }
    if (group > 0) flush();
    if (rp.work && lane == 0) {
        atomicAdd(&rp.work[5], n_entries);
        atomicAdd(&rp.work[1], n_hits);
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
                             uint64_t* pmask, hipStream_t s)
{
    if (cap_c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_masks, dim3(grid256(cap_c)), dim3(256), 0, s, views, nv, cap_c, rp,
                       status, pkey, pvals, cq, cw, pmask);
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
                               const uint32_t* pvals, const uint64_t* pmask, const float4* cq,
                               const float2* cw, float* A, float* tau, uint32_t* nlast,
                               hipStream_t s)
{
    if (tiles_c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_a_fwd, dim3((unsigned)tiles_c), dim3(WAVE), 0, s, views, nv, rp,
                       status, worklist, ranges, pvals, pmask, cq, cw, A, tau, nlast);
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
                               const uint32_t* pvals, const uint64_t* pmask, const float4* cq,
                               const float2* cw, const float* tau, const uint32_t* nlast,
                               const float* grad_i, float* grad_c, int64_t stride,
                               hipStream_t s)
{
    if (tiles_c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_a_bwd, dim3((unsigned)tiles_c), dim3(WAVE), 0, s, views, scenes,
                       nv, rp, status, worklist, ranges, pvals, pmask, cq, cw, tau, nlast,
                       grad_i, grad_c, stride);
    return hipGetLastError();
}

}  // namespace sdgr
