// Tile rasterizers of the SAR Gaussian splatting renderer (paper Sec. II-A,
// scattering intensity and imaging; Sec. II-B, their gradients).
//
// One wave64 owns one 8x8 tile: lane l handles ray / pixel (l % 8, l / 8).
// The tile's Gaussian list is walked in batches of 64: each lane stages one
// record into LDS, then all lanes sweep the batch reading it back as a
// broadcast. Waves of a workgroup are independent (different tiles); no
// workgroup barrier is used, so a wave may leave early.
//
//   pass A forward : per ray, front to back, alpha = 1 - exp(-kappa f),
//                    A_i += alpha * T, T *= exp(-kappa f); the per-Gaussian
//                    sum over the wave's rays is one DPP reduction and one
//                    float atomic per (tile, Gaussian).
//   pass B forward : per pixel, S = sum_i f_i I_i (order-free, no atomics).
//   pass B backward: per record (k_image_bwd): dL/dI and the gradients of the
//                    imaging-plane centre and conic gathered over the
//                    footprint, no atomics. (k_raster_b_bwd is the tile form:
//                    per pixel, reduced over the wave, 6 atomics per
//                    (tile, Gaussian).)
//   pass A backward: per ray, back to front from the last contributing
//                    entry: tau -= kappa f, T = exp(-tau),
//                    dL/dalpha = T (c - U), U <- c alpha + (1 - alpha) U
//                    (division-free), with c = P dL/dI; gradients of kappa
//                    and the computation-plane centre and conic.
#include "common.hpp"

namespace sdgr {
namespace {

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

// Tile coordinates of a bucket: view, the lane's cell, and whether it lies
// inside the grid.
struct TileCell {
    int v;
    int col, row;
    bool inside;
};

template <class OffF>
__device__ __forceinline__ TileCell tile_cell(const DevView* views, int nv, int64_t bucket,
                                              OffF off, bool comp_plane)
{
    TileCell t;
    t.v = find_view(nv, bucket, off);
    const DevView& V = views[t.v];
    const int64_t local = bucket - (comp_plane ? V.tile_c : V.tile_i);
    const int tx_n = comp_plane ? V.txc : V.txi;
    const int tx = (int)(local % tx_n), ty = (int)(local / tx_n);
    const int lane = lane_id();
    t.col = tx * TILE + (lane & (TILE - 1));
    t.row = ty * TILE + (lane / TILE);
    t.inside = comp_plane ? (t.col < V.Wc && t.row < V.Hc) : (t.col < V.W && t.row < V.H);
    return t;
}

__device__ __forceinline__ float quadform(float4 g, float c, float dx, float dy)
{
    return g.z * dx * dx + 2.0f * g.w * dx * dy + c * dy * dy;
}

__global__ void __launch_bounds__(RASTER_THREADS)
k_raster_a_fwd(const DevView* __restrict__ views, int nv, int64_t tiles_c, RasterParams rp,
               const uint2* __restrict__ ranges, const uint32_t* __restrict__ pvals,
               const float4* __restrict__ cq, const float2* __restrict__ cw,
               float* __restrict__ A, float* __restrict__ tau, uint32_t* __restrict__ nlast)
{
    __shared__ float4 s_q[RASTER_WAVES][WAVE];
    __shared__ float2 s_w[RASTER_WAVES][WAVE];
    __shared__ uint32_t s_r[RASTER_WAVES][WAVE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t bucket = (int64_t)blockIdx.x * RASTER_WAVES + w;
    if (bucket >= tiles_c) return;
    const TileCell tc = tile_cell(views, nv, bucket,
                                  [&](int k) { return (int64_t)views[k].tile_c; }, true);
    const DevView& V = views[tc.v];
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    const uint2 rg = ranges[bucket];
    float T = 1.0f, t = 0.0f;
    bool alive = tc.inside;
    uint32_t last = 0;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += WAVE) {
        if (__ballot(alive) == 0) break;
        const uint32_t cnt = min((uint32_t)WAVE, rg.y - b0);
        if (lane < cnt) {
            const uint32_t r = pvals[b0 + lane];
            s_q[w][lane] = cq[r];
            s_w[w][lane] = cw[r];
            s_r[w][lane] = r;
        }
        wave_lds_sync();
        for (uint32_t j = 0; j < cnt; ++j) {
            const float4 g = s_q[w][j];
            const float2 g2 = s_w[w][j];
            const float dx = px - g.x, dy = py - g.y;
            const float q = quadform(g, g2.x, dx, dy);
            const bool hit = alive && q < rp.q_max;
            if (__ballot(hit) == 0) continue;
            float contrib = 0.0f, x = 0.0f, E = 1.0f;
            if (hit) {
                const float f = (__expf(-0.5f * q) - rp.eps) * rp.inv1meps;
                x = g2.y * f;
                E = __expf(-x);
                contrib = (1.0f - E) * T;
            }
            const float s = wave_sum(contrib);
            if (lane == 0 && s != 0.0f) unsafeAtomicAdd(&A[s_r[w][j]], s);
            if (hit) {
                if (rp.shadowing) T *= E;
                t += x;
                last = b0 - rg.x + j + 1;
                if (rp.shadowing && t >= rp.tau_max) alive = false;
            }
        }
        wave_lds_sync();
    }
    if (tc.inside) {
        const int64_t ray = V.ray_off + (int64_t)tc.row * V.Wc + tc.col;
        tau[ray] = t;
        nlast[ray] = last;
    }
}

__global__ void __launch_bounds__(RASTER_THREADS)
k_raster_b_fwd(const DevView* __restrict__ views, int nv, int64_t tiles_c, int64_t tiles_i,
               RasterParams rp, const uint2* __restrict__ ranges,
               const uint32_t* __restrict__ pvals, const float4* __restrict__ iq,
               const float2* __restrict__ iw, float* __restrict__ images)
{
    __shared__ float4 s_q[RASTER_WAVES][WAVE];
    __shared__ float2 s_w[RASTER_WAVES][WAVE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t local = (int64_t)blockIdx.x * RASTER_WAVES + w;
    if (local >= tiles_i) return;
    const int64_t bucket = tiles_c + local;
    const TileCell tc = tile_cell(views, nv, bucket,
                                  [&](int k) { return (int64_t)views[k].tile_i; }, false);
    const DevView& V = views[tc.v];
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    const uint2 rg = ranges[bucket];
    float acc = 0.0f;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += WAVE) {
        const uint32_t cnt = min((uint32_t)WAVE, rg.y - b0);
        if (lane < cnt) {
            const uint32_t r = pvals[b0 + lane];
            s_q[w][lane] = iq[r];
            s_w[w][lane] = iw[r];
        }
        wave_lds_sync();
        for (uint32_t j = 0; j < cnt; ++j) {
            const float4 g = s_q[w][j];
            const float2 g2 = s_w[w][j];
            const float dx = px - g.x, dy = py - g.y;
            const float q = quadform(g, g2.x, dx, dy);
            if (q < rp.q_max) acc += (__expf(-0.5f * q) - rp.eps) * rp.inv1meps * g2.y;
        }
        wave_lds_sync();
    }
    if (tc.inside) images[V.img_off + (int64_t)tc.row * V.W + tc.col] = acc;
}

// Lanes 0..5 add the six wave sums to consecutive floats at dst.
__device__ __forceinline__ void atomic_add6(float* dst, float a0, float a1, float a2, float a3,
                                            float a4, float a5)
{
    const int lane = lane_id();
    if (lane < 6) {
        float v = lane == 0 ? a0 : lane == 1 ? a1 : lane == 2 ? a2 : lane == 3 ? a3
                : lane == 4 ? a4 : a5;
        unsafeAtomicAdd(dst + lane, v);
    }
}

__global__ void __launch_bounds__(RASTER_THREADS)
k_raster_b_bwd(const DevView* __restrict__ views, int nv, int64_t tiles_c, int64_t tiles_i,
               RasterParams rp, const uint2* __restrict__ ranges,
               const uint32_t* __restrict__ pvals, const float4* __restrict__ iq,
               const float2* __restrict__ iw, const float* __restrict__ dimg,
               float* __restrict__ grad_i)
{
    __shared__ float4 s_q[RASTER_WAVES][WAVE];
    __shared__ float2 s_w[RASTER_WAVES][WAVE];
    __shared__ uint32_t s_r[RASTER_WAVES][WAVE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t local = (int64_t)blockIdx.x * RASTER_WAVES + w;
    if (local >= tiles_i) return;
    const int64_t bucket = tiles_c + local;
    const TileCell tc = tile_cell(views, nv, bucket,
                                  [&](int k) { return (int64_t)views[k].tile_i; }, false);
    const DevView& V = views[tc.v];
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    const uint2 rg = ranges[bucket];
    const float G = tc.inside ? dimg[V.img_off + (int64_t)tc.row * V.W + tc.col] : 0.0f;
    const bool live = tc.inside && G != 0.0f;
    if (__ballot(live) == 0) return;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += WAVE) {
        const uint32_t cnt = min((uint32_t)WAVE, rg.y - b0);
        if (lane < cnt) {
            const uint32_t r = pvals[b0 + lane];
            s_q[w][lane] = iq[r];
            s_w[w][lane] = iw[r];
            s_r[w][lane] = r;
        }
        wave_lds_sync();
        for (uint32_t j = 0; j < cnt; ++j) {
            const float4 g = s_q[w][j];
            const float2 g2 = s_w[w][j];
            const float dx = px - g.x, dy = py - g.y;
            const float q = quadform(g, g2.x, dx, dy);
            const bool hit = live && q < rp.q_max;
            if (__ballot(hit) == 0) continue;
            float dI = 0.f, dcx = 0.f, dcy = 0.f, da = 0.f, db = 0.f, dc = 0.f;
            if (hit) {
                const float e = __expf(-0.5f * q);
                dI = G * (e - rp.eps) * rp.inv1meps;
                const float dq = G * g2.y * (-0.5f * e * rp.inv1meps);
                dcx = -2.0f * dq * (g.z * dx + g.w * dy);
                dcy = -2.0f * dq * (g.w * dx + g2.x * dy);
                da = dq * dx * dx;
                db = 2.0f * dq * dx * dy;
                dc = dq * dy * dy;
            }
            const float s0 = wave_sum(dcx), s1 = wave_sum(dcy), s2 = wave_sum(da);
            const float s3 = wave_sum(db), s4 = wave_sum(dc), s5 = wave_sum(dI);
            atomic_add6(grad_i + 8 * (int64_t)s_r[w][j], s0, s1, s2, s3, s4, s5);
        }
        wave_lds_sync();
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
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= records) return;
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
    float4* o = reinterpret_cast<float4*>(grad_i + 8 * r);
    o[0] = make_float4(dcx, dcy, da, db);
    o[1] = make_float4(dc, dI, 0.0f, 0.0f);
}

__global__ void __launch_bounds__(RASTER_THREADS)
k_raster_a_bwd(const DevView* __restrict__ views, const DevScene* __restrict__ scenes, int nv,
               int64_t tiles_c, RasterParams rp, const uint2* __restrict__ ranges,
               const uint32_t* __restrict__ pvals, const float4* __restrict__ cq,
               const float2* __restrict__ cw, const float* __restrict__ tau,
               const uint32_t* __restrict__ nlast, const float* __restrict__ grad_i,
               float* __restrict__ grad_c)
{
    __shared__ float4 s_q[RASTER_WAVES][WAVE];
    __shared__ float2 s_w[RASTER_WAVES][WAVE];
    __shared__ float s_c[RASTER_WAVES][WAVE];
    __shared__ uint32_t s_r[RASTER_WAVES][WAVE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t bucket = (int64_t)blockIdx.x * RASTER_WAVES + w;
    if (bucket >= tiles_c) return;
    const TileCell tc = tile_cell(views, nv, bucket,
                                  [&](int k) { return (int64_t)views[k].tile_c; }, true);
    const DevView& V = views[tc.v];
    const float* amp = scenes[V.scene].amp;
    const float px = tc.col + 0.5f, py = tc.row + 0.5f;
    const uint2 rg = ranges[bucket];
    const int64_t ray = V.ray_off + (int64_t)tc.row * V.Wc + tc.col;
    const uint32_t n_mine = tc.inside ? nlast[ray] : 0u;
    float t = tc.inside ? tau[ray] : 0.0f;
    float U = 0.0f;
    const uint32_t n_max = wave_max_u32(n_mine);
    // batches back to front over list entries [0, n_max)
    for (int64_t be = n_max; be > 0; be -= WAVE) {
        const uint32_t bs = (uint32_t)max((int64_t)0, be - WAVE);
        const uint32_t cnt = (uint32_t)be - bs;
        if (lane < cnt) {
            const uint32_t r = pvals[rg.x + bs + lane];
            s_q[w][lane] = cq[r];
            s_w[w][lane] = cw[r];
            s_c[w][lane] = amp[r - V.rec_off] * grad_i[8 * (int64_t)r + 5];
            s_r[w][lane] = r;
        }
        wave_lds_sync();
        for (int j = (int)cnt - 1; j >= 0; --j) {
            const uint32_t e = bs + (uint32_t)j;
            const float4 g = s_q[w][j];
            const float2 g2 = s_w[w][j];
            const float dx = px - g.x, dy = py - g.y;
            const float q = quadform(g, g2.x, dx, dy);
            const bool hit = e < n_mine && q < rp.q_max;
            if (__ballot(hit) == 0) continue;
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
            const float s0 = wave_sum(dcx), s1 = wave_sum(dcy), s2 = wave_sum(da);
            const float s3 = wave_sum(db), s4 = wave_sum(dc), s5 = wave_sum(dk);
            atomic_add6(grad_c + 8 * (int64_t)s_r[w][j], s0, s1, s2, s3, s4, s5);
        }
        wave_lds_sync();
    }
}

inline unsigned raster_grid(int64_t tiles)
{
    return (unsigned)((tiles + RASTER_WAVES - 1) / RASTER_WAVES);
}

}  // namespace

hipError_t launch_raster_a_fwd(const DevView* views, int nv, int64_t tiles_c,
                               const RasterParams& rp, const uint2* ranges,
                               const uint32_t* pvals, const float4* cq, const float2* cw,
                               float* A, float* tau, uint32_t* nlast, hipStream_t s)
{
    if (tiles_c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_a_fwd, dim3(raster_grid(tiles_c)), dim3(RASTER_THREADS), 0, s,
                       views, nv, tiles_c, rp, ranges, pvals, cq, cw, A, tau, nlast);
    return hipGetLastError();
}

hipError_t launch_raster_b_fwd(const DevView* views, int nv, int64_t tiles_c, int64_t tiles_i,
                               const RasterParams& rp, const uint2* ranges,
                               const uint32_t* pvals, const float4* iq, const float2* iw,
                               float* images, hipStream_t s)
{
    if (tiles_i <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_b_fwd, dim3(raster_grid(tiles_i)), dim3(RASTER_THREADS), 0, s,
                       views, nv, tiles_c, tiles_i, rp, ranges, pvals, iq, iw, images);
    return hipGetLastError();
}

hipError_t launch_raster_b_bwd(const DevView* views, int nv, int64_t tiles_c, int64_t tiles_i,
                               const RasterParams& rp, const uint2* ranges,
                               const uint32_t* pvals, const float4* iq, const float2* iw,
                               const float* dimg, float* grad_i, hipStream_t s)
{
    if (tiles_i <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_b_bwd, dim3(raster_grid(tiles_i)), dim3(RASTER_THREADS), 0, s,
                       views, nv, tiles_c, tiles_i, rp, ranges, pvals, iq, iw, dimg, grad_i);
    return hipGetLastError();
}

hipError_t launch_image_bwd(const DevView* views, int nv, int64_t records,
                            const RasterParams& rp, const float4* iq, const float2* iw,
                            const float* dimg, float* grad_i, hipStream_t s)
{
    if (records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_image_bwd, dim3((unsigned)((records + 255) / 256)), dim3(256), 0, s,
                       views, nv, records, rp, iq, iw, dimg, grad_i);
    return hipGetLastError();
}

hipError_t launch_raster_a_bwd(const DevView* views, const DevScene* scenes, int nv,
                               int64_t tiles_c, const RasterParams& rp, const uint2* ranges,
                               const uint32_t* pvals, const float4* cq, const float2* cw,
                               const float* tau, const uint32_t* nlast, const float* grad_i,
                               float* grad_c, hipStream_t s)
{
    if (tiles_c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_a_bwd, dim3(raster_grid(tiles_c)), dim3(RASTER_THREADS), 0, s,
                       views, scenes, nv, tiles_c, rp, ranges, pvals, cq, cw, tau, nlast,
                       grad_i, grad_c);
    return hipGetLastError();
}

}  // namespace sdgr
