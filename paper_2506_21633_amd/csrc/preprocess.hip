// Per-(view, Gaussian) projection onto the computation and imaging planes
// (paper Sec. II-A: radar rotation R_r, Sigma' = J^T R^T Sigma R J, the
// projections P_C and P_I) and its adjoint (Sec. II-B, gradient of the
// Gaussian parameters, both planes contributing to dL/dSigma).
//
// Forward: a thread per Gaussian and group of views; the projection runs
// in FP32 except the range coordinate that orders the depth lists, which is
// FP64 for a reproducible key; records are stored in FP32. The parameter
// adjoint runs in FP64 (O(views x Gaussians), cheap).
#include "common.hpp"
#include "sh.hpp"

#include <math.h>

namespace sdgr {
namespace {

struct Geo {
    bool valid;
    double mu[3];
    double qn[4], qnorm, s[3], R[9], M[9];
    double S[6];        // 3D covariance xx, xy, xz, yy, yz, zz
};

__device__ __forceinline__ bool finite(double a) { return isfinite(a); }

// Range coordinate z = e_z . mu as ((ez0 mu0 + ez1 mu1) + ez2 mu2), every
// product and sum rounded separately: it decides the depth order, and this
// exact sequence of roundings is the documented key.
__device__ __attribute__((noinline)) double range_coordinate(const double* ez, double m0,
                                                             double m1, double m2)
{
#pragma clang fp contract(off)
    double a = ez[0] * m0;
    double b = ez[1] * m1;
    double c = ez[2] * m2;
    return (a + b) + c;
}

// View-independent frame of Gaussian i: unit quaternion, rotation R,
// M = R diag(s) and Sigma = M M^T.
__device__ void gaussian_frame(const DevScene& S, int64_t i, Geo& g)
{
    const float* mu = S.means + 3 * i;
    const float* sc = S.scales + 3 * i;
    const float* qq = S.quats + 4 * i;
    double m0 = mu[0], m1 = mu[1], m2 = mu[2];
    g.mu[0] = m0; g.mu[1] = m1; g.mu[2] = m2;
    double s0 = sc[0], s1 = sc[1], s2 = sc[2];
    double q0 = qq[0], q1 = qq[1], q2 = qq[2], q3 = qq[3];
    double n2 = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    g.valid = finite(m0) && finite(m1) && finite(m2) && finite(s0) && finite(s1) &&
              finite(s2) && s0 > 0.0 && s1 > 0.0 && s2 > 0.0 && finite(n2) && n2 > 0.0;
    if (!g.valid) return;
    g.qnorm = sqrt(n2);
    double w = q0 / g.qnorm, x = q1 / g.qnorm, y = q2 / g.qnorm, z = q3 / g.qnorm;
    g.qn[0] = w; g.qn[1] = x; g.qn[2] = y; g.qn[3] = z;
    double* R = g.R;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
    g.s[0] = s0; g.s[1] = s1; g.s[2] = s2;
    for (int r = 0; r < 3; ++r) {
        g.M[3 * r + 0] = R[3 * r + 0] * s0;
        g.M[3 * r + 1] = R[3 * r + 1] * s1;
        g.M[3 * r + 2] = R[3 * r + 2] * s2;
    }
    const double* M = g.M;
    auto row = [&](int a, int b) {
        return M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
    };
    g.S[0] = row(0, 0); g.S[1] = row(0, 1); g.S[2] = row(0, 2);
    g.S[3] = row(1, 1); g.S[4] = row(1, 2); g.S[5] = row(2, 2);
}

// u^T Sigma w with Sigma given by its 6 unique entries
__device__ __forceinline__ double quad(const double* u, const double* S, const double* w)
{
    double t0 = S[0] * w[0] + S[1] * w[1] + S[2] * w[2];
    double t1 = S[1] * w[0] + S[3] * w[1] + S[4] * w[2];
    double t2 = S[2] * w[0] + S[4] * w[1] + S[5] * w[2];
    return u[0] * t0 + u[1] * t1 + u[2] * t2;
}

// 2D covariance of one plane spanned by radar axes u, w with spacings su, sw.
// iu, iw: reciprocal spacings along u and w
__device__ __forceinline__ void plane_cov(const Geo& g, const double* u, const double* w,
                                          double iu, double iw, double dil, double* cov)
{
    cov[0] = quad(u, g.S, u) * (iu * iu) + dil;
    cov[1] = quad(u, g.S, w) * (iu * iw);
    cov[2] = quad(w, g.S, w) * (iw * iw) + dil;
}

__device__ __forceinline__ bool conic(const double* cov, double* Q)
{
    double det = cov[0] * cov[2] - cov[1] * cov[1];
    if (!(det > 0.0) || !isfinite(det)) return false;
    const double id = 1.0 / det;
    Q[0] = cov[2] * id; Q[1] = -cov[1] * id; Q[2] = cov[0] * id;
    return true;
}

// Tiles touched by the ellipse q < q_max around centre c (FP32); returns
// the rectangle [tx0, tx1) x [ty0, ty1) packed in a uint2 and its tile count.
// The half extents get a small margin so every cell an FP32 evaluation of
// q < q_max can reach lies inside.
__device__ uint32_t tile_rect(float cx, float cy, float sxx, float syy, float q_max, int cols,
                              int rows, uint2* rect)
{
    const float rx = sqrtf(q_max * sxx) * (1.0f + 1e-4f) + 1e-4f;
    const float ry = sqrtf(q_max * syy) * (1.0f + 1e-4f) + 1e-4f;
    // cells whose centre (k + 1/2) lies within the bounding box, clamped in
    // float before converting
    const float lo_x = fmaxf(ceilf(cx - rx - 0.5f), 0.0f);
    const float hi_x = fminf(floorf(cx + rx - 0.5f), (float)(cols - 1));
    const float lo_y = fmaxf(ceilf(cy - ry - 0.5f), 0.0f);
    const float hi_y = fminf(floorf(cy + ry - 0.5f), (float)(rows - 1));
    if (!(lo_x <= hi_x) || !(lo_y <= hi_y)) { *rect = make_uint2(0, 0); return 0; }
    const uint32_t tx0 = (uint32_t)lo_x / TILE, tx1 = (uint32_t)hi_x / TILE + 1;
    const uint32_t ty0 = (uint32_t)lo_y / TILE, ty1 = (uint32_t)hi_y / TILE + 1;
    *rect = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
    return (tx1 - tx0) * (ty1 - ty0);
}

// Projected 2D covariance and conic of one plane in FP32, spanned by radar
// axes e1, e2 with spacings s1, s2: with u = M^T e1 and w = M^T e2 (M the
// scaled rotation), Sigma' = [[u.u, u.w], [u.w, w.w]] / spacings and
// det = |u x w|^2 / spacings^2 (Lagrange identity), so neither the
// covariance nor its determinant suffers cancellation for flat Gaussians.
struct Conic2 {
    float sxx, sxy, syy;   // covariance (pixels^2)
    float a, b, c;         // inverse
    bool ok;
};

__device__ __forceinline__ Conic2 plane_conic(const float* Mt, const float* e1, const float* e2,
                                              float inv1, float inv2, float dil)
{
    float u[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        u[k] = (Mt[3 * k] * e1[0] + Mt[3 * k + 1] * e1[1] + Mt[3 * k + 2] * e1[2]) * inv1;
        w[k] = (Mt[3 * k] * e2[0] + Mt[3 * k + 1] * e2[1] + Mt[3 * k + 2] * e2[2]) * inv2;
    }
    Conic2 r;
    r.sxx = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    r.sxy = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
    r.syy = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const float c0 = u[1] * w[2] - u[2] * w[1];
    const float c1 = u[2] * w[0] - u[0] * w[2];
    const float c2 = u[0] * w[1] - u[1] * w[0];
    float det = c0 * c0 + c1 * c1 + c2 * c2;
    if (dil > 0.0f) {
        det += dil * (r.sxx + r.syy) + dil * dil;
        r.sxx += dil;
        r.syy += dil;
    }
    r.ok = det > 0.0f && isfinite(det) && r.sxx > 0.0f && r.syy > 0.0f;
    const float inv = r.ok ? 1.0f / det : 0.0f;
    r.a = r.syy * inv;
    r.b = -r.sxy * inv;
    r.c = r.sxx * inv;
    return r;
}

// Unit direction from the centre (m0, m1, m2) to the radar, which sits on
// the line of sight through the origin at slant distance V.range on the near
// side; a plane wave (range 0) arrives from -e_z everywhere.
__device__ __forceinline__ void radar_direction_f(const DevView& V, float m0, float m1, float m2,
                                                  float* d)
{
    const float ez0 = (float)V.ez[0], ez1 = (float)V.ez[1], ez2 = (float)V.ez[2];
    if (V.range > 0.0) {
        const float rr = (float)V.range;
        const float w0 = -rr * ez0 - m0, w1 = -rr * ez1 - m1, w2 = -rr * ez2 - m2;
        const float n2 = w0 * w0 + w1 * w1 + w2 * w2;
        if (n2 > 0.0f) {
            const float inv = rsqrtf(n2);
            d[0] = w0 * inv; d[1] = w1 * inv; d[2] = w2 * inv;
            return;
        }
    }
    d[0] = -ez0; d[1] = -ez1; d[2] = -ez2;
}

// FP32 projection of the records; the range coordinate that orders the
// depth lists is evaluated in FP64 (range_coordinate) for a reproducible
// key. A thread takes one Gaussian and up to PRE_VIEWS views of its scene
// (grid y: the group of views), so the Gaussian's parameters are read and
// its rotation built once per group instead of once per record; writes of
// one view are coalesced across the block's Gaussians. With prec given, it
// also writes each record's phase factor: P (the scalar amplitude or the SH
// expansion at the direction to the radar) times the view's cell-area
// factor.
constexpr int PRE_VIEWS = 8;

__global__ void __launch_bounds__(256)
k_preprocess(const DevView* __restrict__ views, const DevScene* __restrict__ scenes, int nv,
             int nscenes, int64_t items, RasterParams rp, int write_records,
             CRec* __restrict__ crec, float4* __restrict__ iq,
             float2* __restrict__ iw, uint2* __restrict__ rect_c, uint2* __restrict__ rect_i,
             uint32_t* __restrict__ dkey, float* __restrict__ A_zero,
             float* __restrict__ prec, unsigned long long* __restrict__ totals)
{
    __shared__ unsigned long long part[2];
    if (threadIdx.x < 2) part[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t nc = 0, ni = 0;
    if (t < items) {
        const int sc = find_view(nscenes, t, [&](int k) { return scenes[k].item_off; });
        const DevScene& S = scenes[sc];
        const int64_t i = t - S.item_off;
        const float m0 = S.means[3 * i], m1 = S.means[3 * i + 1], m2 = S.means[3 * i + 2];
        const float s0 = S.scales[3 * i], s1 = S.scales[3 * i + 1], s2 = S.scales[3 * i + 2];
        const float* qp = S.quats + 4 * i;
        const float4 q = make_float4(qp[0], qp[1], qp[2], qp[3]);
        // only the sum of the forward and backward extinctions enters
        const float ext = S.ext_back ? S.ext[i] + S.ext_back[i] : S.ext[i];
        const float n2 = q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w;
        const bool valid = isfinite(m0) && isfinite(m1) && isfinite(m2) && isfinite(s0) &&
                           isfinite(s1) && isfinite(s2) && s0 > 0.0f && s1 > 0.0f &&
                           s2 > 0.0f && isfinite(n2) && n2 > 0.0f;
        // rows of M^T: column k of R scaled by s_k
        float Mt[9];
        {
            const float inv_n = valid ? rsqrtf(n2) : 0.0f;
            const float w = q.x * inv_n, x = q.y * inv_n, y = q.z * inv_n, z = q.w * inv_n;
            Mt[0] = (1.f - 2.f * (y * y + z * z)) * s0;
            Mt[1] = 2.f * (x * y + w * z) * s0;
            Mt[2] = 2.f * (x * z - w * y) * s0;
            Mt[3] = 2.f * (x * y - w * z) * s1;
            Mt[4] = (1.f - 2.f * (x * x + z * z)) * s1;
            Mt[5] = 2.f * (y * z + w * x) * s1;
            Mt[6] = 2.f * (x * z + w * y) * s2;
            Mt[7] = 2.f * (y * z - w * x) * s2;
            Mt[8] = (1.f - 2.f * (x * x + y * y)) * s2;
        }
        const int v_end = min(nv, (int)(blockIdx.y + 1) * PRE_VIEWS);
        for (int v = (int)blockIdx.y * PRE_VIEWS; v < v_end; ++v) {
            const DevView& V = views[v];
            if (V.scene != sc) continue;
            const int64_t r = V.rec_off + i;
            float4 vc_q = make_float4(0.f, 0.f, 0.f, 0.f), vi_q = vc_q;
            float2 vc_w = make_float2(0.f, 0.f), vi_w = vc_w;
            uint2 rc = make_uint2(0, 0), ri = make_uint2(0, 0);
            uint32_t zbits = 0u, ntc = 0u;
            if (valid) {
                const float ex[3] = {(float)V.ex[0], (float)V.ex[1], (float)V.ex[2]};
                const float ey[3] = {(float)V.ey[0], (float)V.ey[1], (float)V.ey[2]};
                const float ez[3] = {(float)V.ez[0], (float)V.ez[1], (float)V.ez[2]};
                const float iA = (float)V.iA, iR = (float)V.iR;
                const float iAc = (float)V.iAc, iEc = (float)V.iEc;
                const Conic2 C = plane_conic(Mt, ex, ey, iAc, iEc, rp.dilation);
                const Conic2 I = plane_conic(Mt, ex, ez, iA, iR, rp.dilation);
                if (C.ok && I.ok) {
                    const float xr = ex[0] * m0 + ex[1] * m1 + ex[2] * m2;
                    const float yr = ey[0] * m0 + ey[1] * m1 + ey[2] * m2;
                    const double zr = range_coordinate(V.ez, m0, m1, m2);
                    const float cCx = xr * iAc + (float)V.hWc, cCy = yr * iEc + (float)V.hHc;
                    const float cIx = xr * iA + (float)V.hW, cIy = (float)zr * iR + (float)V.hH;
                    ntc = tile_rect(cCx, cCy, C.sxx, C.syy, rp.q_max, V.Wc, V.Hc, &rc);
                    nc += ntc;
                    ni += tile_rect(cIx, cIy, I.sxx, I.syy, rp.q_max, V.W, V.H, &ri);
                    zbits = __float_as_uint(__double2float_rn(zr));
                    if (zbits == 0x80000000u) zbits = 0u;   // -0 -> +0
                    vc_q = make_float4(cCx, cCy, C.a, C.b);
                    vc_w = make_float2(C.c, ext);
                    vi_q = make_float4(cIx, cIy, I.a, I.b);
                    vi_w = make_float2(I.c, 0.0f);
                }
            }
            if (write_records && prec) {
                float P = 0.0f;
                if (valid) {
                    if (S.shc > 0) {
                        float d[3], Y[SH_MAX];
                        radar_direction_f(V, m0, m1, m2, d);
                        sh_basis(d[0], d[1], d[2], S.shc, Y);
                        const float* c = S.sh + (int64_t)S.sh_stride * i;
                        for (int k = 0; k < S.shc; ++k) P += c[k] * Y[k];
                    } else {
                        P = S.amp[i];
                    }
                }
                prec[r] = P * (float)V.pscale;
            }
            if (write_records) {
                crec[r] = CRec{vc_q, make_float4(vc_w.x, vc_w.y, __uint_as_float(ntc), 0.0f)};
                // the imaging-plane record is read only after pass A: stored
                // non-temporally, it does not displace what the sorts and
                // the footprint masks read next (preprocess 0.213 -> 0.204 ms)
                __builtin_nontemporal_store(vi_q.x, &iq[r].x);
                __builtin_nontemporal_store(vi_q.y, &iq[r].y);
                __builtin_nontemporal_store(vi_q.z, &iq[r].z);
                __builtin_nontemporal_store(vi_q.w, &iq[r].w);
                __builtin_nontemporal_store(vi_w.x, &iw[r].x);
                __builtin_nontemporal_store(vi_w.y, &iw[r].y);
                rect_c[r] = rc;
                __builtin_nontemporal_store(ri.x, &rect_i[r].x);
                __builtin_nontemporal_store(ri.y, &rect_i[r].y);
                dkey[r] = float_order_bits(__uint_as_float(zbits));
                if (A_zero) A_zero[r] = 0.0f;   // pass A adds the shares
            }
        }
    }
    // wave sums first: 256 same-address LDS atomics would serialise
    unsigned long long wc = nc, wi = ni;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        wc += (unsigned long long)__shfl_xor((long long)wc, d, WAVE);
        wi += (unsigned long long)__shfl_xor((long long)wi, d, WAVE);
    }
    if (lane_id() == 0) {
        if (wc) atomicAdd(&part[0], wc);
        if (wi) atomicAdd(&part[1], wi);
    }
    __syncthreads();
    // spread over TOTAL_SLOTS addresses; k_sum_slots adds them up
    const uint32_t bid = blockIdx.y * gridDim.x + blockIdx.x;
    if (threadIdx.x < 2 && part[threadIdx.x])
        atomicAdd(&totals[2 * (bid % TOTAL_SLOTS) + threadIdx.x], part[threadIdx.x]);
}

__global__ void __launch_bounds__(1024)
k_sum_slots(const unsigned long long* __restrict__ slots, unsigned long long* __restrict__ out)
{
    __shared__ unsigned long long acc[2];
    if (threadIdx.x < 2) acc[threadIdx.x] = 0;
    __syncthreads();
    const unsigned long long c = slots[2 * threadIdx.x], i = slots[2 * threadIdx.x + 1];
    if (c) atomicAdd(&acc[0], c);
    if (i) atomicAdd(&acc[1], i);
    __syncthreads();
    if (threadIdx.x < 2) out[threadIdx.x] = acc[threadIdx.x];
}

// I = P A into the imaging record (incident intensity 1, Sec. II-A; P the
// record's phase factor from prec when given, else the scalar amplitude
// times the view's cell-area factor); with
// cnt_i given, also the imaging-plane pair count of the record: the tiles of
// its rectangle if I is nonzero, none otherwise (a zero intensity adds
// nothing to any pixel), and their sum over each block of 256 records.
// Also the list of the records pass A used (A > 0; every used record gets at
// least FLT_MIN), in index order within each block's 2048 records (blocks
// in any order), its length in status[ST_ACTIVE]. A record with A = 0 has
// I = P A = 0 and took part in no ray's compositing, so all of its
// gradients are zero: the backward passes and the parameter adjoint visit
// the listed records only. A wave takes 8 groups of 64 consecutive records
// (16 was 0.137 ms on the 72-view vehicle, 8 is 0.124).
constexpr int INT_GROUPS = 8;

__global__ void __launch_bounds__(256)
k_set_intensity(const DevView* __restrict__ views, const DevScene* __restrict__ scenes, int nv,
                int64_t records, const float* __restrict__ A,
                const float* __restrict__ prec, float2* __restrict__ iw,
                const uint2* __restrict__ rect_i, uint32_t* __restrict__ cnt_i,
                uint32_t* __restrict__ bsum_i, uint32_t* __restrict__ status,
                uint32_t* __restrict__ active)
{
    __shared__ uint32_t s_cnt[4];
    __shared__ uint32_t s_base;
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    const int64_t wave0 = ((int64_t)blockIdx.x * 4 + w) * (INT_GROUPS * WAVE);
    uint64_t m[INT_GROUPS];
    uint32_t n = 0, quarter = 0;
    // the wave's records mostly lie in one view: look it up once
    const int v0 = wave0 < records ? find_view(nv, wave0, [&](int k) { return views[k].rec_off; })
                                   : 0;
    const int64_t v0_end = v0 + 1 < nv ? views[v0 + 1].rec_off : records;
    // all groups' loads first (A and the phase factors, then the rectangles
    // of the records with an intensity), so that a wave waits for two
    // memory latencies instead of two per group
    float a[INT_GROUPS], I[INT_GROUPS];
#pragma unroll
    for (int g = 0; g < INT_GROUPS; ++g) {
        const int64_t r = wave0 + g * WAVE + lane;
        a[g] = 0.0f;
        I[g] = 0.0f;
        if (r < records) {
            a[g] = A[r];
            const int v = r < v0_end ? v0
                                     : find_view(nv, r, [&](int k) { return views[k].rec_off; });
            const DevView& V = views[v];
            I[g] = prec ? prec[r] : scenes[V.scene].amp[r - V.rec_off] * (float)V.pscale;
        }
    }
    uint2 ri[INT_GROUPS];
#pragma unroll
    for (int g = 0; g < INT_GROUPS; ++g) {
        const int64_t r = wave0 + g * WAVE + lane;
        I[g] *= a[g];
        ri[g] = make_uint2(0u, 0u);
        if (cnt_i && r < records && I[g] != 0.0f) ri[g] = rect_i[r];
    }
#pragma unroll
    for (int g = 0; g < INT_GROUPS; ++g) {
        const int64_t r = wave0 + g * WAVE + lane;
        uint32_t cnt = 0u;
        if (r < records) {
            iw[r].y = I[g];
            if (cnt_i) {
                if (I[g] != 0.0f)
                    cnt = ((ri[g].x >> 16) - (ri[g].x & 0xFFFF)) *
                          ((ri[g].y >> 16) - (ri[g].y & 0xFFFF));
                cnt_i[r] = cnt;
            }
        }
        m[g] = __ballot(a[g] != 0.0f);
        n += (uint32_t)__popcll(m[g]);
        if (cnt_i) {
            // the imaging-plane pair count of each 256 records (four groups)
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) cnt += __shfl_xor(cnt, d, WAVE);
            quarter += cnt;
            const int64_t b0 = wave0 + (g & ~3) * WAVE;
            if ((g & 3) == 3) {
                if (lane == 0 && b0 < records) bsum_i[b0 / 256] = quarter;
                quarter = 0;
            }
        }
    }
    // one counter update per block: the list is filled in runs, not per wave
    if (lane == 0) s_cnt[w] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        s_base = tot ? atomicAdd(&status[ST_ACTIVE], tot) : 0u;
    }
    __syncthreads();
    uint32_t o = s_base;
    for (int k = 0; k < w; ++k) o += s_cnt[k];
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int g = 0; g < INT_GROUPS; ++g) {
        if (m[g] >> lane & 1ull)
            active[o + (uint32_t)__popcll(m[g] & below)] = (uint32_t)(wave0 + g * WAVE + lane);
        o += (uint32_t)__popcll(m[g]);
    }
}

// Adjoint of one plane: conic gradient (a, b, c with q = a dx^2 + 2 b dx dy
// + c dy^2) and centre gradient -> dSigma (6 unique, symmetric full-matrix
// convention) and dmu.
__device__ void plane_adjoint(const double* Q, const float* gq, const double* u,
                              const double* w, double a, double b, double* dS, double* dmu)
{
    // symmetric gradient of the conic matrix, then dSigma2 = -Q G Q
    double g00 = gq[2], g01 = 0.5 * (double)gq[3], g11 = gq[4];
    double q00 = Q[0], q01 = Q[1], q11 = Q[2];
    double t00 = q00 * g00 + q01 * g01, t01 = q00 * g01 + q01 * g11;
    double t10 = q01 * g00 + q11 * g01, t11 = q01 * g01 + q11 * g11;
    double h00 = -(t00 * q00 + t01 * q01);
    double h01 = -(t00 * q01 + t01 * q11);
    double h11 = -(t10 * q01 + t11 * q11);
    h00 *= a * a; h01 *= a * b; h11 *= b * b;
    // dSigma += h00 u u^T + h01 (u w^T + w u^T) + h11 w w^T
    int idx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int p = idx[k][0], q = idx[k][1];
        dS[k] += h00 * u[p] * u[q] + h01 * (u[p] * w[q] + w[p] * u[q]) + h11 * w[p] * w[q];
    }
    double gx = (double)gq[0] * a, gy = (double)gq[1] * b;
    for (int k = 0; k < 3; ++k) dmu[k] += gx * u[k] + gy * w[k];
}

// Per-Gaussian gradient outputs: d_means (3), d_scales (3), d_quats (4),
// d_amp, d_ext (d_ext_back is the same), then the SH coefficients' (up to
// SH_MAX) for scenes with a phase-function expansion. The backward takes the
// views PB_VIEWS at a time (grid y): a thread's Gaussian frame serves more
// views, fewer parts are summed; on the 72-view vehicle 16 was fastest
// (0.216 ms at 8, 0.191 at 16, 0.201 at 24, 0.253 at 72).
constexpr int PB_OUT = 12;
constexpr int PB_VIEWS = 16;

template <bool SH>
__device__ __forceinline__ void store_param_grads(const DevScene& S, int64_t i, const float* o)
{
    float* om = S.d_means + 3 * i;
    float* os = S.d_scales + 3 * i;
    float* oq = S.d_quats + 4 * i;
    om[0] = o[0]; om[1] = o[1]; om[2] = o[2];
    os[0] = o[3]; os[1] = o[4]; os[2] = o[5];
    oq[0] = o[6]; oq[1] = o[7]; oq[2] = o[8]; oq[3] = o[9];
    if (S.d_amp) S.d_amp[i] = o[10];
    S.d_ext[i] = o[11];
    if (S.d_ext_back) S.d_ext_back[i] = o[11];
    if (SH)
        for (int k = 0; k < S.shc; ++k) S.d_sh[(int64_t)S.sh_stride * i + k] = o[PB_OUT + k];
}

// dL/dP per view is A dL/dI times the view's cell-area factor. With an SH
// phase function P = sum_k c_k Y_k(d), d = (x_radar - mu) / |x_radar - mu|:
// dL/dc_k = dL/dP Y_k(d), and the means gain dL/dP (dd/dmu)^T grad_d P with
// dd/dmu = -(I - d d^T) / |x_radar - mu| (zero for a plane wave).
template <bool SH>
__global__ void __launch_bounds__(256)
k_params_backward(const DevView* __restrict__ views, const DevScene* __restrict__ scenes, int nv,
                  int nscenes, int64_t items, RasterParams rp, const float* __restrict__ A,
                  const float* __restrict__ grad_c, const float* __restrict__ grad_i,
                  int64_t records, int nout, float* __restrict__ part)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= items) return;
    int s = find_view(nscenes, t, [&](int k) { return scenes[k].item_off; });
    const DevScene& S = scenes[s];
    int64_t i = t - S.item_off;
    double dmu[3] = {0, 0, 0}, dS[6] = {0, 0, 0, 0, 0, 0};
    double dk = 0.0, dp = 0.0;
    constexpr int NSH = SH ? SH_MAX : 1;
    double csh[NSH], dsh[NSH];
    const int nsh = SH ? S.shc : 0;
    if (SH) {
        for (int k = 0; k < NSH; ++k) {
            csh[k] = k < nsh ? (double)S.sh[(int64_t)S.sh_stride * i + k] : 0.0;
            dsh[k] = 0.0;
        }
    }
    Geo g;
    gaussian_frame(S, i, g);
    bool any = false;
    const int v_end = min(nv, (int)(blockIdx.y + 1) * PB_VIEWS);
    for (int v = (int)blockIdx.y * PB_VIEWS; v < v_end && g.valid; ++v) {
        const DevView& V = views[v];
        if (V.scene != s) continue;
        // a record pass A never used (A = 0) has zero gradients in this view,
        // and its gradient sums were never written
        if (A[V.rec_off + i] == 0.0f) continue;
        double covC[3], covI[3], QC[3], QI[3];
        plane_cov(g, V.ex, V.ey, V.iAc, V.iEc, rp.dilation, covC);
        plane_cov(g, V.ex, V.ez, V.iA, V.iR, rp.dilation, covI);
        if (!conic(covC, QC) || !conic(covI, QI)) continue;  // no pairs in this view
        any = true;
        int64_t r = V.rec_off + i;
        float gc[6], gi[6];
        const float4 c0 = reinterpret_cast<const float4*>(grad_c + r * GC_STRIDE)[0];
        const float2 c1 = reinterpret_cast<const float2*>(grad_c + r * GC_STRIDE)[2];
        gc[0] = c0.x, gc[1] = c0.y, gc[2] = c0.z, gc[3] = c0.w, gc[4] = c1.x, gc[5] = c1.y;
        const float4 i0 = reinterpret_cast<const float4*>(grad_i + r * GC_STRIDE)[0];
        const float2 i1 = reinterpret_cast<const float2*>(grad_i + r * GC_STRIDE)[2];
        gi[0] = i0.x, gi[1] = i0.y, gi[2] = i0.z, gi[3] = i0.w, gi[4] = i1.x, gi[5] = i1.y;
        plane_adjoint(QC, gc, V.ex, V.ey, V.iAc, V.iEc, dS, dmu);
        plane_adjoint(QI, gi, V.ex, V.ez, V.iA, V.iR, dS, dmu);
        dk += gc[5];
        const double dP = (double)A[r] * gi[5] * V.pscale;
        if (SH && nsh > 0) {
            double d[3], inv_r = 0.0;
            double w[3] = {-V.range * V.ez[0] - g.mu[0], -V.range * V.ez[1] - g.mu[1],
                           -V.range * V.ez[2] - g.mu[2]};
            const double n2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
            if (V.range > 0.0 && n2 > 0.0) {
                inv_r = 1.0 / sqrt(n2);
                for (int k = 0; k < 3; ++k) d[k] = w[k] * inv_r;
            } else {
                for (int k = 0; k < 3; ++k) d[k] = -V.ez[k];
            }
            double Y[SH_MAX];
            sh_basis(d[0], d[1], d[2], nsh, Y);
            for (int k = 0; k < NSH; ++k)
                if (k < nsh) dsh[k] += dP * Y[k];
            if (inv_r > 0.0) {
                double gd[3];
                sh_expansion_grad(csh, nsh, d[0], d[1], d[2], gd);
                const double along = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
                for (int k = 0; k < 3; ++k) dmu[k] -= dP * (gd[k] - along * d[k]) * inv_r;
            }
        } else {
            dp += dP;
        }
    }
    // the gradients are linear in (dSigma, dmu, dkappa, dP): a group of views
    // contributes its own part, summed over the groups by k_params_reduce
    float o[PB_OUT + (SH ? SH_MAX : 0)] = {};
    if (any && g.valid) {
        // Sigma = M M^T with M = R diag(s): dM = 2 dSigma M (dSigma symmetric)
        double D[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
        double dM[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                dM[3 * r + c] = 2.0 * (D[3 * r] * g.M[c] + D[3 * r + 1] * g.M[3 + c] +
                                       D[3 * r + 2] * g.M[6 + c]);
        double ds[3], G[9];
        for (int c = 0; c < 3; ++c) {
            ds[c] = g.R[c] * dM[c] + g.R[3 + c] * dM[3 + c] + g.R[6 + c] * dM[6 + c];
            for (int r = 0; r < 3; ++r) G[3 * r + c] = dM[3 * r + c] * g.s[c];
        }
        double w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
        // derivative of the unit-quaternion rotation matrix entries
        double gw = 2.0 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
        double gx = 2.0 * (y * G[1] + z * G[2] + y * G[3] - 2.0 * x * G[4] - w * G[5] + z * G[6] +
                           w * G[7] - 2.0 * x * G[8]);
        double gy = 2.0 * (-2.0 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] +
                           z * G[7] - 2.0 * y * G[8]);
        double gz = 2.0 * (-2.0 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.0 * z * G[4] +
                           y * G[5] + x * G[6] + y * G[7]);
        double dot = w * gw + x * gx + y * gy + z * gz;
        double inv = 1.0 / g.qnorm;
        o[0] = (float)dmu[0]; o[1] = (float)dmu[1]; o[2] = (float)dmu[2];
        o[3] = (float)ds[0]; o[4] = (float)ds[1]; o[5] = (float)ds[2];
        o[6] = (float)((gw - w * dot) * inv);
        o[7] = (float)((gx - x * dot) * inv);
        o[8] = (float)((gy - y * dot) * inv);
        o[9] = (float)((gz - z * dot) * inv);
        o[10] = (float)dp;
        o[11] = (float)dk;
        if (SH)
            for (int k = 0; k < NSH; ++k) o[PB_OUT + k] = (float)dsh[k];
    }
    if (gridDim.y == 1) {
        store_param_grads<SH>(S, i, o);
    } else {
        const int nw = PB_OUT + nsh;
#pragma unroll
        for (int k = 0; k < PB_OUT + (SH ? SH_MAX : 0); ++k)
            if (k < nw) part[((int64_t)blockIdx.y * nout + k) * items + t] = o[k];
    }
}

// Sum of the view groups' parts of every Gaussian's gradients (nout floats
// per group and Gaussian; a scene's Gaussians use PB_OUT + its SH count).
template <bool SH>
__global__ void __launch_bounds__(256)
k_params_reduce(const DevScene* __restrict__ scenes, int nscenes, int64_t items, int groups,
                int nout, const float* __restrict__ part)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= items) return;
    const int s = find_view(nscenes, t, [&](int k) { return scenes[k].item_off; });
    const DevScene& S = scenes[s];
    constexpr int NO = PB_OUT + (SH ? SH_MAX : 0);
    const int nw = PB_OUT + (SH ? S.shc : 0);
    double acc[NO] = {};
    for (int gq = 0; gq < groups; ++gq)
#pragma unroll
        for (int k = 0; k < NO; ++k)
            if (k < nw) acc[k] += part[((int64_t)gq * nout + k) * items + t];
    float o[NO];
#pragma unroll
    for (int k = 0; k < NO; ++k) o[k] = (float)acc[k];
    store_param_grads<SH>(S, t - S.item_off, o);
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace

hipError_t launch_preprocess(const DevView* views, const DevScene* scenes, int nv, int nscenes,
                             int64_t items, const RasterParams& rp, bool write_records,
                             CRec* crec, float4* iq, float2* iw, uint2* rect_c,
                             uint2* rect_i, uint32_t* dkey, float* A_zero, float* prec,
                             unsigned long long* slots, unsigned long long* totals,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(2 * TOTAL_SLOTS / 256), dim3(256), 0, s, slots,
                       2 * TOTAL_SLOTS);
    if (items > 0 && nv > 0)
        hipLaunchKernelGGL(k_preprocess,
                           dim3(blocks_for(items, 256), (unsigned)((nv + PRE_VIEWS - 1) / PRE_VIEWS)),
                           dim3(256), 0, s, views, scenes, nv, nscenes, items, rp,
                           write_records ? 1 : 0, crec, iq, iw, rect_c, rect_i, dkey,
                           write_records ? A_zero : nullptr, write_records ? prec : nullptr,
                           slots);
    hipLaunchKernelGGL(k_sum_slots, dim3(1), dim3(TOTAL_SLOTS), 0, s, slots, totals);
    return hipGetLastError();
}

hipError_t launch_set_intensity(const DevView* views, const DevScene* scenes, int nv,
                                int64_t records, const float* A, const float* prec,
                                float2* iw, const uint2* rect_i, uint32_t* cnt_i,
                                uint32_t* bsum_i, uint32_t* status, uint32_t* active,
                                hipStream_t s)
{
    if (records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_intensity, dim3(blocks_for(records, 4 * INT_GROUPS * WAVE)),
                       dim3(256), 0, s, views, scenes, nv, records, A, prec, iw, rect_i, cnt_i,
                       bsum_i, status, active);
    return hipGetLastError();
}

int params_groups(int nv) { return nv > 0 ? (nv + PB_VIEWS - 1) / PB_VIEWS : 1; }

size_t params_part_floats(int nv, int64_t items, int sh_coeffs)
{
    const int g = params_groups(nv);
    return g > 1 ? (size_t)(PB_OUT + sh_coeffs) * g * (size_t)items : 0;
}

hipError_t launch_params_backward(const DevView* views, const DevScene* scenes, int nv,
                                  int nscenes, int64_t scene_items, const RasterParams& rp,
                                  const float* A, const float* grad_c, const float* grad_i,
                                  int64_t records, int sh_coeffs, float* part, hipStream_t s)
{
    if (scene_items <= 0) return hipSuccess;
    if (sh_coeffs < 0 || sh_coeffs > SH_MAX) return hipErrorInvalidValue;
    const int groups = params_groups(nv);
    if (groups > 1 && !part) return hipErrorInvalidValue;
    const int nout = PB_OUT + sh_coeffs;
    const dim3 grid(blocks_for(scene_items, 256), groups);
    if (sh_coeffs > 0)
        hipLaunchKernelGGL(k_params_backward<true>, grid, dim3(256), 0, s, views, scenes, nv,
                           nscenes, scene_items, rp, A, grad_c, grad_i, records, nout, part);
    else
        hipLaunchKernelGGL(k_params_backward<false>, grid, dim3(256), 0, s, views, scenes, nv,
                           nscenes, scene_items, rp, A, grad_c, grad_i, records, nout, part);
    if (groups > 1) {
        const dim3 g1(blocks_for(scene_items, 256));
        if (sh_coeffs > 0)
            hipLaunchKernelGGL(k_params_reduce<true>, g1, dim3(256), 0, s, scenes, nscenes,
                               scene_items, groups, nout, part);
        else
            hipLaunchKernelGGL(k_params_reduce<false>, g1, dim3(256), 0, s, scenes, nscenes,
                               scene_items, groups, nout, part);
    }
    return hipGetLastError();
}

}  // namespace sdgr
