// Reconstruction-loop kernels (Sec. III-B: gradient descent on the
// Gaussians with densification and pruning after Sec. II-B) and evaluation
// metrics (Sec. III-B, "Evaluation Metrics"). Contracts in
// include/sdgr_train.h.
//
// All of it is memory- or launch-bound elementwise work except the
// nearest-neighbour search (exhaustive, LDS-tiled: each workgroup stages
// reference points in LDS and every thread keeps one query's minimum) and
// the SSIM windows (121 taps per position, the window weights in LDS).
#include "common.hpp"
#include "sdgr_train.h"

#include <math.h>

#include <cmath>
#include <string>

namespace sdgr {
namespace {

inline unsigned blocks_for(int64_t n, int b, unsigned cap = 1u << 20)
{
    const int64_t g = (n + b - 1) / b;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

// ------------------------------------------------------------------ Adam

struct AdamGroupDev {
    float* p;
    const float* g;
    float* m;
    float* v;
    int64_t start, count;
    float lr;
    int32_t log_space;
    float lo, hi;
    int32_t clamp;
};

struct AdamArgs {
    AdamGroupDev grp[SDGR_ADAM_MAX_GROUPS];
    int32_t ngroups;
    float b1, b2, eps;
    float bc1, bc2;   // 1 / (1 - b1^t), 1 / (1 - b2^t)
};

__global__ void __launch_bounds__(256) k_adam(AdamArgs a, int64_t total)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int k = 0;
        while (k + 1 < a.ngroups && e >= a.grp[k + 1].start) ++k;
        const AdamGroupDev& G = a.grp[k];
        const int64_t i = e - G.start;
        float x = G.p[i];
        float g = G.g[i];
        if (G.log_space) g *= x;   // d/d(log x) = x d/dx
        const float m = a.b1 * G.m[i] + (1.0f - a.b1) * g;
        const float v = a.b2 * G.v[i] + (1.0f - a.b2) * g * g;
        const float step = G.lr * (m * a.bc1) / (sqrtf(v * a.bc2) + a.eps);
        x = G.log_space ? x * expf(-step) : x - step;
        if (G.clamp) x = fminf(fmaxf(x, G.lo), G.hi);
        G.p[i] = x;
        G.m[i] = m;
        G.v[i] = v;
    }
}

// ------------------------------------------------------ densify statistics

__global__ void __launch_bounds__(256)
k_densify_stats(const float* __restrict__ dmu, int64_t n, float* __restrict__ acc,
                float* __restrict__ cnt, float* __restrict__ dir)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g0 = dmu[3 * i], g1 = dmu[3 * i + 1], g2 = dmu[3 * i + 2];
    const float nn = sqrtf(g0 * g0 + g1 * g1 + g2 * g2);
    if (!(nn > 0.0f)) return;
    acc[i] += nn;
    cnt[i] += 1.0f;
    dir[3 * i] += g0;
    dir[3 * i + 1] += g1;
    dir[3 * i + 2] += g2;
}

// ---------------------------------------------------- densify and prune

constexpr uint8_t ACT_KEEP = 0, ACT_PRUNE = 1, ACT_CLONE = 2, ACT_SPLIT = 3;

struct DensifyArgs {
    sdgr_gaussian_set in, out;
    sdgr_densify_config cfg;
    int64_t n;
};

__device__ __forceinline__ uint32_t outputs_of(uint8_t a)
{
    return a == ACT_PRUNE ? 0u : (a == ACT_KEEP ? 1u : 2u);
}

__device__ __forceinline__ float max3(const float* s)
{
    return fmaxf(s[0], fmaxf(s[1], s[2]));
}

// Action of each Gaussian (FP32 decisions) and the output count of each
// block of 256.
__global__ void __launch_bounds__(256)
k_densify_count(DensifyArgs a, const float* __restrict__ acc, const float* __restrict__ cnt,
                uint8_t* __restrict__ act, uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t s_w[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t nout = 0u;
    if (i < a.n) {
        const float smax = max3(a.in.scales + 3 * i);
        uint8_t c = ACT_KEEP;
        if (a.in.ext[i] < a.cfg.kappa_min || 3.0f * smax > a.cfg.max_radius)
            c = ACT_PRUNE;
        else if (cnt[i] > 0.0f && __fdiv_rn(acc[i], cnt[i]) >= a.cfg.grad_threshold)
            c = smax > a.cfg.split_scale ? ACT_SPLIT : ACT_CLONE;
        act[i] = c;
        nout = outputs_of(c);
    }
    uint32_t total;
    block_excl_scan_256(nout, s_w, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the block counts (one workgroup: each thread sums a
// contiguous run, the runs' sums are scanned in LDS) and the total.
__global__ void __launch_bounds__(1024)
k_densify_scan(const uint32_t* __restrict__ bsum, int64_t nb, uint32_t* __restrict__ boff,
               int64_t* __restrict__ n_out)
{
    __shared__ uint32_t s[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    uint32_t run = 0u;
    for (int64_t b = b0; b < b1; ++b) run += bsum[b];
    s[threadIdx.x] = run;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 run sums
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t t = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t off = s[threadIdx.x] - run;
    for (int64_t b = b0; b < b1; ++b) {
        boff[b] = off;
        off += bsum[b];
    }
    if (threadIdx.x == 1023) *n_out = (int64_t)s[1023];
}

__device__ __forceinline__ void copy_row(const float* src, float* dst, int64_t from, int64_t to,
                                         int width)
{
    if (!src) return;
    for (int k = 0; k < width; ++k) dst[to * width + k] = src[from * width + k];
}

__device__ __forceinline__ void zero_row(float* dst, int64_t to, int width)
{
    if (!dst) return;
    for (int k = 0; k < width; ++k) dst[to * width + k] = 0.0f;
}

// Write Gaussian i's outputs at slot o (and o + 1): the parameters, with
// the means and scales of copies and children changed, and the moments
// (copied for the original, zero for new Gaussians).
__device__ void emit(const DensifyArgs& a, int64_t i, int64_t o, const float* mu,
                     const float* sc, bool fresh)
{
    const sdgr_gaussian_set& I = a.in;
    const sdgr_gaussian_set& O = a.out;
    for (int k = 0; k < 3; ++k) {
        O.means[3 * o + k] = mu[k];
        O.scales[3 * o + k] = sc[k];
    }
    copy_row(I.quats, O.quats, i, o, 4);
    copy_row(I.amp, O.amp, i, o, 1);
    copy_row(I.ext, O.ext, i, o, 1);
    copy_row(I.sh, O.sh, i, o, I.sh_coeffs);
    struct M { const float* im; const float* iv; float* om; float* ov; int w; };
    const M ms[6] = {{I.m_means, I.v_means, O.m_means, O.v_means, 3},
                     {I.m_scales, I.v_scales, O.m_scales, O.v_scales, 3},
                     {I.m_quats, I.v_quats, O.m_quats, O.v_quats, 4},
                     {I.m_amp, I.v_amp, O.m_amp, O.v_amp, 1},
                     {I.m_ext, I.v_ext, O.m_ext, O.v_ext, 1},
                     {I.m_sh, I.v_sh, O.m_sh, O.v_sh, I.sh_coeffs}};
    for (int g = 0; g < 6; ++g) {
        if (!ms[g].om) continue;
        if (fresh) {
            zero_row(ms[g].om, o, ms[g].w);
            zero_row(ms[g].ov, o, ms[g].w);
        } else {
            copy_row(ms[g].im, ms[g].om, i, o, ms[g].w);
            copy_row(ms[g].iv, ms[g].ov, i, o, ms[g].w);
        }
    }
}

__global__ void __launch_bounds__(256)
k_densify_apply(DensifyArgs a, const uint8_t* __restrict__ act,
                const uint32_t* __restrict__ boff, const float* __restrict__ dir)
{
    __shared__ uint32_t s_w[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint8_t c = i < a.n ? act[i] : ACT_PRUNE;
    uint32_t total;
    const uint32_t ex = block_excl_scan_256(outputs_of(c), s_w, total);
    if (i >= a.n || c == ACT_PRUNE) return;
    const int64_t o = (int64_t)boff[blockIdx.x] + ex;
    const float* mu = a.in.means + 3 * i;
    const float* sc = a.in.scales + 3 * i;
    if (c != ACT_SPLIT) emit(a, i, o, mu, sc, false);   // the original stays
    if (c == ACT_KEEP) return;
    // unit accumulated gradient (zero if there is none)
    const float d0 = dir[3 * i], d1 = dir[3 * i + 1], d2 = dir[3 * i + 2];
    const float dn = sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
    const float inv = dn > 0.0f ? 1.0f / dn : 0.0f;
    const float gh[3] = {d0 * inv, d1 * inv, d2 * inv};
    const float smax = max3(sc);
    if (c == ACT_CLONE) {
        const float m2[3] = {mu[0] - smax * gh[0], mu[1] - smax * gh[1], mu[2] - smax * gh[2]};
        emit(a, i, o + 1, m2, sc, true);
        return;
    }
    // split: the largest axis is the column of the rotation for the largest scale
    const float* q = a.in.quats + 4 * i;
    const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
    const int ax = (sc[0] >= sc[1] && sc[0] >= sc[2]) ? 0 : (sc[1] >= sc[2] ? 1 : 2);
    float e[3];
    if (ax == 0) {
        e[0] = 1.f - 2.f * (y * y + z * z); e[1] = 2.f * (x * y + w * z); e[2] = 2.f * (x * z - w * y);
    } else if (ax == 1) {
        e[0] = 2.f * (x * y - w * z); e[1] = 1.f - 2.f * (x * x + z * z); e[2] = 2.f * (y * z + w * x);
    } else {
        e[0] = 2.f * (x * z + w * y); e[1] = 2.f * (y * z - w * x); e[2] = 1.f - 2.f * (x * x + y * y);
    }
    const float f = 1.0f / a.cfg.split_factor;
    const float cs[3] = {sc[0] * f, sc[1] * f, sc[2] * f};
    const float cmax = max3(cs);
    for (int side = 0; side < 2; ++side) {
        const float sg = side == 0 ? 1.0f : -1.0f;
        float m2[3];
        for (int k = 0; k < 3; ++k) m2[k] = mu[k] + sg * smax * e[k] - cmax * gh[k];
        emit(a, i, o + side, m2, cs, true);
    }
}

// ----------------------------------------------------------------- metrics

constexpr int NN_TILE = 1024;

__global__ void __launch_bounds__(256)
k_nearest_sq(const float* __restrict__ q, int64_t nq, const float* __restrict__ ref, int64_t nr,
             float* __restrict__ d2)
{
    __shared__ float s_x[NN_TILE], s_y[NN_TILE], s_z[NN_TILE];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (i < nq) {
        qx = q[3 * i];
        qy = q[3 * i + 1];
        qz = q[3 * i + 2];
    }
    float best = INFINITY;
    for (int64_t t0 = 0; t0 < nr; t0 += NN_TILE) {
        const int cnt = (int)min((int64_t)NN_TILE, nr - t0);
        __syncthreads();
        for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
            s_x[k] = ref[3 * (t0 + k)];
            s_y[k] = ref[3 * (t0 + k) + 1];
            s_z[k] = ref[3 * (t0 + k) + 2];
        }
        __syncthreads();
        for (int k = 0; k < cnt; ++k) {
            const float dx = qx - s_x[k], dy = qy - s_y[k], dz = qz - s_z[k];
            best = fminf(best, dx * dx + dy * dy + dz * dz);
        }
    }
    if (i < nq) d2[i] = best;
}

constexpr int SSIM_WIN = 11;

// One workgroup per image: every thread takes window positions in turn and
// keeps partial sums; the workgroup adds them in a fixed order, so the
// result does not depend on timing.
__global__ void __launch_bounds__(256)
k_image_metrics(const float* __restrict__ x, const float* __restrict__ ref, int h, int w,
                float c1, float c2, float* __restrict__ ssim, float* __restrict__ mse,
                float* __restrict__ rmax)
{
    __shared__ float s_w[SSIM_WIN * SSIM_WIN];
    __shared__ double s_a[256], s_b[256];
    __shared__ float s_m[256];
    if (threadIdx.x < SSIM_WIN * SSIM_WIN) {
        const int r = threadIdx.x / SSIM_WIN - SSIM_WIN / 2, c = threadIdx.x % SSIM_WIN - SSIM_WIN / 2;
        s_w[threadIdx.x] = expf(-(float)(r * r + c * c) / (2.0f * 1.5f * 1.5f));
    }
    __syncthreads();
    float wsum = 0.f;
    for (int k = 0; k < SSIM_WIN * SSIM_WIN; ++k) wsum += s_w[k];
    const float iw = 1.0f / wsum;
    const int64_t img = blockIdx.x;
    const float* X = x + img * (int64_t)h * w;
    const float* Y = ref + img * (int64_t)h * w;
    const int vh = h - SSIM_WIN + 1, vw = w - SSIM_WIN + 1;
    const int64_t npos = (int64_t)vh * vw, npix = (int64_t)h * w;
    double acc = 0.0, err = 0.0;
    float mx = -INFINITY;
    for (int64_t p = threadIdx.x; p < npos; p += blockDim.x) {
        const int r0 = (int)(p / vw), c0 = (int)(p % vw);
        float ma = 0.f, mb = 0.f;
        for (int r = 0; r < SSIM_WIN; ++r)
            for (int c = 0; c < SSIM_WIN; ++c) {
                const float wt = s_w[r * SSIM_WIN + c] * iw;
                ma += wt * X[(int64_t)(r0 + r) * w + c0 + c];
                mb += wt * Y[(int64_t)(r0 + r) * w + c0 + c];
            }
        float va = 0.f, vb = 0.f, cv = 0.f;
        for (int r = 0; r < SSIM_WIN; ++r)
            for (int c = 0; c < SSIM_WIN; ++c) {
                const float wt = s_w[r * SSIM_WIN + c] * iw;
                const float da = X[(int64_t)(r0 + r) * w + c0 + c] - ma;
                const float db = Y[(int64_t)(r0 + r) * w + c0 + c] - mb;
                va += wt * da * da;
                vb += wt * db * db;
                cv += wt * da * db;
            }
        acc += (double)(((2.f * ma * mb + c1) * (2.f * cv + c2)) /
                        ((ma * ma + mb * mb + c1) * (va + vb + c2)));
    }
    for (int64_t p = threadIdx.x; p < npix; p += blockDim.x) {
        const float d = X[p] - Y[p];
        err += (double)d * d;
        mx = fmaxf(mx, Y[p]);
    }
    s_a[threadIdx.x] = acc;
    s_b[threadIdx.x] = err;
    s_m[threadIdx.x] = mx;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            s_a[threadIdx.x] += s_a[threadIdx.x + d];
            s_b[threadIdx.x] += s_b[threadIdx.x + d];
            s_m[threadIdx.x] = fmaxf(s_m[threadIdx.x], s_m[threadIdx.x + d]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ssim[img] = (float)(s_a[0] / (double)npos);
        mse[img] = (float)(s_b[0] / (double)npix);
        rmax[img] = s_m[0];
    }
}

int einval(const char* msg) { return report_error(SDGR_EINVAL, msg); }

#define TRAIN_HIP(expr)                                                              \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return report_error(SDGR_EHIP, (std::string(#expr) + ": " +             \
                                            hipGetErrorString(e_)).c_str());         \
    } while (0)

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

bool set_arrays_ok(const sdgr_gaussian_set& s)
{
    if (!s.means || !s.scales || !s.quats || !s.ext) return false;
    if (!s.m_means || !s.v_means || !s.m_scales || !s.v_scales || !s.m_quats || !s.v_quats ||
        !s.m_ext || !s.v_ext)
        return false;
    if (s.amp && (!s.m_amp || !s.v_amp)) return false;
    if (s.sh && (!s.m_sh || !s.v_sh)) return false;
    return true;
}

}  // namespace
}  // namespace sdgr

using namespace sdgr;

extern "C" {

int sdgr_adam_step(const sdgr_param_group* groups, int32_t ngroups, int64_t t,
                   const sdgr_adam_config* cfg, void* stream)
{
    clear_error();
    if (!cfg || cfg->reserved != 0) return einval("adam config null or reserved not 0");
    if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) ||
        !(cfg->eps > 0.f))
        return einval("adam betas outside [0, 1) or eps not positive");
    if (t < 1) return einval("adam step t must be >= 1");
    if (ngroups < 0 || ngroups > SDGR_ADAM_MAX_GROUPS || (ngroups > 0 && !groups))
        return einval("adam group count outside 0..SDGR_ADAM_MAX_GROUPS");
    AdamArgs a{};
    int64_t total = 0;
    for (int k = 0; k < ngroups; ++k) {
        const sdgr_param_group& G = groups[k];
        if (G.count < 0) return einval("adam group with negative count");
        if (G.count == 0) continue;
        if (!G.param || !G.grad || !G.m || !G.v) return einval("adam group with a null array");
        if (!std::isfinite(G.lr)) return einval("adam learning rate not finite");
        if (G.reserved != 0) return einval("adam group reserved field not 0");
        if (std::isnan(G.lo) || std::isnan(G.hi)) return einval("adam clamp bound is NaN");
        AdamGroupDev& D = a.grp[a.ngroups++];
        D.p = G.param; D.g = G.grad; D.m = G.m; D.v = G.v;
        D.start = total; D.count = G.count; D.lr = G.lr; D.log_space = G.log_space != 0;
        D.lo = G.lo; D.hi = G.hi; D.clamp = G.lo < G.hi;
        total += G.count;
    }
    if (total == 0) return SDGR_OK;
    a.b1 = cfg->beta1; a.b2 = cfg->beta2; a.eps = cfg->eps;
    a.bc1 = (float)(1.0 / (1.0 - pow((double)cfg->beta1, (double)t)));
    a.bc2 = (float)(1.0 / (1.0 - pow((double)cfg->beta2, (double)t)));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(total, 256, 8192)), dim3(256), 0,
                       (hipStream_t)stream, a, total);
    TRAIN_HIP(hipGetLastError());
    return SDGR_OK;
}

int sdgr_densify_stats(const float* d_means, int64_t n, float* grad_acc, float* grad_cnt,
                       float* grad_dir, void* stream)
{
    clear_error();
    if (n < 0) return einval("negative count");
    if (n == 0) return SDGR_OK;
    if (!d_means || !grad_acc || !grad_cnt || !grad_dir) return einval("null array");
    hipLaunchKernelGGL(k_densify_stats, dim3(blocks_for(n, 256)), dim3(256), 0,
                       (hipStream_t)stream, d_means, n, grad_acc, grad_cnt, grad_dir);
    TRAIN_HIP(hipGetLastError());
    return SDGR_OK;
}

size_t sdgr_densify_workspace_bytes(int64_t n)
{
    if (n < 0) return 0;
    const size_t nb = (size_t)((n + 255) / 256) + 1;
    return align256((size_t)n + 1) + 2 * align256(4 * nb);
}

int sdgr_densify(const sdgr_gaussian_set* in, int64_t n, const float* grad_acc,
                 const float* grad_cnt, const float* grad_dir, const sdgr_densify_config* cfg,
                 sdgr_gaussian_set* out, int64_t capacity, int64_t* n_out, void* workspace,
                 size_t workspace_bytes, void* stream)
{
    clear_error();
    if (!in || !out || !cfg || !n_out) return einval("null argument");
    if (cfg->reserved != 0 || in->reserved != 0 || out->reserved != 0)
        return einval("reserved fields must be 0");
    if (n < 0 || n > (int64_t)1 << 30) return einval("count outside [0, 2^30]");
    if (capacity < 2 * n) return einval("output capacity below twice the input count");
    if (!(cfg->split_factor > 1.0f) || !std::isfinite(cfg->split_factor))
        return einval("split_factor must be > 1");
    if (in->sh_coeffs < 0 || in->sh_coeffs > 16 || out->sh_coeffs != in->sh_coeffs)
        return einval("sh_coeffs outside 0..16 or different between in and out");
    if (!set_arrays_ok(*in) || !set_arrays_ok(*out))
        return einval("null parameter or moment array");
    if ((in->amp != nullptr) != (out->amp != nullptr) ||
        (in->sh != nullptr) != (out->sh != nullptr))
        return einval("in and out differ in which optional arrays they have");
    if (n > 0 && (!grad_acc || !grad_cnt || !grad_dir)) return einval("null statistics");
    if (workspace_bytes < sdgr_densify_workspace_bytes(n) || (n > 0 && !workspace))
        return report_error(SDGR_EWORKSPACE, "workspace smaller than sdgr_densify_workspace_bytes");
    if ((uintptr_t)workspace & 255) return einval("workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(k_densify_scan, dim3(1), dim3(1024), 0, s, (const uint32_t*)nullptr,
                           (int64_t)0, (uint32_t*)nullptr, n_out);
        TRAIN_HIP(hipGetLastError());
        return SDGR_OK;
    }
    const int64_t nb = (n + 255) / 256;
    char* w = (char*)workspace;
    uint8_t* act = (uint8_t*)w;
    uint32_t* bsum = (uint32_t*)(w + align256((size_t)n + 1));
    uint32_t* boff = (uint32_t*)(w + align256((size_t)n + 1) + align256(4 * (size_t)(nb + 1)));
    DensifyArgs a{*in, *out, *cfg, n};
    hipLaunchKernelGGL(k_densify_count, dim3((unsigned)nb), dim3(256), 0, s, a, grad_acc,
                       grad_cnt, act, bsum);
    hipLaunchKernelGGL(k_densify_scan, dim3(1), dim3(1024), 0, s, bsum, nb, boff, n_out);
    hipLaunchKernelGGL(k_densify_apply, dim3((unsigned)nb), dim3(256), 0, s, a, act, boff,
                       grad_dir);
    TRAIN_HIP(hipGetLastError());
    return SDGR_OK;
}

int sdgr_nearest_sq(const float* query, int64_t nq, const float* ref, int64_t nr, float* d2,
                    void* stream)
{
    clear_error();
    if (nq < 0 || nr < 0) return einval("negative point count");
    if (nq == 0) return SDGR_OK;
    if (!query || !d2 || (nr > 0 && !ref)) return einval("null array");
    if (nq > (int64_t)1 << 31) return einval("more than 2^31 query points");
    hipLaunchKernelGGL(k_nearest_sq, dim3(blocks_for(nq, 256, 1u << 31)), dim3(256), 0,
                       (hipStream_t)stream, query, nq, ref, nr, d2);
    TRAIN_HIP(hipGetLastError());
    return SDGR_OK;
}

int sdgr_image_metrics(const float* x, const float* ref, int32_t nimg, int32_t h, int32_t w,
                       float data_range, float* ssim, float* mse, float* ref_max, void* stream)
{
    clear_error();
    if (nimg < 0) return einval("negative image count");
    if (h < SSIM_WIN || w < SSIM_WIN) return einval("images smaller than the 11 x 11 window");
    if (!(data_range > 0.0f) || !std::isfinite(data_range)) return einval("data_range must be > 0");
    if (nimg == 0) return SDGR_OK;
    if (!x || !ref || !ssim || !mse || !ref_max) return einval("null array");
    const float c1 = (0.01f * data_range) * (0.01f * data_range);
    const float c2 = (0.03f * data_range) * (0.03f * data_range);
    hipLaunchKernelGGL(k_image_metrics, dim3((unsigned)nimg), dim3(256), 0, (hipStream_t)stream,
                       x, ref, h, w, c1, c2, ssim, mse, ref_max);
    TRAIN_HIP(hipGetLastError());
    return SDGR_OK;
}

}  // extern "C"
