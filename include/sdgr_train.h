/* Reconstruction-loop support of the SDGR library: the steps around the
 * renderer that fit Gaussians to SAR images (Sec. III-B: gradient descent
 * from an initial point cloud, densification and pruning after Sec. II-B,
 * "Densification and Pruning Operation"), and the evaluation metrics of
 * Sec. III-B, "Evaluation Metrics" (PSNR, SSIM, Chamfer distance, F1).
 *
 * Same conventions as sdgr.h: device pointers to contiguous float32 arrays,
 * work enqueued on `stream` (a hipStream_t, NULL = default stream), nothing
 * allocated, SDGR_* return codes with sdgr_last_error() describing the last
 * failure of the calling thread. Argument checks happen before any work is
 * enqueued; a failing call enqueues nothing.
 */
#ifndef SDGR_TRAIN_H
#define SDGR_TRAIN_H

#include "sdgr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One parameter array with its gradient and Adam moments. */
typedef struct sdgr_param_group {
    float* param;        /* [count], updated in place */
    const float* grad;   /* [count] dL/dparam */
    float* m;            /* [count] first moment, 0 before the first step */
    float* v;            /* [count] second moment, 0 before the first step */
    int64_t count;
    float lr;            /* step size */
    int32_t log_space;   /* 1: the parameter is positive and stepped as its
                            logarithm (gradient dL/dparam * param, update
                            param * exp(-step)); 0: stepped as is */
    float lo, hi;        /* after the step the parameter is clamped to
                            [lo, hi] (lo < hi); lo >= hi: no clamp. An
                            extinction stepped in log space has no bound of
                            its own, and an unbounded one overflows */
    int32_t reserved;    /* must be 0 */
} sdgr_param_group;

typedef struct sdgr_adam_config {
    float beta1, beta2;  /* moment decay rates, in [0, 1) */
    float eps;           /* added to the root of the second moment, > 0 */
    int32_t reserved;    /* must be 0 */
} sdgr_adam_config;

/* One Adam step (Kingma and Ba, with bias correction) at iteration t >= 1
 * over all groups, in one launch: m = b1 m + (1 - b1) g, v = b2 v +
 * (1 - b2) g^2, step = lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * then the clamp.
 * At most SDGR_ADAM_MAX_GROUPS groups; a group with count 0 is skipped.
 * SDGR_EINVAL for null arrays of a non-empty group, t < 1, or a config
 * outside the ranges above. */
#define SDGR_ADAM_MAX_GROUPS 16
int sdgr_adam_step(const sdgr_param_group* groups, int32_t ngroups, int64_t t,
                   const sdgr_adam_config* cfg, void* stream);

/* Densification statistics, accumulated after each backward: for every
 * Gaussian whose position gradient d_means[i] is nonzero, grad_acc[i] +=
 * |d_means[i]|, grad_cnt[i] += 1 and grad_dir[i] += d_means[i]. The three
 * arrays ([n], [n], [n,3]) start at zero and are reset by the caller after
 * each densification. */
int sdgr_densify_stats(const float* d_means, int64_t n, float* grad_acc, float* grad_cnt,
                       float* grad_dir, void* stream);

/* Thresholds of densify and prune (Sec. II-B; the ablation study uses a
 * gradient threshold of 0.003 and a largest radius of 0.3 times the radar
 * illumination range). */
typedef struct sdgr_densify_config {
    float grad_threshold;  /* mean position-gradient norm that densifies */
    float split_scale;     /* largest std above which a Gaussian is split
                              rather than cloned [m] */
    float max_radius;      /* 3 x largest std above this is pruned [m] */
    float kappa_min;       /* extinction below this is pruned */
    float split_factor;    /* children's std = parent's / split_factor, > 1 */
    int32_t reserved;      /* must be 0 */
} sdgr_densify_config;

/* A set of Gaussians with the Adam moments of each parameter array.
 * amp and sh (with their moments) may be NULL; rows of sh hold sh_coeffs
 * floats. Moment arrays have the shapes of their parameters. */
typedef struct sdgr_gaussian_set {
    float* means;   float* m_means;  float* v_means;    /* [n,3] */
    float* scales;  float* m_scales; float* v_scales;   /* [n,3] */
    float* quats;   float* m_quats;  float* v_quats;    /* [n,4] */
    float* amp;     float* m_amp;    float* v_amp;      /* [n] or NULL */
    float* ext;     float* m_ext;    float* v_ext;      /* [n] */
    float* sh;      float* m_sh;     float* v_sh;       /* [n,sh_coeffs] or NULL */
    int32_t sh_coeffs;                                  /* 0..16 */
    int32_t reserved;                                   /* must be 0 */
} sdgr_gaussian_set;

/* Densify and prune `in` (n Gaussians) into `out` (capacity >= 2 n rows in
 * every array `in` has), using the statistics of sdgr_densify_stats. Each
 * Gaussian is, in this order of precedence:
 *   pruned  if ext < kappa_min or 3 * max(scale) > max_radius;
 *   cloned  if grad_cnt > 0 and grad_acc / grad_cnt >= grad_threshold and
 *           max(scale) <= split_scale: it stays and a copy displaced by
 *           -max(scale) along the unit accumulated gradient follows it;
 *   split   under the same gradient condition with max(scale) >
 *           split_scale: it is replaced by two children with scales /
 *           split_factor, centred one largest std either side of it along
 *           its largest axis (the + side first), both displaced by the
 *           children's largest std against the accumulated gradient;
 *   kept    otherwise.
 * Decisions are taken in FP32. The outputs keep the input order (each
 * Gaussian's outputs together); copies and children get zero moments, kept
 * and cloned originals keep theirs. The new count is written to the device
 * int64 *n_out (read it after synchronising the stream). `workspace` holds
 * sdgr_densify_workspace_bytes(n) bytes, 256-byte aligned. */
size_t sdgr_densify_workspace_bytes(int64_t n);
int sdgr_densify(const sdgr_gaussian_set* in, int64_t n, const float* grad_acc,
                 const float* grad_cnt, const float* grad_dir, const sdgr_densify_config* cfg,
                 sdgr_gaussian_set* out, int64_t capacity, int64_t* n_out, void* workspace,
                 size_t workspace_bytes, void* stream);

/* Squared distance from each of nq query points to its nearest point among
 * nr reference points ([nq,3], [nr,3]; exhaustive search) into d2[nq]: the
 * directed terms of the Chamfer distance and the matches of precision and
 * recall (Sec. III-B, "Evaluation Metrics"). nr = 0 gives +inf. */
int sdgr_nearest_sq(const float* query, int64_t nq, const float* ref, int64_t nr, float* d2,
                    void* stream);

/* Per image of nimg pairs (x, ref) of h x w floats: SSIM averaged over the
 * positions where an 11 x 11 Gaussian window (sigma 1.5) fits, with C1 =
 * (0.01 L)^2, C2 = (0.03 L)^2, L = data_range; and the mean squared error
 * and the reference's maximum (PSNR = 10 log10(max^2 / mse)). Outputs
 * ssim[nimg], mse[nimg], ref_max[nimg]. SDGR_EINVAL if h or w < 11. */
int sdgr_image_metrics(const float* x, const float* ref, int32_t nimg, int32_t h, int32_t w,
                       float data_range, float* ssim, float* mse, float* ref_max,
                       void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SDGR_TRAIN_H */
