/*
 * sdgr.h -- C ABI of the SAR Differentiable Gaussian Rasterizer (SDGR) on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: SAR-GS, "Gaussian Splatting based SAR Images Rendering and Target
 * Reconstruction" (arXiv 2506.21633), Sec. II.
 *   forward  (Sec. II-A): Gaussians + radar geometry -> SAR images
 *     1. mapping and projection (radar rotation R_r, projections P_C, P_I):
 *        every Gaussian onto the computation plane (perpendicular to the
 *        line of sight) and the imaging plane (slant range x azimuth);
 *     2. scattering intensity (Eq. for I_i): rays from the computation-plane
 *        cells traverse the depth-sorted Gaussians front to back with
 *        two-way extinction; each Gaussian's absorbed share summed over the
 *        rays is A_i, and I_i = P_i * A_i;
 *     3. image formation (Eq. for S_{n,m}): additive layover of footprint-
 *        weighted intensities on the imaging plane.
 *   backward (Sec. II-B): gradients of a scalar loss L, given dL/dS, with
 *     respect to means, scales, rotations, amplitudes P and extinctions.
 *
 * Conventions (the readings of the paper that the implementation fixes):
 *   - grazing angle theta, azimuth phi; image rows = slant range (index
 *     grows away from the radar), columns = azimuth; the world origin maps
 *     to the image centre; pixel and cell centres at +1/2;
 *   - computation plane: same size as the image and spacings
 *     (d_az, d_rg * tan(theta)) unless given;
 *   - footprint f(q) = (exp(-q/2) - eps)/(1 - eps) for q < q_max, else 0,
 *     q the quadratic form of the inverse projected covariance,
 *     eps = exp(-q_max/2);
 *   - alpha = 1 - exp(-kappa f), kappa = k_e+ + k_e- (only their sum is
 *     identifiable: the paper states both derivatives are equal);
 *   - depth order: fl32 of the FP64 range coordinate, ties by ascending
 *     Gaussian index;
 *   - scales are standard deviations in metres (> 0), quaternions (w,x,y,z)
 *     of any nonzero norm, normalised inside. Gaussians with non-finite
 *     parameters, a scale <= 0 or a zero quaternion contribute nothing and
 *     receive zero gradient.
 *
 * Memory: every pointer in sdgr_scene, sdgr_scene_grad, the images and the
 * workspaces is DEVICE memory on the current HIP device; sdgr_view,
 * sdgr_options and sdgr_plan structs live in HOST memory. The caller owns
 * every buffer; the library never allocates or frees device memory. Arrays
 * are contiguous row-major float32.
 *
 * Streams: `stream` is a hipStream_t (NULL = default stream). All work is
 * enqueued on it; sdgr_forward and sdgr_backward do not synchronise the
 * host. sdgr_plan_query synchronises the stream (it reads pair counts).
 *
 * Errors: functions return 0 on success or a negative SDGR_E* code; the
 * message of the last error on the calling thread is sdgr_last_error().
 * Outputs are unspecified after an error.
 */
#ifndef SDGR_H
#define SDGR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDGR_VERSION 1

#define SDGR_OK 0
#define SDGR_EINVAL (-1)       /* invalid argument (null, sizes, angles) */
#define SDGR_EWORKSPACE (-2)   /* workspace smaller than the plan requires */
#define SDGR_EHIP (-3)         /* HIP runtime error */
#define SDGR_EOVERFLOW (-4)    /* pair count exceeds the plan's capacity */
#define SDGR_EUNSUPPORTED (-5) /* option or size outside what is built */

/* One scene of n Gaussians (device pointers, float32).
 *
 * Extinction (Sec. II-A): the forward and backward coefficients k_e+ and
 * k_e- enter the model only through their sum kappa. Give ext = kappa and
 * ext_back = NULL, or the two coefficients separately (ext = k_e+,
 * ext_back = k_e-); both then receive the same gradient dL/dkappa.
 *
 * Phase function (Sec. II-B): the scalar amp, or (sh not NULL) a real
 * spherical-harmonics expansion of degree sh_degree (0..3, orthonormal,
 * without the Condon-Shortley phase, coefficient index l*l + l + m for
 * m = -l..l) evaluated at the unit direction from the Gaussian's centre to
 * the radar (see sdgr_view.radar_range). With sh given, amp is ignored and
 * may be NULL, and the means also receive the gradient through that
 * direction. */
typedef struct sdgr_scene {
    int64_t n;
    const float* means;   /* [n,3] world position, metres */
    const float* scales;  /* [n,3] per-axis standard deviation, metres */
    const float* quats;   /* [n,4] rotation (w,x,y,z) */
    const float* amp;     /* [n]   scattering amplitude P (phase function) */
    const float* ext;     /* [n]   extinction kappa, or k_e+ with ext_back */
    const float* ext_back;   /* [n] backward extinction k_e-, or NULL */
    const float* sh;         /* [n, sh_stride] SH coefficients of the phase
                                function (the first (sh_degree + 1)^2 of
                                each row are used), or NULL */
    int32_t sh_degree;       /* 0..3 when sh is given, else ignored */
    int32_t sh_stride;       /* floats from one Gaussian's row of sh (and
                                of d_sh) to the next: 0 means (sh_degree +
                                1)^2, else at least that (a degree below the
                                array's, e.g. while training raises it) */
} sdgr_scene;

/* Gradient outputs of one scene (device pointers, same shapes as the
 * inputs). They are OVERWRITTEN with the sum over all views of the scene.
 * d_ext_back is required when the scene has ext_back (it receives the same
 * values as d_ext), d_sh when it has sh (rows of sh_stride floats, of which
 * the used (sh_degree + 1)^2 are written and the rest left untouched); with
 * sh, d_amp may be NULL (if given it is filled with zeros: amp takes no
 * part). */
typedef struct sdgr_scene_grad {
    float* d_means;
    float* d_scales;
    float* d_quats;
    float* d_amp;
    float* d_ext;
    float* d_ext_back;
    float* d_sh;
} sdgr_scene_grad;

/* One radar view (host struct). Zero in comp_* takes the default. */
typedef struct sdgr_view {
    double azimuth;      /* phi [rad] */
    double grazing;      /* theta [rad], in (0, pi/2) */
    double d_az, d_rg;   /* image pixel spacings [m], > 0 */
    double comp_d_az;    /* computation-plane azimuth spacing, 0 = d_az */
    double comp_d_el;    /* computation-plane elevation spacing,
                            0 = d_rg * tan(grazing) */
    int64_t img_offset;  /* float offset of this view's H x W image in the
                            images / dL_dimages buffers */
    int32_t img_w, img_h;    /* image columns (azimuth), rows (range) */
    int32_t comp_w, comp_h;  /* computation-plane cells, 0 = image size */
    int32_t scene;           /* index into the scenes array */
    int32_t reserved;        /* must be 0 */
    double radar_range;      /* slant distance [m] of the radar from the
                                scene origin, on the line of sight on the
                                near side; it sets the direction at which a
                                phase-function expansion is evaluated for
                                each Gaussian. 0: a plane wave, the
                                direction the same (-e_z) for all. >= 0 */
} sdgr_view;

typedef struct sdgr_options {
    int32_t shadowing;   /* 1: two-way extinction along the line of sight
                            (Eq. for I_i); 0: every Gaussian sees the full
                            incident wave */
    int32_t recompute;   /* 1: keep only per-ray state and A between forward
                            and backward; the backward re-runs projection,
                            binning and sorting (large scenes) */
    float q_max;         /* footprint cutoff of q, > 0 (9 = 3 sigma) */
    float tau_max;       /* rays stop after their optical depth reaches
                            tau_max (terms below exp(-tau_max) dropped);
                            <= 0 disables early termination */
    float dilation;      /* added to the diagonal of every projected 2D
                            covariance, in pixels^2 (0 = none) */
    int32_t deterministic;  /* 1: repeated calls on the same inputs give
                            bitwise identical images and gradients: every
                            sum over tiles or list segments runs in a fixed
                            order (per-pair partials reduced per Gaussian in
                            list order, one wave per image tile) instead of
                            float atomics; costs extra memory and time */
    int32_t tile;        /* tile side in cells: 0 (default) or 8, the one
                            size built; other values give SDGR_EUNSUPPORTED */
    int32_t cell_area;   /* 1: I = P A times the computation-plane cell area
                            comp_d_az * comp_d_el [m^2], so that intensities
                            measure the absorbing cross-section and do not
                            depend on the cell size; 0: I = P A */
    int32_t reserved;    /* must be 0 */
} sdgr_options;

/* Sizes of one (scenes, views, options) problem; filled by
 * sdgr_plan_query and passed back unchanged to forward/backward. */
typedef struct sdgr_plan {
    size_t state_bytes;        /* kept from forward to backward */
    size_t fwd_scratch_bytes;  /* temporary during forward */
    size_t bwd_scratch_bytes;  /* temporary during backward */
    size_t image_floats;       /* minimum length of images / dL_dimages */
    int64_t records;           /* sum over views of the scene's n */
    int64_t pairs_c;           /* (Gaussian, tile) pairs, computation plane */
    int64_t pairs_i;           /* (Gaussian, tile) pairs, imaging plane, of
                                  all Gaussians: a capacity, since only those
                                  with a nonzero intensity emit pairs */
    int64_t tiles_c, tiles_i;  /* tiles over all views */
    int64_t rays;              /* computation-plane cells over all views */
    int64_t gaussians;         /* sum over the scenes of n */
    int32_t nviews, nscenes;
    int32_t tile;              /* tile side in pixels (8) */
    int32_t recompute;         /* copy of options.recompute */
    int32_t deterministic;     /* copy of options.deterministic */
    int32_t sh_coeffs;         /* most SH coefficients of any scene (0: no
                                  scene has sh); sizes the backward scratch */
    int64_t hit_bytes;         /* part of the state in which the forward keeps
                                  the footprint hits each computation-plane
                                  tile's rays used (Sec. II-A compositing
                                  order), so that the backward (Sec. II-B)
                                  reads them instead of re-deriving them from
                                  the footprint masks. The plan calls set 8
                                  bytes per computation-plane pair plus 16 MiB,
                                  and 0 in recompute or deterministic mode
                                  (where it is always taken as 0). A caller
                                  may lower it (>= 0; the state shrinks to
                                  match): tiles that find it full, and all
                                  tiles at 0, re-derive their hits, with the
                                  same results up to float rounding. */
} sdgr_plan;

/* Library version (SDGR_VERSION). */
int sdgr_version(void);

/* Message of the last error on the calling thread ("" if none). */
const char* sdgr_last_error(void);

/* Fill `opt` with the defaults: shadowing 1, recompute 0, q_max 9,
 * tau_max 16, dilation 0, deterministic 0, tile 0 (8). */
void sdgr_default_options(sdgr_options* opt);

/* Bytes of device scratch that sdgr_plan_query needs for nscenes scenes
 * and nv views (a few KB; host-only computation). */
size_t sdgr_query_bytes(int32_t nscenes, int32_t nv);

/* Plan a problem: validates every argument, projects all Gaussians on the
 * device to count their (Gaussian, tile) pairs on both planes (paper
 * Sec. II-A, the projections P_C and P_I), synchronises `stream`, and fills
 * `plan` with the exact workspace sizes.
 * scenes[nscenes] (host array of structs with device pointers), views[nv]
 * (host), query_scratch: device buffer of at least
 * sdgr_query_bytes(nscenes, nv) bytes, 256-byte aligned, free again when the
 * call returns. Returns SDGR_EINVAL on bad arguments, SDGR_EWORKSPACE if the
 * scratch is too small, SDGR_EUNSUPPORTED if a count exceeds 2^31 - 1. */
int sdgr_plan_query(const sdgr_scene* scenes, int32_t nscenes,
                    const sdgr_view* views, int32_t nv,
                    const sdgr_options* opt, void* query_scratch,
                    size_t query_bytes, void* stream, sdgr_plan* plan);

/* Re-sizes `plan` for pair capacities pairs_c, pairs_i (for instance the
 * counts of a previous query plus headroom, so that a training loop whose
 * Gaussians move a little need not query every step): recomputes the three
 * workspace sizes from the plan's own counts; host-only. A forward that
 * finds more pairs than the capacities reports SDGR_EOVERFLOW through
 * sdgr_status. */
int sdgr_plan_resize(sdgr_plan* plan, int64_t pairs_c, int64_t pairs_i);

/* The plan sdgr_plan_query would return had it counted pairs_c and pairs_i
 * pairs, built from host data alone (no device work, no synchronisation).
 * For callers that know the counts already: the pair counts of a launch
 * that fuses several problems' views are the sums of theirs, so a server
 * can query each request once and plan any batch of them on the host.
 * Same argument checks as sdgr_plan_query; SDGR_EUNSUPPORTED for capacities
 * outside [0, 2^31 - 1]. */
int sdgr_plan_host(const sdgr_scene* scenes, int32_t nscenes, const sdgr_view* views,
                   int32_t nv, const sdgr_options* opt, int64_t pairs_c, int64_t pairs_i,
                   sdgr_plan* plan);

/* Forward and backward return SDGR_EINVAL if `plan` does not belong to the
 * scenes, views and options, and SDGR_EWORKSPACE if its workspace sizes are
 * smaller than its capacities need (a plan edited by hand). */

/* Forward render (Sec. II-A). Writes every view's H x W image at
 * images + view.img_offset (row-major [range row][azimuth column]); other
 * floats of `images` are left untouched. `state` (plan->state_bytes) must
 * be kept unchanged until the matching sdgr_backward; `scratch`
 * (plan->fwd_scratch_bytes) may be reused after the call's work completes
 * on `stream`. Both must be 256-byte aligned. Asynchronous. If the pair
 * counts exceed the plan (inputs changed since the query), the rendering is
 * incomplete and sdgr_status reports SDGR_EOVERFLOW. */
int sdgr_forward(const sdgr_scene* scenes, int32_t nscenes,
                 const sdgr_view* views, int32_t nv, const sdgr_options* opt,
                 const sdgr_plan* plan, void* state, void* scratch,
                 float* images, void* stream);

/* Backward (Sec. II-B) for the cotangent dL_dimages (same layout as the
 * images). Same scenes, views, options, plan and `state` as the forward.
 * `scratch` holds plan->bwd_scratch_bytes. Overwrites grads[s] for every
 * scene s (entries of a scene no view uses are set to zero). Asynchronous. */
int sdgr_backward(const sdgr_scene* scenes, int32_t nscenes,
                  const sdgr_view* views, int32_t nv,
                  const sdgr_options* opt, const sdgr_plan* plan, void* state,
                  void* scratch, const float* dL_dimages,
                  const sdgr_scene_grad* grads, void* stream);

/* Forward render (Sec. II-A) that allocates nothing and takes no workspace:
 * for callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc). Same arguments and
 * result as sdgr_forward without the plan and workspaces: the pair counts,
 * the kept state and the scratch live in one static device array of
 * SDGR_STATIC_SCRATCH_BYTES per GPU, held from the first call on that GPU
 * until the process ends. The call counts the (Gaussian, tile) pairs as
 * sdgr_plan_query does (one synchronisation of `stream`), then enqueues the
 * forward on `stream`. Returns SDGR_EUNSUPPORTED, before enqueuing the
 * forward, when the problem needs more than the array holds (the message
 * gives the size). Calls on one GPU share its array: a call's work must be
 * complete before another call on that GPU starts (calls on one stream are
 * ordered; calls on different streams or threads race). No state is kept
 * for a backward. */
#define SDGR_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int sdgr_forward_static(const sdgr_scene* scenes, int32_t nscenes,
                        const sdgr_view* views, int32_t nv,
                        const sdgr_options* opt, float* images, void* stream);

/* Synchronises `stream` and returns SDGR_EOVERFLOW if a forward or backward
 * that used `state` found more pairs than planned, else SDGR_OK. */
int sdgr_status(const sdgr_plan* plan, const void* state, void* stream);

/* The same check without synchronising: enqueues on `stream` an OR of the
 * state's overflow flag into the device word *flags (a caller-owned uint32
 * that starts at 0). A loop can accumulate the flags of many steps and read
 * the word once: nonzero means some forward or backward found more pairs
 * than planned (its results are incomplete and the step must be redone with
 * a larger plan). */
int sdgr_status_accumulate(const sdgr_plan* plan, const void* state, uint32_t* flags,
                           void* stream);

/* Copies the per-view scattering shares A (float32, plan->records entries,
 * view-major: view v's entries start at the sum of the n of the scenes of
 * views 0..v-1) out of `state` into the device buffer `out`. Asynchronous.
 * I_i = P_i * A_i (Eq. for I_i). */
int sdgr_read_intensity(const sdgr_plan* plan, const void* state, float* out,
                        void* stream);

/* Copies the per-ray total optical depth (float32, plan->rays entries,
 * view-major, each view row-major [row][col] over its computation plane)
 * out of `state` into the device buffer `out`. Asynchronous. */
int sdgr_read_optical_depth(const sdgr_plan* plan, const void* state,
                            float* out, void* stream);

/* ---- instrumentation (for benchmarks; not part of the method) ----------
 * When enabled, every stage of forward/backward/plan_query records a pair of
 * HIP events on the call's stream (a few microseconds of overhead per
 * stage). sdgr_profile_read waits for the recorded events, writes the total
 * milliseconds and the number of timed calls of each stage into ms[i] and
 * calls[i] for i < n (either may be NULL), resets the totals and returns the
 * number of stages. sdgr_profile_stage(i) names stage i. */
int sdgr_profile_enable(int32_t on);
int sdgr_profile_read(double* ms, int64_t* calls, int32_t n);
const char* sdgr_profile_stage(int32_t i);

/* Work counters. While sdgr_profile_count(1) is in effect, forward and
 * backward calls count, in `state`, the (cell, Gaussian) evaluations inside
 * the footprint (q < q_max) of pass A forward, pass A backward, pass B
 * forward and pass B backward (out[0..3]), the rounds of 64 evaluations
 * (pass A forward and backward) or 64 list entries (pass B forward) a wave
 * ran (out[4..6]), the summed length of the tile-list prefixes some ray
 * of pass A used (out[7]), the most batches of list chunks one computation-
 * plane tile read in pass A forward and backward (out[8], out[9]), the
 * batches whose footprint hits did not fit one compaction round, counted
 * once per extra group, in pass A forward and backward (out[10], out[11]),
 * the rays stopped at tau_max (out[12]), the longest list prefix one
 * tile used (out[13]), the tiles the pass A backward ran as long lists
 * (at least 2048 entries) and as short ones (out[14], out[15]), and the
 * tiles whose pass A backward read the forward's stored hits and those
 * that re-derived them from the footprint masks (out[16], out[17]). The
 * counting adds atomics, so timed runs leave it off.
 * sdgr_read_work synchronises `stream` and copies min(n, 18) counters of
 * the last forward (and backward) that used `state`. */
int sdgr_profile_count(int32_t on);
int sdgr_read_work(const sdgr_plan* plan, const void* state, uint64_t* out, int32_t n,
                   void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SDGR_H */
