/*
 * sdgr_oracle.c -- TEST INFRASTRUCTURE, not part of the product path.
 *
 * Plain, slow FP64 CPU reference of the SAR Differentiable Gaussian
 * Rasterizer (SAR-GS, arXiv 2506.21633, Sec. II). Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library.
 * It shares no code with the HIP implementation.
 *
 * What it computes, per view (Sec. II-A):
 *   1. Mapping and projection (Eq. for W, R_r, Sigma' = J^T R^T Sigma R J,
 *      P_C, P_I): every Gaussian is mapped to radar coordinates
 *      (x azimuth, y elevation perpendicular to the line of sight, z slant
 *      range = depth) and projected orthographically onto the computation
 *      plane (x, y) and the imaging plane (x, z), giving 2D centres and 2D
 *      covariances on both planes.
 *   2. Scattering intensity (Eq. for I_i and delta): a ray leaves the centre
 *      of every computation-plane cell along the line of sight; along it the
 *      Gaussians are taken front to back in depth order, each absorbing a
 *      fraction alpha = 1 - exp(-kappa g) of what reaches it, with g the
 *      peak-1 footprint of its projected Gaussian at the ray. Its share of
 *      the incident intensity, summed over all rays, is A_i; I_i = P_i A_i.
 *   3. Image formation (Eq. for S_{n,m}): every imaging-plane pixel sums the
 *      intensities of the Gaussians covering it, weighted by their footprint
 *      there (additive layover, order-free).
 * No tiles, no culling other than the footprint's own cutoff q < q_max, an
 * explicit sort per ray.
 *
 * Backward (Sec. II-B): the exact derivative of the forward above, written
 * out directly. For one ray with depth-ordered Gaussians k and optical
 * depths x_k = kappa_k g_k, the ray's share of the loss is
 *     Phi = sum_k c_k alpha_k T_k,   T_k = exp(-sum_{j<k} x_j),
 * with c_k = dL/dA_k, so that
 *     dPhi/dx_k = c_k (1 - alpha_k) T_k - sum_{j>k} c_j alpha_j T_j,
 * a plain suffix sum (the paper states the two extinction derivatives are
 * equal; only their sum kappa is an input here).
 *
 * Readings of the paper taken here where it is silent or garbled (each one
 * is listed in the design notes of the repository):
 *   - theta in R_r is the grazing (depression) angle; x_r = R_r x_w, the
 *     translation T_r and altitude h only add a constant range offset under
 *     the orthographic projection and are dropped; the image is centred on
 *     the world origin.
 *   - the quadratic form delta uses the inverse 2D covariance (a conic) with
 *     the 1/2 of the Gaussian density: footprint
 *         f(q) = (exp(-q/2) - eps) / (1 - eps) for q < q_max, else 0,
 *     eps = exp(-q_max/2): continuous, peak 1, zero beyond the cutoff.
 *   - alpha_i = 1 - exp(-kappa_i g_i) with kappa = k_e+ + k_e-; transmittance
 *     over the Gaussians strictly in front; incident intensity 1; no
 *     cell-area factor unless asked for (then I = P A dAc dEc, the share
 *     in m^2 of the plane perpendicular to the line of sight).
 *   - the phase function's direction (Sec. II-B, SH coefficients per
 *     Gaussian): from the Gaussian's centre to the radar, which sits on the
 *     line of sight through the origin at the view's slant distance; a view
 *     without one is a plane wave, the direction then -e_z everywhere and
 *     the same for every Gaussian. Real SH to degree 3, orthonormal.
 *   - depth order: key fl32_rn(z computed in FP64), ties by ascending index.
 *   - computation plane spacing (d_az, d_rg tan(theta)) and size of the
 *     image by default (Eq. for P_C); imaging plane rows = slant range at
 *     d_rg, columns = azimuth at d_az (Eq. for P_I, read as a plain
 *     slant-range/azimuth grid); cell and pixel centres at +1/2.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no FMA
 * contraction, so the FP64 depth is the sequence of rounded products and
 * sums written below).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_VERSION 1

typedef struct {
    double az, gr;          /* azimuth phi, grazing theta [rad] */
    int64_t W, H;           /* image columns (azimuth), rows (slant range) */
    double dA, dR;          /* image spacings [m] */
    int64_t Wc, Hc;         /* computation-plane cells */
    double dAc, dEc;        /* computation-plane spacings [m] */
    double range;           /* slant distance of the radar from the scene
                               origin along the line of sight; 0: so far
                               that the incident wave is plane */
    double ex[3], ey[3], ez[3];  /* rows of R_r */
} OView;

/* Per-Gaussian inputs beyond position, shape, the scalar amplitude P and the
 * extinction: the paper's two extinction coefficients (forward and backward
 * along the line of sight) enter only through their sum kappa = ext +
 * ext_back; the phase function P may be a spherical-harmonics expansion in
 * the direction from the Gaussian's centre to the radar; the intensity may
 * be normalised by the computation-plane cell area. */
typedef struct {
    const double* ext_back;   /* [n] backward extinction, or NULL (ext is kappa) */
    const double* sh;         /* [n, (sh_deg + 1)^2] SH coefficients of P, or
                                 NULL (P = amp) */
    int64_t sh_deg;           /* 0 .. 3 */
    int64_t cell_area;        /* 1: I = P A times the cell area [m^2] */
} OExtra;

typedef struct {
    int valid;
    double qn[4], qnorm, s[3], R[9], M[9];
    double Sig[9];               /* 3D covariance, full 3x3 */
    double x, y, z;              /* radar coordinates */
    double cC[2], SC[3], QC[3];  /* plane C: centre, cov (xx,xy,yy), conic */
    double cI[2], SI[3], QI[3];  /* plane I */
    double bxC[4], bxI[4];       /* ellipse bounding boxes (x0,x1,y0,y1) */
    float key;
} OG;

/* ---------------------------------------------------------------- views */

/* Rows of the world-to-radar rotation R_r(phi, theta) (Sec. II-A). */
void orc_axes(double phi, double theta, double* ex, double* ey, double* ez)
{
    double sp = sin(phi), cp = cos(phi), st = sin(theta), ct = cos(theta);
    ex[0] = -sp;      ex[1] = -cp;      ex[2] = 0.0;
    ey[0] = -st * cp; ey[1] = st * sp;  ey[2] = ct;
    ez[0] = -ct * cp; ez[1] = ct * sp;  ez[2] = -st;
}

/* p = [azimuth, grazing, img_w, img_h, d_az, d_rg, comp_w, comp_h,
 *      comp_d_az, comp_d_el, radar_range]; zeros in the comp_* slots take
 * the defaults of the computation-plane projection (same grid, elevation
 * spacing d_rg * tan(theta)); radar_range 0 is a plane incident wave. */
static int view_init(OView* v, const double* p)
{
    v->az = p[0]; v->gr = p[1];
    v->W = (int64_t)p[2]; v->H = (int64_t)p[3];
    v->dA = p[4]; v->dR = p[5];
    v->Wc = p[6] > 0 ? (int64_t)p[6] : v->W;
    v->Hc = p[7] > 0 ? (int64_t)p[7] : v->H;
    v->dAc = p[8] > 0 ? p[8] : v->dA;
    v->dEc = p[9] > 0 ? p[9] : v->dR * tan(v->gr);
    v->range = p[10];
    if (!(v->gr > 0.0 && v->gr < M_PI / 2) || v->W <= 0 || v->H <= 0 ||
        v->Wc <= 0 || v->Hc <= 0 || !(v->dA > 0) || !(v->dR > 0) ||
        !(v->dAc > 0) || !(v->dEc > 0) || !(v->range >= 0.0))
        return -1;
    orc_axes(v->az, v->gr, v->ex, v->ey, v->ez);
    return 0;
}

/* ----------------------------------------------------------- projection */

static double dot3(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* u^T Sigma w for a full 3x3 Sigma */
static double quad3(const double* u, const double* S, const double* w)
{
    double t[3];
    for (int r = 0; r < 3; ++r)
        t[r] = S[3 * r] * w[0] + S[3 * r + 1] * w[1] + S[3 * r + 2] * w[2];
    return dot3(u, t);
}

static void conic_of(const double* S, double* Q, int* ok)
{
    double det = S[0] * S[2] - S[1] * S[1];
    if (!(det > 0.0) || !isfinite(det)) { *ok = 0; Q[0] = Q[1] = Q[2] = 0; return; }
    Q[0] = S[2] / det; Q[1] = -S[1] / det; Q[2] = S[0] / det;
}

static void bbox_of(const double* c, const double* S, double q_max, double* b)
{
    double rx = sqrt(q_max * S[0]), ry = sqrt(q_max * S[2]);
    b[0] = c[0] - rx; b[1] = c[0] + rx; b[2] = c[1] - ry; b[3] = c[1] + ry;
}

static void project(const OView* v, const double* mu, const double* s,
                    const double* q, double dil, double q_max, OG* g)
{
    memset(g, 0, sizeof(*g));
    int ok = 1;
    for (int k = 0; k < 3; ++k)
        ok &= isfinite(mu[k]) && isfinite(s[k]) && s[k] > 0.0;
    double qq = 0;
    for (int k = 0; k < 4; ++k) { ok &= isfinite(q[k]); qq += q[k] * q[k]; }
    if (!ok || !(qq > 0.0)) { g->valid = 0; return; }
    g->qnorm = sqrt(qq);
    for (int k = 0; k < 4; ++k) g->qn[k] = q[k] / g->qnorm;
    double w = g->qn[0], x = g->qn[1], y = g->qn[2], z = g->qn[3];
    double* R = g->R;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) g->M[3 * r + c] = R[3 * r + c] * s[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            g->Sig[3 * r + c] = g->M[3 * r] * g->M[3 * c] +
                                g->M[3 * r + 1] * g->M[3 * c + 1] +
                                g->M[3 * r + 2] * g->M[3 * c + 2];
    for (int k = 0; k < 3; ++k) g->s[k] = s[k];
    g->x = dot3(v->ex, mu);
    g->y = dot3(v->ey, mu);
    /* depth: ((ez0*mu0) + (ez1*mu1)) + (ez2*mu2), each step rounded */
    g->z = (v->ez[0] * mu[0] + v->ez[1] * mu[1]) + v->ez[2] * mu[2];
    float kf = (float)g->z;
    g->key = (kf == 0.0f) ? 0.0f : kf;

    g->cC[0] = g->x / v->dAc + 0.5 * (double)v->Wc;
    g->cC[1] = g->y / v->dEc + 0.5 * (double)v->Hc;
    g->SC[0] = quad3(v->ex, g->Sig, v->ex) / (v->dAc * v->dAc) + dil;
    g->SC[1] = quad3(v->ex, g->Sig, v->ey) / (v->dAc * v->dEc);
    g->SC[2] = quad3(v->ey, g->Sig, v->ey) / (v->dEc * v->dEc) + dil;

    g->cI[0] = g->x / v->dA + 0.5 * (double)v->W;
    g->cI[1] = g->z / v->dR + 0.5 * (double)v->H;
    g->SI[0] = quad3(v->ex, g->Sig, v->ex) / (v->dA * v->dA) + dil;
    g->SI[1] = quad3(v->ex, g->Sig, v->ez) / (v->dA * v->dR);
    g->SI[2] = quad3(v->ez, g->Sig, v->ez) / (v->dR * v->dR) + dil;

    conic_of(g->SC, g->QC, &ok);
    conic_of(g->SI, g->QI, &ok);
    g->valid = ok;
    if (ok) {
        bbox_of(g->cC, g->SC, q_max, g->bxC);
        bbox_of(g->cI, g->SI, q_max, g->bxI);
    }
}

/* ------------------------------------------------ phase and extinction */

/* Real spherical harmonics of degree <= deg at the unit vector d = (x, y, z)
 * (orthonormal on the sphere, no Condon-Shortley phase), index l*l + l + m
 * for m = -l..l, written as polynomials in x, y, z; dY[3 k + j] (if not NULL)
 * is the derivative of polynomial k with respect to component j. */
static void sh_basis(const double* d, int64_t deg, double* Y, double* dY)
{
    const double x = d[0], y = d[1], z = d[2], pi = M_PI;
    const double c0 = 0.5 * sqrt(1.0 / pi);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi),
                 c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi),
                 c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi),
                 c3e = 0.25 * sqrt(105.0 / pi);
    double v[16], g[16][3];
    memset(g, 0, sizeof(g));
    v[0] = c0;
    v[1] = c1 * y;  g[1][1] = c1;
    v[2] = c1 * z;  g[2][2] = c1;
    v[3] = c1 * x;  g[3][0] = c1;
    v[4] = c2a * x * y;  g[4][0] = c2a * y; g[4][1] = c2a * x;
    v[5] = c2a * y * z;  g[5][1] = c2a * z; g[5][2] = c2a * y;
    v[6] = c2b * (3.0 * z * z - 1.0);  g[6][2] = c2b * 6.0 * z;
    v[7] = c2a * x * z;  g[7][0] = c2a * z; g[7][2] = c2a * x;
    v[8] = c2c * (x * x - y * y);  g[8][0] = c2c * 2.0 * x; g[8][1] = -c2c * 2.0 * y;
    v[9] = c3a * y * (3.0 * x * x - y * y);
    g[9][0] = c3a * 6.0 * x * y; g[9][1] = c3a * (3.0 * x * x - 3.0 * y * y);
    v[10] = c3b * x * y * z;
    g[10][0] = c3b * y * z; g[10][1] = c3b * x * z; g[10][2] = c3b * x * y;
    v[11] = c3c * y * (5.0 * z * z - 1.0);
    g[11][1] = c3c * (5.0 * z * z - 1.0); g[11][2] = c3c * 10.0 * y * z;
    v[12] = c3d * z * (5.0 * z * z - 3.0);  g[12][2] = c3d * (15.0 * z * z - 3.0);
    v[13] = c3c * x * (5.0 * z * z - 1.0);
    g[13][0] = c3c * (5.0 * z * z - 1.0); g[13][2] = c3c * 10.0 * x * z;
    v[14] = c3e * z * (x * x - y * y);
    g[14][0] = c3e * 2.0 * x * z; g[14][1] = -c3e * 2.0 * y * z; g[14][2] = c3e * (x * x - y * y);
    v[15] = c3a * x * (x * x - 3.0 * y * y);
    g[15][0] = c3a * (3.0 * x * x - 3.0 * y * y); g[15][1] = -c3a * 6.0 * x * y;
    const int64_t ns = (deg + 1) * (deg + 1);
    for (int64_t k = 0; k < ns; ++k) {
        Y[k] = v[k];
        if (dY)
            for (int j = 0; j < 3; ++j) dY[3 * k + j] = g[k][j];
    }
}

/* Unit vector from the centre mu to the radar, which sits on the line of
 * sight through the origin at slant distance range on the near side
 * (-range e_z); a plane wave (range 0) comes from -e_z everywhere. J (if
 * not NULL) receives the 3x3 Jacobian dd/dmu, row-major. */
static void radar_dir(const OView* v, const double* mu, double* d, double* J)
{
    if (!(v->range > 0.0)) {
        for (int k = 0; k < 3; ++k) d[k] = -v->ez[k];
        if (J) memset(J, 0, 9 * sizeof(double));
        return;
    }
    double w[3], r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        w[k] = -v->range * v->ez[k] - mu[k];
        r2 += w[k] * w[k];
    }
    const double r = sqrt(r2);
    for (int k = 0; k < 3; ++k) d[k] = w[k] / r;
    if (J)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) J[3 * a + b] = -((a == b ? 1.0 : 0.0) - d[a] * d[b]) / r;
}

static int64_t sh_count(const OExtra* ex) { return (ex->sh_deg + 1) * (ex->sh_deg + 1); }

/* The intensity factor of Gaussian i in this view: its phase function P
 * (the scalar amp, or the SH expansion at the direction to the radar)
 * times the cell area when normalised. */
static double phase_of(const OView* v, const OExtra* ex, const double* amp,
                       const double* mu, int64_t i)
{
    double P = amp ? amp[i] : 0.0;
    if (ex->sh) {
        double d[3], Y[16];
        radar_dir(v, mu, d, NULL);
        sh_basis(d, ex->sh_deg, Y, NULL);
        const int64_t ns = sh_count(ex);
        P = 0.0;
        for (int64_t k = 0; k < ns; ++k) P += ex->sh[i * ns + k] * Y[k];
    }
    return ex->cell_area ? P * v->dAc * v->dEc : P;
}

static double kappa_of(const OExtra* ex, const double* ext, int64_t i)
{
    return ex->ext_back ? ext[i] + ex->ext_back[i] : ext[i];
}

/* Per-Gaussian phase factors and extinctions of one view. */
static int prepare(const OView* v, const OExtra* ex, int64_t n, const double* means,
                   const double* amp, const double* ext, double** peff, double** kap)
{
    *peff = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    *kap = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!*peff || !*kap) { free(*peff); free(*kap); *peff = *kap = NULL; return -2; }
    for (int64_t i = 0; i < n; ++i) {
        (*peff)[i] = phase_of(v, ex, amp, means + 3 * i, i);
        (*kap)[i] = kappa_of(ex, ext, i);
    }
    return 0;
}

static OG* project_all(const OView* v, int64_t n, const double* means,
                       const double* scales, const double* quats, double dil,
                       double q_max)
{
    OG* G = (OG*)malloc(sizeof(OG) * (size_t)(n > 0 ? n : 1));
    if (!G) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        project(v, means + 3 * i, scales + 3 * i, quats + 4 * i, dil, q_max, &G[i]);
    return G;
}

/* ------------------------------------------------------------ footprint */

static double quadform(const double* Q, double dx, double dy)
{
    return Q[0] * dx * dx + 2.0 * Q[1] * dx * dy + Q[2] * dy * dy;
}

static double foot(double q, double q_max)
{
    if (!(q < q_max)) return 0.0;
    double eps = exp(-0.5 * q_max);
    return (exp(-0.5 * q) - eps) / (1.0 - eps);
}

static double dfoot(double q, double q_max)
{
    if (!(q < q_max)) return 0.0;
    double eps = exp(-0.5 * q_max);
    return -0.5 * exp(-0.5 * q) / (1.0 - eps);
}

/* ---------------------------------------------------------- ray lists */

typedef struct { float key; int64_t idx; double g, q, dx, dy; } Hit;

static int hit_cmp(const void* a, const void* b)
{
    const Hit* x = (const Hit*)a;
    const Hit* y = (const Hit*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* All Gaussians whose computation-plane footprint reaches the ray through
 * cell (col, row), in depth order. Returns the count. */
static int64_t ray_list(const OG* G, int64_t n, int64_t col, int64_t row,
                        double q_max, Hit* out)
{
    double px = (double)col + 0.5, py = (double)row + 0.5;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!G[i].valid) continue;
        double dx = px - G[i].cC[0], dy = py - G[i].cC[1];
        double q = quadform(G[i].QC, dx, dy);
        if (q < q_max) {
            out[m].key = G[i].key; out[m].idx = i;
            out[m].g = foot(q, q_max); out[m].q = q;
            out[m].dx = dx; out[m].dy = dy;
            ++m;
        }
    }
    qsort(out, (size_t)m, sizeof(Hit), hit_cmp);
    return m;
}

static int nthreads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* ------------------------------------------------------------- exports */

int orc_version(void) { return ORC_VERSION; }
int orc_threads(void) { return nthreads(); }

/* Resolved view: out[0..9] = W, H, dA, dR, Wc, Hc, dAc, dEc, range, 0;
 * out[10..18] = ex, ey, ez. */
int orc_view(const double* p, double* out)
{
    OView v;
    if (view_init(&v, p)) return -1;
    out[0] = (double)v.W; out[1] = (double)v.H; out[2] = v.dA; out[3] = v.dR;
    out[4] = (double)v.Wc; out[5] = (double)v.Hc; out[6] = v.dAc; out[7] = v.dEc;
    out[8] = v.range;
    out[9] = 0.0;
    for (int k = 0; k < 3; ++k) {
        out[10 + k] = v.ex[k]; out[13 + k] = v.ey[k]; out[16 + k] = v.ez[k];
    }
    return 0;
}

/* Per-Gaussian projected quantities, 21 doubles each:
 * [0] valid [1] x [2] y [3] z(depth) [4] key (fl32 of depth)
 * [5,6] cC [7..9] Sigma_C (xx,xy,yy) [10..12] conic_C (a,b,c)
 * [13,14] cI [15..17] Sigma_I [18..20] conic_I                (21 doubles) */
int orc_project(int64_t n, const double* means, const double* scales,
                const double* quats, const double* view, double dil,
                double q_max, double* out)
{
    OView v;
    if (n < 0 || view_init(&v, view)) return -1;
    OG* G = project_all(&v, n, means, scales, quats, dil, q_max);
    if (!G) return -2;
    for (int64_t i = 0; i < n; ++i) {
        double* o = out + 21 * i;
        const OG* g = &G[i];
        o[0] = g->valid; o[1] = g->x; o[2] = g->y; o[3] = g->z; o[4] = g->key;
        o[5] = g->cC[0]; o[6] = g->cC[1];
        for (int k = 0; k < 3; ++k) { o[7 + k] = g->SC[k]; o[10 + k] = g->QC[k]; }
        o[13] = g->cI[0]; o[14] = g->cI[1];
        for (int k = 0; k < 3; ++k) { o[15 + k] = g->SI[k]; o[18 + k] = g->QI[k]; }
    }
    free(G);
    return 0;
}

/* Forward of one view.
 * ext_back, sh, sh_deg, cell_area: see OExtra (NULL, NULL, 0, 0 for the
 * scalar-amplitude model with kappa = ext).
 * A[n]          scattering share of every Gaussian (I_i = P_i * A_i)
 * tau[Hc*Wc]    total optical depth of every ray (row-major [row][col])
 * S[H*W]        SAR image (row-major [range row][azimuth column])
 * shadowing=0 drops the transmittance (every Gaussian sees the full wave). */
int orc_forward(int64_t n, const double* means, const double* scales,
                const double* quats, const double* amp, const double* ext,
                const double* ext_back, const double* sh, int64_t sh_deg,
                int64_t cell_area, const double* view, double q_max, double dil,
                int shadowing, double* A, double* tau, double* S)
{
    OView v;
    if (n < 0 || view_init(&v, view) || !(q_max > 0) || sh_deg < 0 || sh_deg > 3) return -1;
    const OExtra ex = {ext_back, sh, sh_deg, cell_area};
    OG* G = project_all(&v, n, means, scales, quats, dil, q_max);
    if (!G) return -2;
    double *peff = NULL, *kap = NULL;
    if (prepare(&v, &ex, n, means, amp, ext, &peff, &kap)) { free(G); return -2; }
    int nt = nthreads();
    double* At = (double*)calloc((size_t)nt * (size_t)(n > 0 ? n : 1), sizeof(double));
    int err = At ? 0 : -2;
    int64_t nrays = v.Wc * v.Hc;
    if (!err) {
#pragma omp parallel
        {
            Hit* list = (Hit*)malloc(sizeof(Hit) * (size_t)(n > 0 ? n : 1));
            double* Amine = At + (size_t)thread_id() * (size_t)n;
#pragma omp for schedule(dynamic, 8)
            for (int64_t r = 0; r < nrays; ++r) {
                int64_t m = ray_list(G, n, r % v.Wc, r / v.Wc, q_max, list);
                double t = 0.0;
                for (int64_t k = 0; k < m; ++k) {
                    int64_t i = list[k].idx;
                    double x = kap[i] * list[k].g;
                    double alpha = 1.0 - exp(-x);
                    Amine[i] += shadowing ? alpha * exp(-t) : alpha;
                    t += x;
                }
                tau[r] = t;
            }
            free(list);
        }
        for (int64_t i = 0; i < n; ++i) {
            double a = 0.0;
            for (int th = 0; th < nt; ++th) a += At[(size_t)th * (size_t)n + i];
            A[i] = a;
        }
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t p = 0; p < v.W * v.H; ++p) {
            double px = (double)(p % v.W) + 0.5, py = (double)(p / v.W) + 0.5;
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                if (!G[i].valid) continue;
                double q = quadform(G[i].QI, px - G[i].cI[0], py - G[i].cI[1]);
                if (q < q_max) acc += foot(q, q_max) * peff[i] * A[i];
            }
            S[p] = acc;
        }
    }
    free(At);
    free(G);
    free(peff);
    free(kap);
    return err;
}

/* Chain rule from a 2D conic/centre gradient on one plane to the 3D
 * covariance and the mean.  dQ = (d/da, d/db, d/dc) for the conic entries
 * with q = a dx^2 + 2 b dx dy + c dy^2; u, w are the radar axes spanning the
 * plane; su, sw their spacings. Adds into dSig (3x3) and dmu. */
static void plane_to_3d(const double* Q, const double* dQ, const double* dc,
                        const double* u, const double* w, double su, double sw,
                        double* dSig, double* dmu)
{
    /* symmetric-matrix gradient of the conic */
    double Gq[4] = {dQ[0], 0.5 * dQ[1], 0.5 * dQ[1], dQ[2]};
    double Qm[4] = {Q[0], Q[1], Q[1], Q[2]};
    double T[4], G2[4];
    /* dL/dSigma2 = -Q Gq Q */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c)
            T[2 * r + c] = Qm[2 * r] * Gq[c] + Qm[2 * r + 1] * Gq[2 + c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c)
            G2[2 * r + c] = -(T[2 * r] * Qm[c] + T[2 * r + 1] * Qm[2 + c]);
    /* Sigma2 = D B^T Sigma B D  ->  dSigma += B D G2 D B^T */
    double sc[2] = {1.0 / su, 1.0 / sw};
    const double* ax[2] = {u, w};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double gab = G2[2 * a + b] * sc[a] * sc[b];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    dSig[3 * r + c] += ax[a][r] * gab * ax[b][c];
        }
    for (int k = 0; k < 3; ++k) dmu[k] += dc[0] * u[k] / su + dc[1] * w[k] / sw;
}

/* From dL/dSigma (3x3) to scales and the raw quaternion. */
static void cov_to_params(const OG* g, const double* dSig, double* ds, double* dq)
{
    /* Sigma = M M^T, M = R diag(s): dM = (dSig + dSig^T) M */
    double dM[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double a = 0;
            for (int k = 0; k < 3; ++k)
                a += (dSig[3 * r + k] + dSig[3 * k + r]) * g->M[3 * k + c];
            dM[3 * r + c] = a;
        }
    double dR[9];
    for (int c = 0; c < 3; ++c) {
        double a = 0;
        for (int r = 0; r < 3; ++r) {
            a += g->R[3 * r + c] * dM[3 * r + c];
            dR[3 * r + c] = dM[3 * r + c] * g->s[c];
        }
        ds[c] += a;
    }
    double w = g->qn[0], x = g->qn[1], y = g->qn[2], z = g->qn[3];
    double G00 = dR[0], G01 = dR[1], G02 = dR[2], G10 = dR[3], G11 = dR[4],
           G12 = dR[5], G20 = dR[6], G21 = dR[7], G22 = dR[8];
    double gn[4];
    gn[0] = 2 * (-z * G01 + y * G02 + z * G10 - x * G12 - y * G20 + x * G21);
    gn[1] = 2 * (y * G01 + z * G02 + y * G10 - 2 * x * G11 - w * G12 + z * G20 +
                 w * G21 - 2 * x * G22);
    gn[2] = 2 * (-2 * y * G00 + x * G01 + w * G02 + x * G10 + z * G12 - w * G20 +
                 z * G21 - 2 * y * G22);
    gn[3] = 2 * (-2 * z * G00 - w * G01 + x * G02 + w * G10 - 2 * z * G11 +
                 y * G12 + x * G20 + y * G21);
    double proj = 0;
    for (int k = 0; k < 4; ++k) proj += g->qn[k] * gn[k];
    for (int k = 0; k < 4; ++k) dq[k] += (gn[k] - g->qn[k] * proj) / g->qnorm;
}

/* Backward of one view for a cotangent Gimg = dL/dS [H*W].
 * Overwrites dmeans[3n], dscales[3n], dquats[4n], damp[n] (0 with SH),
 * dext[n], dext_back[n] (if not NULL; equal to dext: only the sum of the two
 * extinctions enters) and dsh[n, (sh_deg + 1)^2] (if not NULL and sh is
 * given).
 * aux (may be NULL) receives 16 doubles per Gaussian:
 *   [0] A  [1] dL/dI  [2..3] dL/dcI  [4..6] dL/dconic_I (a,b,c)
 *   [7..8] dL/dcC  [9..11] dL/dconic_C  [12] dL/dkappa  [13] dL/dA (= c)
 *   [14], [15] the smallest |q - q_max| over the Gaussian's imaging-plane
 *   pixels and computation-plane cells (how close a cell comes to the
 *   footprint's cutoff, where the footprint is 0 but its derivative is not;
 *   inf for an invalid Gaussian) */
int orc_backward(int64_t n, const double* means, const double* scales,
                 const double* quats, const double* amp, const double* ext,
                 const double* ext_back, const double* sh, int64_t sh_deg,
                 int64_t cell_area, const double* view, double q_max, double dil,
                 int shadowing, const double* Gimg, double* dmeans, double* dscales,
                 double* dquats, double* damp, double* dext, double* dext_back,
                 double* dsh, double* aux)
{
    OView v;
    if (n < 0 || view_init(&v, view) || !(q_max > 0) || sh_deg < 0 || sh_deg > 3) return -1;
    const OExtra ex = {ext_back, sh, sh_deg, cell_area};
    int64_t nrays = v.Wc * v.Hc, npix = v.W * v.H;
    double* A = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* tau = (double*)malloc(sizeof(double) * (size_t)nrays);
    double* S = (double*)malloc(sizeof(double) * (size_t)npix);
    if (!A || !tau || !S) { free(A); free(tau); free(S); return -2; }
    int err = orc_forward(n, means, scales, quats, amp, ext, ext_back, sh, sh_deg, cell_area,
                          view, q_max, dil, shadowing, A, tau, S);
    free(tau); free(S);
    if (err) { free(A); return err; }
    OG* G = project_all(&v, n, means, scales, quats, dil, q_max);
    double *peff = NULL, *kap = NULL;
    if (!G || prepare(&v, &ex, n, means, amp, ext, &peff, &kap)) {
        free(A); free(G); return -2;
    }
    /* per-Gaussian 2D gradients: dI, dcI(2), dQI(3), dcC(2), dQC(3), dk */
    double* g2 = (double*)calloc((size_t)(n > 0 ? n : 1) * 12, sizeof(double));
    int nt = nthreads();
    double* gt = (double*)calloc((size_t)nt * (size_t)(n > 0 ? n : 1) * 6, sizeof(double));
    if (!g2 || !gt) { free(A); free(G); free(g2); free(gt); free(peff); free(kap); return -2; }

    /* distance of the nearest cell to the footprint cutoff, both planes */
    double* edge = (double*)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
    if (!edge) { free(A); free(G); free(g2); free(gt); free(peff); free(kap); return -2; }
    /* imaging plane: every Gaussian against every pixel */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        edge[2 * i] = edge[2 * i + 1] = INFINITY;
        if (!G[i].valid) continue;
        double I = peff[i] * A[i];
        double* o = g2 + 12 * i;
        for (int64_t p = 0; p < npix; ++p) {
            double dx = (double)(p % v.W) + 0.5 - G[i].cI[0];
            double dy = (double)(p / v.W) + 0.5 - G[i].cI[1];
            double q = quadform(G[i].QI, dx, dy);
            if (fabs(q - q_max) < edge[2 * i]) edge[2 * i] = fabs(q - q_max);
            if (!(q < q_max)) continue;
            double Gp = Gimg[p];
            o[0] += Gp * foot(q, q_max);
            double dq = Gp * I * dfoot(q, q_max);
            const double* Q = G[i].QI;
            o[1] += dq * (-2.0 * (Q[0] * dx + Q[1] * dy));
            o[2] += dq * (-2.0 * (Q[1] * dx + Q[2] * dy));
            o[3] += dq * dx * dx;
            o[4] += dq * 2.0 * dx * dy;
            o[5] += dq * dy * dy;
        }
    }

    /* computation plane: every ray, depth ordered, suffix sums */
#pragma omp parallel
    {
        Hit* list = (Hit*)malloc(sizeof(Hit) * (size_t)(n > 0 ? n : 1));
        double* T = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* al = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* mine = gt + (size_t)thread_id() * (size_t)n * 6;
#pragma omp for schedule(dynamic, 8)
        for (int64_t r = 0; r < nrays; ++r) {
            int64_t m = ray_list(G, n, r % v.Wc, r / v.Wc, q_max, list);
            double t = 0.0;
            for (int64_t k = 0; k < m; ++k) {
                double x = kap[list[k].idx] * list[k].g;
                T[k] = shadowing ? exp(-t) : 1.0;
                al[k] = 1.0 - exp(-x);
                t += x;
            }
            double suffix = 0.0;  /* sum_{j>k} c_j alpha_j T_j */
            for (int64_t k = m - 1; k >= 0; --k) {
                int64_t i = list[k].idx;
                double c = peff[i] * g2[12 * i];
                double dx_ = c * (1.0 - al[k]) * T[k] - (shadowing ? suffix : 0.0);
                suffix += c * al[k] * T[k];
                double g = list[k].g;
                double* o = mine + 6 * i;
                o[0] += dx_ * g;                       /* dL/dkappa */
                double dq = dx_ * kap[i] * dfoot(list[k].q, q_max);
                const double* Q = G[i].QC;
                double ddx = list[k].dx, ddy = list[k].dy;
                o[1] += dq * (-2.0 * (Q[0] * ddx + Q[1] * ddy));
                o[2] += dq * (-2.0 * (Q[1] * ddx + Q[2] * ddy));
                o[3] += dq * ddx * ddx;
                o[4] += dq * 2.0 * ddx * ddy;
                o[5] += dq * ddy * ddy;
            }
        }
        free(list); free(T); free(al);
    }
    for (int64_t i = 0; i < n; ++i)
        for (int th = 0; th < nt; ++th)
            for (int k = 0; k < 6; ++k)
                g2[12 * i + 6 + k] += gt[((size_t)th * (size_t)n + (size_t)i) * 6 + k];
    free(gt);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        if (!G[i].valid) continue;
        const double* b = G[i].bxC;
        int64_t c0 = (int64_t)floor(b[0] - 0.5) - 1, c1 = (int64_t)ceil(b[1] - 0.5) + 1;
        int64_t r0 = (int64_t)floor(b[2] - 0.5) - 1, r1 = (int64_t)ceil(b[3] - 0.5) + 1;
        if (c0 < 0) c0 = 0;
        if (r0 < 0) r0 = 0;
        if (c1 > v.Wc - 1) c1 = v.Wc - 1;
        if (r1 > v.Hc - 1) r1 = v.Hc - 1;
        for (int64_t r = r0; r <= r1; ++r)
            for (int64_t c = c0; c <= c1; ++c) {
                double q = quadform(G[i].QC, (double)c + 0.5 - G[i].cC[0],
                                    (double)r + 0.5 - G[i].cC[1]);
                if (fabs(q - q_max) < edge[2 * i + 1]) edge[2 * i + 1] = fabs(q - q_max);
            }
    }

    /* parameters */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double* dm = dmeans + 3 * i;
        double* dsc = dscales + 3 * i;
        double* dqu = dquats + 4 * i;
        for (int k = 0; k < 3; ++k) dm[k] = dsc[k] = 0.0;
        for (int k = 0; k < 4; ++k) dqu[k] = 0.0;
        damp[i] = dext[i] = 0.0;
        if (dext_back) dext_back[i] = 0.0;
        const int64_t ns = sh_count(&ex);
        if (sh && dsh)
            for (int64_t k = 0; k < ns; ++k) dsh[i * ns + k] = 0.0;
        const double* o = g2 + 12 * i;
        if (aux) {
            double* a = aux + 16 * i;
            a[0] = A[i]; a[1] = o[0];
            a[2] = o[1]; a[3] = o[2]; a[4] = o[3]; a[5] = o[4]; a[6] = o[5];
            a[7] = o[7]; a[8] = o[8]; a[9] = o[9]; a[10] = o[10]; a[11] = o[11];
            a[12] = o[6]; a[13] = peff[i] * o[0];
            a[14] = edge[2 * i]; a[15] = edge[2 * i + 1];
        }
        if (!G[i].valid) continue;
        /* dL/dP_eff = A dL/dI, with P_eff = P (times the cell area) */
        const double scale = cell_area ? v.dAc * v.dEc : 1.0;
        const double dP = A[i] * o[0] * scale;
        if (sh) {
            double d[3], J[9], Y[16], dY[48];
            radar_dir(&v, means + 3 * i, d, J);
            sh_basis(d, sh_deg, Y, dY);
            double gd[3] = {0.0, 0.0, 0.0};   /* dP/dd */
            for (int64_t k = 0; k < ns; ++k) {
                if (dsh) dsh[i * ns + k] = dP * Y[k];
                for (int j = 0; j < 3; ++j) gd[j] += sh[i * ns + k] * dY[3 * k + j];
            }
            for (int j = 0; j < 3; ++j)
                for (int a2 = 0; a2 < 3; ++a2) dm[j] += dP * gd[a2] * J[3 * a2 + j];
        } else {
            damp[i] = dP;
        }
        dext[i] = o[6];
        if (dext_back) dext_back[i] = o[6];
        double dSig[9] = {0};
        plane_to_3d(G[i].QI, o + 3, o + 1, v.ex, v.ez, v.dA, v.dR, dSig, dm);
        plane_to_3d(G[i].QC, o + 9, o + 7, v.ex, v.ey, v.dAc, v.dEc, dSig, dm);
        cov_to_params(&G[i], dSig, dsc, dqu);
    }
    free(g2); free(G); free(A); free(edge); free(peff); free(kap);
    return 0;
}

/* Sampled forward for sizes where the full brute force is too slow.
 * Computes S at `npix` pixels (ids row*W+col) and A for `ng` Gaussians.
 * Exactly the definition restricted to what these outputs depend on:
 * A_i only receives terms from rays where g_i > 0, and every ray used is
 * still brute-forced against all n Gaussians. Candidate rays of a Gaussian
 * are searched inside its exact ellipse bounding box widened by one cell. */
int orc_sparse_forward(int64_t n, const double* means, const double* scales,
                       const double* quats, const double* amp,
                       const double* ext, const double* ext_back, const double* sh,
                       int64_t sh_deg, int64_t cell_area, const double* view,
                       double q_max, double dil, int shadowing, int64_t npix,
                       const int64_t* pix, double* S, int64_t ng,
                       const int64_t* gids, double* Aout)
{
    OView v;
    if (n < 0 || view_init(&v, view) || !(q_max > 0) || sh_deg < 0 || sh_deg > 3) return -1;
    const OExtra ex = {ext_back, sh, sh_deg, cell_area};
    double *peff = NULL, *kap = NULL;
    if (prepare(&v, &ex, n, means, amp, ext, &peff, &kap)) return -2;
    OG* G = project_all(&v, n, means, scales, quats, dil, q_max);
    int64_t nrays = v.Wc * v.Hc;
    char* needA = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    char* ray_on = (char*)calloc((size_t)nrays, 1);
    double* A = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!G || !needA || !ray_on || !A) {
        free(G); free(needA); free(ray_on); free(A); free(peff); free(kap); return -2;
    }
    for (int64_t k = 0; k < ng; ++k) needA[gids[k]] = 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (!G[i].valid) continue;
        for (int64_t k = 0; k < npix; ++k) {
            double px = (double)(pix[k] % v.W) + 0.5, py = (double)(pix[k] / v.W) + 0.5;
            if (quadform(G[i].QI, px - G[i].cI[0], py - G[i].cI[1]) < q_max) {
                needA[i] = 1; break;
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!needA[i] || !G[i].valid) continue;
        const double* b = G[i].bxC;
        int64_t c0 = (int64_t)floor(b[0] - 0.5) - 1, c1 = (int64_t)ceil(b[1] - 0.5) + 1;
        int64_t r0 = (int64_t)floor(b[2] - 0.5) - 1, r1 = (int64_t)ceil(b[3] - 0.5) + 1;
        if (c0 < 0) c0 = 0;
        if (r0 < 0) r0 = 0;
        if (c1 > v.Wc - 1) c1 = v.Wc - 1;
        if (r1 > v.Hc - 1) r1 = v.Hc - 1;
        for (int64_t r = r0; r <= r1; ++r)
            for (int64_t c = c0; c <= c1; ++c) {
                double q = quadform(G[i].QC, (double)c + 0.5 - G[i].cC[0],
                                    (double)r + 0.5 - G[i].cC[1]);
                if (q < q_max) ray_on[r * v.Wc + c] = 1;
            }
    }
    int64_t nsel = 0;
    for (int64_t r = 0; r < nrays; ++r) nsel += ray_on[r];
    int64_t* sel = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nsel > 0 ? nsel : 1));
    nsel = 0;
    for (int64_t r = 0; r < nrays; ++r) if (ray_on[r]) sel[nsel++] = r;
    int nt = nthreads();
    double* At = (double*)calloc((size_t)nt * (size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel
    {
        Hit* list = (Hit*)malloc(sizeof(Hit) * (size_t)(n > 0 ? n : 1));
        double* mine = At + (size_t)thread_id() * (size_t)n;
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nsel; ++s) {
            int64_t r = sel[s];
            int64_t m = ray_list(G, n, r % v.Wc, r / v.Wc, q_max, list);
            double t = 0.0;
            for (int64_t k = 0; k < m; ++k) {
                int64_t i = list[k].idx;
                double x = kap[i] * list[k].g;
                double alpha = 1.0 - exp(-x);
                if (needA[i]) mine[i] += shadowing ? alpha * exp(-t) : alpha;
                t += x;
            }
        }
        free(list);
    }
    for (int64_t i = 0; i < n; ++i)
        for (int th = 0; th < nt; ++th) A[i] += At[(size_t)th * (size_t)n + i];
    free(At);
    for (int64_t k = 0; k < ng; ++k) Aout[k] = A[gids[k]];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < npix; ++k) {
        double px = (double)(pix[k] % v.W) + 0.5, py = (double)(pix[k] / v.W) + 0.5;
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!G[i].valid) continue;
            double q = quadform(G[i].QI, px - G[i].cI[0], py - G[i].cI[1]);
            if (q < q_max) acc += foot(q, q_max) * peff[i] * A[i];
        }
        S[k] = acc;
    }
    free(sel); free(G); free(needA); free(ray_on); free(A); free(peff); free(kap);
    return 0;
}

/* Marks the computation-plane rays on which Gaussian g has a footprint
 * (q < q_max), searched inside its ellipse bounding box widened by one
 * cell. */
static void mark_rays(const OView* v, const OG* g, double q_max, char* on)
{
    if (!g->valid) return;
    const double* b = g->bxC;
    int64_t c0 = (int64_t)floor(b[0] - 0.5) - 1, c1 = (int64_t)ceil(b[1] - 0.5) + 1;
    int64_t r0 = (int64_t)floor(b[2] - 0.5) - 1, r1 = (int64_t)ceil(b[3] - 0.5) + 1;
    if (c0 < 0) c0 = 0;
    if (r0 < 0) r0 = 0;
    if (c1 > v->Wc - 1) c1 = v->Wc - 1;
    if (r1 > v->Hc - 1) r1 = v->Hc - 1;
    for (int64_t r = r0; r <= r1; ++r)
        for (int64_t c = c0; c <= c1; ++c)
            if (quadform(g->QC, (double)c + 0.5 - g->cC[0], (double)r + 0.5 - g->cC[1]) < q_max)
                on[r * v->Wc + c] = 1;
}

/* w = sum_p V[p] f(q(p)) over the imaging plane, the pixels searched inside
 * the footprint's bounding box widened by one pixel. */
static double weighted_footprint(const OView* v, const OG* g, const double* V, double q_max)
{
    if (!g->valid) return 0.0;
    const double* b = g->bxI;
    int64_t c0 = (int64_t)floor(b[0] - 0.5) - 1, c1 = (int64_t)ceil(b[1] - 0.5) + 1;
    int64_t r0 = (int64_t)floor(b[2] - 0.5) - 1, r1 = (int64_t)ceil(b[3] - 0.5) + 1;
    if (c0 < 0) c0 = 0;
    if (r0 < 0) r0 = 0;
    if (c1 > v->W - 1) c1 = v->W - 1;
    if (r1 > v->H - 1) r1 = v->H - 1;
    double w = 0.0;
    for (int64_t r = r0; r <= r1; ++r)
        for (int64_t c = c0; c <= c1; ++c) {
            double q = quadform(g->QI, (double)c + 0.5 - g->cI[0], (double)r + 0.5 - g->cI[1]);
            if (q < q_max) w += V[r * v->W + c] * foot(q, q_max);
        }
    return w;
}

/* Central difference of the linear loss L = sum_p V[p] S[p] of one view when
 * parameter `comp` of Gaussian k moves by +h and by -h.
 *   comp: 0-2 mean, 3-5 scale, 6-9 quaternion (raw), 10 amplitude P,
 *         11 extinction ext, 12 backward extinction ext_back (when given),
 *         13 + k SH coefficient k (when sh is given).
 *   out[0] = L(+h) - L(-h)
 *   out[1] = 1 if, on a ray where Gaussian k has a footprint in both states,
 *            the number of Gaussians in front of it differs between the
 *            states (its depth key crossed another's: the loss jumps, and
 *            the difference is no derivative), else 0.
 * Exact, and cheap at full image sizes, because only what the perturbation
 * changes is recomputed. Every ray on which Gaussian k has no footprint in
 * either state composites identically in both states; the rays on which it
 * has one are brute-forced against all n Gaussians in both states, giving
 * the change dA_i of every share. Writing w_i = sum_p V[p] f_i(p) for the
 * imaging footprint of Gaussian i (unchanged for i != k),
 *   L(+) - L(-) = sum_{i != k} P_i w_i dA_i
 *               + P_k(+) A_k(+) w_k(+) - P_k(-) A_k(-) w_k(-),
 * where all of A_k's terms lie on those rays. */
int orc_fd_linear(int64_t n, const double* means, const double* scales,
                  const double* quats, const double* amp, const double* ext,
                  const double* ext_back, const double* sh, int64_t sh_deg,
                  int64_t cell_area, const double* view, double q_max, double dil,
                  int shadowing, const double* V, int64_t k, int comp, double h, double* out)
{
    OView v;
    const int64_t ns = (sh_deg + 1) * (sh_deg + 1);
    if (n <= 0 || k < 0 || k >= n || comp < 0 || sh_deg < 0 || sh_deg > 3 ||
        comp > (sh ? 12 + (int)ns : 12) || (comp == 12 && !ext_back) ||
        view_init(&v, view) || !(q_max > 0) || !(h > 0))
        return -1;
    const OExtra ex = {ext_back, sh, sh_deg, cell_area};
    double *peff = NULL, *kap = NULL;
    if (prepare(&v, &ex, n, means, amp, ext, &peff, &kap)) return -2;
    OG* G = project_all(&v, n, means, scales, quats, dil, q_max);
    int64_t nrays = v.Wc * v.Hc;
    char* on = (char*)calloc((size_t)nrays, 1);
    double* dA = (double*)calloc((size_t)n, sizeof(double));
    if (!G || !on || !dA) {
        free(G); free(on); free(dA); free(peff); free(kap); return -2;
    }
    /* Gaussian k in the two states */
    OG gs[2];
    double Pk[2], Kk[2];
    for (int st = 0; st < 2; ++st) {
        /* Gaussian k's parameters in this state: mean, scale, quaternion,
         * amp, ext, ext_back, SH coefficients */
        double p[13 + 16];
        for (int j = 0; j < 3; ++j) { p[j] = means[3 * k + j]; p[3 + j] = scales[3 * k + j]; }
        for (int j = 0; j < 4; ++j) p[6 + j] = quats[4 * k + j];
        p[10] = amp ? amp[k] : 0.0;
        p[11] = ext[k];
        p[12] = ext_back ? ext_back[k] : 0.0;
        for (int64_t j = 0; j < ns; ++j) p[13 + j] = sh ? sh[k * ns + j] : 0.0;
        p[comp] += st == 0 ? h : -h;
        project(&v, p, p + 3, p + 6, dil, q_max, &gs[st]);
        /* phase of Gaussian k alone, from its own perturbed values */
        const OExtra exk = {NULL, sh ? p + 13 : NULL, sh_deg, cell_area};
        Pk[st] = phase_of(&v, &exk, p + 10, p, 0);
        Kk[st] = p[11] + p[12];
        mark_rays(&v, &gs[st], q_max, on);
    }
    int64_t nsel = 0;
    for (int64_t r = 0; r < nrays; ++r) nsel += on[r];
    int64_t* sel = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nsel > 0 ? nsel : 1));
    /* per ray and state: entries in front of k (-1: k not on the ray) */
    int64_t* front = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(nsel > 0 ? nsel : 1));
    nsel = 0;
    for (int64_t r = 0; r < nrays; ++r) if (on[r]) sel[nsel++] = r;
    int nt = nthreads();
    double* At = (double*)calloc((size_t)nt * (size_t)n, sizeof(double));
    double Ak[2] = {0.0, 0.0};
    const OG base = G[k];
    for (int st = 0; st < 2 && At && sel && front; ++st) {
        G[k] = gs[st];
        const double sign = st == 0 ? 1.0 : -1.0;
        double akst = 0.0;
#pragma omp parallel reduction(+ : akst)
        {
            Hit* list = (Hit*)malloc(sizeof(Hit) * (size_t)n);
            double* mine = At + (size_t)thread_id() * (size_t)n;
#pragma omp for schedule(dynamic, 1)
            for (int64_t s = 0; s < nsel; ++s) {
                int64_t r = sel[s];
                int64_t m = ray_list(G, n, r % v.Wc, r / v.Wc, q_max, list);
                double t = 0.0;
                front[2 * s + st] = -1;
                for (int64_t j = 0; j < m; ++j) {
                    int64_t i = list[j].idx;
                    double kp = i == k ? Kk[st] : kap[i];
                    double x = kp * list[j].g;
                    double a = (1.0 - exp(-x)) * (shadowing ? exp(-t) : 1.0);
                    if (i == k) {
                        akst += a;
                        front[2 * s + st] = j;
                    } else {
                        mine[i] += sign * a;
                    }
                    t += x;
                }
            }
            free(list);
        }
        Ak[st] = akst;
    }
    G[k] = base;
    int flag = 0;
    for (int64_t s = 0; s < nsel && front; ++s)
        if (front[2 * s] >= 0 && front[2 * s + 1] >= 0 && front[2 * s] != front[2 * s + 1])
            flag = 1;
    double diff = 0.0;
    if (At) {
        for (int64_t i = 0; i < n; ++i)
            for (int th = 0; th < nt; ++th) dA[i] += At[(size_t)th * (size_t)n + i];
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : diff)
        for (int64_t i = 0; i < n; ++i) {
            /* zero for every Gaussian the change does not reach, and for
             * those in front of k (identical terms in both states) */
            if (i == k || dA[i] == 0.0) continue;
            diff += peff[i] * weighted_footprint(&v, &G[i], V, q_max) * dA[i];
        }
        diff += Pk[0] * Ak[0] * weighted_footprint(&v, &gs[0], V, q_max) -
                Pk[1] * Ak[1] * weighted_footprint(&v, &gs[1], V, q_max);
    }
    int err = (At && sel && front) ? 0 : -2;
    out[0] = diff;
    out[1] = (double)flag;
    free(At); free(sel); free(front); free(G); free(on); free(dA); free(peff); free(kap);
    return err;
}

/* The real spherical-harmonics basis of degree <= deg at m unit vectors
 * dirs[3m]: Y[m, (deg + 1)^2] (exported for the tests that check it). */
int orc_sh_basis(int64_t m, const double* dirs, int64_t deg, double* Y)
{
    if (m < 0 || deg < 0 || deg > 3) return -1;
    const int64_t ns = (deg + 1) * (deg + 1);
    for (int64_t j = 0; j < m; ++j) sh_basis(dirs + 3 * j, deg, Y + ns * j, NULL);
    return 0;
}
