// C ABI of the SDGR library: argument validation, workspace layout and the
// launch sequence of the forward (paper Sec. II-A) and backward (Sec. II-B)
// passes. Declarations and contracts are in include/sdgr.h.
#include "common.hpp"
#include "sdgr.h"

#include <math.h>

#include <algorithm>
#include <cstring>
#include <unordered_map>
#include <mutex>
#include <cstdio>
#include <string>
#include <vector>

namespace sdgr {
namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    return fail(SDGR_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define SDGR_HIP(expr)                                          \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);       \
    } while (0)

// ---- optional per-stage timing with HIP events on the caller's stream ----
enum Stage {
    SG_QUERY, SG_PREPROCESS, SG_DEPTH_SORT, SG_BIN, SG_PAIR_SORT, SG_RANGES,
    SG_RASTER_A_FWD, SG_INTENSITY, SG_RASTER_B_FWD, SG_RASTER_B_BWD,
    SG_RASTER_A_BWD, SG_PARAMS_BWD, SG_BIN_I, SG_PAIR_SORT_I, SG_COUNT
};
const char* const kStageNames[SG_COUNT] = {
    "plan_query", "preprocess", "depth_sort", "bin_pairs", "pair_sort", "tile_ranges",
    "raster_a_fwd", "set_intensity", "raster_b_fwd", "raster_b_bwd",
    "raster_a_bwd", "params_bwd", "bin_pairs_i", "pair_sort_i"};

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    double ms[SG_COUNT] = {};
    int64_t calls[SG_COUNT] = {};
};
Profiler g_prof;
bool g_count_work = false;   // fill the work counters of the next calls

hipEvent_t take_event()
{
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around one stage when timing is enabled.
class StageTimer {
public:
    StageTimer(int stage, hipStream_t s) : stage_(stage), s_(s)
    {
        std::lock_guard<std::mutex> g(g_prof.mu);
        if (!g_prof.on) return;
        a_ = take_event();
        b_ = take_event();
        if (a_ && b_) (void)hipEventRecord(a_, s_);
    }
    ~StageTimer()
    {
        if (!a_ || !b_) return;
        std::lock_guard<std::mutex> g(g_prof.mu);
        (void)hipEventRecord(b_, s_);
        g_prof.pending.push_back({stage_, a_, b_});
    }

private:
    int stage_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

int bits_for(int64_t max_value)
{
    int b = 0;
    while (b < 63 && (int64_t(1) << b) <= max_value) ++b;
    return b;
}

// Everything the host knows about a call before touching the device.
struct Problem {
    std::vector<DevView> views;
    std::vector<DevScene> scenes;
    RasterParams rp{};
    int nv = 0, ns = 0;
    int64_t records = 0, rays = 0, tiles_c = 0, tiles_i = 0, items = 0, pixels = 0;
    int64_t image_floats = 0;
    bool recompute = false;
    bool det = false;       // ordered sums instead of float atomics
    int shc = 0;            // most SH coefficients of any scene (0: none has sh)
    bool ikey_vm = false;   // imaging keys (tile within the view << 8) | view
    bool seg = false;       // depth and pair sorts segmented by view
    int cbits = 0;          // bits of the computation-plane tile within a view
    int ikey_bits = 0;      // bits of the tile within a view
    int64_t hit_units = 0;  // 16-byte units of the stored-hit stream (0: none)
};

// The stored-hit stream of a plan (RasterParams::hits): only where the
// forward's lists survive to the backward (not in recompute mode) and the
// sums are unordered (not in deterministic mode, whose results must not
// depend on which tiles found room). The default holds 8 bytes per
// computation-plane pair plus 16 MiB (a used hit takes 8 bytes, and rays
// stop long before using every pair in their tile); a tile that finds the
// stream full has its backward re-derive the hits from the footprint masks.
int64_t hit_units_for(const Problem& P, int64_t pairs_c, int64_t hit_bytes)
{
    if (P.det || P.recompute) return 0;
    const int64_t bytes = hit_bytes < 0 ? 8 * pairs_c + (int64_t(16) << 20) : hit_bytes;
    return std::min<int64_t>(bytes / 16, int64_t(UINT32_MAX) - 64);
}

// Rows of the world-to-radar rotation R_r(phi, theta) (Sec. II-A).
void radar_axes(double phi, double theta, double* ex, double* ey, double* ez)
{
#pragma clang fp contract(off)
    double sp = sin(phi), cp = cos(phi), st = sin(theta), ct = cos(theta);
    ex[0] = -sp;      ex[1] = -cp;     ex[2] = 0.0;
    ey[0] = -st * cp; ey[1] = st * sp; ey[2] = ct;
    ez[0] = -ct * cp; ez[1] = ct * sp; ez[2] = -st;
}

int build_problem(const sdgr_scene* scenes, int32_t nscenes, const sdgr_view* views,
                  int32_t nv, const sdgr_options* opt, Problem& P)
{
    if (!opt) return fail(SDGR_EINVAL, "options is null");
    if (nv <= 0 || !views) return fail(SDGR_EINVAL, "need at least one view");
    if (nscenes <= 0 || !scenes) return fail(SDGR_EINVAL, "need at least one scene");
    if (opt->reserved != 0) return fail(SDGR_EINVAL, "options.reserved must be 0");
    if (!(opt->q_max > 0.0f) || !std::isfinite(opt->q_max))
        return fail(SDGR_EINVAL, "q_max must be positive and finite");
    if (!(opt->dilation >= 0.0f) || !std::isfinite(opt->dilation))
        return fail(SDGR_EINVAL, "dilation must be >= 0");
    if (opt->shadowing != 0 && opt->shadowing != 1)
        return fail(SDGR_EINVAL, "shadowing must be 0 or 1");
    if (opt->recompute != 0 && opt->recompute != 1)
        return fail(SDGR_EINVAL, "recompute must be 0 or 1");
    if (opt->deterministic != 0 && opt->deterministic != 1)
        return fail(SDGR_EINVAL, "deterministic must be 0 or 1");
    if (opt->tile != 0 && opt->tile != TILE)
        return fail(SDGR_EUNSUPPORTED, "tile side must be 0 or 8 (the one size built)");
    if (opt->cell_area != 0 && opt->cell_area != 1)
        return fail(SDGR_EINVAL, "cell_area must be 0 or 1");
    P.nv = nv;
    P.ns = nscenes;
    P.recompute = opt->recompute != 0;
    P.det = opt->deterministic != 0;
    double eps = exp(-0.5 * (double)opt->q_max);
    P.rp.q_max = opt->q_max;
    P.rp.eps = (float)eps;
    P.rp.inv1meps = (float)(1.0 / (1.0 - eps));
    P.rp.tau_max = (opt->tau_max > 0.0f) ? opt->tau_max : INFINITY;
    P.rp.shadowing = opt->shadowing;
    P.rp.dilation = opt->dilation;
    P.rp.work = nullptr;   // set only while work counting is on

    P.scenes.resize(nscenes);
    int64_t items = 0;
    for (int s = 0; s < nscenes; ++s) {
        const sdgr_scene& S = scenes[s];
        if (S.n < 0) return fail(SDGR_EINVAL, "scene " + std::to_string(s) + ": n < 0");
        const std::string tag = "scene " + std::to_string(s) + ": ";
        if (S.sh && (S.sh_degree < 0 || S.sh_degree > 3))
            return fail(SDGR_EUNSUPPORTED, tag + "sh_degree outside 0..3");
        const int shc = S.sh ? (S.sh_degree + 1) * (S.sh_degree + 1) : 0;
        if (S.sh && S.sh_stride != 0 && S.sh_stride < shc)
            return fail(SDGR_EINVAL, tag + "sh_stride below the coefficient count");
        if (S.n > 0 && (!S.means || !S.scales || !S.quats || !S.ext || (!S.amp && !S.sh)))
            return fail(SDGR_EINVAL, tag + "null parameter array");
        DevScene d{};
        d.means = S.means; d.scales = S.scales; d.quats = S.quats; d.amp = S.amp; d.ext = S.ext;
        d.ext_back = S.ext_back;
        d.sh = S.sh;
        d.shc = shc;
        d.sh_stride = S.sh ? (S.sh_stride > 0 ? S.sh_stride : shc) : 0;
        P.shc = std::max(P.shc, (int)d.shc);
        d.n = S.n;
        d.item_off = items;
        items += S.n;
        P.scenes[s] = d;
    }
    P.items = items;

    P.views.resize(nv);
    int64_t rec = 0, rays = 0, tc = 0, ti = 0, img = 0, pix = 0;
    for (int v = 0; v < nv; ++v) {
        const sdgr_view& in = views[v];
        std::string tag = "view " + std::to_string(v) + ": ";
        if (in.reserved != 0) return fail(SDGR_EINVAL, tag + "reserved must be 0");
        if (!(in.grazing > 0.0 && in.grazing < M_PI / 2))
            return fail(SDGR_EINVAL, tag + "grazing angle outside (0, pi/2)");
        if (!std::isfinite(in.azimuth)) return fail(SDGR_EINVAL, tag + "azimuth not finite");
        if (in.img_w <= 0 || in.img_h <= 0 || in.comp_w < 0 || in.comp_h < 0)
            return fail(SDGR_EINVAL, tag + "non-positive image size");
        if (!(in.d_az > 0.0) || !(in.d_rg > 0.0) || !(in.comp_d_az >= 0.0) ||
            !(in.comp_d_el >= 0.0) || !std::isfinite(in.d_az) || !std::isfinite(in.d_rg))
            return fail(SDGR_EINVAL, tag + "non-positive spacing");
        if (in.scene < 0 || in.scene >= nscenes)
            return fail(SDGR_EINVAL, tag + "scene index out of range");
        if (in.img_offset < 0) return fail(SDGR_EINVAL, tag + "negative image offset");
        if (!(in.radar_range >= 0.0) || !std::isfinite(in.radar_range))
            return fail(SDGR_EINVAL, tag + "radar_range must be finite and >= 0");
        DevView d{};
        radar_axes(in.azimuth, in.grazing, d.ex, d.ey, d.ez);
        d.W = in.img_w; d.H = in.img_h;
        d.Wc = in.comp_w > 0 ? in.comp_w : in.img_w;
        d.Hc = in.comp_h > 0 ? in.comp_h : in.img_h;
        d.dA = in.d_az; d.dR = in.d_rg;
        d.dAc = in.comp_d_az > 0.0 ? in.comp_d_az : in.d_az;
        d.dEc = in.comp_d_el > 0.0 ? in.comp_d_el : in.d_rg * tan(in.grazing);
        d.range = in.radar_range;
        d.pscale = opt->cell_area ? d.dAc * d.dEc : 1.0;
        d.iA = 1.0 / d.dA; d.iR = 1.0 / d.dR; d.iAc = 1.0 / d.dAc; d.iEc = 1.0 / d.dEc;
        d.hW = 0.5 * (double)d.W; d.hH = 0.5 * (double)d.H;
        d.hWc = 0.5 * (double)d.Wc; d.hHc = 0.5 * (double)d.Hc;
        d.txc = (d.Wc + TILE - 1) / TILE; d.tyc = (d.Hc + TILE - 1) / TILE;
        d.txi = (d.W + TILE - 1) / TILE;  d.tyi = (d.H + TILE - 1) / TILE;
        if (d.txc >= 65535 || d.tyc >= 65535 || d.txi >= 65535 || d.tyi >= 65535)
            return fail(SDGR_EUNSUPPORTED, tag + "image too large");
        d.scene = in.scene;
        d.n = (int32_t)P.scenes[in.scene].n;
        d.rec_off = rec;
        d.ray_off = rays;
        d.img_off = in.img_offset;
        d.pix_off = pix;
        pix += (int64_t)d.W * d.H;
        d.tile_c = (int32_t)tc;
        rec += P.scenes[in.scene].n;
        rays += (int64_t)d.Wc * d.Hc;
        tc += (int64_t)d.txc * d.tyc;
        ti += (int64_t)d.txi * d.tyi;
        img = std::max<int64_t>(img, in.img_offset + (int64_t)d.W * d.H);
        P.views[v] = d;
    }
    // imaging-plane bucket ids follow all computation-plane ones
    int64_t acc = tc;
    for (int v = 0; v < nv; ++v) {
        P.views[v].tile_i = (int32_t)acc;
        acc += (int64_t)P.views[v].txi * P.views[v].tyi;
    }
    if (rec > INT32_MAX || rays > INT32_MAX || tc + ti > INT32_MAX)
        return fail(SDGR_EUNSUPPORTED, "more than 2^31 - 1 records, rays or tiles");
    P.records = rec;
    P.rays = rays;
    P.tiles_c = tc;
    P.tiles_i = ti;
    int64_t max_ti = 1;
    for (int v = 0; v < nv; ++v)
        max_ti = std::max<int64_t>(max_ti, (int64_t)P.views[v].txi * P.views[v].tyi);
    P.ikey_bits = bits_for(max_ti - 1);
    P.ikey_vm = nv <= IKEY_VIEWS && P.ikey_bits <= 24;
    int64_t max_tc = 1;
    for (int v = 0; v < nv; ++v)
        max_tc = std::max<int64_t>(max_tc, (int64_t)P.views[v].txc * P.views[v].tyc);
    P.cbits = bits_for(max_tc - 1);
    P.seg = nv <= SEG_MAX;
    P.image_floats = img;
    P.pixels = pix;
    return SDGR_OK;
}

// Device buffers of one call, carved out of the caller's workspaces.
struct Bufs {
    uint32_t* status = nullptr;
    DevView* views = nullptr;
    DevScene* scenes = nullptr;
    float* A = nullptr;
    float* tau = nullptr;
    uint32_t* nlast = nullptr;
    // geometry: records, sorted lists and tile ranges
    CRec* crec = nullptr;           // computation-plane records
    float4* iq = nullptr;
    float2* iw = nullptr;
    uint32_t* pval[2] = {nullptr, nullptr};
    uint64_t* pmask = nullptr;      // footprint cells per computation-plane pair
    uint64_t* psum = nullptr;       // OR of the masks of every 64 consecutive pairs
    uint2* ranges = nullptr;
    uint32_t* worklist = nullptr;   // non-empty computation-plane tiles, longest first
    // transient: projection counts and sort buffers
    uint2* rect_c = nullptr;
    uint2* rect_i = nullptr;
    uint32_t* cnt_i = nullptr;
    uint2* rect_c_sorted = nullptr;
    uint32_t* bsum_c = nullptr;     // pair counts per 256 records, then their scan
    uint32_t* bsum_i = nullptr;
    uint32_t* dkey[2] = {nullptr, nullptr};
    uint32_t* dval[2] = {nullptr, nullptr};
    uint32_t* pkey[2] = {nullptr, nullptr};
    uint32_t* hist = nullptr;
    SegTable* segt = nullptr;       // [0] records, [1] computation-plane pairs
    unsigned long long* slots = nullptr;   // spread pair-total accumulators
    // backward accumulators: 13 floats and one list slot per record
    float* grad_c = nullptr;
    float* grad_i = nullptr;
    float* pgrad = nullptr;         // per-view-group parts of the parameter gradients
    float* prec = nullptr;          // phase factor per record (scenes with SH)
    uint32_t* active = nullptr;     // records with A > 0 (backward)
    // the computation-plane pairs' positions before the pair sort (where each
    // (tile, record) partial lands, so that a record's partials are
    // contiguous; deterministic mode and the stored-hit backward), and for
    // deterministic mode only the records in depth order and the first pair
    // of each, the partials of A and of the six plane-C gradient sums, and
    // the imaging-plane tile ranges
    uint32_t* ppos[2] = {nullptr, nullptr};
    uint32_t* dord = nullptr;
    uint32_t* poff = nullptr;
    float* part_a = nullptr;
    float* part_g = nullptr;
    uint2* ranges_i = nullptr;
    // stored hits of pass A's forward for its backward (RasterParams::hits)
    uint4* hits = nullptr;
    uint32_t* hit_tail = nullptr;   // per computation-plane tile
    float* hit_part = nullptr;      // backward: per-pair partials, see RasterParams::hit_part
    unsigned char* hit_touched = nullptr;
};

struct Arena {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(int64_t count)
    {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (size_t)std::max<int64_t>(count, 1);
        return p;
    }
};

enum Phase { FWD, BWD };
constexpr int STATUS_WORDS = 64 + 66;   // status words, then the worklist bins
static_assert(WORK_WORD + 2 * WORK_COUNTERS <= 64, "work counters overlap the worklist bins");
constexpr int ST_RECORDS = 12;   // device copy of the record count (sort length)
constexpr int WL_BINS = WL_BINS_WORD;   // 66 words of worklist bins after the status words

void layout(const Problem& P, int64_t cap_c, int64_t cap_i, Phase ph, char* state,
            char* scratch, Bufs& b, size_t* state_bytes, size_t* scratch_bytes)
{
    Arena st{state}, sc{scratch};
    const int64_t R = P.records, K = cap_c + cap_i;
    b.status = st.take<uint32_t>(STATUS_WORDS);
    b.views = st.take<DevView>(P.nv);
    b.scenes = st.take<DevScene>(P.ns);
    b.A = st.take<float>(R);
    b.tau = st.take<float>(P.rays);
    b.nlast = st.take<uint32_t>(P.rays);
    auto geo = [&](Arena& a) {
        b.active = a.take<uint32_t>(R);   // records pass A used
        b.crec = a.take<CRec>(R);
        b.iq = a.take<float4>(R);
        b.iw = a.take<float2>(R);
        b.pval[0] = a.take<uint32_t>(K);
        b.pval[1] = a.take<uint32_t>(K);
        b.pmask = a.take<uint64_t>(cap_c);
        b.psum = a.take<uint64_t>(cap_c / WAVE + 1);
        b.ranges = a.take<uint2>(P.tiles_c);
        b.worklist = a.take<uint32_t>(P.tiles_c);
        if (P.shc > 0) b.prec = a.take<float>(R);
        if (P.det || P.hit_units > 0) {
            b.ppos[0] = a.take<uint32_t>(cap_c);
            b.ppos[1] = a.take<uint32_t>(cap_c);
        }
        if (P.det) {
            b.dord = a.take<uint32_t>(R);
            b.poff = a.take<uint32_t>(R);
        }
        if (P.hit_units > 0) {
            b.hits = a.take<uint4>(P.hit_units + 16);   // slack for the backward's part copies
            b.hit_tail = a.take<uint32_t>(P.tiles_c);
        }
    };
    auto transient = [&](Arena& a) {
        b.rect_c = a.take<uint2>(R);
        b.rect_i = a.take<uint2>(R);
        b.cnt_i = a.take<uint32_t>(R);
        b.rect_c_sorted = a.take<uint2>(R);
        b.segt = a.take<SegTable>(2);
        b.bsum_c = a.take<uint32_t>(R / 256 + 1);
        b.bsum_i = a.take<uint32_t>(R / 256 + 1);
        b.dkey[0] = a.take<uint32_t>(R);
        b.dkey[1] = a.take<uint32_t>(R);
        b.dval[0] = a.take<uint32_t>(R);
        b.dval[1] = a.take<uint32_t>(R);
        b.pkey[0] = a.take<uint32_t>(K);
        b.pkey[1] = a.take<uint32_t>(K);
        int64_t hw = (int64_t)std::max(radix_hist_words(R), radix_hist_words(K));
        b.hist = a.take<uint32_t>(hw);
        b.slots = a.take<unsigned long long>(2 * TOTAL_SLOTS);
        if (P.det) {
            b.part_a = a.take<float>(cap_c);
            b.ranges_i = a.take<uint2>(P.tiles_i);
        }
    };
    if (!P.recompute) geo(st);
    if (ph == FWD) {
        if (P.recompute) geo(sc);
        transient(sc);
    } else {
        if (P.recompute) {
            geo(sc);
            transient(sc);
        }
        b.grad_c = sc.take<float>(GC_STRIDE * R);   // record-major, see launch_params_backward
        b.grad_i = sc.take<float>(GC_STRIDE * R);   // record-major, as grad_c
        b.pgrad = sc.take<float>((int64_t)params_part_floats(P.nv, P.items, P.shc));
        if (P.det) b.part_g = sc.take<float>(6 * cap_c);
        if (P.hit_units > 0) {
            b.hit_part = sc.take<float>(HIT_PART_STRIDE * cap_c);
            b.hit_touched = sc.take<unsigned char>(cap_c + 4);
        }
    }
    if (state_bytes) *state_bytes = st.off;
    if (scratch_bytes) *scratch_bytes = sc.off;
}

// Host copies of the views table the last forward wrote into each state
// workspace. The state must stay untouched between a forward and its
// backward (the backward reads the forward's records and lists there), so a
// backward given the same views finds an identical table on the device and
// skips its upload (each upload launch reads its argument block from host
// memory). A forward always uploads.
struct ViewsCache {
    std::mutex mu;
    std::unordered_map<const void*, std::vector<char>> last;
};
ViewsCache g_views;
constexpr size_t VIEWS_CACHE_STATES = 64;

int upload_tables(const Problem& P, const Bufs& b, hipStream_t s, const void* state, bool forward)
{
    const size_t nb = sizeof(DevView) * (size_t)P.nv;
    const char* bytes = reinterpret_cast<const char*>(P.views.data());
    bool skip = false;
    if (!forward) {
        std::lock_guard<std::mutex> g(g_views.mu);
        auto it = g_views.last.find(state);
        skip = it != g_views.last.end() && it->second.size() == nb &&
               std::memcmp(it->second.data(), bytes, nb) == 0;
    }
    if (!skip) SDGR_HIP(launch_upload(b.views, P.views.data(), nb, s));
    SDGR_HIP(launch_upload(b.scenes, P.scenes.data(), sizeof(DevScene) * P.ns, s));
    if (forward) {
        std::lock_guard<std::mutex> g(g_views.mu);
        if (g_views.last.size() >= VIEWS_CACHE_STATES && !g_views.last.count(state))
            g_views.last.clear();
        g_views.last[state].assign(bytes, bytes + nb);
    }
    return SDGR_OK;
}

int check_plan(Problem& P, const sdgr_plan* plan)
{
    if (!plan) return fail(SDGR_EINVAL, "plan is null");
    if (plan->records != P.records || plan->rays != P.rays || plan->tiles_c != P.tiles_c ||
        plan->tiles_i != P.tiles_i || plan->gaussians != P.items || plan->nviews != P.nv ||
        plan->nscenes != P.ns ||
        plan->tile != TILE || plan->recompute != (P.recompute ? 1 : 0) ||
        plan->deterministic != (P.det ? 1 : 0) || plan->sh_coeffs != P.shc ||
        plan->pairs_c < 0 || plan->pairs_i < 0 || plan->pairs_c + plan->pairs_i > INT32_MAX ||
        plan->hit_bytes < 0)
        return fail(SDGR_EINVAL, "plan does not match the scenes, views and options");
    P.hit_units = hit_units_for(P, plan->pairs_c, plan->hit_bytes);
    // the workspaces the plan promises must hold the layout of its capacities
    Bufs b;
    size_t st = 0, fs = 0, bs = 0;
    layout(P, plan->pairs_c, plan->pairs_i, FWD, nullptr, nullptr, b, &st, &fs);
    layout(P, plan->pairs_c, plan->pairs_i, BWD, nullptr, nullptr, b, nullptr, &bs);
    if (plan->state_bytes < st || plan->fwd_scratch_bytes < fs || plan->bwd_scratch_bytes < bs)
        return fail(SDGR_EWORKSPACE, "plan's workspace sizes are smaller than its capacities need");
    return SDGR_OK;
}

// Up to SEG_MAX views the depth sort and the pair sort are segmented by
// view (each view's records sorted by depth within the view, the pairs by
// the tile within the view); beyond that the depth sort orders all records
// by depth alone, which is enough since the stable bucket sort of the pairs
// groups them by global tile (and so by view) and keeps the depth order
// within each tile. Computation-plane buckets are [0, tiles_c);
// imaging-plane buckets follow.
int bits_pairs_c(const Problem& P) { return P.seg ? P.cbits : bits_for(P.tiles_c - 1); }
int bits_pairs_i(const Problem& P)
{
    return P.ikey_vm ? P.ikey_bits : bits_for(P.tiles_c + P.tiles_i - 1);
}
int final_buffer_c(const Problem& P) { return radix_passes_for(bits_pairs_c(P)) & 1; }
int final_buffer_i(const Problem& P) { return radix_passes_for(bits_pairs_i(P)) & 1; }

// Projection, depth sort and the computation-plane lists: binning, the
// stable bucket sort, tile ranges, footprint masks and the tile worklist
// (shared by the forward and the recomputing backward).
int build_lists_c(const Problem& P, const sdgr_plan* plan, const Bufs& b, bool zero_A,
                  hipStream_t s)
{
    const int64_t R = P.records;
    // list-building words only: the work counters and the imaging-plane pair
    // count of the forward survive a recomputing backward
    SDGR_HIP(launch_fill_u32(b.status, 0u, ST_PAIRS_I, s));
    SDGR_HIP(launch_fill_u32(b.status + ST_PAIRS_I + 1, 0u, WORK_WORD - ST_PAIRS_I - 1, s));
    SDGR_HIP(launch_fill_u32(b.status + ST_RECORDS, (uint32_t)R, 1, s));
    {
        StageTimer t(SG_PREPROCESS, s);
        SDGR_HIP(launch_preprocess(b.views, b.scenes, P.nv, P.ns, P.items, P.rp, true, b.crec, b.iq,
                                   b.iw, b.rect_c, b.rect_i, b.dkey[0],
                                   zero_A ? b.A : nullptr, b.prec, b.slots,
                                   reinterpret_cast<unsigned long long*>(b.status + ST_COUNT),
                                   s));
    }
    // depth order of the records of every view
    uint32_t* dk[2] = {b.dkey[0], b.dkey[1]};
    uint32_t* dv[2] = {b.dval[0], b.dval[1]};
    int which = 0;
    {
        StageTimer t(SG_DEPTH_SORT, s);
        // segmented by view: view-major depth order, so the rectangle gather
        // below reads one view's records at a time (the per-tile lists are
        // the same either way)
        if (P.seg)
            SDGR_HIP(launch_seg_setup(b.views, P.nv, R, b.status + ST_RECORDS, false, &b.segt[0],
                                      s));
        SDGR_HIP(launch_radix_sort_u32(dk, dv, R, b.status + ST_RECORDS, 32, true, b.hist,
                                       &which, s, 0, P.seg ? &b.segt[0] : nullptr, P.nv,
                                       false));
    }
    uint32_t* pk[2] = {b.pkey[0], b.pkey[1]};
    uint32_t* pv[2] = {b.pval[0], b.pval[1]};
    {
        StageTimer t(SG_BIN, s);
        SDGR_HIP(launch_gather_rects(dv[which], b.rect_c, R, b.rect_c_sorted, b.bsum_c, s));
        SDGR_HIP(launch_scan_blocks(b.bsum_c, (R + 255) / 256, plan->pairs_c, b.status, -1, s));
        SDGR_HIP(launch_pair_total_c(plan->pairs_c, b.status, s));
        SDGR_HIP(launch_emit_pairs_c(b.views, P.nv, R, dv[which], b.rect_c_sorted, b.bsum_c,
                                     plan->pairs_c, b.status, pk[0], pv[0],
                                     P.seg ? b.segt[1].seg : nullptr, b.dord, b.poff, s));
    }
    int pw = 0;
    {
        StageTimer t(SG_PAIR_SORT, s);
        if (P.seg)
            SDGR_HIP(launch_seg_setup(b.views, P.nv, R, b.status + ST_PAIRS_C, true, &b.segt[1],
                                      s, PAIR_SORT_BLOCKS));
        uint32_t* pp[2] = {b.ppos[0], b.ppos[1]};
        SDGR_HIP(launch_radix_sort_u32(pk, pv, plan->pairs_c, b.status + ST_PAIRS_C,
                                       bits_pairs_c(P), false, b.hist, &pw, s, 0,
                                       P.seg ? &b.segt[1] : nullptr, P.nv, true,
                                       b.ppos[0] ? pp : nullptr, PAIR_SORT_BLOCKS));
    }
    if (plan->pairs_c > 0 && pw != final_buffer_c(P))
        return fail(SDGR_EHIP, "internal: pair buffer parity");
    StageTimer t(SG_RANGES, s);
    SDGR_HIP(launch_tile_ranges(pk[pw], plan->pairs_c, b.status + ST_PAIRS_C, P.tiles_c,
                                b.ranges, s));
    SDGR_HIP(launch_pair_masks(b.views, P.nv, plan->pairs_c, P.rp, b.status, pk[pw], pv[pw],
                               b.crec, b.pmask, b.psum, s));
    SDGR_HIP(launch_tile_worklist(b.ranges, P.tiles_c, b.worklist, b.status + WL_BINS, b.status, s));
    return SDGR_OK;
}

// Imaging-plane lists, after pass A: only records with nonzero intensity
// emit pairs (counted by the intensity kernel), which a stable bucket sort
// groups by tile behind the computation-plane part of the pair arrays.
int build_lists_i(const Problem& P, const sdgr_plan* plan, const Bufs& b, hipStream_t s)
{
    const int64_t R = P.records;
    uint32_t* pk[2] = {b.pkey[0] + plan->pairs_c, b.pkey[1] + plan->pairs_c};
    uint32_t* pv[2] = {b.pval[0] + plan->pairs_c, b.pval[1] + plan->pairs_c};
    {
        StageTimer t(SG_BIN_I, s);
        SDGR_HIP(launch_scan_blocks(b.bsum_i, (R + 255) / 256, plan->pairs_i, b.status, ST_PAIRS_I,
                                    s));
        SDGR_HIP(launch_emit_pairs_i(b.views, P.nv, R, b.rect_i, b.cnt_i, b.bsum_i, plan->pairs_c,
                                     plan->pairs_i, P.ikey_vm, b.status, b.pkey[0], b.pval[0], s));
    }
    int pw = 0;
    StageTimer t(SG_PAIR_SORT_I, s);
    SDGR_HIP(launch_radix_sort_u32(pk, pv, plan->pairs_i, b.status + ST_PAIRS_I, bits_pairs_i(P),
                                   false, b.hist, &pw, s, P.ikey_vm ? 8 : 0, nullptr, 0, true,
                                   nullptr, PAIR_SORT_BLOCKS));
    if (plan->pairs_i > 0 && pw != final_buffer_i(P))
        return fail(SDGR_EHIP, "internal: pair buffer parity");
    return SDGR_OK;
}


// Pair counts of the projection (count-only preprocess into `query`, which
// holds sdgr_query_bytes(ns, nv)), read back with one stream
// synchronisation, and the workspace sizes they imply.
void fill_plan(const Problem& P, int64_t pairs_c, int64_t pairs_i, sdgr_plan* plan,
               int64_t hit_bytes = -1);

int count_and_plan(const Problem& P, char* query, hipStream_t s, sdgr_plan* plan)
{
    Arena a{query};
    unsigned long long* totals = a.take<unsigned long long>(8);
    unsigned long long* slots = a.take<unsigned long long>(2 * TOTAL_SLOTS);
    DevView* dviews = a.take<DevView>(P.nv);
    DevScene* dscenes = a.take<DevScene>(P.ns);
    SDGR_HIP(launch_upload(dviews, P.views.data(), sizeof(DevView) * P.nv, s));
    SDGR_HIP(launch_upload(dscenes, P.scenes.data(), sizeof(DevScene) * P.ns, s));
    SDGR_HIP(launch_fill_u32((uint32_t*)totals, 0u, 16, s));
    {
        StageTimer t(SG_QUERY, s);
        SDGR_HIP(launch_preprocess(dviews, dscenes, P.nv, P.ns, P.items, P.rp, false, nullptr,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   slots, totals, s));
    }
    unsigned long long host_tot[2] = {0, 0};
    SDGR_HIP(hipMemcpyAsync(host_tot, totals, sizeof(host_tot), hipMemcpyDeviceToHost, s));
    SDGR_HIP(hipStreamSynchronize(s));
    if (host_tot[0] + host_tot[1] > (unsigned long long)INT32_MAX)
        return fail(SDGR_EUNSUPPORTED, "more than 2^31 - 1 (Gaussian, tile) pairs");
    fill_plan(P, (int64_t)host_tot[0], (int64_t)host_tot[1], plan);
    return SDGR_OK;
}

// The plan of a problem at given pair capacities (host data only);
// hit_bytes < 0 takes the default stored-hit stream.
void fill_plan(const Problem& P0, int64_t pairs_c, int64_t pairs_i, sdgr_plan* plan,
               int64_t hit_bytes)
{
    Problem P = P0;
    P.hit_units = hit_units_for(P, pairs_c, hit_bytes);
    sdgr_plan out{};
    out.hit_bytes = P.hit_units * 16;
    out.records = P.records;
    out.pairs_c = pairs_c;
    out.pairs_i = pairs_i;
    out.tiles_c = P.tiles_c;
    out.tiles_i = P.tiles_i;
    out.rays = P.rays;
    out.gaussians = P.items;
    out.nviews = P.nv;
    out.nscenes = P.ns;
    out.tile = TILE;
    out.recompute = P.recompute ? 1 : 0;
    out.deterministic = P.det ? 1 : 0;
    out.sh_coeffs = P.shc;
    out.image_floats = (size_t)P.image_floats;
    Bufs b;
    layout(P, out.pairs_c, out.pairs_i, FWD, nullptr, nullptr, b, &out.state_bytes,
           &out.fwd_scratch_bytes);
    layout(P, out.pairs_c, out.pairs_i, BWD, nullptr, nullptr, b, nullptr,
           &out.bwd_scratch_bytes);
    *plan = out;
}

// ---- workspace for callers that cannot allocate device memory -----------
// One fixed array per device, held until the process ends. Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol): it takes each device's address once with
// hipGetSymbolAddress and uses that.
constexpr size_t STATIC_SCRATCH_BYTES = SDGR_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

struct StaticScratchPtrs {
    std::mutex mu;
    std::vector<char*> ptr;   // per device ordinal, null until first use
};
StaticScratchPtrs g_static;

int static_scratch(char** out)
{
    int dev = -1;
    SDGR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_static.mu);
    if ((int)g_static.ptr.size() <= dev) g_static.ptr.resize((size_t)dev + 1, nullptr);
    if (!g_static.ptr[dev]) {
        void* p = nullptr;
        SDGR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255))
            return fail(SDGR_EHIP, "static scratch has no usable device address");
        g_static.ptr[dev] = static_cast<char*>(p);
    }
    *out = g_static.ptr[dev];
    return SDGR_OK;
}

}  // namespace
}  // namespace sdgr

namespace sdgr {
// error reporting for the library's other translation units
int report_error(int code, const char* msg) { return fail(code, msg); }
void clear_error() { g_last_error.clear(); }
}  // namespace sdgr

using namespace sdgr;

extern "C" {

int sdgr_version(void) { return SDGR_VERSION; }

const char* sdgr_last_error(void) { return g_last_error.c_str(); }

void sdgr_default_options(sdgr_options* opt)
{
    if (!opt) return;
    opt->shadowing = 1;
    opt->recompute = 0;
    opt->q_max = 9.0f;
    opt->tau_max = 16.0f;
    opt->dilation = 0.0f;
    opt->deterministic = 0;
    opt->tile = 0;
    opt->cell_area = 0;
    opt->reserved = 0;
}

size_t sdgr_query_bytes(int32_t nscenes, int32_t nv)
{
    if (nscenes < 0 || nv < 0) return 0;
    return 4096 + 16 * (size_t)TOTAL_SLOTS + 256 +
           ((sizeof(DevView) * (size_t)nv + 255) & ~size_t(255)) +
           ((sizeof(DevScene) * (size_t)nscenes + 255) & ~size_t(255));
}

int sdgr_plan_query(const sdgr_scene* scenes, int32_t nscenes, const sdgr_view* views,
                    int32_t nv, const sdgr_options* opt, void* query_scratch,
                    size_t query_bytes, void* stream, sdgr_plan* plan)
{
    g_last_error.clear();
    if (!plan) return fail(SDGR_EINVAL, "plan is null");
    Problem P;
    int rc = build_problem(scenes, nscenes, views, nv, opt, P);
    if (rc) return rc;
    if (!query_scratch || query_bytes < sdgr_query_bytes(nscenes, nv))
        return fail(SDGR_EWORKSPACE, "query scratch smaller than sdgr_query_bytes()");
    if ((uintptr_t)query_scratch & 255) return fail(SDGR_EINVAL, "scratch not 256-byte aligned");
    return count_and_plan(P, (char*)query_scratch, (hipStream_t)stream, plan);
}

int sdgr_plan_host(const sdgr_scene* scenes, int32_t nscenes, const sdgr_view* views,
                   int32_t nv, const sdgr_options* opt, int64_t pairs_c, int64_t pairs_i,
                   sdgr_plan* plan)
{
    g_last_error.clear();
    if (!plan) return fail(SDGR_EINVAL, "plan is null");
    if (pairs_c < 0 || pairs_i < 0 || pairs_c + pairs_i > INT32_MAX)
        return fail(SDGR_EUNSUPPORTED, "pair capacities outside [0, 2^31 - 1]");
    Problem P;
    int rc = build_problem(scenes, nscenes, views, nv, opt, P);
    if (rc) return rc;
    fill_plan(P, pairs_c, pairs_i, plan);
    return SDGR_OK;
}

int sdgr_plan_resize(sdgr_plan* plan, int64_t pairs_c, int64_t pairs_i)
{
    g_last_error.clear();
    if (!plan) return fail(SDGR_EINVAL, "plan is null");
    if (pairs_c < 0 || pairs_i < 0 || pairs_c + pairs_i > INT32_MAX)
        return fail(SDGR_EUNSUPPORTED, "pair capacities outside [0, 2^31 - 1]");
    Problem P;
    P.nv = plan->nviews;
    P.ns = plan->nscenes;
    P.records = plan->records;
    P.rays = plan->rays;
    P.tiles_c = plan->tiles_c;
    P.tiles_i = plan->tiles_i;
    P.items = plan->gaussians;   // sizes the parameter-gradient parts
    P.recompute = plan->recompute != 0;
    P.det = plan->deterministic != 0;
    P.shc = plan->sh_coeffs;
    if (P.shc < 0 || P.shc > 16) return fail(SDGR_EINVAL, "plan's sh_coeffs outside 0..16");
    P.hit_units = hit_units_for(P, pairs_c, -1);
    plan->pairs_c = pairs_c;
    plan->pairs_i = pairs_i;
    plan->hit_bytes = P.hit_units * 16;
    Bufs b;
    layout(P, pairs_c, pairs_i, FWD, nullptr, nullptr, b, &plan->state_bytes,
           &plan->fwd_scratch_bytes);
    layout(P, pairs_c, pairs_i, BWD, nullptr, nullptr, b, nullptr, &plan->bwd_scratch_bytes);
    return SDGR_OK;
}

int sdgr_forward(const sdgr_scene* scenes, int32_t nscenes, const sdgr_view* views, int32_t nv,
                 const sdgr_options* opt, const sdgr_plan* plan, void* state, void* scratch,
                 float* images, void* stream)
{
    g_last_error.clear();
    Problem P;
    int rc = build_problem(scenes, nscenes, views, nv, opt, P);
    if (rc) return rc;
    if ((rc = check_plan(P, plan))) return rc;
    if (!state || !scratch || !images) return fail(SDGR_EINVAL, "null workspace or images");
    if (((uintptr_t)state | (uintptr_t)scratch) & 255)
        return fail(SDGR_EINVAL, "workspaces must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    Bufs b;
    layout(P, plan->pairs_c, plan->pairs_i, FWD, (char*)state, (char*)scratch, b, nullptr,
           nullptr);
    if (g_count_work) P.rp.work = reinterpret_cast<unsigned long long*>(b.status + WORK_WORD);
    if ((rc = upload_tables(P, b, s, state, true))) return rc;
    SDGR_HIP(launch_fill_u32(b.status + ST_PAIRS_I, 0u, 1, s));
    SDGR_HIP(launch_fill_u32(b.status + WORK_WORD, 0u, STATUS_WORDS - WORK_WORD, s));
    // the projection also clears A for pass A's sums
    if ((rc = build_lists_c(P, plan, b, true, s))) return rc;
    const int pw = final_buffer_c(P);
    SDGR_HIP(launch_fill_u32((uint32_t*)b.tau, 0u, P.rays, s));   // rays of empty tiles
    SDGR_HIP(launch_fill_u32(b.nlast, 0u, P.rays, s));
    {
        StageTimer t(SG_RASTER_A_FWD, s);
        RasterParams rp = P.rp;
        if (b.hits) {
            rp.hits = b.hits;
            rp.hit_tail = b.hit_tail;
            rp.hit_top = reinterpret_cast<unsigned long long*>(b.status + ST_HIT_TOP);
            rp.hit_cap = (uint32_t)P.hit_units;
        }
        if (P.det) {
            // one partial per (tile, record) pair, summed per record in list order
            SDGR_HIP(launch_fill_u32((uint32_t*)b.part_a, 0u, plan->pairs_c, s));
            rp.ppos = b.ppos[pw];
            rp.part = b.part_a;
        }
        SDGR_HIP(launch_raster_a_fwd(b.views, P.nv, P.tiles_c, rp, b.status, b.worklist,
                                     b.ranges, b.pval[pw], b.pmask, b.psum, b.crec, b.A,
                                     b.tau, b.nlast, s));
        if (P.det)
            SDGR_HIP(launch_reduce_pairs(b.dord, b.poff, P.records, b.status, b.part_a, 1,
                                         plan->pairs_c, b.A, 0, 1, s));
    }
    {
        StageTimer t(SG_INTENSITY, s);
        SDGR_HIP(launch_set_intensity(b.views, b.scenes, P.nv, P.records, b.A, b.prec, b.iw,
                                      b.rect_i, b.cnt_i, b.bsum_i, b.status, b.active, s));
    }
    if ((rc = build_lists_i(P, plan, b, s))) return rc;
    const int pwi = final_buffer_i(P);
    StageTimer t(SG_RASTER_B_FWD, s);
    if (P.det)
        SDGR_HIP(launch_raster_b_tiles(b.views, P.nv, P.pixels, plan->pairs_c, plan->pairs_i,
                                       P.tiles_c, P.tiles_i, P.rp, b.status, b.pkey[pwi],
                                       b.pval[pwi], b.iq, b.iw, b.ranges_i, images, P.ikey_vm,
                                       s));
    else
        SDGR_HIP(launch_raster_b_fwd(b.views, P.nv, P.pixels, plan->pairs_c, plan->pairs_i, P.rp,
                                     b.status, b.pkey[pwi], b.pval[pwi], b.iq, b.iw, images,
                                     P.ikey_vm, s));
    return SDGR_OK;
}

int sdgr_backward(const sdgr_scene* scenes, int32_t nscenes, const sdgr_view* views,
                  int32_t nv, const sdgr_options* opt, const sdgr_plan* plan, void* state,
                  void* scratch, const float* dL_dimages, const sdgr_scene_grad* grads,
                  void* stream)
{
    g_last_error.clear();
    Problem P;
    int rc = build_problem(scenes, nscenes, views, nv, opt, P);
    if (rc) return rc;
    if ((rc = check_plan(P, plan))) return rc;
    if (!state || !scratch || !dL_dimages || !grads)
        return fail(SDGR_EINVAL, "null workspace, cotangent or gradients");
    if (((uintptr_t)state | (uintptr_t)scratch) & 255)
        return fail(SDGR_EINVAL, "workspaces must be 256-byte aligned");
    for (int sidx = 0; sidx < nscenes; ++sidx) {
        const sdgr_scene_grad& g = grads[sidx];
        const sdgr_scene& S = scenes[sidx];
        if (S.n > 0 && (!g.d_means || !g.d_scales || !g.d_quats || !g.d_ext ||
                        (!g.d_amp && !S.sh) || (!g.d_ext_back && S.ext_back) ||
                        (!g.d_sh && S.sh)))
            return fail(SDGR_EINVAL, "scene " + std::to_string(sidx) + ": null gradient array");
        P.scenes[sidx].d_means = g.d_means;
        P.scenes[sidx].d_scales = g.d_scales;
        P.scenes[sidx].d_quats = g.d_quats;
        P.scenes[sidx].d_amp = g.d_amp;
        P.scenes[sidx].d_ext = g.d_ext;
        P.scenes[sidx].d_ext_back = S.ext_back ? g.d_ext_back : nullptr;
        P.scenes[sidx].d_sh = S.sh ? g.d_sh : nullptr;
    }
    hipStream_t s = (hipStream_t)stream;
    Bufs b;
    layout(P, plan->pairs_c, plan->pairs_i, BWD, (char*)state, (char*)scratch, b, nullptr,
           nullptr);
    if (g_count_work) P.rp.work = reinterpret_cast<unsigned long long*>(b.status + WORK_WORD);
    if ((rc = upload_tables(P, b, s, state, false))) return rc;
    if (P.recompute) {
        // the forward's lists are gone: rebuild them (identical, the sorts
        // are deterministic) and refill the intensities from the kept A
        if ((rc = build_lists_c(P, plan, b, false, s))) return rc;
        SDGR_HIP(launch_set_intensity(b.views, b.scenes, P.nv, P.records, b.A, b.prec, b.iw,
                                      nullptr, nullptr, nullptr, b.status, b.active, s));
    }
    const int pw = final_buffer_c(P);
    {
        StageTimer t(SG_RASTER_B_BWD, s);
        // only the records pass A used (listed by the intensity pass) carry
        // gradients; this pass also clears their computation-plane sums
        SDGR_HIP(launch_image_bwd(b.views, b.scenes, P.nv, P.records, P.rp, b.status, b.active,
                                  b.iq, b.iw, b.prec, dL_dimages, b.grad_i, b.crec, b.grad_c,
                                  s));
    }
    {
        StageTimer t(SG_RASTER_A_BWD, s);
        RasterParams rp = P.rp;
        if (b.hits) {
            rp.hits = b.hits;
            rp.hit_tail = b.hit_tail;
            rp.hit_cap = (uint32_t)P.hit_units;
            rp.hit_ppos = b.ppos[pw];
            rp.hit_part = b.hit_part;
            rp.hit_touched = b.hit_touched;
            SDGR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(b.hit_touched), 0u,
                                     (plan->pairs_c + 3) / 4, s));
        }
        if (P.det) {
            SDGR_HIP(launch_fill_u32((uint32_t*)b.part_g, 0u, 6 * plan->pairs_c, s));
            rp.ppos = b.ppos[pw];
            rp.part = b.part_g;
            rp.part_stride = plan->pairs_c;
        }
        // stored hits first (their sums are stored, not added), then the
        // tiles whose hits are re-derived (atomics)
        SDGR_HIP(launch_raster_a_bwd_hits(b.views, P.nv, P.tiles_c, rp, b.status, b.worklist,
                                          b.crec, b.tau, b.grad_c, P.records, s));
        if (b.hits)
            SDGR_HIP(launch_reduce_touched(plan->pairs_c, P.records, b.status,
                                           b.hit_touched, b.hit_part, b.grad_c, s));
        SDGR_HIP(launch_raster_a_bwd(b.views, P.nv, P.tiles_c, rp, b.status, b.worklist,
                                     b.ranges, b.pval[pw], b.pmask, b.psum, b.crec, b.tau,
                                     b.nlast, b.grad_c, P.records, s));
        if (P.det)
            SDGR_HIP(launch_reduce_pairs(b.dord, b.poff, P.records, b.status, b.part_g, 6,
                                         plan->pairs_c, b.grad_c, 1, GC_STRIDE, s));
    }
    StageTimer t(SG_PARAMS_BWD, s);
    SDGR_HIP(launch_params_backward(b.views, b.scenes, P.nv, P.ns, P.items, P.rp, b.A,
                                    b.grad_c, b.grad_i, P.records, P.shc, b.pgrad, s));
    return SDGR_OK;
}

int sdgr_forward_static(const sdgr_scene* scenes, int32_t nscenes, const sdgr_view* views,
                        int32_t nv, const sdgr_options* opt, float* images, void* stream)
{
    g_last_error.clear();
    Problem P;
    int rc = build_problem(scenes, nscenes, views, nv, opt, P);
    if (rc) return rc;
    if (!images) return fail(SDGR_EINVAL, "images is null");
    char* base = nullptr;
    if ((rc = static_scratch(&base))) return rc;
    const size_t qb = (sdgr_query_bytes(nscenes, nv) + 255) & ~size_t(255);
    if (qb > STATIC_SCRATCH_BYTES)
        return fail(SDGR_EUNSUPPORTED, "too many views or scenes for the static workspace");
    hipStream_t s = (hipStream_t)stream;
    sdgr_plan plan{};
    if ((rc = count_and_plan(P, base, s, &plan))) return rc;
    fill_plan(P, plan.pairs_c, plan.pairs_i, &plan, 0);   // forward only: no stored hits
    const size_t sb = (plan.state_bytes + 255) & ~size_t(255);
    const size_t need = qb + sb + plan.fwd_scratch_bytes;
    if (need > STATIC_SCRATCH_BYTES)
        return fail(SDGR_EUNSUPPORTED,
                    "problem needs " + std::to_string(need) + " bytes of workspace; the static "
                    "workspace holds " + std::to_string(STATIC_SCRATCH_BYTES));
    return sdgr_forward(scenes, nscenes, views, nv, opt, &plan, base + qb, base + qb + sb,
                        images, stream);
}

int sdgr_status(const sdgr_plan* plan, const void* state, void* stream)
{
    g_last_error.clear();
    if (!plan || !state) return fail(SDGR_EINVAL, "null plan or state");
    uint32_t flag = 0;
    hipStream_t s = (hipStream_t)stream;
    SDGR_HIP(hipMemcpyAsync(&flag, state, sizeof(flag), hipMemcpyDeviceToHost, s));
    SDGR_HIP(hipStreamSynchronize(s));
    if (flag) return fail(SDGR_EOVERFLOW, "pair count exceeded the planned capacity");
    return SDGR_OK;
}

int sdgr_status_accumulate(const sdgr_plan* plan, const void* state, uint32_t* flags,
                           void* stream)
{
    g_last_error.clear();
    if (!plan || !state || !flags) return fail(SDGR_EINVAL, "null plan, state or flags");
    SDGR_HIP(launch_or_word(reinterpret_cast<const uint32_t*>(state), flags,
                            (hipStream_t)stream));
    return SDGR_OK;
}

static int read_state_array(const sdgr_plan* plan, const void* state, float* out, int which,
                            void* stream)
{
    g_last_error.clear();
    if (!plan || !state || !out) return fail(SDGR_EINVAL, "null argument");
    Problem P;
    P.nv = plan->nviews;
    P.ns = plan->nscenes;
    P.records = plan->records;
    P.rays = plan->rays;
    P.tiles_c = plan->tiles_c;
    P.tiles_i = plan->tiles_i;
    P.recompute = plan->recompute != 0;
    P.det = plan->deterministic != 0;
    Bufs b;
    layout(P, plan->pairs_c, plan->pairs_i, FWD, (char*)state, nullptr, b, nullptr, nullptr);
    const float* src = which == 0 ? b.A : b.tau;
    int64_t n = which == 0 ? plan->records : plan->rays;
    if (n <= 0) return SDGR_OK;
    SDGR_HIP(hipMemcpyAsync(out, src, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice,
                            (hipStream_t)stream));
    return SDGR_OK;
}

int sdgr_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> g(g_prof.mu);
    g_prof.on = on != 0;
    return SDGR_OK;
}

int sdgr_profile_read(double* ms, int64_t* calls, int32_t n)
{
    g_last_error.clear();
    std::vector<Profiler::Rec> recs;
    {
        std::lock_guard<std::mutex> g(g_prof.mu);
        recs.swap(g_prof.pending);
    }
    for (const auto& r : recs) {
        float t = 0.0f;
        SDGR_HIP(hipEventSynchronize(r.b));
        SDGR_HIP(hipEventElapsedTime(&t, r.a, r.b));
        std::lock_guard<std::mutex> g(g_prof.mu);
        g_prof.ms[r.stage] += t;
        g_prof.calls[r.stage] += 1;
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    std::lock_guard<std::mutex> g(g_prof.mu);
    for (int i = 0; i < SG_COUNT; ++i) {
        if (i < n) {
            if (ms) ms[i] = g_prof.ms[i];
            if (calls) calls[i] = g_prof.calls[i];
        }
        g_prof.ms[i] = 0.0;
        g_prof.calls[i] = 0;
    }
    return SG_COUNT;
}

int sdgr_profile_count(int32_t on)
{
    g_count_work = on != 0;
    return SDGR_OK;
}

int sdgr_read_work(const sdgr_plan* plan, const void* state, uint64_t* out, int32_t n,
                   void* stream)
{
    g_last_error.clear();
    if (!plan || !state || !out || n < 0) return fail(SDGR_EINVAL, "null argument");
    uint64_t w[WORK_COUNTERS] = {0};
    hipStream_t s = (hipStream_t)stream;
    SDGR_HIP(hipMemcpyAsync(w, static_cast<const uint32_t*>(state) + WORK_WORD, sizeof(w),
                            hipMemcpyDeviceToHost, s));
    SDGR_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n && i < WORK_COUNTERS; ++i) out[i] = w[i];
    return SDGR_OK;
}

const char* sdgr_profile_stage(int32_t i)
{
    return (i >= 0 && i < SG_COUNT) ? kStageNames[i] : "";
}

int sdgr_read_intensity(const sdgr_plan* plan, const void* state, float* out, void* stream)
{
    return read_state_array(plan, state, out, 0, stream);
}

int sdgr_read_optical_depth(const sdgr_plan* plan, const void* state, float* out, void* stream)
{
    return read_state_array(plan, state, out, 1, stream);
}

}  // extern "C"
