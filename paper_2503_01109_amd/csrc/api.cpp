// C ABI of the FGS HIP library: context, workspace, argument checks and the enqueueing of the
// forward, backward and mapping-step pipelines. See include/fgs.h for the contract of every call.
#include "fgs.h"
#include "fgs_gicp.h"
#include "fgs_internal.h"
#include "fgs_prior.h"
#include "mlp_internal.h"
#include "seed_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace fgs {
void launch_scale(float *x, int64_t n, const float *s, hipStream_t st);
}  // namespace fgs

using namespace fgs;

namespace {

thread_local std::string g_thread_error;

// Device buffer owned by its holder (freed on destruction; movable, not copyable).
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), bytes(o.bytes)
    {
        o.p = nullptr;
        o.bytes = 0;
    }
    DBuf &operator=(DBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    hipError_t ensure(size_t want)
    {
        if (want <= bytes && p) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            bytes = 0;
            if (e != hipSuccess) return e;
        }
        size_t b = want < 256 ? 256 : want;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as(size_t byte_off = 0) const { return (T *)((char *)p + byte_off); }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch of fgs_render_bwd_noalloc: the 2D gradient records of FGS_NOALLOC_MAX_GAUSSIANS
// gaussians (kG2Stride floats each, 32 MiB), one copy per GPU for the life of the process. Host
// code never passes `scratch` itself to a kernel: that name is a host-side stand-in. Its device
// address is looked up once per device (noalloc_scratch_init, from fgs_ctx_create) and kept in
// g_scratch_dev.
constexpr int64_t kNoallocMax = FGS_NOALLOC_MAX_GAUSSIANS;
static __device__ __align__(256) float scratch[kNoallocMax * kG2Stride];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};

// With device `dev` current: the address of that device's copy of `scratch`.
hipError_t noalloc_scratch_init(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[dev]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = (float *)ptr;
    return hipSuccess;
}

float *noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[dev];
}

}  // namespace

struct fgs_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    // workspace of one forward (sized for the largest n / pair capacity seen)
    DBuf rect, count, dkA, dkB, idA, idB, blocksums, offsets, pkA, pkB, pvA, pvB, hist, grad2d;
    DBuf rect_sorted, start_rank, kpart, csum;
    DBuf shist;  // per projection workgroup and super-tile: covering gaussians (views of <= 256 super-tiles)
    DBuf seg[6];  // sorted chunks (depth keys, ids, super-tile keys, twice) of super-tile lists being merged
    // tile lists from super-tile lists (sized for bin_nsup super-tiles, bin_T tiles, bin_cap pairs)
    DBuf bin_sranges, bin_cstart, bin_csuper, bin_chist, bin_tile_total, bin_words, bin_sstart;
    int64_t bin_nsup = -1, bin_T = -1, bin_cap = -1;
    DBuf words;  // status words (ST_WORDS) + small device scalars
    int64_t ws_n = -1, ws_cap = -1;
    // bumped whenever ensure_ws or ensure_bin may have moved a workspace buffer (a captured window
    // graph that baked in the old addresses is then re-captured)
    uint64_t ws_gen = 0;
    int hist_G = 0;  // radix-sort workgroups the hist buffer holds
    // mapping-step buffers
    DBuf ms_state, ms_dl, ms_grad, ms_partials;
    DBuf ms_img, ms_ssim, ms_reg;  // rendered colour, per-tile SSIM sums, regulariser partials
    DBuf ssim_part, ssim_ws;       // SSIM: fgs_ssim's per-tile sums; the partials' workspace
    DBuf prune_ws;                 // pruning: survivor total (int64), chunk counts and offsets
    // tracking: frame-point row counts; a cloud build's sort keys, values and histograms; the
    // Gauss-Newton state and partial sums
    DBuf fp_rows, cl_sort, cl_hist, cl_box, gicp_state, gicp_part;
    void *gicp_host = nullptr;  // pinned copy of the Gauss-Newton state
    DBuf seed_ws, seed_sc;
    // learned prior: network workspace (rows_cap rows) and per-frame tile buffers for seeding
    DBuf mlp_ws, prior_feat, prior_valid, prior_y;
    int64_t mlp_rows = 0;
    int64_t ms_cap = 0;
    uint32_t *host_words = nullptr;  // pinned copy of the status words
    // host-mapped per-view pair counts of mapping steps: [2v] = pairs, [2v+1] = overflow flag
    uint32_t *ms_host = nullptr, *ms_host_dev = nullptr;
    std::vector<bool> ms_seen;
    std::vector<fgs_camera> ms_cams;  // camera last run at each view index
    int64_t ms_n = -1;                // gaussian count of the last step
    int ms_nv_max = 0;                // most views of any step (host-mapped flags in use)
    // Adam step count of mapping steps on the device, in two slots (a step reads one and writes
    // the other, so its kernel never reads what it writes); ms_dev_step is the count the device
    // will hold once the enqueued steps are done, if none of them overflowed (-1: unknown)
    int ms_slot = 0;
    int64_t ms_dev_step = -1;
    int64_t *step_host = nullptr;     // pinned staging of that count
    // profiling: 0 off, 1 rasterizer kernels only, 2 every stage
    int prof = 0;
    std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof_events;
    std::vector<hipEvent_t> event_pool;  // reused by Stage
    DBuf prof_counts;  // 8 x u64 (see fgs_ctx_profile_work)
    int64_t prof_fwd = 0, prof_bwd = 0;
};

namespace {

// device words inside ctx->words
constexpr int W_STATUS = 0;            // ST_WORDS u32
constexpr int W_NDEV = ST_WORDS;       // n for the depth sort
constexpr int W_NPAIRS = ST_WORDS + 1; // pairs to sort
constexpr int W_DSCALE = ST_WORDS + 2; // float: 1/P_v of the depth term
constexpr int W_NSUP = ST_WORDS + 3;   // super-tile pairs to sort
constexpr int W_KTOTAL = ST_WORDS + 4; // (tile, gaussian) pairs counted by the projection
constexpr int W_STEPOVF = ST_WORDS + 5; // a mapping step's overflow word (any view's pairs did not fit)
constexpr int W_STEP = ST_WORDS + 6;   // two int64 slots (8-byte aligned): the mapping step's Adam count
constexpr int W_TOTAL = ST_WORDS + 16;

fgs_status fail(fgs_ctx *ctx, fgs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_thread_error = buf;
    if (ctx) ctx->err = buf;
    return s;
}

#define HIP_TRY(ctx, call)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return fail((ctx), FGS_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool finite_pos(float v) { return isfinite(v) && v > 0.0f; }

fgs_status check_camera(fgs_ctx *ctx, const fgs_camera *c, const char *what)
{
    if (!c) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: camera is NULL", what);
    if (c->width <= 0 || c->height <= 0 || c->width > 16384 || c->height > 16384)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: image size %dx%d outside [1, 16384]", what, c->width, c->height);
    if (!finite_pos(c->fx) || !finite_pos(c->fy))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: focal lengths must be finite and positive", what);
    if (!isfinite(c->cx) || !isfinite(c->cy) || !isfinite(c->z_near) || c->z_near < 0.0f)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: principal point / z_near not finite (or z_near < 0)", what);
    for (int k = 0; k < 9; ++k)
        if (!isfinite(c->R_cw[k])) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: R_cw not finite", what);
    for (int k = 0; k < 3; ++k)
        if (!isfinite(c->t_cw[k])) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: t_cw not finite", what);
    return FGS_OK;
}

fgs_status check_opts(fgs_ctx *ctx, const fgs_render_opts *o, const char *what, int *tw, int *th)
{
    if (!o) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: render options are NULL", what);
    if (!finite_pos(o->sigma_cut)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: sigma_cut must be > 0", what);
    if (!(o->alpha_max > 0.0f && o->alpha_max < 1.0f))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: alpha_max must be in (0, 1)", what);
    if (!(o->alpha_min >= 0.0f && o->alpha_min <= o->alpha_max))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: alpha_min must be in [0, alpha_max]", what);
    if (!(o->T_min >= 0.0f && o->T_min < 1.0f)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: T_min must be in [0, 1)", what);
    if (!(o->lowpass >= 0.0f) || !isfinite(o->lowpass))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: lowpass must be finite and >= 0", what);
    for (int k = 0; k < 3; ++k)
        if (!isfinite(o->bg[k])) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: background not finite", what);
    if (!isfinite(o->bg_depth)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: background depth not finite", what);
    int a = o->tile_w, b = o->tile_h;
    if (a == 0 && b == 0) a = b = 16;
    if (!tile_supported(a, b)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: unsupported tile %dx%d", what, a, b);
    *tw = a;
    *th = b;
    return FGS_OK;
}

fgs_status check_gauss(fgs_ctx *ctx, const fgs_gaussians *g, const char *what, const char *name)
{
    if (!g) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: %s is NULL", what, name);
    if (g->n < 0 || g->n > (int64_t)1 << 30)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: %s.n = %lld outside [0, 2^30]", what, name, (long long)g->n);
    if (g->stride < g->n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: %s.stride < n", what, name);
    if (g->n > 0 && (!g->mean || !g->log_scale || !g->quat || !g->opacity_logit || !g->rgb))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: %s has a NULL plane", what, name);
    return FGS_OK;
}

int key_bits_for(int64_t T)
{
    int b = 1;
    while (((int64_t)1 << b) < T) ++b;
    return b;
}

CamK to_camk(const fgs_camera &c)
{
    CamK k;
    k.W = c.width;
    k.H = c.height;
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy;
    for (int i = 0; i < 9; ++i) k.R[i] = c.R_cw[i];
    for (int i = 0; i < 3; ++i) k.t[i] = c.t_cw[i];
    k.z_near = c.z_near;
    return k;
}

RasterK to_rk(const fgs_render_opts &o, int tw, int th, int W, int H)
{
    RasterK r;
    r.sigma_cut = o.sigma_cut; r.alpha_min = o.alpha_min; r.alpha_max = o.alpha_max;
    r.T_min = o.T_min; r.lowpass = o.lowpass;
    for (int k = 0; k < 3; ++k) r.bg[k] = o.bg[k];
    r.bg_depth = o.bg_depth;
    r.tile_w = tw; r.tile_h = th;
    r.tiles_x = (W + tw - 1) / tw;
    r.tiles_y = (H + th - 1) / th;
    r.supers_x = supers_for(r.tiles_x);
    return r;
}

ParamsK to_pk(const fgs_gaussians &g)
{
    return ParamsK{g.n, g.stride, g.mean, g.log_scale, g.quat, g.opacity_logit, g.rgb};
}

GradK to_gk(const fgs_gaussians &g)
{
    return GradK{g.n, g.stride, g.mean, g.log_scale, g.quat, g.opacity_logit, g.rgb};
}

fgs_status ensure_ws(fgs_ctx *ctx, int64_t n, int64_t cap)
{
    if (n <= ctx->ws_n && cap <= ctx->ws_cap) return FGS_OK;
    const int64_t nn = n > ctx->ws_n ? n : ctx->ws_n;
    const int64_t cc = cap > ctx->ws_cap ? cap : ctx->ws_cap;
    const size_t N = (size_t)(nn > 0 ? nn : 1), C = (size_t)(cc > 0 ? cc : 1);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->ws_gen++;
    HIP_TRY(ctx, ctx->rect.ensure(N * sizeof(uint2)));
    HIP_TRY(ctx, ctx->count.ensure(N * 4));
    HIP_TRY(ctx, ctx->dkA.ensure(N * 4));
    HIP_TRY(ctx, ctx->dkB.ensure(N * 4));
    HIP_TRY(ctx, ctx->idA.ensure(N * 4));
    HIP_TRY(ctx, ctx->idB.ensure(N * 4));
    HIP_TRY(ctx, ctx->blocksums.ensure(((size_t)scan_blocks_cap(nn) + 2) * 4));
    HIP_TRY(ctx, ctx->offsets.ensure((N + 1) * 4));
    HIP_TRY(ctx, ctx->kpart.ensure((size_t)project_blocks(nn) * 2 * 4));
    HIP_TRY(ctx, ctx->csum.ensure((size_t)project_blocks(nn) * 4));
    HIP_TRY(ctx, ctx->shist.ensure(((size_t)project_blocks(nn) + 1) * 256 * 4));
    HIP_TRY(ctx, ctx->rect_sorted.ensure(N * sizeof(uint2)));
    HIP_TRY(ctx, ctx->start_rank.ensure((size_t)emit_chunks((int64_t)C) * 4));
    HIP_TRY(ctx, ctx->pkA.ensure(C * 4));
    HIP_TRY(ctx, ctx->pkB.ensure(C * 4));
    HIP_TRY(ctx, ctx->pvA.ensure(C * 4));
    HIP_TRY(ctx, ctx->pvB.ensure(C * 4));
    for (DBuf &b : ctx->seg) HIP_TRY(ctx, b.ensure(C * 4));
    const int G = std::max(sort_blocks(nn, kDepthSortPerBlock), sort_blocks(cc > nn ? cc : nn, kPairSortPerBlock));
    HIP_TRY(ctx, ctx->hist.ensure(((size_t)G * 256 + 256) * 4));
    ctx->hist_G = G;
    if (nn > ctx->ws_n) {
        // the backward keeps grad2d all-zero between calls (project_bwd clears what it reads)
        HIP_TRY(ctx, ctx->grad2d.ensure(N * kG2Stride * 4));
        HIP_TRY(ctx, hipMemset(ctx->grad2d.p, 0, N * kG2Stride * 4));
    }
    ctx->ws_n = nn;
    ctx->ws_cap = cc;
    return FGS_OK;
}

// Workspace of the tile-list expansion for nsup super-tiles, T tiles and cap pairs (grown on the
// context's stream after it drained).
fgs_status ensure_bin(fgs_ctx *ctx, int64_t nsup, int64_t T, int64_t cap)
{
    if (nsup <= ctx->bin_nsup && T <= ctx->bin_T && cap <= ctx->bin_cap) return FGS_OK;
    const int64_t ns = std::max(nsup, ctx->bin_nsup), tt = std::max(T, ctx->bin_T), cc = std::max(cap, ctx->bin_cap);
    const int64_t mc = bin_max_chunks(cc, ns);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->ws_gen++;
    HIP_TRY(ctx, ctx->bin_sranges.ensure((size_t)ns * 8));
    HIP_TRY(ctx, ctx->bin_cstart.ensure((size_t)(ns + 1) * 4));
    HIP_TRY(ctx, ctx->bin_sstart.ensure((size_t)(ns + 1 + seg_max_chunks(cc, ns)) * 4));
    HIP_TRY(ctx, ctx->bin_csuper.ensure((size_t)mc * 4));
    HIP_TRY(ctx, ctx->bin_chist.ensure((size_t)mc * kSuper * kSuper * 4));
    HIP_TRY(ctx, ctx->bin_tile_total.ensure((size_t)tt * 4));
    HIP_TRY(ctx, ctx->bin_words.ensure((size_t)(16 + kBinGrid) * 4));
    ctx->bin_nsup = ns;
    ctx->bin_T = tt;
    ctx->bin_cap = cc;
    return FGS_OK;
}

BinWS bin_ws(fgs_ctx *ctx)
{
    BinWS b;
    b.cstart = ctx->bin_cstart.as<uint32_t>();
    b.csuper = ctx->bin_csuper.as<uint32_t>();
    b.chist = ctx->bin_chist.as<uint32_t>();
    b.tile_total = ctx->bin_tile_total.as<uint32_t>();
    b.nchunks = ctx->bin_words.as<uint32_t>();
    b.ok = ctx->bin_words.as<uint32_t>() + 1;
    b.vpart = ctx->bin_words.as<uint32_t>() + 16;
    b.max_chunks = bin_max_chunks(ctx->bin_cap, ctx->bin_nsup);
    return b;
}

// Scratch of one radix sort of up to elems elements; the grid is capped by what the workspace
// holds (a smaller grid only gives each workgroup a larger share).
SortWS sort_ws(fgs_ctx *ctx, int64_t elems, int per_block = kPairSortPerBlock)
{
    SortWS s;
    s.G = std::min(sort_blocks(elems, per_block), ctx->hist_G);
    s.hist = ctx->hist.as<uint32_t>();
    s.totals = ctx->hist.as<uint32_t>() + (size_t)ctx->hist_G * 256;
    return s;
}

struct StatePtrs {
    Rec *rec;
    uint32_t *last, *vals;
    uint2 *ranges;
    float *tfinal;
};

StatePtrs state_ptrs(void *state, const StateLayout &L)
{
    char *b = (char *)state;
    return StatePtrs{(Rec *)(b + L.off_rec), (uint32_t *)(b + L.off_last),
                     (uint32_t *)(b + L.off_vals), (uint2 *)(b + L.off_ranges), (float *)(b + L.off_tfinal)};
}

uint32_t *status_words(fgs_ctx *ctx) { return ctx->words.as<uint32_t>() + W_STATUS; }

// Records a pair of HIP events around the work enqueued during its lifetime (profiling only).
struct Stage {
    fgs_ctx *ctx;
    hipEvent_t a = nullptr, b = nullptr;
    static hipEvent_t take(fgs_ctx *c)
    {
        hipEvent_t e = nullptr;
        if (!c->event_pool.empty()) {
            e = c->event_pool.back();
            c->event_pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    Stage(fgs_ctx *c, const char *name) : ctx(c)
    {
        const bool raster = name[0] == 'r' && name[1] == 'a';  // raster_fwd, raster_bwd
        if (ctx->prof < (raster ? 1 : 2)) return;
        a = take(ctx);
        b = take(ctx);
        if (!a || !b) {
            ctx->prof = 0;
            return;
        }
        (void)hipEventRecord(a, ctx->stream);
        ctx->prof_events[name].push_back({a, b});
    }
    ~Stage()
    {
        if (a && b) (void)hipEventRecord(b, ctx->stream);
    }
};

// Work counters of the forward rasterizer: collected at profiling level 3 only, so the kernels
// timed at levels 1 and 2 are the ones that run unprofiled.
unsigned long long *prof_counts(fgs_ctx *ctx)
{
    return ctx->prof >= 3 ? ctx->prof_counts.as<unsigned long long>() : nullptr;
}

void clear_profile(fgs_ctx *ctx, bool destroy = false)
{
    for (auto &kv : ctx->prof_events)
        for (auto &ab : kv.second) {
            ctx->event_pool.push_back(ab.first);
            ctx->event_pool.push_back(ab.second);
        }
    ctx->prof_events.clear();
    ctx->prof_fwd = 0;
    ctx->prof_bwd = 0;
    if (destroy) {
        for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
        ctx->event_pool.clear();
    }
}

fgs_status read_words(fgs_ctx *ctx);

// Network workspace for at least `rows` rows (grown on the context's stream, after it drained).
fgs_status ensure_mlp(fgs_ctx *ctx, int64_t rows)
{
    if (rows <= ctx->mlp_rows && ctx->mlp_ws.p) return FGS_OK;
    const int64_t r = std::max<int64_t>(rows, std::max<int64_t>(ctx->mlp_rows, 64));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, ctx->mlp_ws.ensure(mlp_ws_bytes(r)));
    ctx->mlp_rows = r;
    return FGS_OK;
}

// Unit quaternion (w, x, y, z) of the camera-to-world rotation R_cw^T, so that a gaussian with
// this rotation has its local axes along the camera's x, y and viewing axes.
void camera_to_world_quat(const float R_cw[9], float q[4])
{
    double m[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m[i][j] = R_cw[j * 3 + i];  // transpose
    const double tr = m[0][0] + m[1][1] + m[2][2];
    double w, x, y, z;
    if (tr > 0) {
        const double s = 2.0 * sqrt(tr + 1.0);
        w = 0.25 * s;
        x = (m[2][1] - m[1][2]) / s;
        y = (m[0][2] - m[2][0]) / s;
        z = (m[1][0] - m[0][1]) / s;
    } else if (m[0][0] > m[1][1] && m[0][0] > m[2][2]) {
        const double s = 2.0 * sqrt(1.0 + m[0][0] - m[1][1] - m[2][2]);
        w = (m[2][1] - m[1][2]) / s;
        x = 0.25 * s;
        y = (m[0][1] + m[1][0]) / s;
        z = (m[0][2] + m[2][0]) / s;
    } else if (m[1][1] > m[2][2]) {
        const double s = 2.0 * sqrt(1.0 + m[1][1] - m[0][0] - m[2][2]);
        w = (m[0][2] - m[2][0]) / s;
        x = (m[0][1] + m[1][0]) / s;
        y = 0.25 * s;
        z = (m[1][2] + m[2][1]) / s;
    } else {
        const double s = 2.0 * sqrt(1.0 + m[2][2] - m[0][0] - m[1][1]);
        w = (m[1][0] - m[0][1]) / s;
        x = (m[0][2] + m[2][0]) / s;
        y = (m[1][2] + m[2][1]) / s;
        z = 0.25 * s;
    }
    const double nrm = sqrt(w * w + x * x + y * y + z * z);
    q[0] = (float)(w / nrm);
    q[1] = (float)(x / nrm);
    q[2] = (float)(y / nrm);
    q[3] = (float)(z / nrm);
}

// Where the projection of a view left its per-gaussian tile rectangles and super-tile counts and
// its per-workgroup pair counts (read by the binning).
struct ProjOut {
    uint2 *rect;
    uint32_t *count, *kpart;
};

// Enqueue the binning of a projected view and, with raster, its forward rasterization: one pair
// per covered super-tile in gaussian order, the pairs sorted by super-tile (stably), every
// super-tile list put in (depth, index) order, then expanded into the tile lists. With K_check,
// the call waits for the pair count after the scan and, when it exceeds the state's capacity,
// returns FGS_ERR_CAPACITY with the count in *K_check before enqueueing the rest.
fgs_status enqueue_bin_raster(fgs_ctx *ctx, const fgs_gaussians &g, const fgs_camera &cam, const fgs_render_opts &o,
                              int tw, int th, const ImageK &img, void *state, const StateLayout &L, const ProjOut &po,
                              int64_t *K_check, uint32_t *host_status, bool raster, const LossK *loss,
                              uint32_t *step_ovf, bool first_of_step)
{
    const RasterK rk = to_rk(o, tw, th, cam.width, cam.height);
    const int supers_x = (rk.tiles_x + kSuper - 1) / kSuper, supers_y = (rk.tiles_y + kSuper - 1) / kSuper;
    const int nsup = supers_x * supers_y;
    fgs_status st;
    if ((st = ensure_bin(ctx, nsup, L.T, L.cap)) != FGS_OK) return st;
    hipStream_t s = ctx->stream;
    const StatePtrs sp = state_ptrs(state, L);
    uint32_t *words = ctx->words.as<uint32_t>();
    uint32_t *npairs = words + W_NPAIRS, *nsup_pairs = words + W_NSUP;
    uint32_t *ktotal = words + W_KTOTAL;
    const BinWS bw = bin_ws(ctx);
    const int sbits = key_bits_for(nsup);
    const bool one_pass = sbits <= 8;
    // up to 256 super-tiles the pairs go straight from the projection's histograms to their lists
    const bool direct = nsup <= 256;
    uint32_t *shist = ctx->shist.as<uint32_t>(), *stot = shist + (size_t)project_blocks(g.n) * 256;
    // the super-tile sort leaves its values in svals and its keys in the other key buffer; the
    // depth order goes into the remaining pair of buffers
    uint32_t *svals = one_pass ? ctx->pvB.as<uint32_t>() : ctx->pvA.as<uint32_t>();
    uint32_t *okeys = one_pass ? ctx->pkA.as<uint32_t>() : ctx->pkB.as<uint32_t>();
    uint32_t *ovals = one_pass ? ctx->pvA.as<uint32_t>() : ctx->pvB.as<uint32_t>();
    if (direct) {
        // the projection's super-tile counts per workgroup, scanned; the pair counts summed
        Stage st_(ctx, "bin");
        launch_super_scan(g.n, shist, stot, po.kpart, status_words(ctx), ktotal, s);
    } else {
        // one pair per covered super-tile, in gaussian order (the projection wrote ids 0..n-1 and
        // the block sums of its counts)
        Stage st_(ctx, "bin");
        launch_emit(ctx->idA.as<uint32_t>(), po.count, po.rect, ctx->blocksums.as<uint32_t>(),
                    ctx->offsets.as<uint32_t>(), g.n, supers_x, kSuperShift, L.cap, ctx->pkA.as<uint32_t>(),
                    ctx->pvA.as<uint32_t>(), ctx->rect_sorted.as<uint2>(), ctx->start_rank.as<uint32_t>(),
                    status_words(ctx), nsup_pairs, nullptr, po.kpart, project_blocks(g.n), ktotal, s, nullptr, 0,
                    ctx->csum.as<uint32_t>());
    }
    if (K_check) {
        // the pair count is known once the scan is complete (the emission of an oversized set
        // stops at the capacity; the caller grows the state and starts over)
        fgs_status st2 = read_words(ctx);
        if (st2 != FGS_OK) return st2;
        *K_check = ctx->host_words[ST_PAIRS];
        if (*K_check > L.cap) return FGS_ERR_CAPACITY;
    }
    uint2 *sranges = ctx->bin_sranges.as<uint2>();
    {
        // super-tile lists (stable: each in gaussian order), their ranges and chunk table
        Stage st_(ctx, "tile_sort");
        uint32_t *sstart = ctx->bin_sstart.as<uint32_t>();
        uint32_t *keys;
        if (direct) {
            keys = ctx->pkB.as<uint32_t>();  // (one_pass: svals is pvB)
            launch_super_scatter(po.rect, po.count, g.n, supers_x, shist, stot, ktotal, L.cap, keys, svals, bw,
                                 sranges, nsup, sstart, seg_max_chunks(L.cap, nsup), s);
        } else {
            const SortWS sws = sort_ws(ctx, L.cap, kSuperSortPerBlock);
            keys = launch_radix_sort(ctx->pkA.as<uint32_t>(), ctx->pvA.as<uint32_t>(), ctx->pkB.as<uint32_t>(),
                                     ctx->pvB.as<uint32_t>(), svals, nsup_pairs, L.cap, sbits, sws, s);
            if (!one_pass) launch_ranges(keys, nsup_pairs, sranges, nsup, kSuperKeyMask, s);
            launch_bin_chunks(bw, sranges, one_pass ? sws.totals : nullptr, nsup, s, sstart,
                              seg_max_chunks(L.cap, nsup));
        }
        uint32_t *const tmp[6] = {ctx->seg[0].as<uint32_t>(), ctx->seg[1].as<uint32_t>(), ctx->seg[2].as<uint32_t>(),
                                  ctx->seg[3].as<uint32_t>(), ctx->seg[4].as<uint32_t>(), ctx->seg[5].as<uint32_t>()};
        launch_seg_sort(keys, svals, okeys, ovals, sranges, sstart, nsup, seg_max_chunks(L.cap, nsup),
                        ctx->dkA.as<uint32_t>(), tmp, s);
    }
    {
        // tile ranges, then the tile lists
        Stage st_(ctx, "tile_bin");
        // (with a mapping loss, also the depth term's 1/P_v)
        const bool dsc = loss && loss->ddepth_scale;
        launch_bin_count(bw, okeys, sranges, s, dsc ? loss->tdepth : nullptr, (int64_t)cam.width * cam.height);
        launch_bin_tiles(bw, nsup, L.cap, ktotal, sp.ranges, status_words(ctx), npairs, host_status, step_ovf,
                         first_of_step, s, dsc ? loss->ddepth_scale : nullptr);
        launch_bin_place(bw, okeys, ovals, sranges, sp.ranges, sp.vals, s);
    }
    if (raster) {
        Stage st_(ctx, "raster_fwd");
        const LossK no_loss{};
        launch_raster_fwd(rk, cam.width, cam.height, sp.rec, sp.vals, sp.ranges, sp.last, sp.tfinal, img,
                          loss ? *loss : no_loss, prof_counts(ctx), s);
        if (prof_counts(ctx)) ctx->prof_fwd++;
    }
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

// Enqueue the forward pipeline of one view into a state with layout L: projection, binning
// (enqueue_bin_raster, with its K_check) and, with raster, the rasterization.
fgs_status enqueue_forward(fgs_ctx *ctx, const fgs_gaussians &g, const fgs_camera &cam, const fgs_render_opts &o,
                           int tw, int th, const ImageK &img, void *state, const StateLayout &L,
                           int64_t *K_check = nullptr, uint32_t *host_status = nullptr, bool raster = true,
                           const LossK *loss = nullptr, uint32_t *step_ovf = nullptr, bool first_of_step = false,
                           float *reg_part = nullptr)
{
    fgs_status st = ensure_ws(ctx, g.n, L.cap);
    if (st != FGS_OK) return st;
    const RasterK rk = to_rk(o, tw, th, cam.width, cam.height);
    hipStream_t s = ctx->stream;
    const StatePtrs sp = state_ptrs(state, L);
    uint32_t *ndev = ctx->words.as<uint32_t>() + W_NDEV;
    const ProjOut po{ctx->rect.as<uint2>(), ctx->count.as<uint32_t>(), ctx->kpart.as<uint32_t>()};
    {
        Stage st_(ctx, "project");
        const int supers_x = (rk.tiles_x + kSuper - 1) / kSuper, supers_y = (rk.tiles_y + kSuper - 1) / kSuper;
        const bool direct = supers_x * supers_y <= 256;  // (as enqueue_bin_raster decides)
        launch_project(to_pk(g), to_camk(cam), rk, sp.rec, po.rect, po.count, ctx->dkA.as<uint32_t>(),
                       ctx->idA.as<uint32_t>(), ndev, kSuperShift, po.kpart, s, 0, reg_part, ctx->csum.as<uint32_t>(),
                       direct ? ctx->shist.as<uint32_t>() : nullptr, supers_x);
    }
    return enqueue_bin_raster(ctx, g, cam, o, tw, th, img, state, L, po, K_check, host_status, raster, loss, step_ovf,
                              first_of_step);
}


// Enqueue the backward of one view: grad_out (nullable) = grad_in (nullable) + this view's
// gradient; adam (nullable) applies that sum to g; lf (nullable) is the view's loss reduction,
// done by the projection backward.
fgs_status enqueue_backward(fgs_ctx *ctx, const fgs_gaussians &g, const fgs_camera &cam, const fgs_render_opts &o,
                            int tw, int th, const void *state, const StateLayout &L, const float *drgb,
                            const float *ddepth, const float *dalpha, const float *dscale, const fgs_gaussians *grad_in,
                            const fgs_gaussians *grad_out, const AdamK *adam, const LossFinalK *lf = nullptr)
{
    fgs_status st = ensure_ws(ctx, g.n, 0);
    if (st != FGS_OK) return st;
    hipStream_t s = ctx->stream;
    const CamK ck = to_camk(cam);
    const RasterK rk = to_rk(o, tw, th, cam.width, cam.height);
    const StatePtrs sp = state_ptrs((void *)state, L);
    float *g2 = ctx->grad2d.as<float>();
    {
        Stage st_(ctx, "raster_bwd");
        launch_raster_bwd(rk, cam.width, cam.height, sp.rec, sp.vals, sp.ranges, sp.last, sp.tfinal, drgb,
                          ddepth, dalpha, dscale, g2, prof_counts(ctx), s);
        if (prof_counts(ctx)) ctx->prof_bwd++;
    }
    {
        Stage st_(ctx, "project_bwd");
        const GradK none{g.n, g.n, nullptr, nullptr, nullptr, nullptr, nullptr};
        AdamK no_adam{};
        launch_project_bwd(to_pk(g), ck, rk, g2, grad_in ? to_gk(*grad_in) : none, grad_out ? to_gk(*grad_out) : none,
                           adam ? *adam : no_adam, s, lf ? *lf : LossFinalK{});
    }
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

}  // namespace

namespace fgs {

bool state_layout(int64_t n, int32_t W, int32_t H, int32_t tw, int32_t th, int64_t max_pairs, StateLayout *L)
{
    if (n < 0 || W <= 0 || H <= 0 || tw <= 0 || th <= 0 || max_pairs < 0) return false;
    StateLayout l;
    l.n = n; l.W = W; l.H = H; l.tw = tw; l.th = th;
    l.tiles_x = (W + tw - 1) / tw;
    l.tiles_y = (H + th - 1) / th;
    l.T = tile_items(l.tiles_x, l.tiles_y);
    l.P = (int64_t)W * H;
    size_t o = 0;
    l.off_rec = o; o = align256(o + (size_t)n * sizeof(Rec));
    l.off_ranges = o; o = align256(o + (size_t)l.T * 8);
    l.off_last = o; o = align256(o + (size_t)l.P * 4);
    l.off_tfinal = o; o = align256(o + (size_t)l.P * 4);
    l.fixed = o;
    l.off_vals = o;
    l.cap = max_pairs;
    l.bytes = o + (size_t)max_pairs * 4;
    *L = l;
    return true;
}

int64_t state_capacity(int64_t n, int32_t W, int32_t H, int32_t tw, int32_t th, int64_t bytes, StateLayout *L)
{
    if (!state_layout(n, W, H, tw, th, 0, L)) return -1;
    if (bytes < (int64_t)L->fixed) return -1;
    L->cap = (bytes - (int64_t)L->fixed) / 4;
    if (L->cap > 0xFFFFFFF0ll) L->cap = 0xFFFFFFF0ll;  // pair indices are 32-bit
    L->bytes = L->fixed + (size_t)L->cap * 4;
    return L->cap;
}

}  // namespace fgs

extern "C" {

const char *fgs_status_str(fgs_status s)
{
    switch (s) {
    case FGS_OK: return "ok";
    case FGS_ERR_INVALID_ARG: return "invalid argument";
    case FGS_ERR_CAPACITY: return "capacity exceeded";
    case FGS_ERR_HIP: return "HIP runtime error";
    case FGS_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

fgs_status fgs_last_error(fgs_ctx *ctx, char *buf, size_t len)
{
    if (!buf || len == 0) return FGS_ERR_INVALID_ARG;
    const std::string &e = ctx ? ctx->err : g_thread_error;
    snprintf(buf, len, "%s", e.c_str());
    return FGS_OK;
}

fgs_status fgs_ctx_create(fgs_ctx **out, void *hip_stream)
{
    if (!out) return fail(nullptr, FGS_ERR_INVALID_ARG, "fgs_ctx_create: out is NULL");
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, FGS_ERR_UNSUPPORTED, "fgs_ctx_create: no HIP device (%s)", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(nullptr, FGS_ERR_HIP, "fgs_ctx_create: %s", hipGetErrorString(e));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, FGS_ERR_UNSUPPORTED, "fgs_ctx_create: device is %s, this library is built for gfx950",
                    prop.gcnArchName);
    fgs_ctx *c = new (std::nothrow) fgs_ctx();
    if (!c) return fail(nullptr, FGS_ERR_HIP, "fgs_ctx_create: out of host memory");
    c->device = dev;
    c->stream = (hipStream_t)hip_stream;
    e = noalloc_scratch_init(dev);
    if (e == hipSuccess) e = c->words.ensure(W_TOTAL * 4);
    if (e == hipSuccess) e = hipMemset(c->words.p, 0, W_TOTAL * 4);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->host_words, W_TOTAL * 4, hipHostMallocDefault);
    if (e != hipSuccess) {
        fgs_ctx_destroy(c);
        return fail(nullptr, FGS_ERR_HIP, "fgs_ctx_create: %s", hipGetErrorString(e));
    }
    *out = c;
    return FGS_OK;
}

fgs_status fgs_ctx_destroy(fgs_ctx *ctx)
{
    if (!ctx) return FGS_OK;
    if (ctx->stream || true) (void)hipStreamSynchronize(ctx->stream);
    clear_profile(ctx, true);
    DBuf *bufs[] = {&ctx->prof_counts, &ctx->rect, &ctx->count, &ctx->dkA, &ctx->dkB, &ctx->idA, &ctx->idB,
                    &ctx->blocksums, &ctx->pkA, &ctx->pkB, &ctx->pvA, &ctx->pvB, &ctx->csum, &ctx->shist, &ctx->seg[0], &ctx->seg[1], &ctx->seg[2], &ctx->seg[3], &ctx->seg[4], &ctx->seg[5],
                    &ctx->hist, &ctx->grad2d,
                    &ctx->words, &ctx->ms_state, &ctx->ms_dl, &ctx->ms_grad, &ctx->ms_partials,
                    &ctx->seed_ws, &ctx->seed_sc, &ctx->offsets, &ctx->ms_img, &ctx->ms_ssim, &ctx->ms_reg,
                    &ctx->ssim_part, &ctx->ssim_ws};
    for (DBuf *b : bufs) b->release();
    if (ctx->host_words) (void)hipHostFree(ctx->host_words);
    if (ctx->ms_host) (void)hipHostFree(ctx->ms_host);
    if (ctx->step_host) (void)hipHostFree(ctx->step_host);
    if (ctx->gicp_host) (void)hipHostFree(ctx->gicp_host);
    delete ctx;
    return FGS_OK;
}

fgs_status fgs_ctx_set_stream(fgs_ctx *ctx, void *hip_stream)
{
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "fgs_ctx_set_stream: ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return FGS_OK;
}

}  // extern "C"

namespace {
fgs_status read_words(fgs_ctx *ctx)
{
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_words, ctx->words.p, W_TOTAL * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return FGS_OK;
}
}  // namespace

extern "C" {

fgs_status fgs_ctx_check(fgs_ctx *ctx)
{
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "fgs_ctx_check: ctx is NULL");
    fgs_status st = read_words(ctx);
    if (st != FGS_OK) return st;
    const uint32_t ovf = ctx->host_words[ST_OVERFLOW], sovf = ctx->host_words[ST_SEED_OVF];
    if (ovf || sovf) {
        HIP_TRY(ctx, hipMemsetAsync(ctx->words.as<uint32_t>() + ST_OVERFLOW, 0, 4, ctx->stream));
        HIP_TRY(ctx, hipMemsetAsync(ctx->words.as<uint32_t>() + ST_SEED_OVF, 0, 4, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (ovf)
            return fail(ctx, FGS_ERR_CAPACITY, "forward state too small: %u (tile, gaussian) pairs needed", ovf);
        return fail(ctx, FGS_ERR_CAPACITY, "seed output too small: %u seeds found", sovf);
    }
    return FGS_OK;
}

fgs_status fgs_ctx_stats(fgs_ctx *ctx, int64_t stats[4])
{
    if (!ctx || !stats) return fail(ctx, FGS_ERR_INVALID_ARG, "fgs_ctx_stats: NULL argument");
    fgs_status st = read_words(ctx);
    if (st != FGS_OK) return st;
    stats[0] = ctx->host_words[ST_PAIRS];
    stats[1] = ctx->host_words[ST_VISIBLE];
    stats[2] = ctx->host_words[ST_OVERFLOW];
    stats[3] = ctx->host_words[ST_SEEDS];
    return FGS_OK;
}

fgs_status fgs_ctx_profile(fgs_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "fgs_ctx_profile: ctx is NULL");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    clear_profile(ctx);
    ctx->prof = enable < 0 ? 0 : enable > 3 ? 3 : enable;
    if (ctx->prof && ctx->event_pool.size() < 4096) {
        // events for a few hundred steps up front, so the timed loop does not create any
        while (ctx->event_pool.size() < 4096) {
            hipEvent_t e;
            HIP_TRY(ctx, hipEventCreate(&e));
            ctx->event_pool.push_back(e);
        }
    }
    if (ctx->prof) {
        HIP_TRY(ctx, ctx->prof_counts.ensure(16 * 8));
        HIP_TRY(ctx, hipMemset(ctx->prof_counts.p, 0, 16 * 8));
    }
    return FGS_OK;
}

fgs_status fgs_ctx_profile_stage(fgs_ctx *ctx, const char *stage, double *total_ms, int64_t *launches)
{
    if (!ctx || !stage || !total_ms || !launches)
        return fail(ctx, FGS_ERR_INVALID_ARG, "fgs_ctx_profile_stage: NULL argument");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    double t = 0;
    int64_t k = 0;
    auto it = ctx->prof_events.find(stage);
    if (it != ctx->prof_events.end())
        for (auto &ab : it->second) {
            float ms = 0;
            HIP_TRY(ctx, hipEventElapsedTime(&ms, ab.first, ab.second));
            t += ms;
            ++k;
        }
    *total_ms = t;
    *launches = k;
    return FGS_OK;
}

fgs_status fgs_ctx_profile_counts(fgs_ctx *ctx, int64_t counts[4])
{
    if (!ctx || !counts) return fail(ctx, FGS_ERR_INVALID_ARG, "fgs_ctx_profile_counts: NULL argument");
    unsigned long long c[4] = {0, 0, 0, 0};
    if (ctx->prof_counts.p) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, hipMemcpy(c, ctx->prof_counts.p, sizeof(c), hipMemcpyDeviceToHost));
    }
    for (int k = 0; k < 3; ++k) counts[k] = (int64_t)c[k];
    counts[3] = ctx->prof_fwd;
    return FGS_OK;
}

fgs_status fgs_ctx_profile_work(fgs_ctx *ctx, int64_t counts[12])
{
    if (!ctx || !counts) return fail(ctx, FGS_ERR_INVALID_ARG, "fgs_ctx_profile_work: NULL argument");
    unsigned long long c[10] = {};
    if (ctx->prof_counts.p) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, hipMemcpy(c, ctx->prof_counts.p, sizeof(c), hipMemcpyDeviceToHost));
    }
    for (int k = 0; k < 6; ++k) counts[k] = (int64_t)c[k];
    counts[6] = ctx->prof_fwd;
    for (int k = 6; k < 10; ++k) counts[k + 1] = (int64_t)c[k];
    counts[11] = ctx->prof_bwd;
    return FGS_OK;
}

fgs_status fgs_state_bytes(int64_t n, int32_t width, int32_t height, int64_t max_pairs, const fgs_render_opts *o,
                           int64_t *bytes)
{
    int tw, th;
    if (!bytes) return fail(nullptr, FGS_ERR_INVALID_ARG, "fgs_state_bytes: bytes is NULL");
    fgs_status st = check_opts(nullptr, o, "fgs_state_bytes", &tw, &th);
    if (st != FGS_OK) return st;
    if (max_pairs < 0 || max_pairs > 0xFFFFFFF0ll)
        return fail(nullptr, FGS_ERR_INVALID_ARG, "fgs_state_bytes: max_pairs outside [0, 2^32 - 16]");
    StateLayout L;
    if (n < 0 || width <= 0 || height <= 0 || !state_layout(n, width, height, tw, th, max_pairs, &L))
        return fail(nullptr, FGS_ERR_INVALID_ARG, "fgs_state_bytes: bad sizes");
    *bytes = (int64_t)L.bytes;
    return FGS_OK;
}

fgs_status fgs_render_fwd(fgs_ctx *ctx, const fgs_gaussians *g, const fgs_camera *cam, const fgs_render_opts *o,
                          const fgs_image *out, void *state, int64_t state_bytes)
{
    const char *w = "fgs_render_fwd";
    int tw, th;
    fgs_status st;
    if ((st = check_gauss(ctx, g, w, "g")) != FGS_OK) return st;
    if ((st = check_camera(ctx, cam, w)) != FGS_OK) return st;
    if ((st = check_opts(ctx, o, w, &tw, &th)) != FGS_OK) return st;
    if (!out || !out->rgb || !out->depth) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: image rgb/depth is NULL", w);
    if (!state) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: state is NULL", w);
    StateLayout L;
    if (state_capacity(g->n, cam->width, cam->height, tw, th, state_bytes, &L) < 0)
        return fail(ctx, FGS_ERR_CAPACITY, "%s: state of %lld bytes is smaller than the %zu-byte fixed part", w,
                    (long long)state_bytes, L.fixed);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    ImageK img{out->rgb, out->depth, out->alpha, out->T_final, out->n_contrib};
    return enqueue_forward(ctx, *g, *cam, *o, tw, th, img, state, L);
}

fgs_status fgs_render_bwd(fgs_ctx *ctx, const fgs_gaussians *g, const fgs_camera *cam, const fgs_render_opts *o,
                          const void *state, int64_t state_bytes, const float *dL_drgb, const float *dL_ddepth,
                          const float *dL_dalpha, const fgs_gaussians *grad)
{
    const char *w = "fgs_render_bwd";
    int tw, th;
    fgs_status st;
    if ((st = check_gauss(ctx, g, w, "g")) != FGS_OK) return st;
    if ((st = check_gauss(ctx, grad, w, "grad")) != FGS_OK) return st;
    if (grad->n != g->n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: grad.n != g.n", w);
    if ((st = check_camera(ctx, cam, w)) != FGS_OK) return st;
    if ((st = check_opts(ctx, o, w, &tw, &th)) != FGS_OK) return st;
    if (!dL_drgb || !dL_ddepth) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: dL_drgb/dL_ddepth is NULL", w);
    if (!state) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: state is NULL", w);
    StateLayout L;
    if (state_capacity(g->n, cam->width, cam->height, tw, th, state_bytes, &L) < 0)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: state of %lld bytes does not match n and the image size", w,
                    (long long)state_bytes);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    return enqueue_backward(ctx, *g, *cam, *o, tw, th, state, L, dL_drgb, dL_ddepth, dL_dalpha, nullptr, grad, grad,
                            nullptr);
}

fgs_status fgs_render_bwd_noalloc(fgs_ctx *ctx, const fgs_gaussians *g, const fgs_camera *cam,
                                  const fgs_render_opts *o, const void *state, int64_t state_bytes,
                                  const float *dL_drgb, const float *dL_ddepth, const float *dL_dalpha,
                                  const fgs_gaussians *grad)
{
    const char *w = "fgs_render_bwd_noalloc";
    int tw, th;
    fgs_status st;
    if ((st = check_gauss(ctx, g, w, "g")) != FGS_OK) return st;
    if ((st = check_gauss(ctx, grad, w, "grad")) != FGS_OK) return st;
    if (grad->n != g->n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: grad.n != g.n", w);
    if (g->n > kNoallocMax)
        return fail(ctx, FGS_ERR_CAPACITY, "%s: %lld gaussians exceed the static scratch of %lld", w,
                    (long long)g->n, (long long)kNoallocMax);
    if ((st = check_camera(ctx, cam, w)) != FGS_OK) return st;
    if ((st = check_opts(ctx, o, w, &tw, &th)) != FGS_OK) return st;
    if (!dL_drgb || !dL_ddepth) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: dL_drgb/dL_ddepth is NULL", w);
    if (!state) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: state is NULL", w);
    StateLayout L;
    if (state_capacity(g->n, cam->width, cam->height, tw, th, state_bytes, &L) < 0)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: state of %lld bytes does not match n and the image size", w,
                    (long long)state_bytes);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    float *g2 = noalloc_scratch(ctx->device);
    if (!g2) return fail(ctx, FGS_ERR_HIP, "%s: no scratch address for device %d", w, ctx->device);
    if (g->n == 0) return FGS_OK;
    hipStream_t s = ctx->stream;
    const RasterK rk = to_rk(*o, tw, th, cam->width, cam->height);
    const StatePtrs sp = state_ptrs((void *)state, L);
    // the records of this call's gaussians start at zero (a fill kernel, so the call can be captured)
    launch_zero_f32(g2, g->n * kG2Stride, s);
    launch_raster_bwd(rk, cam->width, cam->height, sp.rec, sp.vals, sp.ranges, sp.last, sp.tfinal, dL_drgb,
                      dL_ddepth, dL_dalpha, nullptr, g2, nullptr, s);
    const GradK gk = to_gk(*grad);
    launch_project_bwd(to_pk(*g), to_camk(*cam), rk, g2, gk, gk, AdamK{}, s);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

fgs_status fgs_loss_l1(fgs_ctx *ctx, int64_t n_pixels, const float *rgb, const float *depth, const fgs_target *target,
                       const fgs_loss_opts *l, float *dL_drgb, float *dL_ddepth, float *loss_dev, float *psnr_dev)
{
    const char *w = "fgs_loss_l1";
    if (n_pixels <= 0) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: n_pixels must be > 0", w);
    if (!rgb || !depth || !target || !target->rgb || !target->depth || !l || !dL_drgb || !dL_ddepth)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: NULL argument", w);
    if (!isfinite(l->lambda_rgb) || !isfinite(l->lambda_depth))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: loss weights not finite", w);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    HIP_TRY(ctx, ctx->ms_partials.ensure((size_t)loss_partials_size(n_pixels) * 4));
    float *dscale = ctx->words.as<float>() + W_DSCALE;
    launch_loss_l1(n_pixels, rgb, depth, target->rgb, target->depth, l->lambda_rgb, l->lambda_depth, dL_drgb,
                   dL_ddepth, dscale, ctx->ms_partials.as<float>(), loss_dev, psnr_dev, ctx->stream);
    launch_scale(dL_ddepth, n_pixels, dscale, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

static fgs_status check_adam(fgs_ctx *ctx, const fgs_adam *opt, int64_t n, const char *w)
{
    if (!opt) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: opt is NULL", w);
    fgs_status st;
    if ((st = check_gauss(ctx, &opt->m, w, "opt.m")) != FGS_OK) return st;
    if ((st = check_gauss(ctx, &opt->v, w, "opt.v")) != FGS_OK) return st;
    if (opt->m.n != n || opt->v.n != n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: Adam moments have n != params.n", w);
    if (opt->step < 0) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: opt.step < 0", w);
    if (!(opt->beta1 >= 0 && opt->beta1 < 1 && opt->beta2 >= 0 && opt->beta2 < 1) || !(opt->eps >= 0))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: beta1, beta2 must be in [0, 1) and eps >= 0", w);
    for (int k = 0; k < 5; ++k)
        if (!isfinite(opt->lr[k])) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: learning rate not finite", w);
    return FGS_OK;
}

static void enqueue_adam(fgs_ctx *ctx, const fgs_gaussians &p, const fgs_gaussians &grad, fgs_adam *opt)
{
    Stage st_(ctx, "adam");
    const double k = (double)(opt->step + 1);
    const float bc1 = (float)(1.0 - pow((double)opt->beta1, k));
    const float bc2 = (float)(1.0 - pow((double)opt->beta2, k));
    launch_adam(to_gk(p), to_pk(grad), to_gk(opt->m), to_gk(opt->v), opt->lr, opt->beta1, opt->beta2, opt->eps, bc1,
                bc2, ctx->stream);
    opt->step += 1;
}

fgs_status fgs_ssim(fgs_ctx *ctx, int32_t width, int32_t height, const float *img, const float *tgt,
                    float *ssim_dev, float *dssim_dimg)
{
    const char *w = "fgs_ssim";
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    if (width <= 0 || height <= 0 || (int64_t)width * height > ((int64_t)1 << 29))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: image size %d x %d outside (0, 2^29] pixels", w, width, height);
    if (!img || !tgt) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: img or tgt is NULL", w);
    if (!ssim_dev && !dssim_dimg) return FGS_OK;
    const int64_t T = ssim_partials(width, height);
    HIP_TRY(ctx, ctx->ssim_part.ensure((size_t)T * 4));
    HIP_TRY(ctx, ctx->ssim_ws.ensure((size_t)ssim_ws_floats(width, height) * 4));
    launch_ssim(width, height, img, tgt, 1.0f, false, dssim_dimg, ssim_dev ? ctx->ssim_part.as<float>() : nullptr,
                ctx->ssim_ws.as<float>(), ctx->stream);
    if (ssim_dev)
        launch_sum_scaled(ctx->ssim_part.as<float>(), (int)T, 1.0 / (3.0 * (double)width * (double)height), ssim_dev,
                          ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

// Byte span [lo, hi) of the planes of a block of n gaussians.
static void block_span(const fgs_gaussians &g, int64_t n, uintptr_t *lo, uintptr_t *hi)
{
    const float *planes[14];
    for (int k = 0; k < 3; ++k) planes[k] = g.mean + k * g.stride;
    for (int k = 0; k < 3; ++k) planes[3 + k] = g.log_scale + k * g.stride;
    for (int k = 0; k < 4; ++k) planes[6 + k] = g.quat + k * g.stride;
    planes[10] = g.opacity_logit;
    for (int k = 0; k < 3; ++k) planes[11 + k] = g.rgb + k * g.stride;
    *lo = UINTPTR_MAX;
    *hi = 0;
    for (const float *q : planes) {
        const uintptr_t a = (uintptr_t)q, b = a + (uintptr_t)n * 4;
        if (a < *lo) *lo = a;
        if (b > *hi) *hi = b;
    }
}

fgs_status fgs_prune(fgs_ctx *ctx, const fgs_prune_opts *o, int32_t n_sets, const fgs_gaussians *src,
                     const fgs_gaussians *dst, int64_t *n_kept_dev, uint8_t *keep, int64_t *n_kept_host)
{
    const char *w = "fgs_prune";
    if (!o) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: options are NULL", w);
    if (n_sets < 1 || n_sets > kPruneSets || !src || !dst)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: n_sets must be in [1, %d] with src and dst given", w, kPruneSets);
    if (!(o->min_opacity >= 0.0f && o->min_opacity < 1.0f))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: min_opacity must be in [0, 1)", w);
    if (std::isnan(o->max_scale)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: max_scale is NaN", w);
    fgs_status st;
    const int64_t n = src[0].n;
    for (int k = 0; k < n_sets; ++k) {
        if ((st = check_gauss(ctx, &src[k], w, "src")) != FGS_OK) return st;
        if (src[k].n != n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: src[%d].n != src[0].n", w, k);
        if (dst[k].stride < n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: dst[%d].stride < n", w, k);
        if (n > 0 && (!dst[k].mean || !dst[k].log_scale || !dst[k].quat || !dst[k].opacity_logit || !dst[k].rgb))
            return fail(ctx, FGS_ERR_INVALID_ARG, "%s: dst[%d] has a NULL plane", w, k);
    }
    if (n > 0) {
        uintptr_t lo[2 * kPruneSets], hi[2 * kPruneSets];
        for (int k = 0; k < n_sets; ++k) {
            block_span(src[k], n, &lo[k], &hi[k]);
            block_span(dst[k], n, &lo[n_sets + k], &hi[n_sets + k]);
        }
        for (int a = n_sets; a < 2 * n_sets; ++a)  // each destination against every other block
            for (int b = 0; b < 2 * n_sets; ++b)
                if (a != b && lo[a] < hi[b] && lo[b] < hi[a])
                    return fail(ctx, FGS_ERR_INVALID_ARG, "%s: dst[%d] overlaps %s[%d]", w, a - n_sets,
                                b < n_sets ? "src" : "dst", b < n_sets ? b : b - n_sets);
    }
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    PruneK pk{};
    pk.n = n;
    const double tau = (double)o->min_opacity, smax = (double)o->max_scale;
    pk.L_o = tau > 0.0 ? (float)log(tau / (1.0 - tau)) : -INFINITY;
    pk.L_s = (smax > 0.0 && std::isfinite(smax)) ? (float)log(smax) : INFINITY;
    pk.logit = src[0].opacity_logit;
    pk.ls0 = src[0].log_scale;
    pk.ls1 = src[0].log_scale + src[0].stride;
    pk.ls2 = src[0].log_scale + 2 * src[0].stride;
    pk.n_planes = 14 * n_sets;
    for (int k = 0; k < n_sets; ++k) {
        const fgs_gaussians &a = src[k], &b = dst[k];
        const float *sp[14] = {a.mean, a.mean + a.stride, a.mean + 2 * a.stride, a.log_scale,
                               a.log_scale + a.stride, a.log_scale + 2 * a.stride, a.quat, a.quat + a.stride,
                               a.quat + 2 * a.stride, a.quat + 3 * a.stride, a.opacity_logit, a.rgb,
                               a.rgb + a.stride, a.rgb + 2 * a.stride};
        float *dp[14] = {b.mean, b.mean + b.stride, b.mean + 2 * b.stride, b.log_scale, b.log_scale + b.stride,
                         b.log_scale + 2 * b.stride, b.quat, b.quat + b.stride, b.quat + 2 * b.stride,
                         b.quat + 3 * b.stride, b.opacity_logit, b.rgb, b.rgb + b.stride, b.rgb + 2 * b.stride};
        for (int j = 0; j < 14; ++j) {
            pk.src[14 * k + j] = sp[j];
            pk.dst[14 * k + j] = dp[j];
        }
    }
    pk.keep = keep;
    const size_t need = 256 + (size_t)prune_ws_words(n) * 4;
    if (need > ctx->prune_ws.bytes) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, ctx->prune_ws.ensure(need));
    }
    int64_t *total = ctx->prune_ws.as<int64_t>();
    {
        Stage st_(ctx, "prune");
        launch_prune(pk, ctx->prune_ws.as<uint32_t>(256), total, n_kept_dev, ctx->stream);
    }
    HIP_TRY(ctx, hipGetLastError());
    if (n_kept_host) {
        int64_t v = -1;
        HIP_TRY(ctx, hipMemcpyAsync(&v, total, 8, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        *n_kept_host = v;
    }
    return FGS_OK;
}

fgs_status fgs_adam_step(fgs_ctx *ctx, const fgs_gaussians *params, const fgs_gaussians *grad, fgs_adam *opt)
{
    const char *w = "fgs_adam_step";
    fgs_status st;
    if ((st = check_gauss(ctx, params, w, "params")) != FGS_OK) return st;
    if ((st = check_gauss(ctx, grad, w, "grad")) != FGS_OK) return st;
    if (grad->n != params->n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: grad.n != params.n", w);
    if ((st = check_adam(ctx, opt, params->n, w)) != FGS_OK) return st;
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    enqueue_adam(ctx, *params, *grad, opt);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

fgs_status fgs_map_step(fgs_ctx *ctx, const fgs_gaussians *params, fgs_adam *opt, int32_t n_views,
                        const fgs_camera *cams, const fgs_target *targets, const fgs_render_opts *o,
                        const fgs_loss_opts *l, float *loss_dev, float *psnr_dev, const fgs_gaussians *grad_out)
{
    const char *w = "fgs_map_step";
    int tw, th;
    fgs_status st;
    if ((st = check_gauss(ctx, params, w, "params")) != FGS_OK) return st;
    if ((st = check_adam(ctx, opt, params->n, w)) != FGS_OK) return st;
    if (n_views <= 0 || n_views > 4096) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: n_views outside [1, 4096]", w);
    if (!cams || !targets) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: cams/targets is NULL", w);
    if ((st = check_opts(ctx, o, w, &tw, &th)) != FGS_OK) return st;
    if (!l || !isfinite(l->lambda_rgb) || !isfinite(l->lambda_depth) || !isfinite(l->lambda_reg))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: loss options NULL or not finite", w);
    if (!(l->lambda_rgb >= 0.0f && l->lambda_rgb <= 1.0f) || l->lambda_reg < 0.0f)
        return fail(ctx, FGS_ERR_INVALID_ARG,
                    "%s: lambda_rgb must lie in [0, 1] (Eq. 16 weights the SSIM term by 1 - lambda_rgb) and "
                    "lambda_reg be >= 0", w);
    int64_t Pmax = 0;
    for (int v = 0; v < n_views; ++v) {
        if ((st = check_camera(ctx, &cams[v], w)) != FGS_OK) return st;
        if (!targets[v].rgb || !targets[v].depth) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: target %d is NULL", w, v);
        const int64_t P = (int64_t)cams[v].width * cams[v].height;
        if (P > Pmax) Pmax = P;
    }
    if (grad_out) {
        if ((st = check_gauss(ctx, grad_out, w, "grad_out")) != FGS_OK) return st;
        if (grad_out->n != params->n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: grad_out.n != params.n", w);
    }
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    hipStream_t s = ctx->stream;
    const int64_t n = params->n;
    if (!ctx->ms_host) {
        HIP_TRY(ctx, hipHostMalloc((void **)&ctx->ms_host, 2 * 4096 * 4, hipHostMallocMapped | hipHostMallocCoherent));
        memset(ctx->ms_host, 0, 2 * 4096 * 4);
        HIP_TRY(ctx, hipHostGetDevicePointer((void **)&ctx->ms_host_dev, ctx->ms_host, 0));
        HIP_TRY(ctx, hipHostMalloc((void **)&ctx->step_host, 8, hipHostMallocDefault));
        ctx->ms_seen.assign(4096, false);
        ctx->ms_cams.assign(4096, fgs_camera{});
    }
    int64_t *dstep = (int64_t *)(ctx->words.as<uint32_t>() + W_STEP);
    uint32_t *step_ovf = ctx->words.as<uint32_t>() + W_STEPOVF;
    // A step whose pair count outgrew a view's state while running unchecked is reported here,
    // once. Such a step (and any step enqueued after it that overflowed as well) left the
    // parameters, the Adam moments and the device step count as they were: opt->step is set back
    // to the device's count, the state is grown, and the caller repeats the step.
    {
        volatile uint32_t *hs = ctx->ms_host;
        bool any = false;
        for (int v = 0; v < ctx->ms_nv_max; ++v) any |= hs[2 * v + 1] != 0;
        if (any) {
            HIP_TRY(ctx, hipStreamSynchronize(s));  // the flags and counts are final now
            int64_t K = 0;
            int vk = 0;
            for (int v = 0; v < ctx->ms_nv_max; ++v)
                if (hs[2 * v + 1]) {
                    if ((int64_t)hs[2 * v] >= K) {
                        K = hs[2 * v];
                        vk = v;
                    }
                    hs[2 * v + 1] = 0;
                }
            if (K + K / 4 + 1024 > ctx->ms_cap) ctx->ms_cap = K + K / 4 + 1024;
            // the context's overflow word saw the same event; this report replaces it
            HIP_TRY(ctx, hipMemsetAsync(ctx->words.as<uint32_t>() + ST_OVERFLOW, 0, 4, s));
            fgs_status st2 = read_words(ctx);
            if (st2 != FGS_OK) return st2;
            if (ctx->ms_dev_step >= 0) {
                int64_t dev;
                memcpy(&dev, ctx->host_words + W_STEP + 2 * ctx->ms_slot, 8);
                opt->step = dev;
                ctx->ms_dev_step = dev;
            }
            return fail(ctx, FGS_ERR_CAPACITY,
                        "%s: an earlier step needed %lld (tile, gaussian) pairs in view %d and was not applied "
                        "(parameters, moments and step count unchanged); the state was grown, repeat that step",
                        w, (long long)K, vk);
        }
    }
    if (n_views > ctx->ms_nv_max) ctx->ms_nv_max = std::min(n_views, 4096);
    // the device's step count follows the host's (a new context, or a caller that reset opt->step)
    if (opt->step != ctx->ms_dev_step) {
        HIP_TRY(ctx, hipStreamSynchronize(s));
        *ctx->step_host = opt->step;
        HIP_TRY(ctx, hipMemcpyAsync(dstep + ctx->ms_slot, ctx->step_host, 8, hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        ctx->ms_dev_step = opt->step;
    }
    // summed gradient: the caller's buffer, or the context's (the first view overwrites it)
    fgs_gaussians grad;
    if (grad_out) {
        grad = *grad_out;
    } else {
        HIP_TRY(ctx, ctx->ms_grad.ensure((size_t)(n > 0 ? n : 1) * 14 * 4));
        float *b = ctx->ms_grad.as<float>();
        grad = fgs_gaussians{n, n, b, b + 3 * n, b + 6 * n, b + 10 * n, b + 11 * n};
    }
    // the loss is fused into each view's forward: per-pixel gradients into ms_dl, one partial
    // quadruple per tile into ms_partials
    int64_t Tmax = 0;
    for (int v = 0; v < n_views; ++v)
        Tmax = std::max<int64_t>(Tmax, tile_items((cams[v].width + tw - 1) / tw, (cams[v].height + th - 1) / th));
    HIP_TRY(ctx, ctx->ms_dl.ensure((size_t)Pmax * 4 * 4));
    HIP_TRY(ctx, ctx->ms_partials.ensure((size_t)Tmax * 4 * 4));
    // the SSIM term needs the rendered colour and one sum per 16x16 tile; the regulariser one
    // partial sum per projection workgroup
    const float ssim_w = 1.0f - l->lambda_rgb;
    const bool use_ssim = ssim_w > 0.0f, use_reg = l->lambda_reg > 0.0f || l->reg_dev;
    if (use_ssim) {
        int64_t St = 0;
        for (int v = 0; v < n_views; ++v) St = std::max<int64_t>(St, ssim_partials(cams[v].width, cams[v].height));
        HIP_TRY(ctx, ctx->ms_img.ensure((size_t)Pmax * 3 * 4));
        HIP_TRY(ctx, ctx->ms_ssim.ensure((size_t)St * 4));
        HIP_TRY(ctx, ctx->ssim_ws.ensure((size_t)9 * Pmax * 4));
    }
    if (use_reg) HIP_TRY(ctx, ctx->ms_reg.ensure((size_t)project_blocks(n) * 4));
    if (ctx->ms_cap == 0) ctx->ms_cap = n * 16 > ((int64_t)1 << 22) ? n * 16 : ((int64_t)1 << 22);
    float *dscale = ctx->words.as<float>() + W_DSCALE;
    for (int v = 0; v < n_views; ++v) {
        const fgs_camera &cam = cams[v];
        const int64_t P = (int64_t)cam.width * cam.height;
        uint32_t *hs_dev = v < 4096 ? ctx->ms_host_dev + 2 * v : nullptr;
        StateLayout L;
        for (int attempt = 0;; ++attempt) {
            state_layout(n, cam.width, cam.height, tw, th, ctx->ms_cap, &L);
            HIP_TRY(ctx, ctx->ms_state.ensure(L.bytes));
            // only the loss reads the image (and the SSIM term the rendered colour)
            const ImageK img{use_ssim ? ctx->ms_img.as<float>() : nullptr, nullptr, nullptr, nullptr, nullptr};
            float *dl = ctx->ms_dl.as<float>();
            LossK lk{};
            lk.trgb = targets[v].rgb;
            lk.tdepth = targets[v].depth;
            lk.drgb = dl;
            lk.ddepth = dl + 3 * P;
            lk.partials = ctx->ms_partials.as<float>();
            lk.lrgb = l->lambda_rgb;
            lk.ldepth = l->lambda_depth;
            lk.inv3P = (float)(1.0 / (3.0 * (double)P));
            lk.ddepth_scale = n > 0 ? dscale : nullptr;  // 1/P_v, written by the binning
            // The pair count is data dependent. A view is checked synchronously (the forward waits
            // for the count after the scan and restarts with a larger state when it does not fit)
            // the first time it is seen (a new index, camera or gaussian count) and whenever its last
            // observed count came within 10% of the capacity; otherwise it runs without a host round
            // trip and an overflow is caught by the flag above on the next call.
            const bool seen = v < 4096 && ctx->ms_seen[v] && n == ctx->ms_n &&
                              memcmp(&ctx->ms_cams[v], &cam, sizeof(fgs_camera)) == 0;
            const int64_t K_obs = v < 4096 ? (int64_t)((volatile uint32_t *)ctx->ms_host)[2 * v] : 0;
            const bool checked = !seen || K_obs * 10 > ctx->ms_cap * 9;
            int64_t K = 0;
            st = enqueue_forward(ctx, *params, cam, *o, tw, th, img, ctx->ms_state.p, L, checked ? &K : nullptr,
                                 hs_dev, true, &lk, step_ovf, v == 0,
                                 use_reg && v == 0 ? ctx->ms_reg.as<float>() : nullptr);
            if (st == FGS_OK) {
                if (v < 4096) {
                    ctx->ms_seen[v] = true;
                    ctx->ms_cams[v] = cam;
                }
                // keep 50% headroom above a count seen within 20% of the capacity (the larger state
                // is allocated before the next step's forward)
                if (checked && K * 5 > ctx->ms_cap * 4) ctx->ms_cap = K + K / 2 + 1024;
                break;
            }
            if (st != FGS_ERR_CAPACITY || attempt > 0) return st;
            ctx->ms_cap = K + K / 4 + 1024;
        }
        float *dl = ctx->ms_dl.as<float>();
        const bool last = v == n_views - 1;
        LossExtraK ex{};
        if (use_ssim) {
            // (1 - lambda_rgb)(1 - ssim): its gradient added to the L1 terms' colour gradient
            Stage st_(ctx, "ssim");
            launch_ssim(cam.width, cam.height, ctx->ms_img.as<float>(), targets[v].rgb, -ssim_w, true, dl,
                        ctx->ms_ssim.as<float>(), ctx->ssim_ws.as<float>(), s);
            ex.ssim_part = ctx->ms_ssim.as<float>();
            ex.ssim_nb = (int)ssim_partials(cam.width, cam.height);
            ex.ssim_w = ssim_w;
        }
        if (use_reg && last) {
            ex.reg_part = ctx->ms_reg.as<float>();
            ex.reg_nb = (int)project_blocks(n);
            ex.reg_scale = n > 0 ? (float)(1.0 / (double)n) : 0.0f;
            ex.reg_out = l->reg_dev;
        }
        // the loss and PSNR: reduced by the projection backward's first workgroup (the backward
        // needs only 1/P_v, which the binning wrote); without gaussians by a launch of their own
        LossFinalK lf{};
        if (n > 0) {
            lf.partials = ctx->ms_partials.as<float>();
            lf.nb = (int)L.T;
            lf.P = P;
            lf.lrgb = l->lambda_rgb;
            lf.ldepth = l->lambda_depth;
            lf.loss = loss_dev ? loss_dev + v : nullptr;
            lf.psnr = psnr_dev ? psnr_dev + v : nullptr;
            lf.extra = ex;
        } else {
            Stage st_(ctx, "loss");
            launch_loss_final(ctx->ms_partials.as<float>(), (int)L.T, P, l->lambda_rgb, l->lambda_depth, dscale,
                              loss_dev ? loss_dev + v : nullptr, psnr_dev ? psnr_dev + v : nullptr, s, ex);
        }
        // views before the last sum their gradients into grad; the last one adds its own (and the
        // regulariser's) and applies Adam in the same kernel (writing the sum only when the caller
        // asked for it)
        AdamK ak{};
        if (last) {
            // update number = the device's count + 1; skipped (and the count kept) when any view
            // of this step overflowed its state
            ak.m = to_gk(opt->m);
            ak.v = to_gk(opt->v);
            ak.step = dstep + ctx->ms_slot;
            ak.step_out = dstep + (1 - ctx->ms_slot);
            ak.skip = step_ovf;
            for (int k = 0; k < 5; ++k) ak.lr[k] = opt->lr[k];
            ak.beta1 = opt->beta1;
            ak.beta2 = opt->beta2;
            ak.eps = opt->eps;
            // the bias corrections of the update the host expects (the kernel recomputes them if
            // the device count differs, after an overflowed step not yet reported)
            ak.step_expect = opt->step;
            const double t = (double)(opt->step + 1);
            ak.bc1 = (float)(1.0 - pow((double)opt->beta1, t));
            ak.bc2 = (float)(1.0 - pow((double)opt->beta2, t));
            ak.reg_w = l->lambda_reg > 0.0f && n > 0 ? (float)((double)l->lambda_reg / (double)n) : 0.0f;
        }
        if ((st = enqueue_backward(ctx, *params, cam, *o, tw, th, ctx->ms_state.p, L, dl, dl + 3 * P, nullptr, dscale,
                                   v > 0 ? &grad : nullptr, !last || grad_out ? &grad : nullptr,
                                   last ? &ak : nullptr, &lf)) != FGS_OK)
            return st;
    }
    ctx->ms_n = n;
    opt->step += 1;
    if (n > 0) {
        ctx->ms_slot ^= 1;  // the projection backward wrote the new count into the other slot
        ctx->ms_dev_step = opt->step;
    } else {
        ctx->ms_dev_step = -1;  // no projection backward ran: the next step uploads the count
    }
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

fgs_status fgs_seed_gaussians(fgs_ctx *ctx, const float *rgb, const float *depth, const fgs_camera *cam,
                              const fgs_seed_opts *o, const fgs_seed_out *out, int64_t *n_seeds_host)
{
    const char *w = "fgs_seed_gaussians";
    fgs_status st;
    if ((st = check_camera(ctx, cam, w)) != FGS_OK) return st;
    if (!rgb || !depth) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: rgb/depth is NULL", w);
    if (!o) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: options are NULL", w);
    if (!(o->D0 > 0) || !isfinite(o->D0)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: D0 must be finite and > 0", w);
    if (o->m <= 0 || o->n <= 0 || o->tile <= 0)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: m, n and tile must be positive", w);
    if (!isfinite(o->alpha_h) || !isfinite(o->alpha_l) || !isfinite(o->opacity_logit) ||
        !(o->depth_min <= o->depth_max))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: radius factors, opacity or depth range invalid", w);
    if (o->use_prior < 0 || o->use_prior > 3)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: use_prior outside 0..3", w);
    if (o->use_prior && !o->prior) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: use_prior without weights", w);
    if (o->render_alpha && (!o->render_depth || !o->render_rgb))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: missing-region check needs the rendered depth and colour", w);
    if (o->render_alpha && (std::isnan(o->miss_alpha) || std::isnan(o->miss_depth) || std::isnan(o->miss_rgb)))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: missing-region thresholds are NaN", w);
    if (o->use_prior && !out->params.mean)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: use_prior needs out->params (the prior writes gaussians)", w);
    if (!out || out->capacity < 0 || (out->capacity > 0 && (!out->pixel || !out->is_high || !out->mean ||
                                                            !out->radius || !out->rgb)))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: seed output incomplete", w);
    if (out->params.mean) {
        if ((st = check_gauss(ctx, &out->params, w, "out.params")) != FGS_OK) return st;
        if (out->params.stride < out->capacity)
            return fail(ctx, FGS_ERR_INVALID_ARG, "%s: out.params.stride < capacity", w);
    }
    const int W = cam->width, H = cam->height;
    if (!seed_size_supported(W, H))
        return fail(ctx, FGS_ERR_UNSUPPORTED, "%s: frame %dx%d: lines must be 2..%d long with prime factors <= 31", w, W,
                    H, kSeedMaxLine);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    HIP_TRY(ctx, ctx->seed_ws.ensure(seed_ws_bytes(W, H)));
    HIP_TRY(ctx, ctx->seed_sc.ensure(sizeof(SeedScalars)));
    SeedK sk;
    sk.m = o->m; sk.n = o->n; sk.tile = o->tile;
    sk.dmin = o->depth_min; sk.dmax = o->depth_max;
    sk.alpha_h = o->alpha_h; sk.alpha_l = o->alpha_l; sk.opacity_logit = o->opacity_logit;
    sk.fx = cam->fx; sk.fy = cam->fy; sk.cx = cam->cx; sk.cy = cam->cy;
    for (int k = 0; k < 9; ++k) sk.R[k] = cam->R_cw[k];
    for (int k = 0; k < 3; ++k) sk.t[k] = cam->t_cw[k];
    sk.ra = o->render_alpha;
    sk.rd = o->render_alpha ? o->render_depth : nullptr;
    sk.rc = o->render_alpha ? o->render_rgb : nullptr;
    sk.tau_a = o->miss_alpha;
    sk.tau_d = o->miss_depth;
    sk.tau_c = o->miss_rgb;
    SeedOutK so;
    so.capacity = out->capacity;
    so.pixel = out->pixel; so.is_high = out->is_high; so.mean = out->mean; so.radius = out->radius; so.rgb = out->rgb;
    so.tile_count = out->tile_count;
    so.n_dev = out->n_dev;
    so.params = out->params.mean ? to_gk(out->params) : GradK{0, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
    so.E = out->E;
    so.hist = out->hist;
    so.missing = out->missing;
    SeedScalars *sc = ctx->seed_sc.as<SeedScalars>();
    launch_seed(rgb, depth, W, H, o->D0, sk, so, ctx->seed_ws.p, sc, status_words(ctx), ctx->stream);
    if (out->threshold)
        HIP_TRY(ctx, hipMemcpyAsync(out->threshold, &sc->thresh, 4, hipMemcpyDeviceToDevice, ctx->stream));
    if (o->use_prior && out->capacity > 0) {
        const int tx = (W + 15) / 16, ty = (H + 15) / 16;
        const int64_t T = (int64_t)tx * ty;
        if ((st = ensure_mlp(ctx, T)) != FGS_OK) return st;
        HIP_TRY(ctx, ctx->prior_feat.ensure((size_t)T * kMlpIn * 4));
        HIP_TRY(ctx, ctx->prior_valid.ensure((size_t)T * 4));
        HIP_TRY(ctx, ctx->prior_y.ensure((size_t)T * kMlpOut * 4));
        MlpWS ws;
        mlp_ws_carve(ctx->mlp_ws.p, ctx->mlp_rows, &ws);
        launch_tile_features(rgb, depth, W, H, o->depth_min, o->depth_max, T, nullptr, ctx->prior_feat.as<float>(),
                             ctx->prior_valid.as<int32_t>(), ctx->stream);
        launch_mlp_forward(ws, T, ctx->prior_feat.as<float>(), (const float *)o->prior, ctx->prior_y.as<float>(),
                           false, ctx->stream);
        PriorApplyK pk;
        pk.tiles_x = tx;
        pk.W = W;
        pk.max_dev = (float)log(4.0);
        pk.min_valid = 4;
        pk.mode = o->use_prior;
        camera_to_world_quat(cam->R_cw, pk.q);
        const int64_t S = out->params.stride;
        launch_prior_apply(pk, seed_count_ptr(ctx->seed_ws.p, W, H), out->capacity, out->pixel,
                           ctx->prior_y.as<float>(), ctx->prior_valid.as<int32_t>(), out->params.log_scale,
                           out->params.quat, out->params.opacity_logit, S, out->from_prior, ctx->stream);
    }
    HIP_TRY(ctx, hipGetLastError());
    if (n_seeds_host) {
        if ((st = read_words(ctx)) != FGS_OK) return st;
        *n_seeds_host = ctx->host_words[ST_SEEDS];
        if (*n_seeds_host > out->capacity) {
            // reported here, so not again by the next fgs_ctx_check
            HIP_TRY(ctx, hipMemsetAsync(ctx->words.as<uint32_t>() + ST_SEED_OVF, 0, 4, ctx->stream));
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            return fail(ctx, FGS_ERR_CAPACITY, "%s: %lld seeds found, capacity %lld", w, (long long)*n_seeds_host,
                        (long long)out->capacity);
        }
    }
    return FGS_OK;
}

/* ------------------------------------ learned prior ------------------------------------ */

fgs_status fgs_tile_features(fgs_ctx *ctx, const float *rgb, const float *depth, int32_t width, int32_t height,
                             float depth_min, float depth_max, int64_t n_tiles, const int32_t *tile_ids, float *feat,
                             int32_t *n_valid)
{
    const char *w = "fgs_tile_features";
    if (width <= 0 || height <= 0 || width > 16384 || height > 16384)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: image size %dx%d outside [1, 16384]", w, width, height);
    if (n_tiles < 0 || n_tiles > ((int64_t)1 << 31) - 1) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: n_tiles", w);
    if (n_tiles > 0 && (!rgb || !depth || !feat)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: NULL plane", w);
    if (!tile_ids && n_tiles > (int64_t)((width + 15) / 16) * ((height + 15) / 16))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: more tiles than the frame has", w);
    if (!(depth_min <= depth_max)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: depth range", w);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    launch_tile_features(rgb, depth, width, height, depth_min, depth_max, n_tiles, tile_ids, feat, n_valid,
                         ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

fgs_status fgs_prior_forward(fgs_ctx *ctx, int64_t rows, const float *x, const float *weights, float *y)
{
    const char *w = "fgs_prior_forward";
    if (rows < 0 || rows > ((int64_t)1 << 24)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: rows outside [0, 2^24]", w);
    if (rows > 0 && (!x || !weights || !y)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: NULL argument", w);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    if (rows == 0) return FGS_OK;
    fgs_status st;
    if ((st = ensure_mlp(ctx, rows)) != FGS_OK) return st;
    MlpWS ws;
    mlp_ws_carve(ctx->mlp_ws.p, ctx->mlp_rows, &ws);
    launch_mlp_forward(ws, rows, x, weights, y, false, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

fgs_status fgs_prior_train_step(fgs_ctx *ctx, int64_t rows, const float *x, const float *target, float *weights,
                                fgs_prior_adam *opt, float *loss_dev, float *grad_out)
{
    const char *w = "fgs_prior_train_step";
    if (rows <= 0 || rows > ((int64_t)1 << 24)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: rows outside [1, 2^24]", w);
    if (!x || !target || !weights) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: NULL argument", w);
    if (!opt || !opt->m || !opt->v) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: Adam state incomplete", w);
    if (opt->step < 0 || !isfinite(opt->lr) || !(opt->beta1 >= 0 && opt->beta1 < 1) ||
        !(opt->beta2 >= 0 && opt->beta2 < 1) || !(opt->eps >= 0))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: Adam hyper-parameters", w);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    fgs_status st;
    if ((st = ensure_mlp(ctx, rows)) != FGS_OK) return st;
    MlpWS ws;
    mlp_ws_carve(ctx->mlp_ws.p, ctx->mlp_rows, &ws);
    const double k = (double)(opt->step + 1);
    const float bc1 = (float)(1.0 - pow((double)opt->beta1, k));
    const float bc2 = (float)(1.0 - pow((double)opt->beta2, k));
    launch_mlp_train_step(ws, rows, x, target, weights, opt->m, opt->v, opt->lr, opt->beta1, opt->beta2, opt->eps,
                          bc1, bc2, loss_dev, grad_out, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    opt->step += 1;
    return FGS_OK;
}

}  // extern "C"

/* ------------------------------------ keyframe window ------------------------------------ */

struct fgs_window {
    fgs_ctx *ctx = nullptr;
    int nv = 0;
    std::vector<fgs_camera> cams;
    std::vector<int> tw, th;
    int blocks = 0;
    int64_t n = -1;
    std::vector<int64_t> cap;
    std::vector<StateLayout> L;
    std::vector<DBuf> state;
    std::vector<int64_t> pix_off;  // float offset of view v's 4 planes in img and dl
    std::vector<uint32_t> tile_base;
    uint32_t total_tiles = 0;
    DBuf dl, grad2d, views, cams_dev, words, partials;
    // all views binned at once: the projection's per-workgroup pair counts of every view, the
    // views' key tables (x: super-tiles per row, y: first super-tile), and the tile ranges (by
    // window item) and tile lists of all views
    DBuf kpart, bintab, wranges, wvals;
    int64_t nsup_all = 0, cap_all = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> sig;        // what the captured graph baked in
    std::vector<uintptr_t> table_sig;  // what the device view table was built from
    ViewK *views_host = nullptr;       // pinned, rewritten only after the window stream drained
    CamK *cams_host = nullptr;
    int64_t *step_host = nullptr;      // pinned staging of the device Adam step counter
    int64_t dev_step = -1;             // value of the device counter once enqueued work is done
    uint32_t *hs = nullptr, *hs_dev = nullptr;  // host-mapped: [0] pairs of all views, [1] overflow
};

namespace {

// device words of a window: item counter of the persistent rasterizer, the step's overflow word,
// Adam step (int64, 8-byte aligned), per-view 1/P_v
constexpr int WW_COUNTER = 0, WW_OVF = 1, WW_STEP = 2, WW_DSCALE = 4;

void window_drop_graph(fgs_window *w)
{
    if (w->exec) (void)hipGraphExecDestroy(w->exec);
    if (w->graph) (void)hipGraphDestroy(w->graph);
    w->exec = nullptr;
    w->graph = nullptr;
    w->sig.clear();
}

float *view_dl(fgs_window *w, int v) { return w->dl.as<float>() + w->pix_off[v]; }

// Size every view's state from a synchronous pair count (50% headroom) for this n.
fgs_status window_size(fgs_window *w, const fgs_gaussians &params, const fgs_render_opts &o)
{
    fgs_ctx *ctx = w->ctx;
    const int64_t n = params.n;
    fgs_status st;
    if ((st = ensure_ws(ctx, std::max<int64_t>(n, w->total_tiles), 0)) != FGS_OK) return st;
    for (int v = 0; v < w->nv; ++v) {
        const fgs_camera &cam = w->cams[v];
        int64_t cap = std::max<int64_t>(w->cap[v], std::max<int64_t>(n * 8, (int64_t)1 << 20));
        for (int attempt = 0;; ++attempt) {
            state_layout(n, cam.width, cam.height, w->tw[v], w->th[v], cap, &w->L[v]);
            HIP_TRY(ctx, w->state[v].ensure(w->L[v].bytes));
            const ImageK img{nullptr, nullptr, nullptr, nullptr, nullptr};  // binning only: no image
            int64_t K = 0;
            st = enqueue_forward(ctx, params, cam, o, w->tw[v], w->th[v], img, w->state[v].p, w->L[v], &K, nullptr,
                                 false);
            if (st == FGS_OK || st == FGS_ERR_CAPACITY) {
                if (st == FGS_ERR_CAPACITY && attempt > 0) return fail(ctx, st, "fgs_window_step: sizing failed");
                w->cap[v] = std::max<int64_t>(w->cap[v], K + K / 2 + 1024);
                if (st == FGS_OK) break;
                cap = w->cap[v];
                continue;
            }
            return st;
        }
        state_layout(n, cam.width, cam.height, w->tw[v], w->th[v], w->cap[v], &w->L[v]);
        HIP_TRY(ctx, w->state[v].ensure(w->L[v].bytes));
    }
    // the context's sort and binning buffers hold every view's gaussians and pairs at once
    int64_t capsum = 0;
    for (int v = 0; v < w->nv; ++v) capsum += w->cap[v];
    w->cap_all = std::max(w->cap_all, capsum);
    const int64_t all = (int64_t)w->nv * n;
    if (all >= ((int64_t)1 << 31) || w->cap_all >= ((int64_t)1 << 32) - 1)
        return fail(ctx, FGS_ERR_UNSUPPORTED, "fgs_window_step: views x gaussians = %lld or pairs = %lld too many",
                    (long long)all, (long long)w->cap_all);
    if ((st = ensure_ws(ctx, std::max<int64_t>(all, w->total_tiles), w->cap_all)) != FGS_OK) return st;
    if ((st = ensure_bin(ctx, w->nsup_all, w->total_tiles, w->cap_all)) != FGS_OK) return st;
    const size_t g2 = (size_t)w->nv * kG2Stride * (size_t)(n > 0 ? n : 1) * 4;
    HIP_TRY(ctx, hipStreamSynchronize(w->stream));
    HIP_TRY(ctx, w->kpart.ensure((size_t)w->nv * 2 * project_blocks(n) * 4));
    HIP_TRY(ctx, w->wvals.ensure((size_t)std::max<int64_t>(w->cap_all, 1) * 4));
    HIP_TRY(ctx, w->grad2d.ensure(g2));
    HIP_TRY(ctx, hipMemset(w->grad2d.p, 0, g2));  // the backward keeps it all-zero between steps
    w->n = n;
    window_drop_graph(w);
    w->table_sig.clear();
    return FGS_OK;
}

// Build and upload the device table of views (pointers, shapes, options, the fused loss's
// targets) when it changed.
fgs_status window_tables(fgs_window *w, const fgs_gaussians &params, const fgs_render_opts &o,
                         const fgs_target *targets, const fgs_loss_opts &l)
{
    fgs_ctx *ctx = w->ctx;
    std::vector<uintptr_t> sig = {(uintptr_t)params.n, (uintptr_t)ctx->prof};
    uint32_t ob[sizeof(fgs_render_opts) / 4];
    memcpy(ob, &o, sizeof(ob));
    for (uint32_t x : ob) sig.push_back(x);
    uint32_t lb[2];
    memcpy(&lb[0], &l.lambda_rgb, 4);
    memcpy(&lb[1], &l.lambda_depth, 4);
    for (uint32_t x : lb) sig.push_back(x);
    for (int v = 0; v < w->nv; ++v) {
        sig.push_back((uintptr_t)w->state[v].p);
        sig.push_back((uintptr_t)targets[v].rgb);
        sig.push_back((uintptr_t)targets[v].depth);
    }
    if (sig == w->table_sig) return FGS_OK;
    HIP_TRY(ctx, hipStreamSynchronize(w->stream));  // earlier copies out of the pinned tables are done
    const int64_t n = params.n;
    for (int v = 0; v < w->nv; ++v) {
        const fgs_camera &cam = w->cams[v];
        const int64_t P = (int64_t)cam.width * cam.height;
        const StatePtrs sp = state_ptrs(w->state[v].p, w->L[v]);
        ViewK V = {};
        V.rk = to_rk(o, w->tw[v], w->th[v], cam.width, cam.height);
        V.W = cam.width;
        V.H = cam.height;
        V.rec = sp.rec;
        V.vals = w->wvals.as<uint32_t>();
        V.ranges = w->wranges.as<uint2>() + w->tile_base[v];
        V.last = sp.last;
        V.tfinal = sp.tfinal;
        V.img = ImageK{nullptr, nullptr, nullptr, nullptr, nullptr};  // only the fused loss reads the image
        V.loss.trgb = targets[v].rgb;
        V.loss.tdepth = targets[v].depth;
        V.loss.drgb = view_dl(w, v);
        V.loss.ddepth = view_dl(w, v) + 3 * P;
        V.loss.partials = w->partials.as<float>() + 4 * (size_t)w->tile_base[v];
        V.loss.lrgb = l.lambda_rgb;
        V.loss.ldepth = l.lambda_depth;
        V.loss.inv3P = (float)(1.0 / (3.0 * (double)P));
        V.drgb = view_dl(w, v);
        V.ddepth = view_dl(w, v) + 3 * P;
        V.ddepth_scale = w->words.as<float>() + WW_DSCALE + v;
        V.loss.ddepth_scale = w->words.as<float>() + WW_DSCALE + v;
        V.grad2d = w->grad2d.as<float>() + (size_t)v * kG2Stride * (size_t)n;
        V.counts = prof_counts(ctx);
        V.tile_base = w->tile_base[v];
        w->views_host[v] = V;
        w->cams_host[v] = to_camk(cam);
    }
    HIP_TRY(ctx, hipMemcpyAsync(w->views.p, w->views_host, sizeof(ViewK) * w->nv, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(ctx, hipMemcpyAsync(w->cams_dev.p, w->cams_host, sizeof(CamK) * w->nv, hipMemcpyHostToDevice, w->stream));
    w->table_sig = sig;
    return FGS_OK;
}

// Enqueue one window step on the context's stream (rebound to the window's stream by the caller).
// Only kernel launches: the sequence can be captured into a graph.
fgs_status window_enqueue(fgs_window *w, const fgs_gaussians &params, const fgs_adam &opt, const fgs_target *targets,
                          const fgs_render_opts &o, const fgs_loss_opts &l, float *loss_dev, float *psnr_dev,
                          const fgs_gaussians *grad_out)
{
    fgs_ctx *ctx = w->ctx;
    hipStream_t s = ctx->stream;
    const int64_t n = params.n;
    uint32_t *words = w->words.as<uint32_t>();
    // every view's projection into consecutive ranges of the depth-sort buffers
    const int64_t pb = project_blocks(n), all = (int64_t)w->nv * n;
    uint32_t *ndev = ctx->words.as<uint32_t>() + W_NDEV;
    auto proj_out = [&](int v) {
        return ProjOut{ctx->rect.as<uint2>() + (size_t)v * n, ctx->count.as<uint32_t>() + (size_t)v * n,
                       w->kpart.as<uint32_t>() + (size_t)v * 2 * pb};
    };
    for (int v = 0; v < w->nv; ++v) {
        const fgs_camera &cam = w->cams[v];
        const ProjOut po = proj_out(v);
        Stage st_(ctx, "project");
        launch_project(to_pk(params), to_camk(cam), to_rk(o, w->tw[v], w->th[v], cam.width, cam.height),
                       state_ptrs(w->state[v].p, w->L[v]).rec, po.rect, po.count, ctx->dkA.as<uint32_t>() + (size_t)v * n,
                       ctx->idA.as<uint32_t>() + (size_t)v * n, ndev, kSuperShift, po.kpart, s, (uint32_t)((size_t)v * n));
    }
    {
        // one stable sort of all views' values v n + i by depth (2,048 keys per workgroup: measured
        // faster than 512 or 1,024 at 4M keys)
        Stage st_(ctx, "depth_sort");
        // (four passes: the last one writes its values to idA, as it would without v_final)
        launch_radix_sort(ctx->dkA.as<uint32_t>(), ctx->idA.as<uint32_t>(), ctx->dkB.as<uint32_t>(),
                          ctx->idB.as<uint32_t>(), ctx->idA.as<uint32_t>(), ndev, all, 32,
                          sort_ws(ctx, all, kPairSortPerBlock), s);
    }
    {
        // All views binned at once: the pairs of one super-tile come from one view, so the depth
        // order of all views' values, kept by the stable super-tile sort, is each view's depth order.
        uint32_t *cw = ctx->words.as<uint32_t>();
        const uint2 *view_tab = w->bintab.as<uint2>();
        const int nsup = (int)w->nsup_all, sbits = key_bits_for(nsup);
        uint32_t *svals = (sbits + 7) / 8 == 1 ? ctx->pvB.as<uint32_t>() : ctx->pvA.as<uint32_t>();
        const BinWS bw = bin_ws(ctx);
        {
            Stage st_(ctx, "bin");
            launch_scan_counts(ctx->idA.as<uint32_t>(), ctx->count.as<uint32_t>(), all, ctx->blocksums.as<uint32_t>(),
                               s);
            launch_emit(ctx->idA.as<uint32_t>(), ctx->count.as<uint32_t>(), ctx->rect.as<uint2>(),
                        ctx->blocksums.as<uint32_t>(), ctx->offsets.as<uint32_t>(), all, 0, kSuperShift, w->cap_all,
                        ctx->pkA.as<uint32_t>(), ctx->pvA.as<uint32_t>(), ctx->rect_sorted.as<uint2>(),
                        ctx->start_rank.as<uint32_t>(), status_words(ctx), cw + W_NSUP, nullptr,
                        w->kpart.as<uint32_t>(), (int64_t)w->nv * pb, cw + W_KTOTAL, s, view_tab, (uint32_t)n);
        }
        {
            Stage st_(ctx, "tile_sort");
            const SortWS sws = sort_ws(ctx, w->cap_all);
            uint32_t *keys = launch_radix_sort(ctx->pkA.as<uint32_t>(), ctx->pvA.as<uint32_t>(),
                                               ctx->pkB.as<uint32_t>(), ctx->pvB.as<uint32_t>(), svals, cw + W_NSUP,
                                               w->cap_all, sbits, sws, s);
            const bool one_pass = sbits <= 8;
            if (!one_pass) launch_ranges(keys, cw + W_NSUP, ctx->bin_sranges.as<uint2>(), nsup, kSuperKeyMask, s);
            launch_bin_counts(bw, keys, ctx->bin_sranges.as<uint2>(), one_pass ? sws.totals : nullptr, nsup, s);
            launch_bin_tiles(bw, nsup, w->cap_all, cw + W_KTOTAL, w->wranges.as<uint2>(), status_words(ctx),
                             cw + W_NPAIRS, w->hs_dev, words + WW_OVF, true, s);
            launch_bin_place(bw, keys, svals, ctx->bin_sranges.as<uint2>(), w->wranges.as<uint2>(),
                             w->wvals.as<uint32_t>(), s);
        }
    }
    {
        Stage st_(ctx, "raster_fwd");
        launch_raster_window(true, prof_counts(ctx) != nullptr, w->views.as<ViewK>(), w->nv, w->total_tiles,
                             words + WW_COUNTER, w->blocks, s);
        if (prof_counts(ctx)) ctx->prof_fwd += w->nv;
    }
    {
        // the forward wrote the L1 terms' gradients and one partial quadruple per tile
        Stage st_(ctx, "loss");
        launch_loss_final_views(w->views.as<ViewK>(), w->nv, w->total_tiles, loss_dev, psnr_dev, s);
    }
    {
        Stage st_(ctx, "raster_bwd");
        launch_raster_window(false, false, w->views.as<ViewK>(), w->nv, w->total_tiles, words + WW_COUNTER,
                             w->blocks, s);
    }
    int64_t *step = (int64_t *)(words + WW_STEP);
    AdamK ak{};
    ak.m = to_gk(opt.m);
    ak.v = to_gk(opt.v);
    ak.step = step;
    ak.step_expect = -1;       // a replayed graph meets a new count every time: always recomputed
    ak.skip = words + WW_OVF;  // an overflowed step changes no parameter, moment or step count
    for (int k = 0; k < 5; ++k) ak.lr[k] = opt.lr[k];
    ak.beta1 = opt.beta1;
    ak.beta2 = opt.beta2;
    ak.eps = opt.eps;
    const GradK gk = grad_out ? to_gk(*grad_out) : GradK{n, n, nullptr, nullptr, nullptr, nullptr, nullptr};
    {
        Stage st_(ctx, "project_bwd");
        launch_project_bwd_window(to_pk(params), w->cams_dev.as<CamK>(), w->nv, o.lowpass, w->grad2d.as<float>(),
                                  (int64_t)kG2Stride * n, gk, ak, s);
    }
    launch_step_advance(step, words + WW_OVF, s);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

}  // namespace

extern "C" {

fgs_status fgs_window_create(fgs_ctx *ctx, int32_t n_views, const fgs_camera *cams, const int32_t *tiles,
                             int32_t blocks_per_cu, fgs_window **out)
{
    const char *w_ = "fgs_window_create";
    if (!out) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: out is NULL", w_);
    *out = nullptr;
    if (n_views <= 0 || n_views > 64) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: n_views outside [1, 64]", w_);
    if (!cams) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: cams is NULL", w_);
    if (blocks_per_cu < 0 || blocks_per_cu > 16)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: blocks_per_cu outside [0, 16]", w_);
    fgs_status st;
    for (int v = 0; v < n_views; ++v) {
        if ((st = check_camera(ctx, &cams[v], w_)) != FGS_OK) return st;
        const int a = tiles ? tiles[2 * v] : 16, b = tiles ? tiles[2 * v + 1] : 16;
        if (!tile_supported_window(a, b))
            return fail(ctx, FGS_ERR_INVALID_ARG, "%s: view %d: window tiles are 16x16, 32x8 or 8x32 (got %dx%d)", w_,
                        v, a, b);
    }
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w_);
    fgs_window *w = new (std::nothrow) fgs_window();
    if (!w) return fail(ctx, FGS_ERR_HIP, "%s: out of host memory", w_);
    w->ctx = ctx;
    w->nv = n_views;
    w->cams.assign(cams, cams + n_views);
    int64_t pix = 0;
    uint64_t tb = 0;
    for (int v = 0; v < n_views; ++v) {
        w->tw.push_back(tiles ? tiles[2 * v] : 16);
        w->th.push_back(tiles ? tiles[2 * v + 1] : 16);
        w->pix_off.push_back(4 * pix);
        const int64_t P = (int64_t)cams[v].width * cams[v].height;
        pix += P;
        w->tile_base.push_back((uint32_t)tb);
        tb += (uint64_t)tile_items((cams[v].width + w->tw[v] - 1) / w->tw[v], (cams[v].height + w->th[v] - 1) / w->th[v]);
    }
    if (tb >= ((uint64_t)1 << 31)) {
        delete w;
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: too many tiles in the window", w_);
    }
    w->total_tiles = (uint32_t)tb;
    // key table of the joint binning: view v's super-tiles follow those of the views before it
    std::vector<uint32_t> bintab(2 * (size_t)n_views);
    for (int v = 0; v < n_views; ++v) {
        const int sx = supers_for((cams[v].width + w->tw[v] - 1) / w->tw[v]);
        const int sy = supers_for((cams[v].height + w->th[v] - 1) / w->th[v]);
        bintab[2 * v] = (uint32_t)sx;
        bintab[2 * v + 1] = (uint32_t)w->nsup_all;
        w->nsup_all += (int64_t)sx * sy;
    }
    if (w->nsup_all > ((int64_t)1 << kBoxShift)) {  // not reached with 64 views of at most 16384^2 pixels
        delete w;
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: too many super-tiles in the window", w_);
    }
    w->cap.assign(n_views, 0);
    w->L.resize(n_views);
    w->state.resize(n_views);
    int cus = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    w->blocks = blocks_per_cu * cus;  // 0: one workgroup per (view, tile) item
    const size_t wbytes = (size_t)(WW_DSCALE + n_views) * 4 + 64;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = w->dl.ensure((size_t)pix * 4 * 4);
    if (e == hipSuccess) e = w->views.ensure(sizeof(ViewK) * n_views);
    if (e == hipSuccess) e = w->cams_dev.ensure(sizeof(CamK) * n_views);
    if (e == hipSuccess) e = w->words.ensure(wbytes);
    if (e == hipSuccess) e = hipMemset(w->words.p, 0, wbytes);
    if (e == hipSuccess) e = w->partials.ensure((size_t)w->total_tiles * 4 * 4);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w->step_host, 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w->views_host, sizeof(ViewK) * n_views, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w->cams_host, sizeof(CamK) * n_views, hipHostMallocDefault);
    if (e == hipSuccess) e = w->bintab.ensure(bintab.size() * 4);
    if (e == hipSuccess) e = hipMemcpy(w->bintab.p, bintab.data(), bintab.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = w->wranges.ensure((size_t)w->total_tiles * 8);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&w->hs, 2 * 4, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
        memset(w->hs, 0, 2 * 4);
        e = hipHostGetDevicePointer((void **)&w->hs_dev, w->hs, 0);
    }
    if (e != hipSuccess) {
        fgs_window_destroy(w);
        return fail(ctx, FGS_ERR_HIP, "%s: %s", w_, hipGetErrorString(e));
    }
    *out = w;
    return FGS_OK;
}

fgs_status fgs_window_destroy(fgs_window *w)
{
    if (!w) return FGS_OK;
    if (w->stream) (void)hipStreamSynchronize(w->stream);
    window_drop_graph(w);
    for (DBuf &b : w->state) b.release();
    DBuf *bufs[] = {&w->dl,       &w->grad2d, &w->views,   &w->cams_dev, &w->words,
                    &w->partials, &w->kpart,  &w->bintab, &w->wranges,  &w->wvals};
    for (DBuf *b : bufs) b->release();
    if (w->ev_in) (void)hipEventDestroy(w->ev_in);
    if (w->ev_out) (void)hipEventDestroy(w->ev_out);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    if (w->step_host) (void)hipHostFree(w->step_host);
    if (w->views_host) (void)hipHostFree(w->views_host);
    if (w->cams_host) (void)hipHostFree(w->cams_host);
    if (w->hs) (void)hipHostFree(w->hs);
    delete w;
    return FGS_OK;
}

fgs_status fgs_window_step(fgs_window *w, const fgs_gaussians *params, fgs_adam *opt, const fgs_target *targets,
                           const fgs_render_opts *o, const fgs_loss_opts *l, float *loss_dev, float *psnr_dev,
                           const fgs_gaussians *grad_out, int32_t use_graph)
{
    const char *w_ = "fgs_window_step";
    if (!w) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: window is NULL", w_);
    fgs_ctx *ctx = w->ctx;
    int tw, th;
    fgs_status st;
    if ((st = check_gauss(ctx, params, w_, "params")) != FGS_OK) return st;
    if ((st = check_adam(ctx, opt, params->n, w_)) != FGS_OK) return st;
    if ((st = check_opts(ctx, o, w_, &tw, &th)) != FGS_OK) return st;
    if (!targets) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: targets is NULL", w_);
    for (int v = 0; v < w->nv; ++v)
        if (!targets[v].rgb || !targets[v].depth)
            return fail(ctx, FGS_ERR_INVALID_ARG, "%s: target %d has a NULL plane", w_, v);
    if (!l || !std::isfinite(l->lambda_rgb) || !std::isfinite(l->lambda_depth))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: loss options NULL or not finite", w_);
    if (l->lambda_rgb != 1.0f || l->lambda_reg != 0.0f || l->reg_dev)
        return fail(ctx, FGS_ERR_UNSUPPORTED,
                    "%s: the window takes the L1 terms only (lambda_rgb = 1, lambda_reg = 0, no reg_dev); use "
                    "fgs_map_step for the SSIM term and the scale regulariser", w_);
    if (grad_out) {
        if ((st = check_gauss(ctx, grad_out, w_, "grad_out")) != FGS_OK) return st;
        if (grad_out->n != params->n) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: grad_out.n != params.n", w_);
    }
    // a step already run that outgrew the window's pair capacity changed no parameter, moment or
    // device step count: opt->step is set back to that count, the window grows, and the caller
    // hears of it once
    if (((volatile uint32_t *)w->hs)[1]) {
        HIP_TRY(ctx, hipStreamSynchronize(w->stream));  // the flag and count are final now
        volatile uint32_t *hs = w->hs;
        const int64_t K = hs[0];
        hs[0] = 0;
        hs[1] = 0;
        w->cap_all = std::max<int64_t>(w->cap_all, K + K / 2 + 1024);
        // the context's own overflow word saw the same event; this report replaces it
        HIP_TRY(ctx, hipMemsetAsync(ctx->words.as<uint32_t>() + ST_OVERFLOW, 0, 4, w->stream));
        HIP_TRY(ctx, hipMemcpyAsync(w->step_host, w->words.as<char>() + 4 * WW_STEP, 8, hipMemcpyDeviceToHost,
                                    w->stream));
        HIP_TRY(ctx, hipStreamSynchronize(w->stream));
        if (w->dev_step >= 0) opt->step = *w->step_host;
        w->dev_step = opt->step;
        w->n = -1;  // the next step resizes
        return fail(ctx, FGS_ERR_CAPACITY,
                    "%s: an earlier step needed %lld pairs over its views and was not applied (parameters, moments "
                    "and step count unchanged); the window has grown, repeat that step", w_, (long long)K);
    }
    hipStream_t user = ctx->stream;
    HIP_TRY(ctx, hipEventRecord(w->ev_in, user));
    HIP_TRY(ctx, hipStreamWaitEvent(w->stream, w->ev_in, 0));
    ctx->stream = w->stream;
    struct Rebind {
        fgs_ctx *c;
        hipStream_t s;
        ~Rebind() { c->stream = s; }
    } rebind{ctx, user};
    if (params->n != w->n && (st = window_size(w, *params, *o)) != FGS_OK) return st;
    if ((st = window_tables(w, *params, *o, targets, *l)) != FGS_OK) return st;
    const int64_t dev_step = w->dev_step;
    w->dev_step = -1;  // unknown until this step is enqueued whole
    if (opt->step != dev_step) {  // the device counter follows the host's
        HIP_TRY(ctx, hipStreamSynchronize(w->stream));
        *w->step_host = opt->step;
        HIP_TRY(ctx, hipMemcpyAsync(w->words.as<char>() + 4 * WW_STEP, w->step_host, 8, hipMemcpyHostToDevice,
                                    w->stream));
    }
    if (use_graph && ctx->prof) use_graph = 0;  // profiled steps run eagerly
    if (use_graph) {
        std::vector<uintptr_t> sig = w->table_sig;
        sig.push_back((uintptr_t)ctx->ws_gen);  // the context's sort and binning buffers are baked in
        const void *ptrs[] = {params->mean, params->log_scale, params->quat, params->opacity_logit, params->rgb,
                              opt->m.mean, opt->m.log_scale, opt->m.quat, opt->m.opacity_logit, opt->m.rgb,
                              opt->v.mean, opt->v.log_scale, opt->v.quat, opt->v.opacity_logit, opt->v.rgb,
                              loss_dev, psnr_dev};
        for (const void *q : ptrs) sig.push_back((uintptr_t)q);
        sig.push_back((uintptr_t)params->stride);
        sig.push_back((uintptr_t)opt->m.stride);
        sig.push_back((uintptr_t)opt->v.stride);
        if (grad_out) {
            const void *gp[] = {grad_out->mean, grad_out->log_scale, grad_out->quat, grad_out->opacity_logit,
                                grad_out->rgb};
            for (const void *q : gp) sig.push_back((uintptr_t)q);
            sig.push_back((uintptr_t)grad_out->stride);
        } else {
            sig.push_back(0);
        }
        for (int v = 0; v < w->nv; ++v) {
            sig.push_back((uintptr_t)targets[v].rgb);
            sig.push_back((uintptr_t)targets[v].depth);
        }
        uint32_t fb[10];
        memcpy(&fb[0], &l->lambda_rgb, 4);
        memcpy(&fb[1], &l->lambda_depth, 4);
        memcpy(&fb[2], opt->lr, 20);
        memcpy(&fb[7], &opt->beta1, 4);
        memcpy(&fb[8], &opt->beta2, 4);
        memcpy(&fb[9], &opt->eps, 4);
        for (uint32_t x : fb) sig.push_back(x);
        if (!w->exec || sig != w->sig) {
            window_drop_graph(w);
            HIP_TRY(ctx, hipStreamBeginCapture(w->stream, hipStreamCaptureModeThreadLocal));
            st = window_enqueue(w, *params, *opt, targets, *o, *l, loss_dev, psnr_dev, grad_out);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(w->stream, &g);
            if (st != FGS_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return fail(ctx, FGS_ERR_HIP, "%s: capture: %s", w_, hipGetErrorString(e));
            w->graph = g;
            const hipError_t e2 = hipGraphInstantiate(&w->exec, g, nullptr, nullptr, 0);
            if (e2 != hipSuccess) {
                window_drop_graph(w);
                return fail(ctx, FGS_ERR_HIP, "%s: instantiate: %s", w_, hipGetErrorString(e2));
            }
            w->sig = sig;
        }
        const hipError_t e = hipGraphLaunch(w->exec, w->stream);
        if (e != hipSuccess) return fail(ctx, FGS_ERR_HIP, "%s: graph launch: %s", w_, hipGetErrorString(e));
    } else if ((st = window_enqueue(w, *params, *opt, targets, *o, *l, loss_dev, psnr_dev, grad_out)) != FGS_OK) {
        return st;
    }
    HIP_TRY(ctx, hipEventRecord(w->ev_out, w->stream));
    HIP_TRY(ctx, hipStreamWaitEvent(user, w->ev_out, 0));
    opt->step += 1;
    w->dev_step = opt->step;
    return FGS_OK;
}

}  // extern "C"

/* ------------------------------------ GICP tracking ------------------------------------ */

struct fgs_cloud {
    fgs_ctx *ctx = nullptr;
    int64_t n = 0;
    int32_t k = 0;
    GridK grid{};
    int64_t cells = 0;
    DBuf xyz, pts, ranges, cov, knn;
};

namespace {

// Gauss-Newton iterations enqueued before the first and between later reads of the done flag.
constexpr int kGicpFirstBatch = 4, kGicpBatch = 2;

// Grows a context buffer after the stream has drained (work in flight may still use the old one).
hipError_t grow(fgs_ctx *ctx, DBuf &b, size_t bytes)
{
    if (bytes <= b.bytes && b.p) return hipSuccess;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? b.ensure(bytes) : e;
}

bool finite_pose(const double *T)
{
    for (int q = 0; q < 16; ++q)
        if (!std::isfinite(T[q])) return false;
    return true;
}

fgs_status gicp_setup(fgs_ctx *ctx, const fgs_cloud *src, const fgs_cloud *tgt, const double *T, float d_max,
                      const char *w, GicpK *K)
{
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    if (!src || !tgt) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: source or target cloud is NULL", w);
    if (!T || !finite_pose(T)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: pose is NULL or not finite", w);
    if (!(d_max > 0.0f) || !std::isfinite(d_max)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: d_max must be > 0", w);
    const double rings = floor((double)d_max / (double)tgt->grid.c + (double)tgt->grid.margin) + 1.0;
    if (rings > 8.0)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: d_max %g spans more than 8 cells of the target grid (cell %g)", w,
                    (double)d_max, (double)tgt->grid.c);
    K->g = tgt->grid;
    K->ranges = tgt->ranges.as<uint2>();
    K->tpts = tgt->pts.as<float4>();
    K->tx = tgt->xyz.as<float>();
    K->ty = K->tx + tgt->n;
    K->tz = K->tx + 2 * tgt->n;
    K->tcov = tgt->cov.as<double>();
    K->nt = tgt->n;
    K->sx = src->xyz.as<float>();
    K->sy = K->sx + src->n;
    K->sz = K->sx + 2 * src->n;
    K->scov = src->cov.as<double>();
    K->ns = src->n;
    K->dm2 = d_max * d_max;
    K->rings = (int32_t)rings;
    HIP_TRY(ctx, grow(ctx, ctx->gicp_state, sizeof(GicpState)));
    HIP_TRY(ctx, grow(ctx, ctx->gicp_part, (size_t)std::max<int64_t>(gicp_partials(src->n), 1) * 29 * 8));
    double R[9], t[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R[3 * r + c] = T[4 * r + c];
        t[r] = T[4 * r + 3];
    }
    launch_gicp_init(ctx->gicp_state.as<GicpState>(), R, t, ctx->stream);
    return FGS_OK;
}

}  // namespace

extern "C" {

fgs_status fgs_frame_points(fgs_ctx *ctx, const float *depth, const fgs_camera *cam, const double *pose_wc,
                            int32_t stride, float depth_min, float depth_max, float *xyz, int64_t capacity,
                            int64_t *n_dev, int64_t *n_host)
{
    const char *w = "fgs_frame_points";
    fgs_status st;
    if ((st = check_camera(ctx, cam, w)) != FGS_OK) return st;
    if (!depth) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: depth is NULL", w);
    if (stride <= 0) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: stride must be positive", w);
    if (capacity < 0 || (capacity > 0 && !xyz)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: bad output", w);
    if (std::isnan(depth_min) || std::isnan(depth_max))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: depth range is NaN", w);
    if (pose_wc && !finite_pose(pose_wc)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: pose not finite", w);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    FrameK f{};
    f.depth = depth;
    f.W = cam->width;
    f.H = cam->height;
    f.stride = stride;
    f.fx = cam->fx;
    f.fy = cam->fy;
    f.cx = cam->cx;
    f.cy = cam->cy;
    f.dmin = depth_min;
    f.dmax = depth_max;
    f.has_pose = pose_wc != nullptr;
    if (pose_wc)
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) f.R[3 * r + c] = (float)pose_wc[4 * r + c];
            f.t[r] = (float)pose_wc[4 * r + 3];
        }
    const int rows = (cam->height + stride - 1) / stride;
    HIP_TRY(ctx, grow(ctx, ctx->fp_rows, (size_t)rows * 4 + 8));
    int64_t *cnt = n_dev ? n_dev : ctx->fp_rows.as<int64_t>();
    uint32_t *row_count = ctx->fp_rows.as<uint32_t>(8);
    launch_frame_points(f, row_count, xyz, capacity, cnt, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    if (n_host) {
        int64_t v = -1;
        HIP_TRY(ctx, hipMemcpyAsync(&v, cnt, 8, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        *n_host = v;
        if (v > capacity)
            return fail(ctx, FGS_ERR_CAPACITY, "%s: %lld points, capacity %lld", w, (long long)v, (long long)capacity);
    }
    return FGS_OK;
}

fgs_status fgs_cloud_create(fgs_ctx *ctx, int64_t n, int64_t stride, const float *xyz, const fgs_cloud_opts *o,
                            fgs_cloud **out)
{
    const char *w = "fgs_cloud_create";
    if (!out) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: out is NULL", w);
    *out = nullptr;
    if (!o) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: options are NULL", w);
    if (o->k < 3 || o->k > 32) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: k must be in [3, 32]", w);
    if (n < o->k || n > ((int64_t)1 << 30))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: n = %lld outside [k, 2^30]", w, (long long)n);
    if (stride < n || !xyz) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: xyz is NULL or stride < n", w);
    if (!(o->cell > 0.0f) || !std::isfinite(o->cell)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: cell must be > 0", w);
    if (!(o->eps > 0.0 && o->eps <= 1.0)) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: eps must be in (0, 1]", w);
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: ctx is NULL", w);
    fgs_cloud *c = new (std::nothrow) fgs_cloud();
    if (!c) return fail(ctx, FGS_ERR_HIP, "%s: out of host memory", w);
    std::unique_ptr<fgs_cloud> own(c);
    c->ctx = ctx;
    c->n = n;
    c->k = o->k;
    hipStream_t s = ctx->stream;
    HIP_TRY(ctx, c->xyz.ensure((size_t)n * 3 * 4));
    for (int r = 0; r < 3; ++r)
        HIP_TRY(ctx, hipMemcpyAsync(c->xyz.as<float>() + r * n, xyz + r * stride, (size_t)n * 4,
                                    hipMemcpyDeviceToDevice, s));
    const float *X = c->xyz.as<float>(), *Y = X + n, *Z = X + 2 * n;
    // bounding box -> grid
    // cl_box: the box and the non-finite count (7 floats, padded to 8), the partial results, then
    // the point count for the sort
    HIP_TRY(ctx, grow(ctx, ctx->cl_box, ((size_t)8 + (size_t)bbox_partials() + 8) * 4));
    float *box = ctx->cl_box.as<float>();
    uint32_t *ndev = (uint32_t *)(box + 8 + bbox_partials());
    launch_bbox(X, Y, Z, n, box + 8, box, s);
    float hb[7];
    HIP_TRY(ctx, hipMemcpyAsync(hb, box, 28, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (hb[6] != 0.0f)
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: %.0f points have a non-finite coordinate", w, (double)hb[6]);
    for (int q = 0; q < 6; ++q)
        if (!std::isfinite(hb[q])) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: points are not finite", w);
    const double cell = (double)o->cell;
    GridK &g = c->grid;
    g.c = o->cell;
    g.inv_c = 1.0f / o->cell;
    g.ox = (float)(hb[0] - 0.5 * cell);
    g.oy = (float)(hb[1] - 0.5 * cell);
    g.oz = (float)(hb[2] - 0.5 * cell);
    const double dims[3] = {floor(((double)hb[3] - g.ox) / cell) + 2.0, floor(((double)hb[4] - g.oy) / cell) + 2.0,
                            floor(((double)hb[5] - g.oz) / cell) + 2.0};
    const double cells = dims[0] * dims[1] * dims[2];
    if (cells > (double)((int64_t)1 << 25))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: %.0f grid cells of %g over the cloud's extent (at most 2^25)", w,
                    cells, cell);
    g.gx = (int32_t)dims[0];
    g.gy = (int32_t)dims[1];
    g.gz = (int32_t)dims[2];
    c->cells = (int64_t)cells;
    const double gmax = std::max(dims[0], std::max(dims[1], dims[2]));
    g.margin = (float)(1e-3 + 6.0 * ldexp(1.0, -24) * gmax);
    // points sorted by cell
    const int G = sort_blocks(n, kPairSortPerBlock);
    HIP_TRY(ctx, grow(ctx, ctx->cl_sort, (size_t)n * 5 * 4 + 16));
    HIP_TRY(ctx, grow(ctx, ctx->cl_hist, ((size_t)G * 256 + 256) * 4));
    uint32_t *ka = ctx->cl_sort.as<uint32_t>(), *va = ka + n, *kb = va + n, *vb = kb + n, *vf = vb + n;
    HIP_TRY(ctx, hipMemsetD32Async((hipDeviceptr_t)ndev, (int)n, 1, s));
    launch_cell_keys(g, X, Y, Z, n, ka, va, s);
    SortWS sws;
    sws.G = G;
    sws.hist = ctx->cl_hist.as<uint32_t>();
    sws.totals = sws.hist + (size_t)G * 256;
    int bits = 1;
    while (((int64_t)1 << bits) < c->cells) ++bits;
    uint32_t *sk = launch_radix_sort(ka, va, kb, vb, vf, ndev, n, bits, sws, s);
    HIP_TRY(ctx, c->ranges.ensure((size_t)c->cells * sizeof(uint2)));
    launch_ranges(sk, ndev, c->ranges.as<uint2>(), c->cells, 0xffffffffu, s);
    HIP_TRY(ctx, c->pts.ensure((size_t)n * sizeof(float4)));
    launch_gather_cells(vf, X, Y, Z, n, c->pts.as<float4>(), s);
    HIP_TRY(ctx, c->cov.ensure((size_t)n * 6 * 8));
    if (o->keep_knn) HIP_TRY(ctx, c->knn.ensure((size_t)n * o->k * 4));
    launch_knn_cov(g, c->ranges.as<uint2>(), c->pts.as<float4>(), n, o->k, o->eps, X, Y, Z,
                   o->keep_knn ? c->knn.as<int32_t>() : nullptr, c->cov.as<double>(), s);
    HIP_TRY(ctx, hipGetLastError());
    *out = own.release();
    return FGS_OK;
}

fgs_status fgs_cloud_destroy(fgs_cloud *c)
{
    if (!c) return FGS_OK;
    if (c->ctx) (void)hipStreamSynchronize(c->ctx->stream);
    delete c;
    return FGS_OK;
}

fgs_status fgs_cloud_read(const fgs_cloud *c, double *cov, int32_t *knn, int64_t *n_out, int32_t *k_out)
{
    const char *w = "fgs_cloud_read";
    if (!c) return fail(nullptr, FGS_ERR_INVALID_ARG, "%s: cloud is NULL", w);
    fgs_ctx *ctx = c->ctx;
    if (knn && !c->knn.p) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: the cloud kept no neighbour lists", w);
    if (n_out) *n_out = c->n;
    if (k_out) *k_out = c->k;
    if (cov) HIP_TRY(ctx, hipMemcpyAsync(cov, c->cov.p, (size_t)c->n * 6 * 8, hipMemcpyDeviceToDevice, ctx->stream));
    if (knn)
        HIP_TRY(ctx, hipMemcpyAsync(knn, c->knn.p, (size_t)c->n * c->k * 4, hipMemcpyDeviceToDevice, ctx->stream));
    return FGS_OK;
}

fgs_status fgs_gicp_linearize(fgs_ctx *ctx, const fgs_cloud *source, const fgs_cloud *target, const double T[16],
                              float d_max, double *out, int32_t *corr)
{
    const char *w = "fgs_gicp_linearize";
    if (!out) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: out is NULL", w);
    GicpK K;
    fgs_status st = gicp_setup(ctx, source, target, T, d_max, w, &K);
    if (st != FGS_OK) return st;
    launch_gicp_iteration(K, ctx->gicp_state.as<GicpState>(), ctx->gicp_part.as<double>(), corr, 0, 1, 0.0, 0.0, out,
                          ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

fgs_status fgs_gicp_align(fgs_ctx *ctx, const fgs_cloud *source, const fgs_cloud *target, const double T_init[16],
                          const fgs_gicp_opts *o, fgs_gicp_result *result)
{
    const char *w = "fgs_gicp_align";
    if (!o || !result) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: options or result is NULL", w);
    if (o->max_iter < 1 || o->max_iter > 1000) return fail(ctx, FGS_ERR_INVALID_ARG, "%s: max_iter outside [1, 1000]", w);
    if (!(o->eps_rot >= 0.0) || !(o->eps_trans >= 0.0))
        return fail(ctx, FGS_ERR_INVALID_ARG, "%s: eps_rot and eps_trans must be >= 0", w);
    GicpK K;
    fgs_status st = gicp_setup(ctx, source, target, T_init, o->d_max, w, &K);
    if (st != FGS_OK) return st;
    GicpState *sd = ctx->gicp_state.as<GicpState>();
    if (!ctx->gicp_host) HIP_TRY(ctx, hipHostMalloc(&ctx->gicp_host, sizeof(GicpState), hipHostMallocDefault));
    {
        // Iterations are enqueued a few at a time and the done flag is read back between batches:
        // once the pose has converged the rest of the iterations are not launched at all (each
        // would still cost two launches that find the flag set).
        Stage st_(ctx, "gicp");
        int launched = 0;
        volatile int32_t *done_host = &((GicpState *)ctx->gicp_host)->done;
        while (launched < o->max_iter) {
            const int batch = std::min(launched == 0 ? kGicpFirstBatch : kGicpBatch, o->max_iter - launched);
            for (int it = 0; it < batch; ++it)
                launch_gicp_iteration(K, sd, ctx->gicp_part.as<double>(), nullptr, 1, o->max_iter, o->eps_rot,
                                      o->eps_trans, nullptr, ctx->stream);
            launched += batch;
            if (launched >= o->max_iter) break;
            HIP_TRY(ctx, hipMemcpyAsync((void *)done_host, &sd->done, 4, hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            if (*done_host) break;
        }
    }
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->gicp_host, sd, sizeof(GicpState), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const GicpState &hs = *(const GicpState *)ctx->gicp_host;
    for (int q = 0; q < 16; ++q) result->T[q] = 0.0;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) result->T[4 * r + c] = hs.R[3 * r + c];
        result->T[4 * r + 3] = hs.t[r];
    }
    result->T[15] = 1.0;
    result->iterations = hs.iters;
    result->status = hs.status;
    result->correspondences = hs.count;
    result->cost = hs.cost;
    return FGS_OK;
}

}  // extern "C"

