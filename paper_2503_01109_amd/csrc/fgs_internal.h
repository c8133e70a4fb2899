// Internal declarations of the FGS HIP library (gfx950): device helpers, kernel launchers,
// and the layout of a forward state. Not part of the public ABI (include/fgs.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fgs {

constexpr int kWave = 64;

// Camera and cutoffs as kernel arguments (by value). Projection runs in FP64, so the pose and
// intrinsics are carried in double.
struct CamK {
    int32_t W, H;
    double fx, fy, cx, cy;
    double R[9];
    double t[3];
    double z_near;
};

struct RasterK {
    float sigma_cut, alpha_min, alpha_max, T_min, lowpass;
    float bg[3];
    float bg_depth;
    int32_t tile_w, tile_h, tiles_x, tiles_y, supers_x;
};

// Tiles are grouped in super-tiles of kSuper x kSuper and numbered super-tile-major: item
// g = kSuper^2 s + kSuper ly + lx is tile (kSuper (s % supers_x) + lx, kSuper (s / supers_x) + ly);
// items beyond the image's tiles have empty lists. Tile ranges, rasterizer grids and window items
// all use this numbering.
constexpr int kSuper = 4, kSuperShift = 2;
// super-tile keys carry the entry's coverage box (4 x 2 bits) above bit kBoxShift; the super-tile
// index itself stays below 2^kBoxShift (at most 64 views of at most 2^18 super-tiles)
constexpr int kBoxShift = 24;
constexpr uint32_t kSuperKeyMask = (1u << kBoxShift) - 1u;
inline int32_t supers_for(int32_t tiles) { return (tiles + kSuper - 1) / kSuper; }
inline int64_t tile_items(int32_t tiles_x, int32_t tiles_y)
{
    return (int64_t)supers_for(tiles_x) * supers_for(tiles_y) * kSuper * kSuper;
}

// 2D gradients of one view: one record of kG2Stride floats per gaussian id, terms d/d(mean2 x, y;
// conic a, b, c; opacity; r, g, b; depth) in slots 0..9, the rest padding (a record is one 64-byte
// line, so the rasterizer's atomics for one gaussian land in one line).
constexpr int kG2Stride = 16;

// Gaussian parameter planes (device).
struct ParamsK {
    int64_t n, stride;
    const float *mean, *log_scale, *quat, *logit, *rgb;
};
struct GradK {
    int64_t n, stride;
    float *mean, *log_scale, *quat, *logit, *rgb;
};

// Projected record of one gaussian, 3 x float4, by gaussian id inside a forward state:
//  r0 = {ix, iy (int bits), fx, fy}: the projected mean as integer pixel + fraction
//  r1 = {conic a, conic b, conic c, opacity}
//  r2 = {r, g, b, depth}
struct Rec {
    float4 r0, r1, r2;
};

// Device status words of a context.
enum : int {
    ST_PAIRS = 0,      // (tile, gaussian) pairs of the last forward (may exceed capacity)
    ST_VISIBLE = 1,    // gaussians kept by the last forward
    ST_OVERFLOW = 2,   // largest pair count that did not fit (sticky until checked)
    ST_SEEDS = 3,      // seeds found by the last seeding (may exceed capacity)
    ST_SEED_OVF = 4,   // largest seed count that did not fit (sticky)
    ST_WORDS = 16
};

// Layout of a forward state (one view). Everything the backward needs lives here; temporaries
// live in the context's workspace.
struct StateLayout {
    int64_t n = 0, P = 0, T = 0;
    int32_t W = 0, H = 0, tw = 0, th = 0, tiles_x = 0, tiles_y = 0;
    size_t off_rec = 0;    // Rec x n, by gaussian id
    size_t off_ranges = 0; // uint2 x T: [start, end) into vals per tile item (super-tile-major)
    size_t off_last = 0;   // u32 x P: list position after a pixel's last blended gaussian
    size_t off_tfinal = 0; // f32 x P: final transmittance
    size_t off_vals = 0;   // u32 x cap: gaussian ids, per tile in (depth, index) order
    int64_t cap = 0;
    size_t fixed = 0, bytes = 0;
};

bool state_layout(int64_t n, int32_t W, int32_t H, int32_t tw, int32_t th, int64_t max_pairs,
                  StateLayout *L);
// Capacity of a state of `bytes` bytes (pairs that fit), or -1 when even the fixed part does not.
int64_t state_capacity(int64_t n, int32_t W, int32_t H, int32_t tw, int32_t th, int64_t bytes,
                       StateLayout *L);

// ---------------------------------- launchers ----------------------------------
// All take the stream last and only enqueue work.

struct SortWS {  // radix-sort scratch of one sort
    uint32_t *hist;    // 256 x G
    uint32_t *totals;  // 256
    int G;
};
// Radix-sort grid for up to cap elements at about per_block elements per workgroup (1..4096
// workgroups). Any grid sorts correctly: each workgroup takes a contiguous share of the actual
// element count. The depth sort (n known on the host) uses small shares so that every compute
// unit takes part; pair sorts are sized from their capacity and use larger ones. The super-tile
// sort of one view is sized at 8,192 per workgroup of its capacity: its keys number about a
// sixth of the capacity (a quarter of the tile pairs, with 50% headroom), so a workgroup takes
// some 1,300 of them (measured: 3% faster per mapping step than 2,048 per workgroup).
constexpr int kDepthSortPerBlock = 512, kPairSortPerBlock = 2048, kSuperSortPerBlock = 8192;
int sort_blocks(int64_t cap, int per_block);

void launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);
void launch_zero_f32(float *p, int64_t n, hipStream_t s);

// Projects every gaussian into rec (by id: the forward state's records); writes the depth key
// dkey[i] and ids[i] = id_base + i, and id_base + n to *n_out (the element count of the depth
// sort: views sorted together are projected into consecutive ranges). count[i] receives the
// number of tiles (shift 0) or super-tiles (tile rectangle >> shift) covered, rect[i] the tile
// rectangle; kpart (2 words per workgroup, project_blocks(n) workgroups) the workgroups'
// (tile, gaussian) pair and visible gaussian counts, summed by launch_scan_counts. reg_part
// (nullable, project_blocks(n) floats): each workgroup's sum of the scale regulariser's terms
// |s1 - s2| + s3 (s = exp(log-scale); Eq. 15). csum (nullable, project_blocks(n) words): each
// workgroup's sum of count[], the block sums of a scan of the counts in gaussian order (see
// launch_emit). shist (nullable; at most 256 super-tiles, supers_x per row; 256 x
// project_blocks(n) words): shist[s project_blocks(n) + b] = the number of workgroup b's gaussians
// that cover super-tile s (see launch_super_pairs).
int64_t project_blocks(int64_t n);
void launch_project(const ParamsK &g, const CamK &cam, const RasterK &rk, Rec *rec,
                    uint2 *rect, uint32_t *count, uint32_t *dkey, uint32_t *ids, uint32_t *n_out, int shift,
                    uint32_t *kpart, hipStream_t s, uint32_t id_base = 0, float *reg_part = nullptr,
                    uint32_t *csum = nullptr, uint32_t *shist = nullptr, int supers_x = 0);

// LSD radix sort of (key, value) pairs over key bits [0, key_bits) with 8-bit digits; the
// element count is read from *n_dev (clamped to n_cap). Ping-pongs between (ka, va) and
// (kb, vb); the last pass writes the values to v_final and the keys to the returned buffer.
uint32_t *launch_radix_sort(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, uint32_t *v_final,
                            const uint32_t *n_dev, int64_t n_cap, int key_bits, const SortWS &ws,
                            hipStream_t s);

// Per-block sums of count[ids[r]] over ranks r (scan_blocks(n) words of blocksums, at most
// scan_blocks_cap(n) for any count up to n), the first half of the scan that launch_emit completes.
int64_t scan_blocks(int64_t n);
int64_t scan_blocks_cap(int64_t n);
void launch_scan_counts(const uint32_t *ids, const uint32_t *count, int64_t n, uint32_t *blocksums, hipStream_t s);

// Completes the scan (each block adds the block sums before it) and emits one (key, gaussian id)
// pair per covered tile in the order of ids (rank r: gaussian ids[r]); with shift > 0 the keys are
// super-tiles (tile rectangle >> shift, keys_x super-tiles per row) and carry, above bit
// kBoxShift, the box of the super-tile's tiles that the gaussian covers. Several views binned at
// once (view_tab non-null): ids are values v view_n + i, view v's keys are view_tab[v].y + its
// own key with view_tab[v].x keys per row (keys_x unused), and the value emitted is i. offsets is scratch of n + 1
// words (per-rank exclusive offsets). If the pairs exceed cap, nothing is emitted for sorting
// (*n_pairs_dev = 0) and the required count is recorded in status. host_status (nullable,
// host-mapped): [0] = pairs, [1] |= overflow. rect_sorted (n) receives the tile rectangles in
// rank order, start_rank (emit_chunks(cap) words) the first rank of every emission chunk. The
// projection's per-workgroup counts kpart (proj_blocks workgroups) are summed into *ktotal and
// status[ST_PAIRS] ((tile, gaussian) pairs) and status[ST_VISIBLE]. csum (nullable): the
// projection's per-workgroup sums of count[] when ids is the identity (ranks in gaussian order),
// used as the scan's block sums in place of launch_scan_counts' (which then need not run); it is
// scanned in place when there are more than 4,096 scan blocks.
int64_t emit_chunks(int64_t cap);
void launch_emit(const uint32_t *ids, const uint32_t *count, const uint2 *rect, uint32_t *blocksums,
                 uint32_t *offsets, int64_t n, int32_t keys_x, int shift, int64_t cap, uint32_t *keys, uint32_t *vals,
                 uint2 *rect_sorted, uint32_t *start_rank, uint32_t *status, uint32_t *n_pairs_dev,
                 uint32_t *host_status, const uint32_t *kpart, int64_t proj_blocks, uint32_t *ktotal, hipStream_t s,
                 const uint2 *view_tab = nullptr, uint32_t view_n = 0, uint32_t *csum = nullptr);

// Tile lists from super-tile lists (kSuper x kSuper tiles per super-tile). The gaussians' pairs
// are emitted per covered super-tile (launch_emit with shift log2(kSuper)), sorted by the key bits
// below kBoxShift into (skeys, svals) with ranges sranges; then:
//   launch_bin_counts: chunk table and per-chunk tile counts;
//   launch_bin_tiles:  prefixes over chunks and tiles, the tile ranges, and the capacity check of
//                      K = *ktotal pairs (status, n_pairs_dev, host_status; empty ranges on
//                      overflow). step_ovf (nullable) is the overflow word of a mapping step
//                      whose views are binned one after another: the step's first binning
//                      writes 0 or 1 to it, later ones set it to 1 on overflow;
//   launch_bin_place:  every entry's gaussian id into the lists of its tiles (vals, K entries).
// The tiles an entry covers come from the box in its key.
struct BinWS {
    uint32_t *cstart;      // nsup + 1
    uint32_t *csuper;      // max_chunks
    uint32_t *chist;       // max_chunks x kSuper^2
    uint32_t *tile_total;  // T
    uint32_t *nchunks;     // 1 word
    uint32_t *ok;          // 1 word
    uint32_t *vpart;       // kBinGrid: valid target-depth pixels per counting workgroup
    int64_t max_chunks;
};
constexpr int kBinGrid = 4096;  // workgroups of the expansion kernels (each loops over chunks)
int64_t bin_max_chunks(int64_t cap, int64_t nsup);
// digit_totals (nullable): the per-digit totals of a single-pass super-tile sort, from which the
// super-tile ranges are written into sranges; else sranges holds them already.
void launch_bin_counts(const BinWS &b, const uint32_t *skeys, uint2 *sranges, const uint32_t *digit_totals, int nsup,
                       hipStream_t s);
// The two halves of launch_bin_counts: the chunk table (and sranges from digit_totals; with
// sstart non-null, also the first depth-order chunk of every super-tile list, nsup + 1 words,
// followed by the super-tile of each of the at most smax depth-order chunks), then the per-chunk
// tile counts.
void launch_bin_chunks(const BinWS &b, uint2 *sranges, const uint32_t *digit_totals, int nsup, hipStream_t s,
                       uint32_t *sstart = nullptr, int64_t smax = 0, const uint32_t *ktotal = nullptr,
                       int64_t cap = 0);
// Super-tile lists of one view with at most 256 super-tiles, straight from the projection
// (launch_project with shist): launch_super_scan scans the per-workgroup super-tile counts hist
// (256 x project_blocks(n) words) over the workgroups in place, writes the super-tile totals
// (256 words) and sums the projection's counts kpart (into *ktotal, status[ST_PAIRS] and
// status[ST_VISIBLE], as launch_emit does); launch_super_scatter then writes every covered
// super-tile's (key with box, gaussian id) pair to (keys, vals), each super-tile's list in
// gaussian order, or nothing when *ktotal exceeds cap, and writes what launch_bin_chunks would
// (the ranges sranges, the chunk table of b and sstart; empty lists on overflow).
void launch_super_scan(int64_t n, uint32_t *hist, uint32_t *totals, const uint32_t *kpart, uint32_t *status,
                       uint32_t *ktotal, hipStream_t s);
void launch_super_scatter(const uint2 *rect, const uint32_t *count, int64_t n, int32_t supers_x, const uint32_t *hist,
                          const uint32_t *totals, const uint32_t *ktotal, int64_t cap, uint32_t *keys, uint32_t *vals,
                          const BinWS &b, uint2 *sranges, int nsup, uint32_t *sstart, int64_t smax, hipStream_t s);
// With tdepth set (P target depths of the view), the count also sums the valid pixels of the
// mapping loss's depth term per workgroup, and launch_bin_tiles with dscale set turns them into
// the term's scale 1/P_v before the rasterizer runs.
void launch_bin_count(const BinWS &b, const uint32_t *skeys, const uint2 *sranges, hipStream_t s,
                      const float *tdepth = nullptr, int64_t P = 0);
// Depth order inside every super-tile list: (kin, vin) hold the lists in ascending gaussian id
// (ranges sranges, nsup lists, chunk table sstart from launch_bin_chunks); each list is written
// to (kout, vout) at the same place, stably reordered by dkey[gaussian id] (so in (depth, id)
// order). t[0..5] (as many words as the pairs each) hold the sorted chunks of lists longer than
// one chunk (depth keys, gaussian ids, super-tile keys, and a second set for merge levels in
// global memory) while they are merged. max_chunks = seg_max_chunks(pair capacity, nsup).
int64_t seg_max_chunks(int64_t cap, int64_t nsup);
void launch_seg_sort(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, const uint2 *sranges,
                     const uint32_t *sstart, int nsup, int64_t max_chunks, const uint32_t *dkey, uint32_t *const t[6],
                     hipStream_t s);
void launch_bin_tiles(const BinWS &b, int nsup, int64_t cap, const uint32_t *ktotal, uint2 *ranges, uint32_t *status,
                      uint32_t *n_pairs_dev, uint32_t *host_status, uint32_t *step_ovf, bool first_of_step,
                      hipStream_t s, float *dscale = nullptr);
void launch_bin_place(const BinWS &b, const uint32_t *skeys, const uint32_t *svals, const uint2 *sranges,
                      const uint2 *ranges, uint32_t *vals, hipStream_t s);

// [start, end) of the runs of keys 0..T-1 in the sorted keys (n_dev of them), comparing key & mask.
void launch_ranges(const uint32_t *keys, const uint32_t *n_dev, uint2 *ranges, int64_t T, uint32_t mask,
                   hipStream_t s);

struct ImageK {
    float *rgb, *depth, *alpha, *T_final;  // rgb, depth: nullable when the loss below is fused
    int32_t *n_contrib;
};

// The L1 terms of the mapping loss fused into the forward's per-pixel epilogue (partials ==
// nullptr: none). For each pixel: drgb = lrgb sgn(C - C*) inv3P per channel, ddepth = ldepth
// sgn(D - D*) where D* > 0 (else 0; the 1/P_v factor is applied by the backward); each tile's
// workgroup writes partials[4 tile + q] = its sums of |C - C*|, (C - C*)^2, |D - D*| over valid
// depth, and the valid-depth count, which launch_loss_final reduces.
struct LossK {
    const float *trgb, *tdepth;
    float *drgb, *ddepth, *partials;
    float *ddepth_scale;  // where the loss reduction of a window view writes its 1/P_v
    float lrgb, ldepth, inv3P;
};

// Everything the rasterizer needs for one view (kernel argument, or an entry of a device array
// for the persistent window kernels).
struct ViewK {
    RasterK rk;
    int32_t W, H;
    const Rec *rec;
    const uint32_t *vals;  // tile lists of gaussian ids
    const uint2 *ranges;
    uint32_t *last;
    float *tfinal;
    ImageK img;
    const float *drgb, *ddepth, *dalpha, *ddepth_scale;
    float *grad2d;
    unsigned long long *counts;
    LossK loss;
    uint32_t tile_base;  // index of this view's first tile in the window's item numbering
};

bool tile_supported(int tw, int th);
bool tile_supported_window(int tw, int th);

// Window rasterizer over the items g < total of all views (item g is tile g - views[v].tile_base
// of view v, views in order). blocks > 0: a persistent grid of that many workgroups pulls items
// through counter, zeroed first with a kernel so the sequence can be captured in a graph;
// blocks <= 0: one workgroup per item. count: the forward adds its work counters to
// views[v].counts (which must then be non-null).
void launch_raster_window(bool fwd, bool count, const ViewK *views_dev, int nv, uint32_t total, uint32_t *counter,
                          int blocks, hipStream_t s);

// counts (nullable, profiling): [0] += pairs within the cutoff examined before each pixel
// stopped, [1] += pairs blended, [2] += list entries staged, [3] += (tile, gaussian) entries that
// some pixel blended (K_c), [4] += per tile the list entries up to the last one a pixel examined
// (L_f), [5] += per tile the list entries up to the last blended one (L_b).
void launch_raster_fwd(const RasterK &rk, int32_t W, int32_t H, const Rec *rec, const uint32_t *vals,
                       const uint2 *ranges, uint32_t *last, float *tfinal, const ImageK &img, const LossK &loss,
                       unsigned long long *counts, hipStream_t s);

// dL planes: drgb 3 planes of P, ddepth P, dalpha P (nullable). ddepth_scale (nullable) points
// to a device float multiplying ddepth (the 1/P_v of the mean depth term). grad2d: records of
// kG2Stride floats by gaussian id (the tile lists hold ids). counts (nullable, profiling): [6] +=
// wave-entry evaluations (a wave evaluating one list entry for its 64 pixels), [7] += those in
// which some pixel blended, [8] += those in which 1 to 8 pixels blended, [9] += pairs blended.
void launch_raster_bwd(const RasterK &rk, int32_t W, int32_t H, const Rec *rec, const uint32_t *vals,
                       const uint2 *ranges, const uint32_t *last, const float *tfinal,
                       const float *drgb, const float *ddepth, const float *dalpha,
                       const float *ddepth_scale, float *grad2d, unsigned long long *counts, hipStream_t s);

// Adam hyper-parameters of an update fused into a projection backward. step (nullable) points
// to the device count of updates already applied (the kernel applies update *step + 1): bc1 and
// bc2 are the bias corrections of update step_expect + 1, used when *step == step_expect (the
// count the host expects) and recomputed otherwise; without step, bc1 and bc2 are used as given. skip (nullable) points to a step's
// overflow word: when it is non-zero the step's gradient is incomplete and no parameter or moment
// changes. step_out (nullable, not aliasing step) receives the count after this step: *step + 1,
// or *step when skipped (a captured window step advances its counter in a launch of its own).
struct AdamK {
    GradK m, v;
    const int64_t *step;
    int64_t step_expect;
    int64_t *step_out;
    const uint32_t *skip;
    float lr[5];
    float beta1, beta2, eps;
    float bc1, bc2;
    // scale regulariser of Eq. 15 applied with the update: reg_w = lambda_r / n (0: none)
    float reg_w;
};

// The structural-similarity term and the scale regulariser (Sec. III-D, Eq. 15 and 16) as reduced
// by launch_loss_final: ssim_part (ssim_nb per-tile sums of the index, nullable) adds
// ssim_w (1 - sum / (3 P)) to the loss; reg_part (reg_nb per-workgroup sums of |s1 - s2| + s3,
// nullable) gives reg_out = reg_scale sum (nullable).
struct LossExtraK {
    const float *ssim_part;
    int ssim_nb;
    float ssim_w;
    const float *reg_part;
    int reg_nb;
    float reg_scale;
    float *reg_out;
};

// A loss reduction handed to the projection backward (partials null: none): the nb per-tile
// quadruples of the fused forward loss of a W x H = P view with weights lrgb, ldepth (and the
// extra terms) into the device scalars loss and psnr (nullable), as launch_loss_final computes them.
struct LossFinalK {
    const float *partials;
    int nb;
    int64_t P;
    float lrgb, ldepth;
    float *loss, *psnr;
    LossExtraK extra;
};

// Chain rule from the 2D gradient records (by gaussian id) to the 14 parameter gradients of every
// gaussian: grad_out (nullable) = grad_in (nullable: an earlier views' sum) + this view's, and
// Adam (when adam.m.mean is set) applies that sum. grad2d is left zeroed. grad_in may equal
// grad_out (accumulation in place). With lf.partials set, one more workgroup reduces the view's
// loss (it reads nothing the gradient work writes).
void launch_project_bwd(const ParamsK &g, const CamK &cam, const RasterK &rk, float *grad2d, const GradK &grad_in,
                        const GradK &grad_out, const AdamK &adam, hipStream_t s, const LossFinalK &lf = LossFinalK{});


// Window backward: sums every view's 2D gradients through its projection per gaussian (view v's
// records at grad2d + v * view_stride, cleared after use), writes grad when grad.mean is set,
// and applies Adam when adam.m.mean is set.
void launch_project_bwd_window(const ParamsK &g, const CamK *cams_dev, int nv, float lowpass, float *grad2d,
                               int64_t view_stride, const GradK &grad, const AdamK &adam, hipStream_t s);

// L1 loss of Eq. 16 (colour + depth terms) with its gradient; partials is scratch of
// loss_partials_size(P) floats; writes loss/psnr device scalars (nullable) and the depth-gradient
// scale 1/P_v into *ddepth_scale.
int64_t loss_partials_size(int64_t P);
// Reduction of nb partial quadruples (as written by the fused forward loss) into loss, psnr and
// the depth term's 1/P_v (all device scalars, nullable).
void launch_loss_final(const float *partials, int nb, int64_t P, float lrgb, float ldepth, float *ddepth_scale,
                       float *loss, float *psnr, hipStream_t s, const LossExtraK &extra = LossExtraK{});

// Structural similarity of img to tgt (3 planes of W x H each; Sec. III-D, Eq. 16): grad (3
// planes, nullable) = (accumulate ? grad : 0) + gscale d ssim / d img; partials (nullable,
// ssim_partials(W, H) floats): per channel and 32x32 tile the sum of the index over the tile's
// pixels; ws: ssim_ws_floats(W, H) floats of scratch.
int64_t ssim_partials(int32_t W, int32_t H);
int64_t ssim_ws_floats(int32_t W, int32_t H);
// *out = scale * the sum of n floats (one workgroup, FP64, fixed order)
void launch_sum_scaled(const float *a, int n, double scale, float *out, hipStream_t s);
void launch_ssim(int32_t W, int32_t H, const float *img, const float *tgt, float gscale, bool accumulate, float *grad,
                 float *partials, float *ws, hipStream_t s);
// The same for every view of a window at once (view v: its partials, tile count, pixel count,
// loss weights and 1/P_v slot from views_dev[v]; loss[v], psnr[v], nullable).
void launch_loss_final_views(const ViewK *views_dev, int nv, uint32_t total_items, float *loss, float *psnr,
                             hipStream_t s);
void launch_loss_l1(int64_t P, const float *rgb, const float *depth, const float *trgb,
                    const float *tdepth, float lrgb, float ldepth, float *drgb, float *ddepth,
                    float *ddepth_scale, float *partials, float *loss, float *psnr, hipStream_t s);

void launch_adam(const GradK &p, const ParamsK &g, const GradK &m, const GradK &v, const float lr[5],
                 float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s);

// *step += 1 on the device unless *skip (nullable) is non-zero (the Adam step counter a captured
// window step reads and advances; an overflowed step leaves it unchanged).
// Pruning (prune.hip): survivors have logit >= L_o and every log-scale <= L_s in the test planes;
// their columns of the n_planes source planes are packed in index order into the destination
// planes (which must not overlap the sources). keep (nullable): one byte per gaussian.
constexpr int kPruneSets = 4, kPrunePlanes = 14 * kPruneSets;
struct PruneK {
    int64_t n;
    float L_o, L_s;
    const float *logit, *ls0, *ls1, *ls2;  // the test planes
    int32_t n_planes;
    const float *src[kPrunePlanes];
    float *dst[kPrunePlanes];
    uint8_t *keep;
};
int64_t prune_chunks(int64_t n);
// Workspace of launch_prune in 32-bit words for n gaussians.
int64_t prune_ws_words(int64_t n);
// ws: prune_ws_words(n) words (256-byte aligned); total: the survivor count (int64, device), also
// written to total_out when that is not null.
void launch_prune(const PruneK &k, uint32_t *ws, int64_t *total, int64_t *total_out, hipStream_t s);
// ---------------------------- GICP tracking (gicp.hip) ----------------------------
// Lattice points of a depth frame (Sec. III-B): row_count holds one word per lattice row.
struct FrameK {
    const float *depth;
    int32_t W, H, stride;
    float fx, fy, cx, cy, dmin, dmax;
    int32_t has_pose;
    float R[9], t[3];  // camera to world
};
void launch_frame_points(const FrameK &f, uint32_t *row_count, float *xyz, int64_t capacity, int64_t *n_dev,
                         hipStream_t s);
// Uniform grid of cubic cells: cell (floor((x - ox) inv_c), ...) in binary32, dims gx, gy, gz;
// margin: the slack in cells of that rounding plus the distances', kept off every ring bound.
struct GridK {
    float ox, oy, oz, inv_c, c;
    int32_t gx, gy, gz;
    float margin;
};
int bbox_partials();  // floats of launch_bbox's partial results
// min x, y, z, max x, y, z of n points and (as a float) the number of points with a non-finite
// coordinate into out (7 floats); part: bbox_partials() floats.
void launch_bbox(const float *x, const float *y, const float *z, int64_t n, float *part, float *out, hipStream_t s);
void launch_cell_keys(const GridK &g, const float *x, const float *y, const float *z, int64_t n, uint32_t *keys,
                      uint32_t *vals, hipStream_t s);
// pts[r] = (x, y, z, index bits) of the point vals[r] (the points in cell order).
void launch_gather_cells(const uint32_t *vals, const float *x, const float *y, const float *z, int64_t n, float4 *pts,
                         hipStream_t s);
// k (<= 32) nearest neighbours of every point of the cloud and its plane-regularised covariance
// (6 FP64 planes of stride n, by point index); knn_out (nullable): [n][k] indices.
void launch_knn_cov(const GridK &g, const uint2 *ranges, const float4 *pts, int64_t n, int k, double eps,
                    const float *x, const float *y, const float *z, int32_t *knn_out, double *cov, hipStream_t s);
// Pose and progress of a Gauss-Newton alignment, on the device.
struct GicpState {
    double R[9], t[3];
    float R32[9], t32[3];
    int32_t done, iters, status, pad;
    int64_t count;
    double cost;
};
struct GicpK {
    GridK g;  // the target's grid
    const uint2 *ranges;
    const float4 *tpts;
    const float *tx, *ty, *tz;
    const double *tcov;
    int64_t nt;
    const float *sx, *sy, *sz;
    const double *scov;
    int64_t ns;
    float dm2;
    int32_t rings;  // search block of (2 rings + 1)^3 cells
};
int64_t gicp_partials(int64_t ns);  // partial sums of 29 doubles
// Starts an alignment at (R, t): not done, no iterations, status 1 (iteration limit).
void launch_gicp_init(GicpState *st, const double R[9], const double t[3], hipStream_t s);
// One Gauss-Newton iteration: correspondences and partial sums, then (update != 0) the solve and
// pose update in st, or (update == 0) only the totals into out (29 doubles, nullable otherwise).
void launch_gicp_iteration(const GicpK &k, GicpState *st, double *partials, int32_t *corr, int update, int max_iter,
                           double eps_rot, double eps_trans, double *out, hipStream_t s);
void launch_step_advance(int64_t *step, const uint32_t *skip, hipStream_t s);

}  // namespace fgs
