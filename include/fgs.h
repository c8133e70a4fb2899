/*
 * fgs.h - C ABI of the MI355X (gfx950) implementation of the mapping hot path of
 * "FGS-SLAM: Fourier-based Gaussian Splatting for Real-time SLAM with Sparse and
 * Dense Map Fusion" (arXiv 2503.01109).
 *
 * The library renders a set of 3D gaussians G{mu, S, R, alpha, c} (Sec. III) by front-to-
 * back alpha blending (Eq. 1, with gamma = colour, depth and 1), differentiates that
 * rendering, optimises the map against an RGB-D frame with the L1 colour and depth terms of
 * the mapping loss (Eq. 16) and Adam, and seeds new gaussians from a frame by the Fourier
 * high-pass analysis of Sec. III-A (Eq. 2-8, the triangle threshold, the missing-region check of
 * Eq. 9-10, Eq. 11).
 *
 * Conventions shared by every call:
 *  - Pointers are DEVICE pointers unless a parameter is marked [host].
 *  - The caller owns every buffer it passes; the library never frees them.
 *  - Gaussian parameters are SoA float32 planes. A block of k planes with plane stride s holds
 *    plane j at ptr + j*s. Quaternions are (w, x, y, z); scales are log-scales; opacity is a
 *    logit (opacity = sigmoid); colour is RGB without view dependence.
 *  - Images are float32 planes of width*height, row-major (index y*width + x). Pixel (x, y)
 *    samples the continuous point (x + 0.5, y + 0.5).
 *  - Every call enqueues its work on the context's HIP stream and returns without waiting;
 *    outputs are valid once that stream reaches the point of the call.
 *  - Argument checks run on the host before anything is enqueued; a rejected call enqueues
 *    nothing and returns FGS_ERR_INVALID_ARG. Conditions only the device can see (more
 *    (tile, gaussian) pairs than a buffer holds, more seeds than the output holds) are
 *    recorded on the device and reported by fgs_ctx_check. No C++ exception crosses the ABI.
 *  - A context is not thread-safe; use one context per host thread and stream.
 */
#ifndef FGS_H
#define FGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FGS_OK = 0,
    FGS_ERR_INVALID_ARG = -1, /* bad size, stride, null pointer or option; nothing enqueued */
    FGS_ERR_CAPACITY = -2,    /* a device buffer was too small; fgs_last_error gives the size */
    FGS_ERR_HIP = -3,         /* a HIP runtime call failed; fgs_last_error gives its message */
    FGS_ERR_UNSUPPORTED = -5  /* no gfx950 device, or an option the library does not provide */
} fgs_status;

typedef struct fgs_ctx fgs_ctx; /* opaque: stream, workspace, device status words */

/* [host] Pinhole camera. World to camera: x_c = R_cw x_w + t_cw (R_cw row-major); the camera
 * looks along +z with x to the right and y down. Gaussians with camera z <= z_near are culled. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R_cw[9];
    float t_cw[3];
    float z_near;
} fgs_camera;

/* Gaussian parameters (device). n gaussians; every plane has stride `stride` >= n elements.
 * mean: 3 planes, log_scale: 3 planes, quat: 4 planes, opacity_logit: 1 plane, rgb: 3 planes.
 * The same struct carries gradients (same layout) and Adam moments. */
typedef struct {
    int64_t n;
    int64_t stride;
    float *mean;
    float *log_scale;
    float *quat;
    float *opacity_logit;
    float *rgb;
} fgs_gaussians;

/* [host] Rendering cutoffs. A gaussian reaches a pixel when its Mahalanobis distance there is
 * at most sigma_cut; its alpha = min(alpha_max, opacity * exp(-Q/2)) is skipped below alpha_min;
 * a pixel stops before the first gaussian that would take its transmittance below T_min.
 * lowpass is added to the diagonal of every projected 2D covariance (pixels^2). The background
 * (bg, bg_depth) fills the remaining transmittance. tile_w x tile_h is the screen tile of the
 * rasterizer (0, 0 = 16 x 16); supported shapes: 16x16, 32x8, 8x32, 32x16, 16x32, 8x8. */
typedef struct {
    float sigma_cut;
    float alpha_min;
    float alpha_max;
    float T_min;
    float lowpass;
    float bg[3];
    float bg_depth;
    int32_t tile_w, tile_h;
} fgs_render_opts;

/* Rendered planes (device), each width*height; rgb holds 3 planes (stride width*height).
 * alpha = sum_i w_i (Eq. 1 with gamma = 1), T_final = the remaining transmittance, n_contrib =
 * the number of gaussians blended. alpha, T_final and n_contrib may be NULL. */
typedef struct {
    float *rgb;
    float *depth;
    float *alpha;
    float *T_final;
    int32_t *n_contrib;
} fgs_image;

/* [host] Adam state. m and v have the parameters' layout. step = updates already applied; a
 * call applies update step+1 and increments step. lr per group: mean, log-scale, quaternion,
 * opacity logit, rgb. */
typedef struct {
    fgs_gaussians m, v;
    int64_t step;
    float lr[5];
    float beta1, beta2, eps;
} fgs_adam;

/* One RGB-D target view (device): rgb 3 planes and depth, width*height each. Depth <= 0 marks
 * pixels without a depth measurement; they are left out of the depth term. */
typedef struct {
    const float *rgb;
    const float *depth;
} fgs_target;

/* [host] Weights of the mapping loss of Eq. 16 (Sec. III-D):
 *   lambda_rgb ||C - C*||_1 + lambda_depth ||D - D*||_1 + (1 - lambda_rgb)(1 - ssim(C, C*))
 *   + lambda_reg L_reg,
 * the L1 terms as means over pixels (the depth mean over pixels with target depth > 0). ssim is
 * the windowed structural-similarity index averaged over pixels and channels (11x11 gaussian
 * window, sigma 1.5, zero outside the image, C1 = 0.01^2, C2 = 0.03^2); its weight 1 - lambda_rgb
 * follows Eq. 16, so lambda_rgb = 1 leaves only the L1 terms. L_reg is the scale regulariser of
 * Eq. 15, 1/n sum_i (|s_i1 - s_i2| + s_i3) over the n gaussians with s = exp(log-scale) (the
 * in-plane mean taken per gaussian, epsilon = 0), counted once per step. reg_dev (device float,
 * may be NULL) receives L_reg of the parameters a mapping step started from (unweighted).
 * The SSIM and L_reg terms are taken by fgs_map_step only; fgs_loss_l1 takes the L1 terms. */
typedef struct {
    float lambda_rgb, lambda_depth;
    float lambda_reg;
    float *reg_dev;
} fgs_loss_opts;

/* ------------------------------------------------------------------------------------------ */

/* Create a context on the current HIP device bound to `hip_stream` (a hipStream_t; NULL = the
 * null stream). Fails with FGS_ERR_UNSUPPORTED when the device is not gfx950. */
fgs_status fgs_ctx_create(fgs_ctx **out, void *hip_stream);
fgs_status fgs_ctx_destroy(fgs_ctx *ctx);
/* Rebind the context to another stream (work already enqueued stays where it is). */
fgs_status fgs_ctx_set_stream(fgs_ctx *ctx, void *hip_stream);

/* Waits for the context's stream, then reports device-side conditions recorded since the last
 * check: FGS_ERR_CAPACITY when a forward state or a seed output was too small (the required
 * size is in fgs_last_error and fgs_ctx_stats). Clears the recorded conditions. */
fgs_status fgs_ctx_check(fgs_ctx *ctx);

/* [host] stats[0] = (tile, gaussian) pairs of the last forward, stats[1] = gaussians that
 * survived culling, stats[2] = the largest pair count that overflowed a state (0 if none).
 * Waits for the stream. */
fgs_status fgs_ctx_stats(fgs_ctx *ctx, int64_t stats[4]);

const char *fgs_status_str(fgs_status s);
/* Copies the context's last error message (NUL-terminated, truncated to len). */
fgs_status fgs_last_error(fgs_ctx *ctx, char *buf, size_t len);

/* [host] Profiling. While enabled, the context records HIP events around pipeline stages it
 * enqueues. level 1: the rasterizer kernels only ("raster_fwd", "raster_bwd"), which then run
 * exactly as unprofiled; level 2: every stage: "project", "depth_sort", "bin" (scan + pair
 * emission), "tile_sort" (with tile ranges), "raster_fwd", "ssim" (the SSIM term of a mapping
 * step), "loss", "raster_bwd", "project_bwd",
 * "adam", every kernel still the unprofiled one; level 3: as level 2, and the rasterizers count
 * their work (fgs_ctx_profile_counts, fgs_ctx_profile_work) in variants that run longer.
 * 0 disables. Every call clears previous records. */
fgs_status fgs_ctx_profile(fgs_ctx *ctx, int32_t level);
/* Waits for the stream; total milliseconds and number of launches of one stage since enabling. */
fgs_status fgs_ctx_profile_stage(fgs_ctx *ctx, const char *stage, double *total_ms, int64_t *launches);
/* Waits for the stream; work counters since enabling level 3 (zero below): counts[0] =
 * (pixel, gaussian) pairs within the sigma_cut ellipse that each pixel examined before it
 * stopped, counts[1] = pairs blended, counts[2] = list entries staged by the forward rasterizer,
 * counts[3] = forward launches counted. */
fgs_status fgs_ctx_profile_counts(fgs_ctx *ctx, int64_t counts[4]);
/* Waits for the stream; the full work counters since enabling level 3 (zero below), summed
 * over the single-view forwards and backwards: counts[0] = E_f, (pixel, gaussian) pairs within the
 * sigma_cut ellipse examined before each pixel stopped; counts[1] = E_c, pairs blended; counts[2] =
 * list entries staged (read from HBM) by the forward rasterizer; counts[3] = K_c, (tile, gaussian)
 * list entries that some pixel of the tile blended; counts[4] = L_f, per tile the list entries up to
 * the last one any pixel examined (all, for a pixel that never stops), summed; counts[5] = L_b, per
 * tile the list entries up to the last blended one, summed; counts[6] = forwards counted;
 * counts[7] = backward wave-entry evaluations (a wave of 64 pixels evaluating one list entry);
 * counts[8] = those in which some pixel blended; counts[9] = those in which 1 to 8 pixels blended;
 * counts[10] = pairs the backward found blended (E_c again); counts[11] = backwards counted. */
fgs_status fgs_ctx_profile_work(fgs_ctx *ctx, int64_t counts[12]);

/* ---------------------------- rendering (Eq. 1) and its gradient ---------------------------- */

/* [host] Size in bytes of a forward state for n gaussians, a width x height image, the tile of
 * `o` and room for max_pairs (tile, gaussian) pairs. */
fgs_status fgs_state_bytes(int64_t n, int32_t width, int32_t height, int64_t max_pairs,
                           const fgs_render_opts *o, int64_t *bytes);

/* Forward render of g through cam (Sec. III, Eq. 1): EWA projection of every gaussian
 * (covariance R S S^T R^T), binning into screen tiles, ordering of every tile's list by
 * (depth, index), and front-to-back blending of colour, depth and opacity into `out`.
 * `state` (device, state_bytes, caller-owned) receives what the backward needs; its pair
 * capacity is what fgs_state_bytes reserved. If the scene needs more pairs than that, the
 * image is incomplete and the next fgs_ctx_check returns FGS_ERR_CAPACITY. */
fgs_status fgs_render_fwd(fgs_ctx *ctx, const fgs_gaussians *g, const fgs_camera *cam,
                          const fgs_render_opts *o, const fgs_image *out, void *state,
                          int64_t state_bytes);

/* Gradient of a scalar loss through the forward that filled `state` (same g, cam and o).
 * dL_drgb (3 planes), dL_ddepth and dL_dalpha (may be NULL) are the loss's gradients with
 * respect to the rendered planes. The parameter gradients are ADDED to `grad` (same n;
 * any stride >= n), so several views accumulate into one buffer. */
fgs_status fgs_render_bwd(fgs_ctx *ctx, const fgs_gaussians *g, const fgs_camera *cam,
                          const fgs_render_opts *o, const void *state, int64_t state_bytes,
                          const float *dL_drgb, const float *dL_ddepth, const float *dL_dalpha,
                          const fgs_gaussians *grad);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the computation, arguments and result of
 * fgs_render_bwd, with no allocation inside the call. Its one scratch buffer, the 2D gradient
 * records (64 bytes per gaussian), is a static device array of FGS_NOALLOC_MAX_GAUSSIANS records
 * that each GPU holds until the process ends (32 MiB); the call clears the first g->n records
 * with a fill kernel before using them. Every call on one GPU shares that array: calls that
 * overlap on one GPU (two streams or two threads) race and produce wrong gradients. g->n above
 * FGS_NOALLOC_MAX_GAUSSIANS returns FGS_ERR_CAPACITY and enqueues nothing. ctx must have been
 * created on the GPU the call runs on (fgs_ctx_create looks up that GPU's copy of the array). */
#define FGS_NOALLOC_MAX_GAUSSIANS (1 << 19)
fgs_status fgs_render_bwd_noalloc(fgs_ctx *ctx, const fgs_gaussians *g, const fgs_camera *cam,
                                  const fgs_render_opts *o, const void *state, int64_t state_bytes,
                                  const float *dL_drgb, const float *dL_ddepth, const float *dL_dalpha,
                                  const fgs_gaussians *grad);

/* ------------------------------------ mapping step ------------------------------------ */

/* One mapping iteration over a window of n_views keyframes (Sec. III-D, map optimization):
 * for every view, render (Eq. 1), take the image terms of Eq. 16 (L1 colour and depth, and the
 * SSIM term when l->lambda_rgb < 1) against the view's target, and accumulate the gradient; add
 * the scale regulariser's (l->lambda_reg > 0) once; then one Adam update of `params`
 * (opt->step is incremented on the host). cams and targets are [host] arrays of n_views.
 * l->lambda_rgb must lie in [0, 1] and l->lambda_reg be >= 0. loss_dev and psnr_dev (device,
 * n_views floats each, may be NULL) receive each view's image terms and PSNR.
 * grad_out (may be NULL) receives the summed gradient (overwritten). The context keeps the
 * per-view states; it grows them when a scene needs more pairs than before. Adam's step count is
 * kept on the device too (the update applied is that count + 1; a caller that changes opt->step
 * between calls is followed). A view seen before (same index, camera and gaussian count) runs
 * without waiting for its pair count; if its pairs outgrow the state, that step applies nothing:
 * parameters, moments and the device count stay as they were. The next call then returns
 * FGS_ERR_CAPACITY without running, with opt->step set back to the device's count and the state
 * grown; the caller repeats the step. */
fgs_status fgs_map_step(fgs_ctx *ctx, const fgs_gaussians *params, fgs_adam *opt,
                        int32_t n_views, const fgs_camera *cams, const fgs_target *targets,
                        const fgs_render_opts *o, const fgs_loss_opts *l, float *loss_dev,
                        float *psnr_dev, const fgs_gaussians *grad_out);

/* L1 loss of one rendered view (the L1 terms of Eq. 16) and its gradient: writes dL_drgb
 * (3 planes), dL_ddepth, and the loss and PSNR (device floats, may be NULL). */
fgs_status fgs_loss_l1(fgs_ctx *ctx, int64_t n_pixels, const float *rgb, const float *depth,
                       const fgs_target *target, const fgs_loss_opts *l, float *dL_drgb,
                       float *dL_ddepth, float *loss_dev, float *psnr_dev);

/* Structural similarity of a rendered image to a target (Sec. III-D, the SSIM term of Eq. 16),
 * device planes of width*height: img and tgt 3 planes each. ssim_dev (device float, may be NULL)
 * receives the index averaged over pixels and channels (11x11 gaussian window, sigma 1.5, zero
 * outside the image, C1 = 0.01^2, C2 = 0.03^2); dssim_dimg (device, 3 planes, may be NULL) its
 * gradient with respect to img (overwritten). */
fgs_status fgs_ssim(fgs_ctx *ctx, int32_t width, int32_t height, const float *img, const float *tgt,
                    float *ssim_dev, float *dssim_dimg);

/* One Adam update of params with gradient grad (opt->step is incremented on the host). */
fgs_status fgs_adam_step(fgs_ctx *ctx, const fgs_gaussians *params, const fgs_gaussians *grad,
                         fgs_adam *opt);

/* ------------------------------------ keyframe window ------------------------------------ */

/* [host] Pruning thresholds (Sec. III-D, "Gaussian Pruning": gaussians grown too large in any
 * dimension and gaussians of low opacity are removed; the paper gives no values). A gaussian is
 * removed when sigmoid(opacity logit) < min_opacity or when any of its three scales
 * exp(log-scale) exceeds max_scale (world units). min_opacity in [0, 1) (0: no opacity test);
 * max_scale <= 0 or +inf: no size test. The tests compare the stored values with the thresholds
 * carried into their domains: a gaussian is kept when logit >= (float)log(min_opacity / (1 -
 * min_opacity)) and every log-scale <= (float)log(max_scale), each threshold computed in double
 * and rounded to float; a NaN logit or log-scale removes the gaussian. */
typedef struct {
    float min_opacity;
    float max_scale;
} fgs_prune_opts;

/* Prunes src[0] (Sec. III-D) by stream compaction: the survivors are packed, in index order, into
 * dst[0] at [0, kept), and the same columns of src[1 .. n_sets) (blocks of the same layout and n,
 * such as the Adam moments m and v) into dst[1 .. n_sets). 1 <= n_sets <= 4. Each dst[k].stride
 * must be at least src[0].n (dst[k].n is ignored); no destination block may overlap a source block
 * or another destination. n_kept_dev (device int64, nullable) receives the survivor count; keep
 * (device, src[0].n bytes, nullable) receives 1 for each survivor and 0 for each removed gaussian.
 * n_kept_host [host] (nullable) waits for the stream and receives the count. */
fgs_status fgs_prune(fgs_ctx *ctx, const fgs_prune_opts *o, int32_t n_sets, const fgs_gaussians *src,
                     const fgs_gaussians *dst, int64_t *n_kept_dev, uint8_t *keep, int64_t *n_kept_host);

typedef struct fgs_window fgs_window; /* opaque: per-view states, item counter, captured graph */

/* A keyframe window (Sec. III-C, III-D: the co-visible and random keyframes optimised together)
 * of n_views cameras ([host] array, copied) that may differ in size. tiles ([host], 2 ints per
 * view: tile_w, tile_h; NULL = 16x16) picks each view's rasterizer tile among 16x16, 32x8 and
 * 8x32. blocks_per_cu > 0 makes the rasterizer launches persistent grids of that many workgroups
 * per compute unit pulling (view, tile) items from a counter; 0 launches one workgroup per item.
 * The window keeps its own stream for graph capture and orders it against the context's stream. */
fgs_status fgs_window_create(fgs_ctx *ctx, int32_t n_views, const fgs_camera *cams, const int32_t *tiles,
                             int32_t blocks_per_cu, fgs_window **out);
fgs_status fgs_window_destroy(fgs_window *w);

/* One mapping iteration over the window, with the semantics of fgs_map_step: all views' gaussians
 * are ordered by depth in one sort and binned together, all views' tiles are rendered (Eq. 1) by
 * ONE launch over the (view, tile) items, the L1 terms of Eq. 16 are taken per view, ONE launch
 * runs every view's backward over the same items, and one pass per gaussian sums the views'
 * gradients through their projections and applies Adam. targets: [host] array of n_views. use_graph != 0 captures
 * the step in a hipGraph on its first call and replays it afterwards (re-captured when a pointer,
 * n, an option, the profiling level or the context's own sort and binning buffers change). The
 * first call for a given n sizes the window's pair capacity from a synchronous count per view (50%
 * headroom). A later step that outgrows it applies nothing (parameters, moments and the device
 * step count stay as they were); the next call returns FGS_ERR_CAPACITY without running, with
 * opt->step set back to the device's count and the window grown, and the caller repeats the step.
 * The window takes the L1 terms only: l->lambda_rgb other than 1 or l->lambda_reg other than 0
 * returns FGS_ERR_UNSUPPORTED and enqueues nothing. */
fgs_status fgs_window_step(fgs_window *w, const fgs_gaussians *params, fgs_adam *opt, const fgs_target *targets,
                           const fgs_render_opts *o, const fgs_loss_opts *l, float *loss_dev, float *psnr_dev,
                           const fgs_gaussians *grad_out, int32_t use_graph);

/* ------------------------------ Fourier seeding (Sec. III-A) ------------------------------ */

/* [host] Seeding constants. D0: cutoff radius of the Gaussian high-pass of Eq. 5, in frequency
 * samples. m < n: lattice strides inside the high- and low-frequency masks. tile: edge of the
 * square tiles of the per-tile seed count. alpha_h, alpha_l: radius factors of Eq. 11 (a seed's
 * radius is alpha d / fx, alpha pixels at its depth). opacity_logit: initial opacity logit.
 * Seeds need a finite depth in [depth_min, depth_max]. use_prior = 1 replaces the radius rule and
 * the constant opacity of the gaussians written into out->params (required then) by the learned
 * prior of fgs_prior.h, evaluated on the frame's 16x16 tiles, whose packed FP32 weights `prior`
 * points to (device); 2 takes only its shape (log-scales and the camera-aligned rotation), 3 only
 * its opacity; the seed set and the seed arrays are unchanged.
 * Missing-region check (Sec. III-A, Eq. 9, 10): render_alpha, render_depth (width*height) and
 * render_rgb (3 planes) are the current map rendered at cam with a black background and background
 * depth 0 (fgs_render_fwd's opacity A, depth and colour planes; device). A pixel is missing when
 * A < miss_alpha (M_i), or A > 0 and either its depth is valid and |rendered depth / A - depth| >
 * miss_depth (M_d) or (|dr| + |dg|) + |db| > miss_rgb for the rendered colour / A minus the frame
 * colour (M_c), each a binary32 operation; only missing pixels seed (both frequency masks are
 * intersected with M_m). render_alpha NULL: no map yet, every pixel is missing (the other two
 * pointers are then ignored). */
typedef struct {
    double D0;
    int32_t m, n, tile;
    float alpha_h, alpha_l, opacity_logit;
    float depth_min, depth_max;
    int32_t use_prior;
    const void *prior;
    const float *render_alpha, *render_depth, *render_rgb;
    float miss_alpha, miss_depth, miss_rgb;
} fgs_seed_opts;

/* Seed output (device). Seeds are written in ascending pixel order (y * width + x), at most
 * `capacity`: pixel index, is_high (1 = high-frequency mask), mean (3 planes of stride capacity,
 * world coordinates), radius, rgb (3 planes). tile_count (ceil(W/tile) * ceil(H/tile) ints,
 * row-major tiles) and n_dev (one int64: the number of seeds, which may exceed capacity) may be
 * NULL. When params.mean is not NULL the seeds are also written as gaussians into params at
 * [0, count): the mean, log-scale log(radius) on all axes, identity rotation, the initial opacity
 * logit and the pixel colour (params.stride >= capacity). E (width*height doubles: |I_h|), hist
 * (256 uint32: histogram of q = floor(255 E / E_max)) and threshold (one int32: the triangle
 * threshold, -1 for a flat frame) are optional diagnostics. With the learned prior, from_prior
 * (capacity bytes, nullable) marks the seeds whose shape and opacity came from the prior. missing
 * (width*height bytes, nullable) receives the missing-region mask M_m (1 = missing). */
typedef struct {
    int64_t capacity;
    int32_t *pixel;
    uint8_t *is_high;
    float *mean;
    float *radius;
    float *rgb;
    int32_t *tile_count;
    int64_t *n_dev;
    fgs_gaussians params;
    double *E;
    uint32_t *hist;
    int32_t *threshold;
    uint8_t *from_prior;
    uint8_t *missing;
} fgs_seed_out;

/* Seeds gaussians from one RGB-D frame (rgb: 3 planes, depth: 1 plane, width*height of cam) by the
 * frequency analysis of Sec. III-A: luma DFT (Eq. 2), Gaussian high-pass centred on DC (Eq. 3, 5,
 * 7), inverse DFT (Eq. 8), the triangle threshold of the magnitude histogram, the missing-region
 * check against the current map (Eq. 9, 10; see fgs_seed_opts), lattice sampling with strides m
 * and n, and back-projection through cam with the radius rule of Eq. 11. Frame
 * lines must be at most 1920 pixels with prime factors up to 31. n_seeds_host [host] (may be NULL)
 * waits for the stream and receives the number of seeds; more seeds than capacity then returns
 * FGS_ERR_CAPACITY (otherwise the next fgs_ctx_check reports it). */
fgs_status fgs_seed_gaussians(fgs_ctx *ctx, const float *rgb, const float *depth, const fgs_camera *cam,
                              const fgs_seed_opts *o, const fgs_seed_out *out, int64_t *n_seeds_host);

#ifdef __cplusplus
}
#endif
#endif /* FGS_H */
