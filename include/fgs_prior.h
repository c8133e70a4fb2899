/*
 * The learned seeding prior of libfgs: a small network that maps a 16x16 tile's spectrum and
 * depth statistics to the initial shape and opacity of the gaussians seeded in that tile.
 *
 * The paper gives every seed the radius rule of Eq. 11 and one opacity; this prior is an addition
 * that keeps that rule as its fallback and as the reference its output is judged against:
 *
 *  - features (260 per tile): log(1 + |F_c|) of the tile's 16x16 luma DFT (Eq. 2 on the tile,
 *    centred as in Eq. 3 with DC at (8, 8), magnitude as in Eq. 4), 256 values in row-major
 *    (v, u) order; then mean, standard deviation, minimum and maximum of the tile's valid depth;
 *  - network: h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), y = W3 h2 + b3, GELU(a) =
 *    a (1 + erf(a / sqrt 2)) / 2, sizes 260 -> 256 -> 256 -> 4. Every product rounds its operands
 *    to bfloat16 (round to nearest even) and accumulates in FP32 on the matrix cores;
 *  - outputs: y[0..2] are log-scale offsets from the log of the seed's Eq. 11 radius
 *    (alpha d / fx, alpha by the seed's frequency class) along the camera's x, y and viewing axes;
 *    y[3] is the opacity logit;
 *  - fallback: a tile with fewer than 4 valid-depth pixels, or an offset larger than log 4 in
 *    magnitude on some axis, keeps the radius rule and the constant opacity.
 *
 * Weights are one packed FP32 vector of FGS_PRIOR_PARAMS floats (device): W1 [256][260] row-major,
 * b1 [256], W2 [256][256], b2 [256], W3 [4][256], b3 [4]. All calls enqueue on the context's
 * stream. Pointers are device pointers unless marked [host].
 */
#ifndef FGS_PRIOR_H
#define FGS_PRIOR_H

#include "fgs.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FGS_PRIOR_INPUTS 260
#define FGS_PRIOR_HIDDEN 256
#define FGS_PRIOR_OUTPUTS 4
#define FGS_PRIOR_PARAMS 133636

/* [host] Adam state of the prior's weights: m, v (device, FGS_PRIOR_PARAMS floats each), the
 * number of updates done, one learning rate, betas and epsilon. */
typedef struct {
    float *m, *v;
    int64_t step;
    float lr, beta1, beta2, eps;
} fgs_prior_adam;

/* Features of n_tiles 16x16 tiles of one frame (rgb: 3 planes, depth: 1 plane, width x height).
 * tile_ids (n_tiles ints, row-major tile index over ceil(width/16) columns) may be NULL for all
 * tiles in order. feat: [n_tiles][260] floats; n_valid (nullable): valid-depth pixel count per tile,
 * -1 for an id outside the frame (whose features are zero). Depth is valid when finite and in
 * [depth_min, depth_max]. */
fgs_status fgs_tile_features(fgs_ctx *ctx, const float *rgb, const float *depth, int32_t width, int32_t height,
                             float depth_min, float depth_max, int64_t n_tiles, const int32_t *tile_ids, float *feat,
                             int32_t *n_valid);

/* y [rows][4] = network(x [rows][260]) with the packed FP32 weights. */
fgs_status fgs_prior_forward(fgs_ctx *ctx, int64_t rows, const float *x, const float *weights, float *y);

/* One training step of the network on the mean squared error (1 / (4 rows)) sum (y - target)^2
 * against target [rows][4]: forward, backward, and an Adam update of weights (in place; bias
 * corrections for update opt->step + 1, then opt->step is incremented). loss_dev (nullable): the
 * loss before the update (one float). grad_out (nullable): the gradient (FGS_PRIOR_PARAMS floats). */
fgs_status fgs_prior_train_step(fgs_ctx *ctx, int64_t rows, const float *x, const float *target, float *weights,
                                fgs_prior_adam *opt, float *loss_dev, float *grad_out);

#ifdef __cplusplus
}
#endif
#endif /* FGS_PRIOR_H */
