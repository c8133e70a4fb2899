/*
 * FGS oracle: a plain, slow, FP64 CPU implementation of the mapping hot path of
 * "FGS-SLAM: Fourier-based Gaussian Splatting for Real-time SLAM with Sparse and
 * Dense Map Fusion" (arXiv 2503.01109).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The product path (the
 * HIP library) never calls it, and the two share no code.
 *
 * Every function takes host pointers. Gaussian parameters are one SoA block of
 * 14 planes of length n (stride n):
 *   0-2 mean, 3-5 log-scale, 6-9 quaternion (w,x,y,z), 10 opacity logit, 11-13 rgb.
 * Images are planes of width*height doubles, row-major (index y*width + x).
 * Functions return 0 on success and a negative value on invalid arguments.
 */
#ifndef FGSO_H
#define FGSO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9];   /* world -> camera rotation, row-major: x_c = R x_w + t */
    double t[3];
    double z_near; /* gaussians with camera-space z <= z_near are culled */
} fgso_camera;

typedef struct {
    double sigma_cut;  /* per-pixel cutoff: Mahalanobis distance <= sigma_cut (3) */
    double alpha_min;  /* contributions with alpha < alpha_min are skipped (1/255) */
    double alpha_max;  /* alpha is clamped to alpha_max (0.99) */
    double T_min;      /* stop before transmittance would drop below T_min (1e-4) */
    double lowpass;    /* added to the diagonal of the screen-space covariance (0.3 px^2) */
    double bg[3];      /* background colour */
    double bg_depth;   /* background depth */
} fgso_render_opts;

/* Per-gaussian projection, 16 doubles per gaussian:
 * valid, t_x, t_y, t_z, cov2_xx, cov2_xy, cov2_yy, conic_a, conic_b, conic_c,
 * mean2_x, mean2_y, depth, opacity, reserved, reserved. */
#define FGSO_PROJ_STRIDE 16
int fgso_project(int64_t n, const double *params, const fgso_camera *cam,
                 const fgso_render_opts *o, double *proj);

/* Forward render (Eq. 1 with gamma = colour, depth and 1).
 * mode 0: tile-bucketed candidate lists (a conservative pre-cull); mode 1: brute force.
 * pix: optional list of n_pix pixel indices to render (NULL = all pixels); outputs are
 * then indexed by list position. Outputs: rgb (3 planes), depth, alpha, T_final, n_contrib.
 * Candidates are ordered by (depth rounded to binary32, index).
 * amb (nullable): per-pixel flags: bit 0 (ambiguous) when a cutoff decision at this pixel (Q
 * against sigma_cut^2, alpha against alpha_min or alpha_max, T against T_min) lies within a
 * relative amb_rel of its threshold; bit 1 (information only) when two consecutive contributors
 * have equal binary32 depths and so blend in index order.
 * stats (nullable, 4 doubles): pairs tested until termination (E_f), contributing pairs
 * (E_c), pixels with bit 0 set, pixels rendered. */
int fgso_render_fwd(int64_t n, const double *params, const fgso_camera *cam,
                    const fgso_render_opts *o, int mode, int64_t n_pix, const int64_t *pix,
                    double *rgb, double *depth, double *alpha, double *T_final,
                    int32_t *n_contrib, uint8_t *amb, double amb_rel, double *stats);

/* Analytic backward of fgso_render_fwd. g_rgb (3 planes), g_depth, g_alpha (nullable) are the
 * upstream gradients of the rendered planes (indexed like the forward's outputs when pix is
 * given). grad (14 planes) receives dL/dparams (overwritten). grad2d (nullable, 10 planes of n):
 * dL/d(mean2_x, mean2_y, conic_a, conic_b, conic_c, opacity, r, g, b, depth).
 * mass (nullable, 14 planes of n, a diagnostic): the absolute mass of every gradient entry, which
 * bounds the rounding error of an evaluation of that sum in a precision of unit roundoff u as
 * c u mass for a modest c: per 2D entry the sum over pixels of the absolute value of each term, with
 * dL/dalpha replaced by the sum of the absolute values of its parts (the pair's own share and
 * everything blended behind it) and the mean terms a dx + b dy split as |a dx| + |b dy|; then
 * mass_k = sum_j |d grad_k / d grad2d_j| mass2d_j through the per-gaussian chain rule. It does not
 * model the sensitivity of the terms to rounded inputs, which dominates for splats just past the
 * near plane (very elongated, far off-centre projections). */
int fgso_render_bwd(int64_t n, const double *params, const fgso_camera *cam,
                    const fgso_render_opts *o, int mode, int64_t n_pix, const int64_t *pix,
                    const double *g_rgb, const double *g_depth, const double *g_alpha,
                    double *grad, double *grad2d, double *mass);

/* Work counts of the tile formulation (16x16 tiles, lists of the gaussians whose sigma_cut box
 * reaches the tile, in (binary32 depth, index) order): counts[0] = K_c, the (tile, gaussian) pairs
 * with at least one blended pixel; counts[1] = L_f, per tile the list entries up to the last one
 * any pixel examined (a pixel examines up to the entry at which it stops, the whole list when it
 * never stops), summed; counts[2] = L_b, per tile the list entries up to the last blended one,
 * summed; counts[3] = the list entries of all tiles. A diagnostic of the work the method implies. */
int fgso_tile_counts(int64_t n, const double *params, const fgso_camera *cam, const fgso_render_opts *o,
                     int64_t counts[4]);

/* Number of (tile, gaussian) duplicates under axis-aligned 3-sigma-box binning. */
int64_t fgso_count_duplicates(int64_t n, const double *params, const fgso_camera *cam,
                              const fgso_render_opts *o, int32_t tile_w, int32_t tile_h);

/* L1 colour + depth loss (the L1 terms of the mapping loss, Eq. 16), mean-reduced.
 * Writes dL/d(rgb planes) and dL/d(depth) and returns loss and PSNR. */
int fgso_loss_l1(int64_t P, const double *rgb, const double *depth, const double *rgb_t,
                 const double *depth_t, double lambda_rgb, double lambda_depth,
                 double *g_rgb, double *g_depth, double *loss, double *psnr);

/* Structural similarity of img to tgt (3 planes each), Sec. III-D, Eq. 16: the mean over the
 * 3 P (channel, pixel) values of the windowed index (11x11 gaussian window, sigma 1.5, zero
 * outside the image, C1 = 0.01^2, C2 = 0.03^2). grad (nullable, 3 planes): d ssim / d img;
 * smap (nullable, 3 planes): the per-pixel index. */
int fgso_ssim(int32_t W, int32_t H, const double *img, const double *tgt, double *ssim, double *grad,
              double *smap);

/* Scale regulariser of Eq. 15 over n gaussians (log_scale: 3 planes of n): value = 1/n sum_i
 * (|s_i1 - s_i2| + s_i3) with s = exp(log-scale); grad (nullable, 3 planes): d value / d log-scale. */
int fgso_scale_reg(int64_t n, const double *log_scale, double *value, double *grad);

/* Adam (Kingma and Ba) over 14 parameter planes; lr per group (mean, log-scale, quat,
 * opacity, rgb). step = number of updates already done; this update is step+1. */
int fgso_adam(int64_t n, double *params, double *m, double *v, const double *grad,
              int64_t step, const double lr[5], double beta1, double beta2, double eps);

/* ---------------------------- Fourier seeding (Sec. III-A) ---------------------------- */
typedef struct {
    double D0;               /* high-pass cutoff radius, frequency samples (Eq. 5) */
    int32_t m, n;            /* lattice strides in high- and low-frequency regions */
    int32_t tile;            /* tile edge for the per-tile seed count (16) */
    double alpha_h, alpha_l; /* radius factors in pixels (Eq. 11) */
    double opacity_logit;    /* initial opacity logit of every seed */
    double depth_min, depth_max;
} fgso_seed_opts;

/* Seeding diagnostics (all outputs nullable):
 *  E       (W*H) high-pass magnitude |I_h|
 *  hist    (256) histogram of q = floor(255 (E / E_max))
 *  thresh  triangle threshold t (q > t is high frequency); -1 when E_max == 0
 *  margin  min over pixels (the maximum's aside) of the distance of 255 (E / E_max) to the
 *          nearest integer k >= 1, the only values where q can change */
int fgso_highpass(int32_t W, int32_t H, const float *rgb, double D0, double *E,
                  int64_t *hist, int32_t *thresh, double *margin);

/* Triangle threshold over a 256-bin histogram. */
int32_t fgso_triangle(const int64_t *hist);

/* Missing-region check (Sec. III-A, Eq. 9 and 10) against the current map rendered at the
 * frame's pose (black background, background depth 0): binary32 planes of W*H, the rendered
 * opacity A (Eq. 1 with gamma = 1), depth (gamma = d) and 3 colour planes. A pixel is missing
 * (M_m = M_i | M_d | M_c, Eq. 9) when
 *   M_i: A < tau_alpha (too little gaussian there);
 *   M_d: A > 0, its frame depth is valid and |rendered depth / A - frame depth| > tau_depth
 *        (foreground that the map lacks);
 *   M_c: A > 0 and (|dr| + |dg|) + |db| > tau_rgb over the rendered colour / A minus the frame's;
 * each division, difference, absolute value and sum a binary32 operation, comparisons strict. */
typedef struct {
    const float *alpha, *depth, *rgb;
    float tau_alpha, tau_depth, tau_rgb;
} fgso_missing;

/* Full seeding: returns the number of seeds (or < 0 on error). Seeds are written in
 * ascending pixel order, at most `capacity`: pixel id, class (1 = high frequency),
 * mean (3 planes of capacity), radius, rgb (3 planes of capacity). tile_count has
 * ceil(W/tile)*ceil(H/tile) entries. Float outputs are binary32 values. miss (nullable: no map
 * yet, every pixel missing) restricts the high- and low-frequency masks to the missing region
 * (Eq. 10); missing_out (nullable, W*H) receives M_m. */
int64_t fgso_seed(int32_t W, int32_t H, const float *rgb, const float *depth,
                  const float cam_R[9], const float cam_t[3], float fx, float fy, float cx, float cy,
                  const fgso_seed_opts *o, int64_t capacity, int32_t *pixel, uint8_t *is_high,
                  float *mean, float *radius, float *seed_rgb, int32_t *tile_count,
                  int32_t *thresh_out, double *margin_out, const fgso_missing *miss, uint8_t *missing_out);

/* ------------------------------- Learned prior MLP ------------------------------- */
/* Tile features: 256 values log(1 + |F_c|) of the tile's 16x16 luma DFT (Eq. 2-4, centred),
 * then mean, std, min, max of valid depth. Returns the number of valid-depth pixels. */
int fgso_tile_features(int32_t W, int32_t H, const float *rgb, const float *depth,
                       int32_t tx, int32_t ty, double depth_min, double depth_max, double *feat);

/* MLP 260 -> 256 -> 256 -> 4 with exact-erf GELU. Weights row-major W1[256][260], b1[256],
 * W2[256][256], b2[256], W3[4][256], b3[4], packed in that order (133,636 doubles).
 * bf16 != 0 rounds every GEMM operand (weights, activations, upstream gradients) to
 * bfloat16 (round to nearest even) before use; accumulation is FP64. */
#define FGSO_MLP_PARAMS 133636
int fgso_mlp_fwd(int64_t rows, const double *x, const double *w, int bf16, double *y,
                 double *h1, double *h2, double *a1, double *a2);
/* Backward of the mean-squared error 1/(rows*4) sum (y - target)^2; writes dL/dw (FP64). */
int fgso_mlp_bwd(int64_t rows, const double *x, const double *w, int bf16, const double *target,
                 double *gw, double *loss);

/* ---------------------------------- Pruning ---------------------------------- */
/* Thresholds of the pruning test (Sec. III-D) in the domains of the stored values: L_o on the
 * opacity logit, L_s on each log-scale (binary32 values; -inf / +inf when a test is off).
 * Returns -1 unless min_opacity is in [0, 1) and max_scale is not NaN. */
int fgso_prune_thresholds(double min_opacity, double max_scale, double *L_o, double *L_s);
/* keep[i] = 1 when gaussian i of the (14, n) block survives: logit >= L_o and every log-scale
 * <= L_s. Returns the number kept (or < 0 on error). */
int64_t fgso_prune_keep(int64_t n, const double *params, double min_opacity, double max_scale, uint8_t *keep);
/* Stable compaction of `planes` planes of length n (stride n) to out (stride out_stride >= kept):
 * the j-th kept index goes to position j. Returns the number kept. */
int64_t fgso_compact(int64_t n, int32_t planes, const double *in, const uint8_t *keep, double *out,
                     int64_t out_stride);

/* ------------------------------ GICP tracking (Sec. III-B) ------------------------------ */
/* Points are 3 binary32 planes (x, y, z) of stride n; covariances 6 FP64 planes (xx, xy, xz, yy,
 * yz, zz) of stride n; rotations row-major. See gicp.c for the readings. */
/* Lattice points of a depth frame (camera frame, or world with R_wc, t_wc both given); returns
 * the count (the first `capacity` are written, planes of stride capacity). */
int64_t fgso_frame_points(int32_t W, int32_t H, const float *depth, float fx, float fy, float cx, float cy,
                          const float *R_wc, const float *t_wc, int32_t stride, float dmin, float dmax,
                          int64_t capacity, float *xyz);
/* k nearest points of every point in its own cloud (itself included): idx [n][k], d2 [n][k]
 * (nullable) in (binary32 squared distance, index) order. */
int fgso_knn(int64_t n, const float *xyz, int32_t k, int32_t *idx, float *d2);
/* The same for the nq points q[] only (q NULL: the first nq); idx [nq][k], d2 [nq][k]. */
int fgso_knn_some(int64_t n, const float *xyz, int32_t k, int64_t nq, const int64_t *q, int32_t *idx, float *d2);
/* Jacobi eigen-decomposition of a symmetric 3x3 (6 values); evecs column-major. */
int fgso_sym3_eigen(const double A6[6], double evals[3], double evecs[9]);
/* Regularised local covariances (eigenvalues 1, 1, eps) from k nearest neighbours. */
int fgso_cloud_cov(int64_t n, const float *xyz, int32_t k, double eps, double *cov);
/* The covariances of the nq points q[] only: 6 planes of stride nq. */
int fgso_cloud_cov_some(int64_t n, const float *xyz, int32_t k, double eps, int64_t nq, const int64_t *q,
                        double *cov);
/* Correspondences (target index or -1) of the nq source points q[] at (R, t). */
int fgso_gicp_corr_some(int64_t ns, const float *src, int64_t nt, const float *tgt, const double R[9],
                        const double t[3], float d_max, int64_t nq, const int64_t *q, int32_t *corr);
/* One Gauss-Newton linearisation of Eq. 14 at (R, t): H (6x6 row-major), b (6), cost, the number
 * of correspondences, corr (nullable, ns: target index or -1). */
int fgso_gicp_linearize(int64_t ns, const float *src, const double *src_cov, int64_t nt, const float *tgt,
                        const double *tgt_cov, const double R[9], const double t[3], float d_max, double H[36],
                        double b[6], double *cost, int64_t *count, int32_t *corr);
/* Rotation Exp(w) (Rodrigues). */
void fgso_so3_exp(const double w[3], double E[9]);
/* Gauss-Newton alignment from (R0, t0); status 0 converged, 1 iteration limit, 2 degenerate. */
int fgso_gicp_align(int64_t ns, const float *src, const double *src_cov, int64_t nt, const float *tgt,
                    const double *tgt_cov, const double R0[9], const double t0[3], float d_max, int32_t max_iter,
                    double eps_rot, double eps_trans, double R[9], double t[3], int32_t *iters, int32_t *status,
                    double *cost, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif
