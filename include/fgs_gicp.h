/*
 * GICP tracking of libfgs (Sec. III-B "Tracking", Eq. 12-14): the current frame's points (the
 * source, uniformly downsampled) are aligned to the sparse map (the target: downsampled keyframe
 * points) by the pose T that minimises sum_i d_i^T (C_q + T C_p T^T)^-1 d_i, d_i = q_i - T p_i.
 *
 * The paper gives the objective and names the method; the rest follows standard GICP:
 *  - frame points: the pixels on a stride-s lattice (x % s == 0 and y % s == 0) whose depth is
 *    finite and in [depth_min, depth_max], back-projected at the pixel centre in binary32,
 *    X = ((x + 0.5 - cx) d) / fx, Y = ((y + 0.5 - cy) d) / fy, Z = d, in pixel order, optionally
 *    moved to the world by a camera-to-world pose: ((R_r0 X + R_r1 Y) + R_r2 Z) + t_r;
 *  - local covariances C_p, C_q: the k nearest points of the same cloud, the point itself
 *    included (squared distances (dx dx + dy dy) + dz dz in binary32, ties by index), their
 *    sample covariance (1/k), regularised to eigenvalues (1, 1, eps): I - (1 - eps) n n^T with n
 *    the eigenvector of its smallest eigenvalue (defined when that eigenvalue is simple);
 *  - correspondence of source point i at pose (R, t): the nearest target point to T p_i (computed
 *    in binary32 with the pose rounded to binary32: ((R_r0 x + R_r1 y) + R_r2 z) + t_r) within
 *    squared distance d_max^2 (binary32, ties by index), or none;
 *  - Gauss-Newton on Eq. 14: residual d_i = q_j - (R p_i + t) and weight W_i = (C_q + R C_p R^T)^-1
 *    in FP64, Jacobian J_i = [[R p_i + t]_x, -I] for the update R <- Exp(w) R, t <- Exp(w) t + v;
 *    H = sum J^T W J, b = sum J^T W d, cost = sum d^T W d; (w, v) solves H (w, v) = -b.
 *
 * Points are three float32 planes (x, y, z) with a plane stride; covariances six FP64 planes
 * (xx, xy, xz, yy, yz, zz); poses row-major 4x4 FP64 [host] mapping the source frame to the
 * target frame. Pointers are device pointers unless marked [host]; calls enqueue on the context's
 * stream unless they say that they wait.
 */
#ifndef FGS_GICP_H
#define FGS_GICP_H

#include "fgs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Lattice points of one depth frame (width x height of cam; cam's pose is not used). pose_wc
 * [host] (nullable): camera-to-world pose, row-major 4x4 (its top 3x4 is rounded to float and
 * applied); NULL leaves the points in the camera frame. xyz: 3 planes of stride `capacity`; at
 * most `capacity` points are written. n_dev (device int64, nullable) receives the count, which may
 * exceed capacity; n_host [host] (nullable) waits for the stream and receives it, and then a count
 * above capacity returns FGS_ERR_CAPACITY. */
fgs_status fgs_frame_points(fgs_ctx *ctx, const float *depth, const fgs_camera *cam, const double *pose_wc,
                            int32_t stride, float depth_min, float depth_max, float *xyz, int64_t capacity,
                            int64_t *n_dev, int64_t *n_host);

typedef struct fgs_cloud fgs_cloud; /* opaque: a point cloud with its grid and covariances */

/* [host] Cloud options: cell, the edge of the uniform grid's cubic cells (world units; the grid
 * spans the cloud's bounding box and may hold at most 2^25 cells); k in [3, 32] neighbours per
 * covariance (at most n); eps in (0, 1], the regularised covariance's smallest eigenvalue;
 * keep_knn != 0 keeps the neighbour lists for fgs_cloud_read. The cell is best near the distance
 * of the k-th neighbour: a point whose k neighbours are not settled within 4 rings of cells around
 * its own scans the whole cloud. A correspondence search with d_max below about cell (1 - 1e-3)
 * examines one ring of cells around the query's; larger radii examine more (at most 8 rings). */
typedef struct {
    float cell;
    int32_t k;
    double eps;
    int32_t keep_knn;
} fgs_cloud_opts;

/* Builds a cloud from n >= k points (xyz: 3 planes of stride `stride`, copied; the caller's
 * buffer may be reused afterwards): bounding box, grid (points sorted by cell), neighbours and
 * covariances. Waits for the stream once (for the bounding box that sizes the grid); points with a
 * non-finite coordinate make it return FGS_ERR_INVALID_ARG. */
fgs_status fgs_cloud_create(fgs_ctx *ctx, int64_t n, int64_t stride, const float *xyz, const fgs_cloud_opts *o,
                            fgs_cloud **out);
fgs_status fgs_cloud_destroy(fgs_cloud *c);
/* Copies the cloud's covariances (cov: 6 planes of stride n, FP64; nullable) and, when kept,
 * its neighbour lists (knn: [n][k] int32 in (distance, index) order; nullable) into caller
 * buffers; *n_out and *k_out [host] (nullable) receive n and k. */
fgs_status fgs_cloud_read(const fgs_cloud *c, double *cov, int32_t *knn, int64_t *n_out, int32_t *k_out);

/* [host] Alignment options: d_max > 0 the correspondence radius; max_iter >= 1 Gauss-Newton
 * updates at most; stop after an update with |w| < eps_rot and |v| < eps_trans. */
typedef struct {
    float d_max;
    int32_t max_iter;
    double eps_rot, eps_trans;
} fgs_gicp_opts;

/* [host] Alignment result. status: 0 converged, 1 iteration limit, 2 degenerate (fewer than 6
 * correspondences or H not positive definite: the pose of the last good update is kept).
 * correspondences and cost belong to the last linearisation. */
typedef struct {
    double T[16];
    int32_t iterations;
    int32_t status;
    int64_t correspondences;
    double cost;
} fgs_gicp_result;

/* Aligns the source cloud to the target cloud (Eq. 14) from T_init [host] by Gauss-Newton, every
 * iteration on the GPU (correspondences and the sums of H, b in one launch, the 6x6 solve and the
 * pose update in a second). Iterations are enqueued in small batches with a wait for the stream
 * between batches, and none is enqueued once the pose has converged. Waits for the stream and
 * fills *result [host]. */
fgs_status fgs_gicp_align(fgs_ctx *ctx, const fgs_cloud *source, const fgs_cloud *target, const double T_init[16],
                          const fgs_gicp_opts *o, fgs_gicp_result *result);

/* One linearisation of Eq. 14 at pose T [host] without an update: out (device, 29 doubles) gets
 * H's upper triangle row by row (21), b (6), the cost and the correspondence count; corr (device,
 * source n ints, nullable) the target index of each source point's correspondence, or -1. */
fgs_status fgs_gicp_linearize(fgs_ctx *ctx, const fgs_cloud *source, const fgs_cloud *target, const double T[16],
                              float d_max, double *out, int32_t *corr);

#ifdef __cplusplus
}
#endif
#endif /* FGS_GICP_H */
