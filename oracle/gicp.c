/*
 * Oracle: GICP tracking on a sparse point map (Sec. III-B "Tracking", Eq. 12-14). FP64 plain
 * loops and brute-force searches; the decisions that pick points (lattice validity, nearest
 * neighbours, correspondences) are taken in binary32, as the GPU takes them.
 *
 * TEST INFRASTRUCTURE ONLY (see fgso.h).
 *
 * The paper gives the objective (Eq. 12-14) and names GICP, the uniform downsampling of frames
 * and the sparse map built from keyframes; the rest is read as the standard method:
 *  1. Frame points: the pixels of a depth frame on a stride-s lattice (x % s == 0, y % s == 0)
 *     with a finite depth d in [dmin, dmax], back-projected at the pixel centre in binary32,
 *     X = ((x + 0.5 - cx) d) / fx, Y = ((y + 0.5 - cy) d) / fy, Z = d, in pixel order; with a
 *     pose (R_wc, t_wc) moved to the world as ((R_r0 X + R_r1 Y) + R_r2 Z) + t_r. The current
 *     frame's points (camera frame) are the source P; the sparse map Q is the union of keyframe
 *     points (world frame).
 *  2. Local covariances C_p, C_q of Eq. 13: the k nearest points of the same cloud, the point
 *     itself included (squared distance (dx dx + dy dy) + dz dz in binary32, ties by index); their
 *     sample covariance (1/k, FP64); regularised to eigenvalues (1, 1, eps) along its eigenvectors,
 *     i.e. C = I - (1 - eps) n n^T with n the eigenvector of the smallest eigenvalue (the local
 *     surface normal). Defined when that eigenvalue is simple.
 *  3. Correspondence of source point i at pose (R, t): T p_i in binary32 with the pose rounded to
 *     binary32, ((R_r0 x + R_r1 y) + R_r2 z) + t_r; its nearest target point with squared distance
 *     <= d_max^2 (binary32, ties by index), or none.
 *  4. Eq. 14 by Gauss-Newton. Residual d_i = q_j - (R p_i + t) (Eq. 12, FP64); weight
 *     W_i = (C_q + R C_p R^T)^-1 (Eq. 13), fixed within a linearisation; for the update
 *     R <- Exp(w) R, t <- Exp(w) t + v the residual's Jacobian is J_i = [[R p_i + t]_x, -I]
 *     ([a]_x w = a x w). H = sum J^T W J, b = sum J^T W d, cost = sum d^T W d; (w, v) solves
 *     H (w, v) = -b (Cholesky). Stop after an update with |w| < eps_rot and |v| < eps_trans
 *     (status 0), after max_iter updates (status 1), or, without updating, when fewer than 6
 *     source points have a correspondence or H is not positive definite (status 2).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "fgso.h"

/* binary32 operations evaluated in FP64 and rounded once (exact binary32 results for + - * /) */
static float b_add(float a, float b) { return (float)((double)a + (double)b); }
static float b_sub(float a, float b) { return (float)((double)a - (double)b); }
static float b_mul(float a, float b) { return (float)((double)a * (double)b); }
static float b_div(float a, float b) { return (float)((double)a / (double)b); }

static float dist2_b32(float ax, float ay, float az, float bx, float by, float bz)
{
    const float dx = b_sub(bx, ax), dy = b_sub(by, ay), dz = b_sub(bz, az);
    return b_add(b_add(b_mul(dx, dx), b_mul(dy, dy)), b_mul(dz, dz));
}

/* (d, j) before (e, l) */
static int before(float d, int64_t j, float e, int64_t l) { return d < e || (d == e && j < l); }

int64_t fgso_frame_points(int32_t W, int32_t H, const float *depth, float fx, float fy, float cx, float cy,
                          const float *R_wc, const float *t_wc, int32_t stride, float dmin, float dmax,
                          int64_t capacity, float *xyz)
{
    if (W <= 0 || H <= 0 || !depth || stride <= 0 || capacity < 0 || (capacity > 0 && !xyz)) return -1;
    if ((R_wc == NULL) != (t_wc == NULL)) return -1;
    int64_t count = 0;
    for (int32_t y = 0; y < H; y += stride)
        for (int32_t x = 0; x < W; x += stride) {
            const float d = depth[(int64_t)y * W + x];
            if (!isfinite(d) || !(d >= dmin && d <= dmax)) continue;
            if (count < capacity) {
                const float X = b_div(b_mul(b_sub(b_add((float)x, 0.5f), cx), d), fx);
                const float Y = b_div(b_mul(b_sub(b_add((float)y, 0.5f), cy), d), fy);
                float P[3] = {X, Y, d};
                if (R_wc) {
                    for (int r = 0; r < 3; ++r)
                        P[r] = b_add(b_add(b_add(b_mul(R_wc[3 * r], X), b_mul(R_wc[3 * r + 1], Y)),
                                           b_mul(R_wc[3 * r + 2], d)),
                                     t_wc[r]);
                }
                for (int r = 0; r < 3; ++r) xyz[r * capacity + count] = P[r];
            }
            count++;
        }
    return count;
}

int fgso_knn_some(int64_t n, const float *xyz, int32_t k, int64_t nq, const int64_t *q, int32_t *idx, float *d2)
{
    if (n < 0 || k <= 0 || k > n || !xyz || !idx || nq < 0) return -1;
    const float *X = xyz, *Y = xyz + n, *Z = xyz + 2 * n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < nq; ++a) {
        const int64_t i = q ? q[a] : a;
        int32_t *bi = idx + a * k;
        float bd[256];
        float *bdp = k <= 256 ? bd : (float *)malloc(sizeof(float) * (size_t)k);
        int32_t m = 0; /* entries held, sorted by (distance, index) */
        for (int64_t j = 0; j < n; ++j) {
            const float e = dist2_b32(X[i], Y[i], Z[i], X[j], Y[j], Z[j]);
            if (m == k && !before(e, j, bdp[k - 1], bi[k - 1])) continue;
            int32_t s = m < k ? m++ : k - 1;
            while (s > 0 && before(e, j, bdp[s - 1], bi[s - 1])) {
                bdp[s] = bdp[s - 1];
                bi[s] = bi[s - 1];
                --s;
            }
            bdp[s] = e;
            bi[s] = (int32_t)j;
        }
        if (d2)
            for (int32_t s = 0; s < k; ++s) d2[a * k + s] = bdp[s];
        if (bdp != bd) free(bdp);
    }
    return 0;
}

int fgso_knn(int64_t n, const float *xyz, int32_t k, int32_t *idx, float *d2)
{
    return fgso_knn_some(n, xyz, k, n, NULL, idx, d2);
}

/* Eigen-decomposition of the symmetric matrix A (xx, xy, xz, yy, yz, zz) by cyclic Jacobi
 * rotations; evals unsorted, evecs column-major (column c is the eigenvector of evals[c]). */
int fgso_sym3_eigen(const double A6[6], double evals[3], double evecs[9])
{
    double a[3][3] = {{A6[0], A6[1], A6[2]}, {A6[1], A6[3], A6[4]}, {A6[2], A6[4], A6[5]}};
    double v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        const double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off == 0.0 || off <= 1e-32 * diag) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                /* the rotation in the (p, q) plane that zeroes a[p][q]: tan of its angle is the
                 * smaller root of t^2 + 2 theta t - 1 = 0 */
                const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- G^T A G with G the rotation by (c, s) in the (p, q) plane */
                const double apq = a[p][q];
                a[p][p] -= t * apq;
                a[q][q] += t * apq;
                a[p][q] = a[q][p] = 0.0;
                for (int r = 0; r < 3; ++r) {
                    if (r == p || r == q) continue;
                    const double arp = a[r][p], arq = a[r][q];
                    a[r][p] = a[p][r] = c * arp - s * arq;
                    a[r][q] = a[q][r] = s * arp + c * arq;
                }
                for (int r = 0; r < 3; ++r) { /* V <- V G */
                    const double vp = v[r][p], vq = v[r][q];
                    v[r][p] = c * vp - s * vq;
                    v[r][q] = s * vp + c * vq;
                }
            }
    }
    for (int c = 0; c < 3; ++c) {
        evals[c] = a[c][c];
        for (int r = 0; r < 3; ++r) evecs[3 * c + r] = v[r][c];
    }
    return 0;
}

int fgso_cloud_cov_some(int64_t n, const float *xyz, int32_t k, double eps, int64_t nq, const int64_t *q,
                        double *cov)
{
    if (n < 0 || k <= 0 || k > n || !xyz || !cov || nq < 0) return -1;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)((nq > 0 ? nq : 1) * k));
    if (!idx) return -2;
    if (fgso_knn_some(n, xyz, k, nq, q, idx, NULL) != 0) {
        free(idx);
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nq; ++i) {
        double mu[3] = {0, 0, 0};
        for (int32_t s = 0; s < k; ++s)
            for (int r = 0; r < 3; ++r) mu[r] += (double)xyz[r * n + idx[i * k + s]];
        for (int r = 0; r < 3; ++r) mu[r] /= (double)k;
        double C[6] = {0, 0, 0, 0, 0, 0};
        for (int32_t s = 0; s < k; ++s) {
            double e[3];
            for (int r = 0; r < 3; ++r) e[r] = (double)xyz[r * n + idx[i * k + s]] - mu[r];
            C[0] += e[0] * e[0]; C[1] += e[0] * e[1]; C[2] += e[0] * e[2];
            C[3] += e[1] * e[1]; C[4] += e[1] * e[2]; C[5] += e[2] * e[2];
        }
        for (int q = 0; q < 6; ++q) C[q] /= (double)k;
        double ev[3], V[9];
        fgso_sym3_eigen(C, ev, V);
        int lo = 0;
        for (int c = 1; c < 3; ++c)
            if (ev[c] < ev[lo]) lo = c;
        const double *nrm = V + 3 * lo, f = 1.0 - eps;
        cov[0 * nq + i] = 1.0 - f * nrm[0] * nrm[0];
        cov[1 * nq + i] = -f * nrm[0] * nrm[1];
        cov[2 * nq + i] = -f * nrm[0] * nrm[2];
        cov[3 * nq + i] = 1.0 - f * nrm[1] * nrm[1];
        cov[4 * nq + i] = -f * nrm[1] * nrm[2];
        cov[5 * nq + i] = 1.0 - f * nrm[2] * nrm[2];
    }
    free(idx);
    return 0;
}

int fgso_cloud_cov(int64_t n, const float *xyz, int32_t k, double eps, double *cov)
{
    return fgso_cloud_cov_some(n, xyz, k, eps, n, NULL, cov);
}

/* full symmetric 3x3 from 6 planes at index i */
static void sym_at(const double *c6, int64_t n, int64_t i, double M[3][3])
{
    M[0][0] = c6[i]; M[0][1] = M[1][0] = c6[n + i]; M[0][2] = M[2][0] = c6[2 * n + i];
    M[1][1] = c6[3 * n + i]; M[1][2] = M[2][1] = c6[4 * n + i]; M[2][2] = c6[5 * n + i];
}

static int inverse3(const double A[3][3], double B[3][3])
{
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    if (!(det != 0.0) || !isfinite(det)) return -1;
    const double id = 1.0 / det;
    B[0][0] = c00 * id;
    B[1][0] = c01 * id;
    B[2][0] = c02 * id;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    return 0;
}

/* Correspondence of source point i at the pose rounded to binary32 (R32, t32): the nearest
 * target point within d_max (binary32 squared distances, ties by index), or -1. */
static int32_t corr_of(int64_t i, int64_t ns, const float *src, int64_t nt, const float *tgt, const float R32[9],
                       const float t32[3], float dm2)
{
    const float x = src[i], y = src[ns + i], z = src[2 * ns + i];
    float P[3];
    for (int r = 0; r < 3; ++r)
        P[r] = b_add(b_add(b_add(b_mul(R32[3 * r], x), b_mul(R32[3 * r + 1], y)), b_mul(R32[3 * r + 2], z)), t32[r]);
    int64_t best = -1;
    float bd = 0.0f;
    for (int64_t j = 0; j < nt; ++j) {
        const float e = dist2_b32(P[0], P[1], P[2], tgt[j], tgt[nt + j], tgt[2 * nt + j]);
        if (!(e <= dm2)) continue;
        if (best < 0 || before(e, j, bd, best)) {
            best = j;
            bd = e;
        }
    }
    return (int32_t)best;
}

int fgso_gicp_corr_some(int64_t ns, const float *src, int64_t nt, const float *tgt, const double R[9],
                        const double t[3], float d_max, int64_t nq, const int64_t *q, int32_t *corr)
{
    if (ns < 0 || nt < 0 || nq < 0 || !src || (nt > 0 && !tgt) || !R || !t || !corr) return -1;
    float R32[9], t32[3];
    for (int k = 0; k < 9; ++k) R32[k] = (float)R[k];
    for (int k = 0; k < 3; ++k) t32[k] = (float)t[k];
    const float dm2 = b_mul(d_max, d_max);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < nq; ++a) corr[a] = corr_of(q ? q[a] : a, ns, src, nt, tgt, R32, t32, dm2);
    return 0;
}

int fgso_gicp_linearize(int64_t ns, const float *src, const double *src_cov, int64_t nt, const float *tgt,
                        const double *tgt_cov, const double R[9], const double t[3], float d_max, double H[36],
                        double b[6], double *cost, int64_t *count, int32_t *corr)
{
    if (ns < 0 || nt < 0 || (ns > 0 && (!src || !src_cov)) || (nt > 0 && (!tgt || !tgt_cov)) || !R || !t || !H ||
        !b)
        return -1;
    int32_t *cj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ns > 0 ? ns : 1));
    if (!cj) return -2;
    fgso_gicp_corr_some(ns, src, nt, tgt, R, t, d_max, ns, NULL, cj);
    for (int q = 0; q < 36; ++q) H[q] = 0.0;
    for (int q = 0; q < 6; ++q) b[q] = 0.0;
    double c = 0.0;
    int64_t m = 0;
    for (int64_t i = 0; i < ns; ++i) {
        if (corr) corr[i] = cj[i];
        const int64_t j = cj[i];
        if (j < 0) continue;
        const double p[3] = {src[i], src[ns + i], src[2 * ns + i]};
        double Tp[3], d[3];
        for (int r = 0; r < 3; ++r) Tp[r] = R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2] + t[r];
        for (int r = 0; r < 3; ++r) d[r] = (double)tgt[r * nt + j] - Tp[r];
        double Cp[3][3], Cq[3][3], RC[3][3], C[3][3], Wm[3][3];
        sym_at(src_cov, ns, i, Cp);
        sym_at(tgt_cov, nt, j, Cq);
        for (int r = 0; r < 3; ++r)
            for (int s = 0; s < 3; ++s) {
                RC[r][s] = 0.0;
                for (int u = 0; u < 3; ++u) RC[r][s] += R[3 * r + u] * Cp[u][s];
            }
        for (int r = 0; r < 3; ++r)
            for (int s = 0; s < 3; ++s) {
                double a = 0.0;
                for (int u = 0; u < 3; ++u) a += RC[r][u] * R[3 * s + u];
                C[r][s] = Cq[r][s] + a;
            }
        if (inverse3(C, Wm) != 0) continue;
        /* J = [[Tp]_x, -I]: [a]_x = [[0, -a2, a1], [a2, 0, -a0], [-a1, a0, 0]] */
        double J[3][6] = {{0, -Tp[2], Tp[1], -1, 0, 0}, {Tp[2], 0, -Tp[0], 0, -1, 0}, {-Tp[1], Tp[0], 0, 0, 0, -1}};
        double WJ[3][6], Wd[3];
        for (int r = 0; r < 3; ++r) {
            Wd[r] = Wm[r][0] * d[0] + Wm[r][1] * d[1] + Wm[r][2] * d[2];
            for (int q = 0; q < 6; ++q) WJ[r][q] = Wm[r][0] * J[0][q] + Wm[r][1] * J[1][q] + Wm[r][2] * J[2][q];
        }
        for (int q = 0; q < 6; ++q) {
            for (int s = 0; s < 6; ++s) H[6 * q + s] += J[0][q] * WJ[0][s] + J[1][q] * WJ[1][s] + J[2][q] * WJ[2][s];
            b[q] += J[0][q] * Wd[0] + J[1][q] * Wd[1] + J[2][q] * Wd[2];
        }
        c += d[0] * Wd[0] + d[1] * Wd[1] + d[2] * Wd[2];
        m++;
    }
    free(cj);
    if (cost) *cost = c;
    if (count) *count = m;
    return 0;
}

void fgso_so3_exp(const double w[3], double E[9])
{
    const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    /* E = I + A [w]_x + B [w]_x^2 with A = sin(th)/th, B = (1 - cos(th))/th^2 (series near 0) */
    double A, B;
    if (th < 1e-5) {
        A = 1.0 - th * th / 6.0;
        B = 0.5 - th * th / 24.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / (th * th);
    }
    const double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double K2 = 0.0;
            for (int u = 0; u < 3; ++u) K2 += K[r][u] * K[u][c];
            E[3 * r + c] = (r == c ? 1.0 : 0.0) + A * K[r][c] + B * K2;
        }
}

/* Cholesky solve of the 6x6 system H x = rhs; -1 when H is not positive definite. */
static int chol_solve6(const double H[36], const double rhs[6], double x[6])
{
    double L[6][6] = {{0}};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = H[6 * i + j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0)) return -1;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = rhs[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return 0;
}

int fgso_gicp_align(int64_t ns, const float *src, const double *src_cov, int64_t nt, const float *tgt,
                    const double *tgt_cov, const double R0[9], const double t0[3], float d_max, int32_t max_iter,
                    double eps_rot, double eps_trans, double R[9], double t[3], int32_t *iters, int32_t *status,
                    double *cost, int64_t *count)
{
    if (!R0 || !t0 || !R || !t || max_iter < 0) return -1;
    memcpy(R, R0, sizeof(double) * 9);
    memcpy(t, t0, sizeof(double) * 3);
    int32_t it = 0, st = 1;
    double c = 0.0;
    int64_t m = 0;
    while (it < max_iter) {
        double H[36], b[6], x[6], rhs[6];
        if (fgso_gicp_linearize(ns, src, src_cov, nt, tgt, tgt_cov, R, t, d_max, H, b, &c, &m, NULL) != 0) return -1;
        for (int q = 0; q < 6; ++q) rhs[q] = -b[q];
        if (m < 6 || chol_solve6(H, rhs, x) != 0) {
            st = 2;
            break;
        }
        double E[9], Rn[9], tn[3];
        fgso_so3_exp(x, E);
        for (int r = 0; r < 3; ++r) {
            for (int s = 0; s < 3; ++s) Rn[3 * r + s] = E[3 * r] * R[s] + E[3 * r + 1] * R[3 + s] + E[3 * r + 2] * R[6 + s];
            tn[r] = E[3 * r] * t[0] + E[3 * r + 1] * t[1] + E[3 * r + 2] * t[2] + x[3 + r];
        }
        memcpy(R, Rn, sizeof(Rn));
        memcpy(t, tn, sizeof(tn));
        it++;
        const double nw = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double nv = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
        if (nw < eps_rot && nv < eps_trans) {
            st = 0;
            break;
        }
    }
    if (iters) *iters = it;
    if (status) *status = st;
    if (cost) *cost = c;
    if (count) *count = m;
    return 0;
}
