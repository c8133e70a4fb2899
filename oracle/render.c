/*
 * FGS oracle, rendering part: projection of 3D gaussians, front-to-back alpha
 * compositing (Eq. 1) and its analytic backward, in FP64.
 *
 * TEST INFRASTRUCTURE ONLY (see fgso.h): not linked into the product library.
 *
 * What is computed (the gaussian set of Sec. III, covariance C = R S S^T R^T):
 *  - q_hat = q/|q|, R = R(q_hat), S = diag(exp(s)), Sigma = R S S^T R^T.
 *  - t = R_cw mu + t_cw; culled when t_z <= z_near.
 *  - EWA projection: J = [[fx/tz, 0, -fx tx/tz^2], [0, fy/tz, -fy ty/tz^2]], A = J R_cw,
 *    Sigma' = A Sigma A^T + lowpass * I; conic = Sigma'^-1; culled when det Sigma' <= 0.
 *  - mean2 = (fx tx/tz + cx, fy ty/tz + cy); pixel (x, y) samples (x + 0.5, y + 0.5).
 *  - Per pixel, the candidates are the gaussians with Q = d^T conic d <= sigma_cut^2,
 *    ordered by (depth, index). The order is a decision that floating point takes; it is taken
 *    on the depth rounded to binary32, the precision of the rasterizer's sort key (the depth
 *    itself, as blended, stays FP64), so that equal binary32 depths blend in index order. Eq. 1 is evaluated front to back with
 *    alpha = min(alpha_max, o exp(-Q/2)), skipping alpha < alpha_min, and stopping
 *    (without compositing) at the first gaussian that would take T below T_min.
 *  - Colour = sum w_i c_i + T bg, depth = sum w_i d_i + T bg_depth, opacity = sum w_i,
 *    with w_i = alpha_i prod_{j<i}(1 - alpha_j) (Eq. 1 with gamma = c, d, 1).
 * The backward is the chain rule through exactly these steps with the set of
 * contributors held fixed.
 */
#include "fgso.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int valid;
    double t[3];
    double cov2[3];   /* Sigma'_xx, Sigma'_xy, Sigma'_yy */
    double conic[3];  /* a, b, c of Sigma'^-1 */
    double m2[2];
    double depth, opacity;
    double qn[4], qnorm;
    double Rq[9];     /* R(q_hat), row-major */
    double s[3];      /* exp(log-scale) */
    double Sig[9];    /* 3D covariance */
    double A[6];      /* J R_cw, 2x3 row-major */
} proj_t;

static int opts_ok(const fgso_camera *cam, const fgso_render_opts *o)
{
    if (!cam || !o) return 0;
    if (cam->width <= 0 || cam->height <= 0) return 0;
    if (!(cam->fx > 0) || !(cam->fy > 0)) return 0;
    if (!(o->sigma_cut > 0) || !(o->alpha_max > 0) || !(o->alpha_max < 1)) return 0;
    if (!(o->T_min >= 0) || !(o->lowpass >= 0)) return 0;
    return 1;
}

/* Unit-quaternion rotation matrix, q = (w, x, y, z). */
static void quat_to_rot(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void project_one(int64_t n, int64_t i, const double *params, const fgso_camera *cam,
                        const fgso_render_opts *o, proj_t *p)
{
    memset(p, 0, sizeof(*p));
    const double *mean = params, *ls = params + 3 * n, *quat = params + 6 * n;
    const double *logit = params + 10 * n;
    double mu[3] = {mean[i], mean[n + i], mean[2 * n + i]};
    double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
    double qq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(qq > 0) || !isfinite(qq)) return;
    p->qnorm = qq;
    for (int k = 0; k < 4; ++k) p->qn[k] = q[k] / qq;
    quat_to_rot(p->qn, p->Rq);
    for (int k = 0; k < 3; ++k) p->s[k] = exp(ls[k * n + i]);
    /* Sigma = (R S)(R S)^T */
    double M[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = p->Rq[3 * r + c] * p->s[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += M[3 * r + k] * M[3 * c + k];
            p->Sig[3 * r + c] = acc;
        }
    const double *W = cam->R;
    for (int r = 0; r < 3; ++r)
        p->t[r] = W[3 * r] * mu[0] + W[3 * r + 1] * mu[1] + W[3 * r + 2] * mu[2] + cam->t[r];
    double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    if (!(tz > cam->z_near)) return;
    double J[6] = {cam->fx / tz, 0, -cam->fx * tx / (tz * tz),
                   0, cam->fy / tz, -cam->fy * ty / (tz * tz)};
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += J[3 * r + k] * W[3 * k + c];
            p->A[3 * r + c] = acc;
        }
    double AS[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += p->A[3 * r + k] * p->Sig[3 * k + c];
            AS[3 * r + c] = acc;
        }
    double S2[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += AS[3 * r + k] * p->A[3 * c + k];
            S2[2 * r + c] = acc;
        }
    p->cov2[0] = S2[0] + o->lowpass;
    p->cov2[1] = 0.5 * (S2[1] + S2[2]);
    p->cov2[2] = S2[3] + o->lowpass;
    double det = p->cov2[0] * p->cov2[2] - p->cov2[1] * p->cov2[1];
    if (!(det > 0) || !isfinite(det)) return;
    p->conic[0] = p->cov2[2] / det;
    p->conic[1] = -p->cov2[1] / det;
    p->conic[2] = p->cov2[0] / det;
    p->m2[0] = cam->fx * tx / tz + cam->cx;
    p->m2[1] = cam->fy * ty / tz + cam->cy;
    p->depth = tz;
    p->opacity = 1.0 / (1.0 + exp(-logit[i]));
    if (!isfinite(p->m2[0]) || !isfinite(p->m2[1]) || !isfinite(p->opacity)) return;
    p->valid = 1;
}

int fgso_project(int64_t n, const double *params, const fgso_camera *cam,
                 const fgso_render_opts *o, double *proj)
{
    if (n < 0 || (n > 0 && (!params || !proj)) || !opts_ok(cam, o)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        proj_t p;
        project_one(n, i, params, cam, o, &p);
        double *d = proj + FGSO_PROJ_STRIDE * i;
        d[0] = p.valid;
        for (int k = 0; k < 3; ++k) { d[1 + k] = p.t[k]; d[4 + k] = p.cov2[k]; d[7 + k] = p.conic[k]; }
        d[10] = p.m2[0]; d[11] = p.m2[1]; d[12] = p.depth; d[13] = p.opacity; d[14] = 0; d[15] = 0;
    }
    return 0;
}

/* ------------------------------ candidate lists ------------------------------ */

typedef struct {
    int32_t tiles_x, tiles_y;
    int64_t *start;   /* tiles+1 */
    int32_t *idx;     /* gaussian indices, per tile sorted by (depth, index) */
} buckets_t;

#define BUCKET 16

/* Pixel-index range [lo, hi] whose centres x+0.5 lie within [c - r, c + r]. */
static int px_range(double c, double r, int32_t size, int32_t *lo, int32_t *hi)
{
    double a = ceil(c - r - 0.5), b = floor(c + r - 0.5);
    if (!(a <= b)) return 0;
    if (b < 0 || a > size - 1) return 0;
    *lo = a < 0 ? 0 : (int32_t)a;
    *hi = b > size - 1 ? size - 1 : (int32_t)b;
    return 1;
}

typedef struct {
    double d;
    int32_t i;
} dkey_t;

static int cmp_key(const void *a, const void *b)
{
    const dkey_t *x = (const dkey_t *)a, *y = (const dkey_t *)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->i > y->i) - (x->i < y->i);
}

/* The depth that orders the blending: the camera-space depth rounded to binary32. */
static double order_key(double depth) { return (double)(float)depth; }

/* Order idx[0..cnt) by (binary32 depth, index) ascending; tmp holds cnt keys. */
static void sort_by_depth(const proj_t *P, int32_t *idx, int64_t cnt, dkey_t *tmp)
{
    for (int64_t k = 0; k < cnt; ++k) { tmp[k].d = order_key(P[idx[k]].depth); tmp[k].i = idx[k]; }
    qsort(tmp, (size_t)cnt, sizeof(dkey_t), cmp_key);
    for (int64_t k = 0; k < cnt; ++k) idx[k] = tmp[k].i;
}

static int build_buckets(int64_t n, const proj_t *P, const fgso_camera *cam, double cut,
                         buckets_t *b)
{
    b->tiles_x = (cam->width + BUCKET - 1) / BUCKET;
    b->tiles_y = (cam->height + BUCKET - 1) / BUCKET;
    int64_t T = (int64_t)b->tiles_x * b->tiles_y;
    b->start = (int64_t *)calloc((size_t)T + 1, sizeof(int64_t));
    if (!b->start) return -1;
    int32_t *rect = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(n > 0 ? n : 1));
    if (!rect) return -1;
    for (int64_t i = 0; i < n; ++i) {
        rect[4 * i] = 1; rect[4 * i + 1] = 0;
        if (!P[i].valid) continue;
        int32_t x0, x1, y0, y1;
        double rx = cut * sqrt(P[i].cov2[0]) * (1 + 1e-9) + 1e-9;
        double ry = cut * sqrt(P[i].cov2[2]) * (1 + 1e-9) + 1e-9;
        if (!px_range(P[i].m2[0], rx, cam->width, &x0, &x1)) continue;
        if (!px_range(P[i].m2[1], ry, cam->height, &y0, &y1)) continue;
        rect[4 * i] = x0 / BUCKET; rect[4 * i + 1] = x1 / BUCKET;
        rect[4 * i + 2] = y0 / BUCKET; rect[4 * i + 3] = y1 / BUCKET;
        for (int32_t ty = rect[4 * i + 2]; ty <= rect[4 * i + 3]; ++ty)
            for (int32_t tx = rect[4 * i]; tx <= rect[4 * i + 1]; ++tx)
                b->start[(int64_t)ty * b->tiles_x + tx + 1]++;
    }
    for (int64_t k = 0; k < T; ++k) b->start[k + 1] += b->start[k];
    b->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(b->start[T] > 0 ? b->start[T] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)T);
    if (!b->idx || !fill) return -1;
    memcpy(fill, b->start, sizeof(int64_t) * (size_t)T);
    for (int64_t i = 0; i < n; ++i) {
        if (rect[4 * i] > rect[4 * i + 1]) continue;
        for (int32_t ty = rect[4 * i + 2]; ty <= rect[4 * i + 3]; ++ty)
            for (int32_t tx = rect[4 * i]; tx <= rect[4 * i + 1]; ++tx)
                b->idx[fill[(int64_t)ty * b->tiles_x + tx]++] = (int32_t)i;
    }
    free(fill);
    free(rect);
    return 0;
}

static void sort_buckets(const proj_t *P, buckets_t *b, const uint8_t *need)
{
    int64_t T = (int64_t)b->tiles_x * b->tiles_y;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < T; ++k) {
        if (need && !need[k]) continue;
        int64_t cnt = b->start[k + 1] - b->start[k];
        dkey_t *tmp = (dkey_t *)malloc(sizeof(dkey_t) * (size_t)(cnt > 0 ? cnt : 1));
        sort_by_depth(P, b->idx + b->start[k], cnt, tmp);
        free(tmp);
    }
}

/* ------------------------------ per-pixel compositing ------------------------------ */

typedef struct {
    int32_t i;
    int clamped;
    double alpha, G, dx, dy;
} contrib_t;

typedef struct {
    double C[3], D, A, T;
    int32_t nc;
    int amb;
    double ef;
    int64_t consumed; /* list entries up to the one at which the pixel stopped (all when it never did) */
    int64_t last_pos; /* 1 + list position of the last contributor (0: none) */
} pixel_out_t;

/* Upper bound on contributors per pixel: every contributor has alpha >= alpha_min, so T
 * falls below T_min after at most log(T_min)/log(1 - alpha_min) of them (2,344 for the
 * default cutoffs); the buffers below hold this many. */
static int64_t max_contrib(const fgso_render_opts *o)
{
    double am = o->alpha_min > 1e-6 ? o->alpha_min : 1e-6;
    double tm = o->T_min > 1e-300 ? o->T_min : 1e-300;
    double k = ceil(log(tm) / log1p(-am)) + 2;
    return (int64_t)(k < 1e7 ? k : 1e7);
}

/* Eq. 1 for one pixel over an ordered candidate list (a superset of the gaussians with
 * Q <= cut^2, ordered by (depth, index)). Contributors are appended to seq. */
static void composite(const proj_t *P, const double *col, int64_t n, const int32_t *list,
                      int64_t cnt, double px, double py, const fgso_render_opts *o,
                      double amb_rel, pixel_out_t *out, contrib_t *seq, int64_t cap)
{
    double cut2 = o->sigma_cut * o->sigma_cut;
    double T = 1, C[3] = {0, 0, 0}, D = 0, A = 0, prev_d = -1;
    int32_t nc = 0;
    int amb = 0;
    double ef = 0;
    int64_t consumed = cnt, last_pos = 0;
    for (int64_t k = 0; k < cnt; ++k) {
        int32_t i = list[k];
        const proj_t *g = &P[i];
        if (!g->valid) continue;
        double dx = px - g->m2[0], dy = py - g->m2[1];
        double Q = g->conic[0] * dx * dx + 2 * g->conic[1] * dx * dy + g->conic[2] * dy * dy;
        if (amb_rel > 0 && fabs(Q - cut2) <= amb_rel * cut2) amb |= 1;
        if (!(Q <= cut2)) continue;
        ef += 1;
        double G = exp(-0.5 * Q);
        double ar = g->opacity * G;
        if (amb_rel > 0 && (fabs(ar - o->alpha_min) <= amb_rel * o->alpha_min ||
                            fabs(ar - o->alpha_max) <= amb_rel * o->alpha_max)) amb |= 1;
        int clamped = ar > o->alpha_max;
        double alpha = clamped ? o->alpha_max : ar;
        if (alpha < o->alpha_min) continue;
        double Tn = T * (1 - alpha);
        if (amb_rel > 0 && fabs(Tn - o->T_min) <= amb_rel * o->T_min) amb |= 1;
        if (Tn < o->T_min) { consumed = k + 1; break; }
        if (amb_rel > 0 && prev_d >= 0 && order_key(g->depth) == prev_d) amb |= 2;
        prev_d = order_key(g->depth);
        double w = alpha * T;
        for (int ch = 0; ch < 3; ++ch) C[ch] += w * col[ch * n + i];
        D += w * g->depth;
        A += w;
        if (seq && nc < cap) {
            seq[nc].i = i; seq[nc].clamped = clamped; seq[nc].alpha = alpha;
            seq[nc].G = G; seq[nc].dx = dx; seq[nc].dy = dy;
        }
        T = Tn;
        nc++;
        last_pos = k + 1;
    }
    for (int ch = 0; ch < 3; ++ch) out->C[ch] = C[ch];
    out->T = T; out->A = A; out->D = D; out->nc = nc; out->amb = amb; out->ef = ef;
    out->consumed = consumed; out->last_pos = last_pos;
}

/* Candidate list for a brute-force pixel: all valid gaussians with Q <= cut2_ext, ordered
 * by (depth, index). */
static int64_t brute_list(int64_t n, const proj_t *P, double px, double py, double cut2_ext,
                          int32_t *list, dkey_t *tmp)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!P[i].valid) continue;
        double dx = px - P[i].m2[0], dy = py - P[i].m2[1];
        double Q = P[i].conic[0] * dx * dx + 2 * P[i].conic[1] * dx * dy + P[i].conic[2] * dy * dy;
        if (Q <= cut2_ext) list[cnt++] = (int32_t)i;
    }
    sort_by_depth(P, list, cnt, tmp);
    return cnt;
}

typedef struct {
    proj_t *P;
    buckets_t b;
    int have_b;
    int64_t n_out;
} setup_t;

static int setup(int64_t n, const double *params, const fgso_camera *cam, const fgso_render_opts *o,
                 int mode, int64_t n_pix, const int64_t *pix, double amb_rel, setup_t *s)
{
    memset(s, 0, sizeof(*s));
    int64_t P_all = (int64_t)cam->width * cam->height;
    s->n_out = pix ? n_pix : P_all;
    s->P = (proj_t *)malloc(sizeof(proj_t) * (size_t)(n > 0 ? n : 1));
    if (!s->P) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) project_one(n, i, params, cam, o, &s->P[i]);
    if (mode == 0) {
        double cut = o->sigma_cut * sqrt(1 + (amb_rel > 0 ? 2 * amb_rel : 0));
        if (build_buckets(n, s->P, cam, cut, &s->b)) return -1;
        s->have_b = 1;
        uint8_t *need = NULL;
        if (pix) {
            int64_t T = (int64_t)s->b.tiles_x * s->b.tiles_y;
            need = (uint8_t *)calloc((size_t)T, 1);
            for (int64_t k = 0; k < n_pix; ++k) {
                int64_t x = pix[k] % cam->width, y = pix[k] / cam->width;
                need[(y / BUCKET) * s->b.tiles_x + x / BUCKET] = 1;
            }
        }
        sort_buckets(s->P, &s->b, need);
        free(need);
    }
    return 0;
}

static void teardown(setup_t *s)
{
    free(s->P);
    if (s->have_b) { free(s->b.start); free(s->b.idx); }
}

/* The ordered candidate list of pixel (x, y). */
static int64_t pixel_list(const setup_t *s, int64_t n, int mode, int32_t x, int32_t y,
                          double cut2_ext, int32_t *buf, dkey_t *tmp, const int32_t **L)
{
    if (mode == 0) {
        int64_t tile = (int64_t)(y / BUCKET) * s->b.tiles_x + x / BUCKET;
        *L = s->b.idx + s->b.start[tile];
        return s->b.start[tile + 1] - s->b.start[tile];
    }
    *L = buf;
    return brute_list(n, s->P, x + 0.5, y + 0.5, cut2_ext, buf, tmp);
}

int fgso_render_fwd(int64_t n, const double *params, const fgso_camera *cam,
                    const fgso_render_opts *o, int mode, int64_t n_pix, const int64_t *pix,
                    double *rgb, double *depth, double *alpha, double *T_final,
                    int32_t *n_contrib, uint8_t *amb, double amb_rel, double *stats)
{
    if (n < 0 || (n > 0 && !params) || !opts_ok(cam, o) || (mode != 0 && mode != 1)) return -1;
    if (pix && n_pix < 0) return -1;
    if (!rgb || !depth || !alpha || !T_final || !n_contrib) return -1;
    int64_t P_all = (int64_t)cam->width * cam->height;
    if (pix)
        for (int64_t k = 0; k < n_pix; ++k)
            if (pix[k] < 0 || pix[k] >= P_all) return -1;
    setup_t s;
    if (setup(n, params, cam, o, mode, n_pix, pix, amb_rel, &s)) { teardown(&s); return -2; }
    int64_t n_out = s.n_out;
    const double *col = params + 11 * n;
    double cut2_ext = o->sigma_cut * o->sigma_cut * (1 + (amb_rel > 0 ? 2 * amb_rel : 0));
    double ef_tot = 0, ec_tot = 0, amb_tot = 0;
    int64_t cap = max_contrib(o);
#pragma omp parallel reduction(+ : ef_tot, ec_tot, amb_tot)
    {
        int32_t *buf = mode == 1 ? (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)) : NULL;
        dkey_t *tmp = mode == 1 ? (dkey_t *)malloc(sizeof(dkey_t) * (size_t)(n > 0 ? n : 1)) : NULL;
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < n_out; ++k) {
            int64_t p = pix ? pix[k] : k;
            int32_t x = (int32_t)(p % cam->width), y = (int32_t)(p / cam->width);
            const int32_t *L;
            int64_t cnt = pixel_list(&s, n, mode, x, y, cut2_ext, buf, tmp, &L);
            pixel_out_t po;
            composite(s.P, col, n, L, cnt, x + 0.5, y + 0.5, o, amb_rel, &po, NULL, 0);
            for (int c = 0; c < 3; ++c) rgb[c * n_out + k] = po.C[c] + po.T * o->bg[c];
            depth[k] = po.D + po.T * o->bg_depth;
            alpha[k] = po.A;
            T_final[k] = po.T;
            n_contrib[k] = po.nc;
            if (amb) amb[k] = (uint8_t)po.amb;
            ef_tot += po.ef;
            ec_tot += po.nc;
            amb_tot += (po.amb & 1) != 0;
        }
        free(buf);
        free(tmp);
    }
    (void)cap;
    if (stats) { stats[0] = ef_tot; stats[1] = ec_tot; stats[2] = amb_tot; stats[3] = (double)n_out; }
    teardown(&s);
    return 0;
}

/* ------------------------------ backward ------------------------------ */

/* dL/dparams for one gaussian from its 2D gradient g2 = dL/d(m2x, m2y, ca, cb, cc, o, r, g, b, d). */
static void chain_one(const proj_t *p, const fgso_camera *cam, const double *g2, double out[14])
{
    memset(out, 0, sizeof(double) * 14);
    if (!p->valid) return;
    double a = p->conic[0], b = p->conic[1], c = p->conic[2];
    double X[4] = {a, b, b, c};
    double Gh[4] = {g2[2], 0.5 * g2[3], 0.5 * g2[3], g2[4]};
    /* dSigma' = - X Gh X */
    double XG[4], dS2[4];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 2; ++k) XG[2 * r + k] = X[2 * r] * Gh[k] + X[2 * r + 1] * Gh[2 + k];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 2; ++k) dS2[2 * r + k] = -(XG[2 * r] * X[k] + XG[2 * r + 1] * X[2 + k]);
    /* dSigma = A^T dSigma' A ; dA = 2 dSigma' A Sigma */
    const double *A = p->A;
    double dSig[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0;
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) acc += A[3 * u + r] * dS2[2 * u + v] * A[3 * v + k];
            dSig[3 * r + k] = acc;
        }
    double dA[6];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0;
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 3; ++v) acc += dS2[2 * r + u] * A[3 * u + v] * p->Sig[3 * v + k];
            dA[3 * r + k] = 2 * acc;
        }
    /* A = J W: dJ = dA W^T */
    const double *W = cam->R;
    double dJ[6];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0;
            for (int v = 0; v < 3; ++v) acc += dA[3 * r + v] * W[3 * k + v];
            dJ[3 * r + k] = acc;
        }
    double tx = p->t[0], ty = p->t[1], tz = p->t[2], fx = cam->fx, fy = cam->fy;
    double dt[3] = {0, 0, 0};
    /* J entries as functions of t */
    dt[2] += dJ[0] * (-fx / (tz * tz));
    dt[0] += dJ[2] * (-fx / (tz * tz));
    dt[2] += dJ[2] * (2 * fx * tx / (tz * tz * tz));
    dt[2] += dJ[4] * (-fy / (tz * tz));
    dt[1] += dJ[5] * (-fy / (tz * tz));
    dt[2] += dJ[5] * (2 * fy * ty / (tz * tz * tz));
    /* projected mean and depth */
    dt[0] += g2[0] * fx / tz;
    dt[2] += g2[0] * (-fx * tx / (tz * tz));
    dt[1] += g2[1] * fy / tz;
    dt[2] += g2[1] * (-fy * ty / (tz * tz));
    dt[2] += g2[9];
    /* t = W mu + t_cw */
    for (int k = 0; k < 3; ++k) out[k] = W[k] * dt[0] + W[3 + k] * dt[1] + W[6 + k] * dt[2];
    /* Sigma = M M^T, M = R S */
    double M[9], dM[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) M[3 * r + k] = p->Rq[3 * r + k] * p->s[k];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0;
            for (int v = 0; v < 3; ++v) acc += dSig[3 * r + v] * M[3 * v + k];
            dM[3 * r + k] = 2 * acc;
        }
    for (int k = 0; k < 3; ++k) {
        double acc = 0;
        for (int r = 0; r < 3; ++r) acc += p->Rq[3 * r + k] * dM[3 * r + k];
        out[3 + k] = acc * p->s[k];
    }
    double dR[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) dR[3 * r + k] = dM[3 * r + k] * p->s[k];
    double w = p->qn[0], x = p->qn[1], y = p->qn[2], z = p->qn[3];
    double dq[4];
    dq[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] +
                 w * dR[7] - 2 * x * dR[8]);
    dq[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                 z * dR[7] - 2 * y * dR[8]);
    dq[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] +
                 x * dR[6] + y * dR[7]);
    double dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    for (int k = 0; k < 4; ++k) out[6 + k] = (dq[k] - p->qn[k] * dot) / p->qnorm;
    out[10] = g2[5] * p->opacity * (1 - p->opacity);
    out[11] = g2[6]; out[12] = g2[7]; out[13] = g2[8];
}

int fgso_render_bwd(int64_t n, const double *params, const fgso_camera *cam,
                    const fgso_render_opts *o, int mode, int64_t n_pix, const int64_t *pix,
                    const double *g_rgb, const double *g_depth, const double *g_alpha,
                    double *grad, double *grad2d, double *mass)
{
    if (n < 0 || (n > 0 && (!params || !grad)) || !opts_ok(cam, o) || (mode != 0 && mode != 1))
        return -1;
    if (!g_rgb || !g_depth) return -1;
    int64_t P_all = (int64_t)cam->width * cam->height;
    if (pix)
        for (int64_t k = 0; k < n_pix; ++k)
            if (pix[k] < 0 || pix[k] >= P_all) return -1;
    setup_t s;
    if (setup(n, params, cam, o, mode, n_pix, pix, 0, &s)) { teardown(&s); return -2; }
    int64_t n_out = s.n_out;
    const double *col = params + 11 * n;
    double cut2 = o->sigma_cut * o->sigma_cut;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nthr * 10 * (size_t)(n > 0 ? n : 1), sizeof(double));
    if (!acc) { teardown(&s); return -2; }
    /* with mass: the same sums over the absolute values of every term (see fgso.h) */
    double *macc = mass ? (double *)calloc((size_t)nthr * 10 * (size_t)(n > 0 ? n : 1), sizeof(double)) : NULL;
    if (mass && !macc) { free(acc); teardown(&s); return -2; }
    int64_t seq_cap = max_contrib(o);
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g2 = acc + (size_t)tid * 10 * (size_t)n;
        double *m2 = macc ? macc + (size_t)tid * 10 * (size_t)n : NULL;
        int32_t *buf = mode == 1 ? (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)) : NULL;
        dkey_t *tmp = mode == 1 ? (dkey_t *)malloc(sizeof(dkey_t) * (size_t)(n > 0 ? n : 1)) : NULL;
        contrib_t *seq = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)seq_cap);
        double *Ts = (double *)malloc(sizeof(double) * (size_t)(seq_cap + 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < n_out; ++k) {
            int64_t p = pix ? pix[k] : k;
            int32_t x = (int32_t)(p % cam->width), y = (int32_t)(p / cam->width);
            const int32_t *L;
            int64_t cnt = pixel_list(&s, n, mode, x, y, cut2, buf, tmp, &L);
            pixel_out_t po;
            composite(s.P, col, n, L, cnt, x + 0.5, y + 0.5, o, 0, &po, seq, seq_cap);
            int32_t m = po.nc;
            Ts[0] = 1;
            for (int32_t j = 0; j < m; ++j) Ts[j + 1] = Ts[j] * (1 - seq[j].alpha);
            double Tf = Ts[m];
            double gC[3] = {g_rgb[k], g_rgb[n_out + k], g_rgb[2 * n_out + k]};
            double gD = g_depth[k], gA = g_alpha ? g_alpha[k] : 0;
            /* suffix sums of what lies behind contributor j */
            double BC[3] = {Tf * o->bg[0], Tf * o->bg[1], Tf * o->bg[2]};
            double BD = Tf * o->bg_depth;
            /* absolute mass of what lies behind (for the mass diagnostic) */
            double Babs = Tf * (fabs(gC[0] * o->bg[0]) + fabs(gC[1] * o->bg[1]) + fabs(gC[2] * o->bg[2]) +
                                fabs(gD * o->bg_depth) + fabs(gA));
            for (int32_t j = m - 1; j >= 0; --j) {
                const contrib_t *e = &seq[j];
                const proj_t *g = &s.P[e->i];
                double Tj = Ts[j], a = e->alpha, w = a * Tj;
                double c3[3] = {col[e->i], col[n + e->i], col[2 * n + e->i]};
                double dalpha = 0;
                for (int ch = 0; ch < 3; ++ch) dalpha += gC[ch] * (Tj * c3[ch] - BC[ch] / (1 - a));
                dalpha += gD * (Tj * g->depth - BD / (1 - a));
                dalpha += gA * Tf / (1 - a);
                double *d = g2;
                for (int ch = 0; ch < 3; ++ch) d[(6 + ch) * n + e->i] += gC[ch] * w;
                d[9 * n + e->i] += gD * w;
                if (!e->clamped) {
                    d[5 * n + e->i] += dalpha * e->G;
                    double dQ = -0.5 * a * dalpha;
                    double ca = g->conic[0], cb = g->conic[1], cc = g->conic[2];
                    d[0 * n + e->i] += dQ * (-2 * (ca * e->dx + cb * e->dy));
                    d[1 * n + e->i] += dQ * (-2 * (cb * e->dx + cc * e->dy));
                    d[2 * n + e->i] += dQ * e->dx * e->dx;
                    d[3 * n + e->i] += dQ * 2 * e->dx * e->dy;
                    d[4 * n + e->i] += dQ * e->dy * e->dy;
                }
                if (m2) {
                    double Xabs = fabs(gC[0] * c3[0]) + fabs(gC[1] * c3[1]) + fabs(gC[2] * c3[2]) +
                                  fabs(gD * g->depth);
                    for (int ch = 0; ch < 3; ++ch) m2[(6 + ch) * n + e->i] += fabs(gC[ch] * w);
                    m2[9 * n + e->i] += fabs(gD * w);
                    if (!e->clamped) {
                        double dam = Tj * Xabs + Babs / (1 - a); /* mass of dL/dalpha */
                        double dQm = 0.5 * a * dam;
                        double ca = fabs(g->conic[0]), cb = fabs(g->conic[1]), cc = fabs(g->conic[2]);
                        double adx = fabs(e->dx), ady = fabs(e->dy);
                        m2[5 * n + e->i] += dam * e->G;
                        m2[0 * n + e->i] += dQm * 2 * (ca * adx + cb * ady);
                        m2[1 * n + e->i] += dQm * 2 * (cb * adx + cc * ady);
                        m2[2 * n + e->i] += dQm * adx * adx;
                        m2[3 * n + e->i] += dQm * 2 * adx * ady;
                        m2[4 * n + e->i] += dQm * ady * ady;
                    }
                    Babs += w * Xabs;
                }
                for (int ch = 0; ch < 3; ++ch) BC[ch] += w * c3[ch];
                BD += w * g->depth;
            }
        }
        free(buf);
        free(tmp);
        free(seq);
        free(Ts);
    }
    /* reduce per-thread buffers and apply the per-gaussian chain rule */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double g2[10];
        for (int k = 0; k < 10; ++k) {
            double t = 0;
            for (int th = 0; th < nthr; ++th) t += acc[(size_t)th * 10 * (size_t)n + (size_t)k * n + i];
            g2[k] = t;
        }
        if (grad2d)
            for (int k = 0; k < 10; ++k) grad2d[k * n + i] = g2[k];
        double out[14];
        chain_one(&s.P[i], cam, g2, out);
        for (int k = 0; k < 14; ++k) grad[k * n + i] = out[k];
        if (mass) {
            /* parameter mass: sum_j |d grad_k / d g2_j| * mass of g2_j (the chain rule is linear) */
            double mk[14] = {0};
            for (int j = 0; j < 10; ++j) {
                double mj = 0;
                for (int th = 0; th < nthr; ++th) mj += macc[(size_t)th * 10 * (size_t)n + (size_t)j * n + i];
                if (mj == 0) continue;
                double unit[10] = {0}, col_j[14];
                unit[j] = 1;
                chain_one(&s.P[i], cam, unit, col_j);
                for (int k = 0; k < 14; ++k) mk[k] += fabs(col_j[k]) * mj;
            }
            for (int k = 0; k < 14; ++k) mass[k * n + i] = mk[k];
        }
    }
    free(acc);
    free(macc);
    teardown(&s);
    return 0;
}

int64_t fgso_count_duplicates(int64_t n, const double *params, const fgso_camera *cam,
                              const fgso_render_opts *o, int32_t tile_w, int32_t tile_h)
{
    if (n < 0 || !opts_ok(cam, o) || tile_w <= 0 || tile_h <= 0) return -1;
    int64_t K = 0;
#pragma omp parallel for reduction(+ : K) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        proj_t p;
        project_one(n, i, params, cam, o, &p);
        if (!p.valid) continue;
        int32_t x0, x1, y0, y1;
        if (!px_range(p.m2[0], o->sigma_cut * sqrt(p.cov2[0]), cam->width, &x0, &x1)) continue;
        if (!px_range(p.m2[1], o->sigma_cut * sqrt(p.cov2[2]), cam->height, &y0, &y1)) continue;
        K += (int64_t)(x1 / tile_w - x0 / tile_w + 1) * (y1 / tile_h - y0 / tile_h + 1);
    }
    return K;
}

/* Work counts of the tile formulation (16x16 tiles, lists of the gaussians whose sigma_cut box
 * reaches the tile, in (binary32 depth, index) order): counts[0] = K_c, the (tile, gaussian) pairs
 * with at least one blended pixel; counts[1] = L_f, per tile the list entries up to the last one
 * any pixel examined (a pixel examines up to the entry at which it stops, the whole list when it
 * never stops), summed; counts[2] = L_b, per tile the list entries up to the last blended one,
 * summed; counts[3] = K, the list entries of all tiles. */
int fgso_tile_counts(int64_t n, const double *params, const fgso_camera *cam, const fgso_render_opts *o,
                     int64_t counts[4])
{
    if (n < 0 || (n > 0 && !params) || !opts_ok(cam, o) || !counts) return -1;
    setup_t s;
    if (setup(n, params, cam, o, 0, 0, NULL, 0, &s)) { teardown(&s); return -2; }
    const double *col = params + 11 * n;
    int64_t T = (int64_t)s.b.tiles_x * s.b.tiles_y;
    int64_t kc = 0, lf = 0, lb = 0;
    int64_t cap = max_contrib(o);
#pragma omp parallel reduction(+ : kc, lf, lb)
    {
        contrib_t *seq = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)cap);
        uint8_t *seen = NULL;
        int64_t seen_cap = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < T; ++t) {
            int64_t cnt = s.b.start[t + 1] - s.b.start[t];
            const int32_t *L = s.b.idx + s.b.start[t];
            if (cnt > seen_cap) {
                free(seen);
                seen = (uint8_t *)malloc((size_t)cnt);
                seen_cap = cnt;
            }
            if (cnt) memset(seen, 0, (size_t)cnt);
            int32_t tx = (int32_t)(t % s.b.tiles_x), ty = (int32_t)(t / s.b.tiles_x);
            int64_t tf = 0, tb = 0;
            for (int32_t y = ty * BUCKET; y < (ty + 1) * BUCKET && y < cam->height; ++y)
                for (int32_t x = tx * BUCKET; x < (tx + 1) * BUCKET && x < cam->width; ++x) {
                    pixel_out_t po;
                    composite(s.P, col, n, L, cnt, x + 0.5, y + 0.5, o, 0, &po, seq, cap);
                    if (po.consumed > tf) tf = po.consumed;
                    if (po.last_pos > tb) tb = po.last_pos;
                    /* mark the contributors' list positions (the list holds each gaussian once) */
                    for (int32_t j = 0, k = 0; j < po.nc && j < cap; ++j) {
                        while (k < cnt && L[k] != seq[j].i) ++k;
                        if (k < cnt) seen[k] = 1;
                    }
                }
            for (int64_t k = 0; k < cnt; ++k) kc += seen[k];
            lf += tf;
            lb += tb;
        }
        free(seq);
        free(seen);
    }
    counts[0] = kc;
    counts[1] = lf;
    counts[2] = lb;
    counts[3] = s.b.start[T];
    teardown(&s);
    return 0;
}
