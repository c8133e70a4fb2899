/*
 * FGS oracle: the learned seeding prior, in FP64.
 *
 * TEST INFRASTRUCTURE ONLY (see fgso.h).
 *
 * The paper assigns every seed the radius of Eq. 11 and a constant opacity. The learned
 * prior replaces that with a small network evaluated per 16x16 tile:
 *  - features: the tile's 16x16 luma DFT (Eq. 2 applied to the tile), centred so that DC sits
 *    at index (8, 8) (Eq. 3), magnitude (Eq. 4), as log(1 + |F_c|), 256 values in row-major
 *    (v, u) order; then mean, standard deviation, minimum and maximum of the tile's valid depth;
 *  - network: h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), y = W3 h2 + b3, with
 *    GELU(a) = a/2 (1 + erf(a/sqrt 2)); sizes 260 -> 256 -> 256 -> 4;
 *  - with bf16 set, every GEMM operand (weights, input, hidden activations, and the upstream
 *    gradients in the backward) is rounded to bfloat16, round-to-nearest-even; sums are FP64.
 */
#include "fgso.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NI 260
#define NH 256
#define NO 4

static double bf16(double v)
{
    if (v == 0 || !isfinite(v)) return v;
    int e;
    frexp(v, &e);                 /* v = m 2^e, 0.5 <= |m| < 1 */
    double s = ldexp(1.0, 8 - e); /* 8 significant bits */
    return nearbyint(v * s) / s;  /* default rounding mode: to nearest, ties to even */
}

static double op(double v, int on) { return on ? bf16(v) : v; }

static double gelu(double a) { return 0.5 * a * (1.0 + erf(a / sqrt(2.0))); }

static double gelu_grad(double a)
{
    return 0.5 * (1.0 + erf(a / sqrt(2.0))) + a * exp(-0.5 * a * a) / sqrt(2.0 * M_PI);
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3;
} net_t;

static void unpack(const double *w, net_t *n)
{
    n->W1 = w;
    n->b1 = n->W1 + NH * NI;
    n->W2 = n->b1 + NH;
    n->b2 = n->W2 + NH * NH;
    n->W3 = n->b2 + NH;
    n->b3 = n->W3 + NO * NH;
}

int fgso_mlp_fwd(int64_t rows, const double *x, const double *w, int bf, double *y,
                 double *h1_out, double *h2_out, double *a1_out, double *a2_out)
{
    if (rows < 0 || (rows > 0 && (!x || !w || !y))) return -1;
    net_t n;
    unpack(w, &n);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        double a1[NH], h1[NH], a2[NH], h2[NH];
        const double *xr = x + r * NI;
        for (int j = 0; j < NH; ++j) {
            double s = 0;
            for (int k = 0; k < NI; ++k) s += op(n.W1[j * NI + k], bf) * op(xr[k], bf);
            a1[j] = s + n.b1[j];
            h1[j] = gelu(a1[j]);
        }
        for (int j = 0; j < NH; ++j) {
            double s = 0;
            for (int k = 0; k < NH; ++k) s += op(n.W2[j * NH + k], bf) * op(h1[k], bf);
            a2[j] = s + n.b2[j];
            h2[j] = gelu(a2[j]);
        }
        for (int j = 0; j < NO; ++j) {
            double s = 0;
            for (int k = 0; k < NH; ++k) s += op(n.W3[j * NH + k], bf) * op(h2[k], bf);
            y[r * NO + j] = s + n.b3[j];
        }
        if (h1_out) memcpy(h1_out + r * NH, h1, sizeof(h1));
        if (h2_out) memcpy(h2_out + r * NH, h2, sizeof(h2));
        if (a1_out) memcpy(a1_out + r * NH, a1, sizeof(a1));
        if (a2_out) memcpy(a2_out + r * NH, a2, sizeof(a2));
    }
    return 0;
}

int fgso_mlp_bwd(int64_t rows, const double *x, const double *w, int bf, const double *target,
                 double *gw, double *loss)
{
    if (rows <= 0 || !x || !w || !target || !gw) return -1;
    net_t n;
    unpack(w, &n);
    double *y = (double *)malloc(sizeof(double) * (size_t)rows * NO);
    double *h1 = (double *)malloc(sizeof(double) * (size_t)rows * NH);
    double *h2 = (double *)malloc(sizeof(double) * (size_t)rows * NH);
    double *a1 = (double *)malloc(sizeof(double) * (size_t)rows * NH);
    double *a2 = (double *)malloc(sizeof(double) * (size_t)rows * NH);
    double *dy = (double *)malloc(sizeof(double) * (size_t)rows * NO);
    double *da2 = (double *)malloc(sizeof(double) * (size_t)rows * NH);
    double *da1 = (double *)malloc(sizeof(double) * (size_t)rows * NH);
    if (!y || !h1 || !h2 || !a1 || !a2 || !dy || !da2 || !da1) return -2;
    fgso_mlp_fwd(rows, x, w, bf, y, h1, h2, a1, a2);
    double L = 0, scale = 1.0 / ((double)rows * NO);
    for (int64_t k = 0; k < rows * NO; ++k) {
        double r = y[k] - target[k];
        L += r * r * scale;
        dy[k] = 2 * r * scale;
    }
    if (loss) *loss = L;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        for (int j = 0; j < NH; ++j) {
            double s = 0;
            for (int o = 0; o < NO; ++o) s += op(dy[r * NO + o], bf) * op(n.W3[o * NH + j], bf);
            da2[r * NH + j] = s * gelu_grad(a2[r * NH + j]);
        }
        for (int j = 0; j < NH; ++j) {
            double s = 0;
            for (int o = 0; o < NH; ++o) s += op(da2[r * NH + o], bf) * op(n.W2[o * NH + j], bf);
            da1[r * NH + j] = s * gelu_grad(a1[r * NH + j]);
        }
    }
    double *gW1 = gw, *gb1 = gW1 + NH * NI, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH;
    double *gW3 = gb2 + NH, *gb3 = gW3 + NO * NH;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < NH; ++j) {
        for (int k = 0; k < NI; ++k) {
            double s = 0;
            for (int64_t r = 0; r < rows; ++r) s += op(da1[r * NH + j], bf) * op(x[r * NI + k], bf);
            gW1[j * NI + k] = s;
        }
        for (int k = 0; k < NH; ++k) {
            double s = 0;
            for (int64_t r = 0; r < rows; ++r) s += op(da2[r * NH + j], bf) * op(h1[r * NH + k], bf);
            gW2[j * NH + k] = s;
        }
        double s1 = 0, s2 = 0;
        for (int64_t r = 0; r < rows; ++r) { s1 += da1[r * NH + j]; s2 += da2[r * NH + j]; }
        gb1[j] = s1;
        gb2[j] = s2;
    }
    for (int o = 0; o < NO; ++o) {
        for (int k = 0; k < NH; ++k) {
            double s = 0;
            for (int64_t r = 0; r < rows; ++r) s += op(dy[r * NO + o], bf) * op(h2[r * NH + k], bf);
            gW3[o * NH + k] = s;
        }
        double s = 0;
        for (int64_t r = 0; r < rows; ++r) s += dy[r * NO + o];
        gb3[o] = s;
    }
    free(y); free(h1); free(h2); free(a1); free(a2); free(dy); free(da2); free(da1);
    return 0;
}

int fgso_tile_features(int32_t W, int32_t H, const float *rgb, const float *depth,
                       int32_t tx, int32_t ty, double depth_min, double depth_max, double *feat)
{
    if (W <= 0 || H <= 0 || !rgb || !depth || !feat || tx < 0 || ty < 0) return -1;
    int64_t P = (int64_t)W * H;
    double Y[16][16];
    int valid = 0;
    double sum = 0, sum2 = 0, mn = INFINITY, mx = -INFINITY;
    for (int y = 0; y < 16; ++y)
        for (int x = 0; x < 16; ++x) {
            int64_t gx = (int64_t)tx * 16 + x, gy = (int64_t)ty * 16 + y;
            Y[y][x] = 0;
            if (gx >= W || gy >= H) continue;
            int64_t p = gy * W + gx;
            Y[y][x] = 0.299 * (double)rgb[p] + 0.587 * (double)rgb[P + p] + 0.114 * (double)rgb[2 * P + p];
            double d = depth[p];
            if (isfinite(d) && d >= depth_min && d <= depth_max) {
                valid++;
                sum += d;
                sum2 += d * d;
                if (d < mn) mn = d;
                if (d > mx) mx = d;
            }
        }
    const double two_pi = 6.283185307179586476925286766559;
    for (int v = 0; v < 16; ++v)
        for (int u = 0; u < 16; ++u) {
            double re = 0, im = 0;
            for (int y = 0; y < 16; ++y)
                for (int x = 0; x < 16; ++x) {
                    double ang = two_pi * (double)((u * x + v * y) % 16) / 16.0;
                    re += Y[y][x] * cos(ang);
                    im -= Y[y][x] * sin(ang);
                }
            int i = (u + 8) % 16, j = (v + 8) % 16;
            feat[j * 16 + i] = log1p(sqrt(re * re + im * im));
        }
    if (valid) {
        double mean = sum / valid, var = sum2 / valid - mean * mean;
        feat[256] = mean;
        feat[257] = sqrt(var > 0 ? var : 0);
        feat[258] = mn;
        feat[259] = mx;
    } else {
        feat[256] = feat[257] = feat[258] = feat[259] = 0;
    }
    return valid;
}
