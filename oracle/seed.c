/*
 * FGS oracle: Fourier seeding of new gaussians (Sec. III-A, "Mapping": Eq. 2-8, the triangle
 * threshold and Eq. 11), in FP64 with a naive separable DFT.
 *
 * TEST INFRASTRUCTURE ONLY (see fgso.h).
 *
 * Steps, in the paper's order:
 *  1. The frame I(x, y) is the BT.601 luma of the RGB frame (colours in [0, 1]).
 *  2. F = DFT of I (Eq. 2), evaluated as row DFTs followed by column DFTs; the twiddle
 *     angle uses (u x mod W)/W so its reduction is exact.
 *  3. Centring (Eq. 3) places the filter centre at DC: D^2(u, v) = ub^2 + vb^2 with
 *     ub = u for u < W/2 else u - W (vb likewise); the Gaussian high-pass of Eq. 5,
 *     H = 1 - exp(-D^2/(2 D0^2)), multiplies the spectrum (Eq. 7).
 *  4. The inverse DFT with the 1/(HW) factor (Eq. 8) gives I_h; E = |I_h|.
 *  5. E is quantised to q = floor(255 (E / E_max)) and histogrammed in 256 bins (the ratio first,
 *     so the pixel at the maximum maps exactly to 255: x / x = 1 in IEEE arithmetic). A frame whose
 *     E_max is at rounding level, E_max <= 1e-9 max|I|, is flat: it has no high-frequency
 *     region (a constant frame gives E == 0 in exact arithmetic).
 *  6. The triangle method picks the threshold t (the bin furthest below the line from the
 *     histogram's peak to the end of its longer tail); M_h = {q > t}, M_l its complement.
 *  7. Seeds lie on a stride-m lattice inside M_h and a stride-n lattice inside M_l, where the
 *     depth is finite and inside [depth_min, depth_max].
 *  8. Each seed is back-projected at its pixel centre with its depth, and gets the radius
 *     r = alpha d / f of Eq. 11 (alpha = alpha_h in M_h, alpha_l in M_l) and the pixel colour.
 *     Every value of step 8 is a fixed sequence of IEEE binary32 operations without fused
 *     multiply-add; each operation is evaluated in FP64 and rounded to binary32, which equals
 *     the binary32 operation for +, -, *, / (53 >= 2*24 + 2).
 */
#include "fgso.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* binary32 operations evaluated in FP64 and rounded once */
static float f_add(float a, float b) { return (float)((double)a + (double)b); }
static float f_sub(float a, float b) { return (float)((double)a - (double)b); }
static float f_mul(float a, float b) { return (float)((double)a * (double)b); }
static float f_div(float a, float b) { return (float)((double)a / (double)b); }

/* One naive DFT pass over `count` sequences of length L (stride `step` between elements,
 * `dist` between sequences); sign = -1 forward, +1 inverse. */
static void dft_pass(int64_t count, int64_t L, int64_t step, int64_t dist, int sign,
                     const double *re_in, const double *im_in, double *re_out, double *im_out)
{
    double *c = (double *)malloc(sizeof(double) * (size_t)L);
    double *s = (double *)malloc(sizeof(double) * (size_t)L);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t k = 0; k < L; ++k) {
        double ang = two_pi * (double)k / (double)L;
        c[k] = cos(ang);
        s[k] = sign * sin(ang);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < count; ++j) {
        const double *xr = re_in + j * dist, *xi = im_in ? im_in + j * dist : NULL;
        for (int64_t u = 0; u < L; ++u) {
            double ar = 0, ai = 0;
            for (int64_t x = 0; x < L; ++x) {
                int64_t k = (u * x) % L;
                double vr = xr[x * step], vi = xi ? xi[x * step] : 0.0;
                ar += vr * c[k] - vi * s[k];
                ai += vr * s[k] + vi * c[k];
            }
            re_out[j * dist + u * step] = ar;
            im_out[j * dist + u * step] = ai;
        }
    }
    free(c);
    free(s);
}

int fgso_highpass(int32_t W, int32_t H, const float *rgb, double D0, double *E_out,
                  int64_t *hist_out, int32_t *thresh_out, double *margin_out)
{
    if (W <= 0 || H <= 0 || !rgb || !(D0 > 0)) return -1;
    int64_t P = (int64_t)W * H;
    double *Y = (double *)malloc(sizeof(double) * (size_t)P);
    double *ar = (double *)malloc(sizeof(double) * (size_t)P), *ai = (double *)malloc(sizeof(double) * (size_t)P);
    double *br = (double *)malloc(sizeof(double) * (size_t)P), *bi = (double *)malloc(sizeof(double) * (size_t)P);
    double *E = (double *)malloc(sizeof(double) * (size_t)P);
    if (!Y || !ar || !ai || !br || !bi || !E) return -2;
    for (int64_t p = 0; p < P; ++p)
        Y[p] = 0.299 * (double)rgb[p] + 0.587 * (double)rgb[P + p] + 0.114 * (double)rgb[2 * P + p];
    /* Eq. 2: rows (length W, stride 1) then columns (length H, stride W) */
    dft_pass(H, W, 1, W, -1, Y, NULL, ar, ai);
    dft_pass(W, H, W, 1, -1, ar, ai, br, bi);
    /* Eq. 3, 5, 7 */
    for (int32_t v = 0; v < H; ++v) {
        double vb = v < H / 2.0 ? v : v - H;
        for (int32_t u = 0; u < W; ++u) {
            double ub = u < W / 2.0 ? u : u - W;
            double D2 = ub * ub + vb * vb;
            double Hf = 1.0 - exp(-D2 / (2.0 * D0 * D0));
            br[(int64_t)v * W + u] *= Hf;
            bi[(int64_t)v * W + u] *= Hf;
        }
    }
    /* Eq. 8: inverse columns then rows, 1/(HW) */
    dft_pass(W, H, W, 1, +1, br, bi, ar, ai);
    dft_pass(H, W, 1, W, +1, ar, ai, br, bi);
    double Emax = 0, Ymax = 0;
    for (int64_t p = 0; p < P; ++p) {
        double re = br[p] / (double)P, im = bi[p] / (double)P;
        E[p] = sqrt(re * re + im * im);
        if (E[p] > Emax) Emax = E[p];
        if (fabs(Y[p]) > Ymax) Ymax = fabs(Y[p]);
    }
    if (Emax <= 1e-9 * Ymax) Emax = 0; /* flat frame */
    int64_t hist[256];
    memset(hist, 0, sizeof(hist));
    double margin = INFINITY;
    int32_t t = -1;
    if (Emax > 0) {
        int64_t arg = -1;
        for (int64_t p = 0; p < P; ++p)
            if (E[p] == Emax) { arg = p; break; }
        for (int64_t p = 0; p < P; ++p) {
            double r = 255.0 * (E[p] / Emax);
            int32_t q = (int32_t)floor(r);
            if (q > 255) q = 255;
            hist[q]++;
            /* distance to the nearest integer k >= 1 (floor cannot change on [0, 1), E >= 0) */
            double k = nearbyint(r);
            if (p != arg && k >= 1.0) {
                double d = fabs(r - k);
                if (d < margin) margin = d;
            }
        }
        t = fgso_triangle(hist);
    }
    if (E_out) memcpy(E_out, E, sizeof(double) * (size_t)P);
    if (hist_out) memcpy(hist_out, hist, sizeof(hist));
    if (thresh_out) *thresh_out = t;
    if (margin_out) *margin_out = margin;
    free(Y); free(ar); free(ai); free(br); free(bi); free(E);
    return 0;
}

/* Triangle threshold: peak p (first maximum), endpoint e = the last non-empty bin of the longer
 * side (the right one on equal lengths). For bins strictly between p and e, the distance below
 * the line from (p, h_p) to (e, h_e) is proportional to the cross product taken with the sign
 * that makes "below" positive; the largest wins, the bin nearest the peak on ties. */
int32_t fgso_triangle(const int64_t *h)
{
    int32_t a = -1, b = -1, p = 0;
    for (int32_t i = 0; i < 256; ++i) {
        if (h[i] > 0) { if (a < 0) a = i; b = i; }
        if (h[i] > h[p]) p = i;
    }
    if (a < 0) return 0;
    int32_t e = (b - p >= p - a) ? b : a;
    int32_t dir = e > p ? 1 : -1;
    int32_t best = p;
    int64_t best_val = INT64_MIN;
    for (int32_t i = p + dir; i != e && (e - i) * dir > 0; i += dir) {
        int64_t cross = (int64_t)(e - p) * (h[i] - h[p]) - (h[e] - h[p]) * (int64_t)(i - p);
        int64_t below = dir > 0 ? -cross : cross;
        if (below > best_val) { best_val = below; best = i; }
    }
    return best;
}

int64_t fgso_seed(int32_t W, int32_t H, const float *rgb, const float *depth,
                  const float cam_R[9], const float cam_t[3], float fx, float fy, float cx, float cy,
                  const fgso_seed_opts *o, int64_t capacity, int32_t *pixel, uint8_t *is_high,
                  float *mean, float *radius, float *seed_rgb, int32_t *tile_count,
                  int32_t *thresh_out, double *margin_out, const fgso_missing *miss, uint8_t *missing_out)
{
    if (miss && (!miss->alpha || !miss->depth || !miss->rgb)) return -1;
    if (W <= 0 || H <= 0 || !rgb || !depth || !o || !cam_R || !cam_t) return -1;
    if (o->m <= 0 || o->n <= 0 || o->tile <= 0 || capacity < 0) return -1;
    if (!(fx > 0) || !(fy > 0)) return -1;
    int64_t P = (int64_t)W * H;
    double *E = (double *)malloc(sizeof(double) * (size_t)P);
    int32_t t;
    double margin;
    if (fgso_highpass(W, H, rgb, o->D0, E, NULL, &t, &margin)) { free(E); return -1; }
    double Emax = 0;
    if (t >= 0)
        for (int64_t p = 0; p < P; ++p)
            if (E[p] > Emax) Emax = E[p];
    int32_t tiles_x = (W + o->tile - 1) / o->tile, tiles_y = (H + o->tile - 1) / o->tile;
    if (tile_count) memset(tile_count, 0, sizeof(int32_t) * (size_t)tiles_x * tiles_y);
    float ah = (float)o->alpha_h, al = (float)o->alpha_l;
    int64_t count = 0;
    for (int32_t y = 0; y < H; ++y)
        for (int32_t x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            float d = depth[p];
            int valid = isfinite(d) && d >= o->depth_min && d <= o->depth_max;
            /* Eq. 9: the missing region; without a map every pixel is missing */
            int missing = 1;
            if (miss) {
                /* M_d and M_c compare the surface the map shows: the rendered depth and colour over
                   the rendered opacity (Eq. 1 with gamma = d, c divided by gamma = 1) */
                float A = miss->alpha[p];
                int Mi = A < miss->tau_alpha, Md = 0, Mc = 0;
                if (A > 0) {
                    Md = valid && fabsf(f_sub(f_div(miss->depth[p], A), d)) > miss->tau_depth;
                    float dc = 0;
                    for (int c = 0; c < 3; ++c)
                        dc = f_add(dc, fabsf(f_sub(f_div(miss->rgb[c * P + p], A), rgb[c * P + p])));
                    Mc = dc > miss->tau_rgb;
                }
                missing = Mi || Md || Mc;
            }
            if (missing_out) missing_out[p] = (uint8_t)missing;
            if (!valid) continue;
            /* Eq. 10: both frequency masks are restricted to the missing region */
            if (!missing) continue;
            int high = 0;
            if (Emax > 0) {
                int32_t q = (int32_t)floor(255.0 * (E[p] / Emax));
                if (q > 255) q = 255;
                high = q > t;
            }
            int32_t stride = high ? o->m : o->n;
            if (x % stride || y % stride) continue;
            if (tile_count) tile_count[(y / o->tile) * tiles_x + x / o->tile]++;
            if (count < capacity) {
                float X = f_div(f_mul(f_sub(f_add((float)x, 0.5f), cx), d), fx);
                float Yc = f_div(f_mul(f_sub(f_add((float)y, 0.5f), cy), d), fy);
                float u0 = f_sub(X, cam_t[0]), u1 = f_sub(Yc, cam_t[1]), u2 = f_sub(d, cam_t[2]);
                for (int r = 0; r < 3; ++r)
                    mean[r * capacity + count] =
                        f_add(f_add(f_mul(cam_R[r], u0), f_mul(cam_R[3 + r], u1)), f_mul(cam_R[6 + r], u2));
                radius[count] = f_div(f_mul(high ? ah : al, d), fx);
                pixel[count] = (int32_t)p;
                is_high[count] = (uint8_t)high;
                for (int c = 0; c < 3; ++c) seed_rgb[c * capacity + count] = rgb[c * P + p];
            }
            count++;
        }
    if (thresh_out) *thresh_out = t;
    if (margin_out) *margin_out = margin;
    free(E);
    return count;
}
