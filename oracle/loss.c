/*
 * Oracle: the structural-similarity term and the scale regulariser of the mapping loss
 * (Sec. III-D "Map Optimization", Eq. 15 and Eq. 16). FP64, plain loops.
 *
 * TEST INFRASTRUCTURE ONLY (see fgso.h).
 *
 * SSIM (the paper names it without a definition; the standard windowed index is used): per
 * channel and pixel p, window moments over the 11x11 gaussian window w (sigma 1.5, normalised to
 * sum 1) centred on p, pixels outside the image counting as zero:
 *   mu_x = sum w x,  mu_y = sum w y,  m_xx = sum w x^2,  m_yy = sum w y^2,  m_xy = sum w x y,
 *   S_p = (2 mu_x mu_y + C1)(2 (m_xy - mu_x mu_y) + C2)
 *         / ((mu_x^2 + mu_y^2 + C1)((m_xx - mu_x^2) + (m_yy - mu_y^2) + C2)),
 * with C1 = 0.01^2, C2 = 0.03^2 (intensities in [0, 1]); ssim = the mean of S over the 3 P
 * (pixel, channel) values. Its gradient with respect to x_q: S_p depends on x only through
 * mu_x, m_xx and m_xy at p, each a window sum, so
 *   d ssim / d x_q = 1/(3P) sum_p w(p - q) (dS/dmu_x + 2 x_q dS/dm_xx + y_q dS/dm_xy)_p,
 * the sum over the image pixels p whose window contains q.
 *
 * Scale regulariser (Eq. 15), with S the gaussians' scales exp(log-scale) in their stored axis
 * order, the mean of the first two taken per gaussian and epsilon = 0:
 *   L_reg = 1/n sum_i (|s_i1 - m_i| + |s_i2 - m_i|) + 1/n sum_i s_i3,  m_i = (s_i1 + s_i2)/2,
 * i.e. 1/n sum_i (|s_i1 - s_i2| + s_i3).
 */
#include <math.h>
#include <stdlib.h>

#include "fgso.h"

#define SSIM_R 5
#define SSIM_K (2 * SSIM_R + 1)

static double sgn(double v) { return (double)((v > 0) - (v < 0)); }

/* The 11x11 window: w[(dy + R) K + (dx + R)] = exp(-(dx^2 + dy^2) / (2 sigma^2)) / sum. */
static void ssim_window(double w[SSIM_K * SSIM_K])
{
    const double sigma = 1.5;
    double sum = 0.0;
    for (int dy = -SSIM_R; dy <= SSIM_R; ++dy)
        for (int dx = -SSIM_R; dx <= SSIM_R; ++dx) {
            const double v = exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma * sigma));
            w[(dy + SSIM_R) * SSIM_K + dx + SSIM_R] = v;
            sum += v;
        }
    for (int k = 0; k < SSIM_K * SSIM_K; ++k) w[k] /= sum;
}

int fgso_ssim(int32_t W, int32_t H, const double *img, const double *tgt, double *ssim, double *grad,
              double *smap)
{
    if (W <= 0 || H <= 0 || !img || !tgt) return -1;
    const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
    const int64_t P = (int64_t)W * H;
    double w[SSIM_K * SSIM_K];
    ssim_window(w);
    /* per (channel, pixel): S and the three partial derivatives */
    double *dA = malloc(sizeof(double) * 3 * P), *dB = malloc(sizeof(double) * 3 * P);
    double *dC = malloc(sizeof(double) * 3 * P), *S = malloc(sizeof(double) * 3 * P);
    if (!dA || !dB || !dC || !S) {
        free(dA); free(dB); free(dC); free(S);
        return -2;
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < 3; ++c)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const double *X = img + (int64_t)c * P, *Y = tgt + (int64_t)c * P;
                double mx = 0, my = 0, mxx = 0, myy = 0, mxy = 0;
                for (int dy = -SSIM_R; dy <= SSIM_R; ++dy)
                    for (int dx = -SSIM_R; dx <= SSIM_R; ++dx) {
                        const int xx = x + dx, yy = y + dy;
                        if (xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
                        const double wv = w[(dy + SSIM_R) * SSIM_K + dx + SSIM_R];
                        const double a = X[(int64_t)yy * W + xx], b = Y[(int64_t)yy * W + xx];
                        mx += wv * a;
                        my += wv * b;
                        mxx += wv * a * a;
                        myy += wv * b * b;
                        mxy += wv * a * b;
                    }
                const double a1 = 2.0 * mx * my + C1, a2 = 2.0 * (mxy - mx * my) + C2;
                const double b1 = mx * mx + my * my + C1, b2 = (mxx - mx * mx) + (myy - my * my) + C2;
                const double s = (a1 * a2) / (b1 * b2);
                const int64_t k = (int64_t)c * P + (int64_t)y * W + x;
                S[k] = s;
                /* d log S = d a1 / a1 + d a2 / a2 - d b1 / b1 - d b2 / b2, with
                 * d(a1, a2, b1, b2)/d mu_x = (2 mu_y, -2 mu_y, 2 mu_x, -2 mu_x),
                 * d/d m_xx = (0, 0, 0, 1), d/d m_xy = (0, 2, 0, 0) */
                dA[k] = s * (2.0 * my / a1 - 2.0 * my / a2 - 2.0 * mx / b1 + 2.0 * mx / b2);
                dB[k] = -s / b2;
                dC[k] = s * 2.0 / a2;
            }
    double sum = 0.0;
    for (int64_t k = 0; k < 3 * P; ++k) sum += S[k];
    if (ssim) *ssim = sum / (3.0 * (double)P);
    if (smap)
        for (int64_t k = 0; k < 3 * P; ++k) smap[k] = S[k];
    if (grad) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int c = 0; c < 3; ++c)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    const int64_t q = (int64_t)c * P + (int64_t)y * W + x;
                    double a = 0, b = 0, cc = 0;
                    for (int dy = -SSIM_R; dy <= SSIM_R; ++dy)
                        for (int dx = -SSIM_R; dx <= SSIM_R; ++dx) {
                            const int px = x + dx, py = y + dy;  /* a pixel p whose window holds q */
                            if (px < 0 || px >= W || py < 0 || py >= H) continue;
                            const double wv = w[(-dy + SSIM_R) * SSIM_K + (-dx + SSIM_R)];  /* w(q - p) */
                            const int64_t k = (int64_t)c * P + (int64_t)py * W + px;
                            a += wv * dA[k];
                            b += wv * dB[k];
                            cc += wv * dC[k];
                        }
                    grad[q] = (a + 2.0 * img[q] * b + tgt[q] * cc) / (3.0 * (double)P);
                }
    }
    free(dA); free(dB); free(dC); free(S);
    return 0;
}

int fgso_scale_reg(int64_t n, const double *log_scale, double *value, double *grad)
{
    if (n < 0 || (n > 0 && !log_scale)) return -1;
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double s1 = exp(log_scale[i]), s2 = exp(log_scale[n + i]), s3 = exp(log_scale[2 * n + i]);
        const double m = 0.5 * (s1 + s2);
        sum += fabs(s1 - m) + fabs(s2 - m) + s3;
        if (grad) {
            /* d/d log s_k = s_k d/d s_k; d(|s1 - m| + |s2 - m|)/d s1 = sgn(s1 - m)/2 - sgn(s2 - m)/2 */
            const double d1 = 0.5 * sgn(s1 - m) - 0.5 * sgn(s2 - m);
            const double d2 = 0.5 * sgn(s2 - m) - 0.5 * sgn(s1 - m);
            grad[i] = s1 * d1 / (double)n;
            grad[n + i] = s2 * d2 / (double)n;
            grad[2 * n + i] = s3 / (double)n;
        }
    }
    if (value) *value = n > 0 ? sum / (double)n : 0.0;
    return 0;
}
