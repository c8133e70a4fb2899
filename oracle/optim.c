/*
 * FGS oracle: the L1 colour and depth terms of the mapping loss (Eq. 16) and the
 * Adam update, in FP64.
 *
 * TEST INFRASTRUCTURE ONLY (see fgso.h).
 *
 * Loss (mean-reduced): L = l_rgb/(3P) sum |C - C*| + l_d/P_v sum_{D* > 0} |D - D*|, where P_v
 * counts pixels with a positive target depth; sign(0) is taken as 0 in the gradient.
 * PSNR = 10 log10(1 / MSE) over the three colour planes (colours in [0, 1]).
 * Adam: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, p <- p - lr mhat/(sqrt(vhat) + eps),
 * with mhat = m/(1-b1^k), vhat = v/(1-b2^k) for update number k = step + 1.
 */
#include "fgso.h"

#include <math.h>

static double sgn(double x) { return (x > 0) - (x < 0); }

int fgso_loss_l1(int64_t P, const double *rgb, const double *depth, const double *rgb_t,
                 const double *depth_t, double lambda_rgb, double lambda_depth,
                 double *g_rgb, double *g_depth, double *loss, double *psnr)
{
    if (P <= 0 || !rgb || !depth || !rgb_t || !depth_t) return -1;
    int64_t Pv = 0;
    for (int64_t p = 0; p < P; ++p) Pv += depth_t[p] > 0;
    double l1c = 0, l1d = 0, se = 0;
    for (int64_t k = 0; k < 3 * P; ++k) {
        double r = rgb[k] - rgb_t[k];
        l1c += fabs(r);
        se += r * r;
        if (g_rgb) g_rgb[k] = lambda_rgb * sgn(r) / (3.0 * (double)P);
    }
    for (int64_t p = 0; p < P; ++p) {
        double r = depth[p] - depth_t[p];
        int valid = depth_t[p] > 0;
        if (valid) l1d += fabs(r);
        if (g_depth) g_depth[p] = (valid && Pv > 0) ? lambda_depth * sgn(r) / (double)Pv : 0.0;
    }
    double L = lambda_rgb * l1c / (3.0 * (double)P) + (Pv > 0 ? lambda_depth * l1d / (double)Pv : 0.0);
    double mse = se / (3.0 * (double)P);
    if (loss) *loss = L;
    if (psnr) *psnr = mse > 0 ? 10.0 * log10(1.0 / mse) : INFINITY;
    return 0;
}

int fgso_adam(int64_t n, double *params, double *m, double *v, const double *grad,
              int64_t step, const double lr[5], double beta1, double beta2, double eps)
{
    if (n < 0 || step < 0 || !lr) return -1;
    if (n > 0 && (!params || !m || !v || !grad)) return -1;
    static const int group_of_row[14] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 3, 4, 4, 4};
    double k = (double)(step + 1);
    double bc1 = 1.0 - pow(beta1, k), bc2 = 1.0 - pow(beta2, k);
    for (int row = 0; row < 14; ++row) {
        double a = lr[group_of_row[row]];
        for (int64_t i = 0; i < n; ++i) {
            int64_t j = (int64_t)row * n + i;
            double g = grad[j];
            m[j] = beta1 * m[j] + (1 - beta1) * g;
            v[j] = beta2 * v[j] + (1 - beta2) * g * g;
            double mh = m[j] / bc1, vh = v[j] / bc2;
            params[j] -= a * mh / (sqrt(vh) + eps);
        }
    }
    return 0;
}
