/*
 * Oracle: gaussian pruning (Sec. III-D, "Gaussian Pruning"). FP64 values of binary32 parameters,
 * plain loops.
 *
 * TEST INFRASTRUCTURE ONLY (see fgso.h).
 *
 * The paper removes two kinds of gaussians: those grown too large in any dimension, and those
 * whose opacity is below a threshold. It gives neither threshold a value nor says how "too large"
 * is measured; the reading taken here:
 *   - a gaussian is too large when any of its three scales exp(log-scale) exceeds max_scale
 *     (world units); max_scale <= 0 or +inf turns the test off;
 *   - its opacity is too low when sigmoid(opacity logit) < min_opacity, min_opacity in [0, 1).
 * Both thresholds are binary32 values, as the parameters are. The decisions are taken on the
 * stored binary32 values, against the thresholds carried into their domains (sigmoid and exp are
 * increasing): the gaussian is kept when
 *   logit >= L_o = fl(log(min_opacity / (1 - min_opacity)))  (L_o = -inf for min_opacity = 0), and
 *   log-scale_k <= L_s = fl(log(max_scale)) for k = 1, 2, 3  (L_s = +inf when the test is off),
 * each threshold computed in FP64 and rounded to binary32 (fl). A NaN in the logit or a log-scale
 * fails its comparison, so such a gaussian is removed.
 *
 * Survivors keep their order: compaction writes the j-th kept gaussian (in index order) to
 * position j of every plane.
 */
#include <math.h>

#include "fgso.h"

static double to_binary32(double v) { return (double)(float)v; }

int fgso_prune_thresholds(double min_opacity, double max_scale, double *L_o, double *L_s)
{
    /* the thresholds are binary32 values, as the parameters are */
    min_opacity = to_binary32(min_opacity);
    max_scale = to_binary32(max_scale);
    if (!(min_opacity >= 0.0 && min_opacity < 1.0) || isnan(max_scale)) return -1;
    *L_o = min_opacity > 0.0 ? to_binary32(log(min_opacity / (1.0 - min_opacity))) : -INFINITY;
    *L_s = (max_scale > 0.0 && isfinite(max_scale)) ? to_binary32(log(max_scale)) : INFINITY;
    return 0;
}

int64_t fgso_prune_keep(int64_t n, const double *params, double min_opacity, double max_scale, uint8_t *keep)
{
    double L_o, L_s;
    if (n < 0 || (n > 0 && (!params || !keep))) return -1;
    if (fgso_prune_thresholds(min_opacity, max_scale, &L_o, &L_s) != 0) return -1;
    const double *log_scale = params + 3 * n, *logit = params + 10 * n;
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) {
        int ok = logit[i] >= L_o;
        for (int k = 0; k < 3; ++k) ok = ok && log_scale[k * n + i] <= L_s;
        keep[i] = (uint8_t)ok;
        kept += ok;
    }
    return kept;
}

int64_t fgso_compact(int64_t n, int32_t planes, const double *in, const uint8_t *keep, double *out,
                     int64_t out_stride)
{
    if (n < 0 || planes <= 0 || (n > 0 && (!in || !keep || !out))) return -1;
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) kept += keep[i] != 0;
    if (out_stride < kept) return -1;
    for (int32_t k = 0; k < planes; ++k) {
        int64_t j = 0;
        for (int64_t i = 0; i < n; ++i)
            if (keep[i]) out[(int64_t)k * out_stride + j++] = in[(int64_t)k * n + i];
    }
    return kept;
}
