// Internal declarations of the learned seeding prior (mlp.hip): per-tile spectral features, the
// 260 -> 256 -> 256 -> 4 GELU network with BF16 GEMM operands and FP32 accumulation on MFMA, its
// backward pass and Adam.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace fgs {

constexpr int kMlpIn = 260, kMlpHidden = 256, kMlpOut = 4;
constexpr int kMlpInPad = 288;  // input width padded to the MFMA k step (32)
constexpr int kMlpOutPad = 16;  // output rows of W3 padded to one MFMA tile
constexpr int kMlpOutK = 32;    // output width padded to the MFMA k step, as a reduction dimension
constexpr int64_t kMlpParams = (int64_t)kMlpHidden * kMlpIn + kMlpHidden + (int64_t)kMlpHidden * kMlpHidden +
                               kMlpHidden + kMlpOut * kMlpHidden + kMlpOut;  // 133,636
// offsets of the packed FP32 parameter vector: W1[256][260], b1, W2[256][256], b2, W3[4][256], b3
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + (int64_t)kMlpHidden * kMlpIn, kOffW2 = kOffB1 + kMlpHidden,
                  kOffB2 = kOffW2 + (int64_t)kMlpHidden * kMlpHidden, kOffW3 = kOffB2 + kMlpHidden,
                  kOffB3 = kOffW3 + kMlpOut * kMlpHidden;
constexpr int kMlpSplits = 16;  // split-K factor of the weight-gradient GEMMs

inline int64_t mlp_rows_padded(int64_t rows) { return (rows + 63) / 64 * 64; }

// Device workspace of the network for up to rows_cap rows (Rp = mlp_rows_padded(rows_cap)).
struct MlpWS {
    int64_t Rp = 0;
    uint16_t *W1b, *W2b, *W3b, *W2T, *W3T;  // BF16 shadow weights (padded, zero filled)
    uint16_t *Xb, *XT;                      // [Rp][288], [288][Rp]
    float *a1, *a2;                         // pre-activations [Rp][256]
    uint16_t *h1b, *h1T, *h2b, *h2T;        // activations [Rp][256], [256][Rp]
    uint16_t *dYb, *dYT;                    // [Rp][32], [16][Rp]
    uint16_t *da2b, *da2T, *da1T;           // [Rp][256], [256][Rp], [256][Rp]
    float *y;                               // [Rp][4]
    float *grad;                            // packed FP32 gradient
    float *partial;                         // split-K partials [kMlpSplits][256][288]
    double *loss;                           // one FP64 scalar
};
size_t mlp_ws_bytes(int64_t rows_cap);
void mlp_ws_carve(void *base, int64_t rows_cap, MlpWS *ws);

// Tile features: 256 log(1 + |DFT|) values of the tile's 16x16 luma, centred, then mean, std,
// min and max of valid depth; feat [n_tiles][260] FP32, n_valid [n_tiles] (nullable).
void launch_tile_features(const float *rgb, const float *depth, int W, int H, float dmin, float dmax, int64_t n_tiles,
                          const int32_t *tile_ids, float *feat, int32_t *n_valid, hipStream_t s);

// y [rows][4] = network(x [rows][260]) with the FP32 packed weights w.
void launch_mlp_forward(const MlpWS &ws, int64_t rows, const float *x, const float *w, float *y, bool keep_for_backward,
                        hipStream_t s);

// One training step on the mean squared error against target [rows][4]: forward, backward
// (gradient into ws.grad), Adam on w/m/v with bias corrections bc1, bc2. loss (nullable, FP32).
void launch_mlp_train_step(const MlpWS &ws, int64_t rows, const float *x, const float *target, float *w, float *m,
                           float *v, float lr, float beta1, float beta2, float eps, float bc1, float bc2, float *loss,
                           float *grad_out, hipStream_t s);

struct PriorApplyK {
    int tiles_x, W;
    float max_dev;    // fallback when a predicted offset exceeds this in magnitude
    float q[4];       // camera-to-world rotation (w, x, y, z): local axes = camera axes
    int32_t min_valid;  // fallback when a tile has fewer valid-depth pixels
    int32_t mode;       // 1: shape (log-scales, rotation) and opacity; 2: shape only; 3: opacity only
};

// Rewrites the seeds' log-scales, rotation and opacity logit from per-tile predictions y
// [tiles][4] (offsets from the radius rule's log-radius on the camera's x, y and viewing axes,
// opacity logit), keeping the radius rule where the tile or the prediction is rejected. The seed
// emission must have written log(radius) into log_scale. count: number of seeds (device), capped
// by capacity. from_prior (nullable): 1 where the prior was used.
void launch_prior_apply(const PriorApplyK &pk, const uint32_t *count, int64_t capacity, const int32_t *pixel,
                        const float *y, const int32_t *n_valid, float *log_scale, float *quat, float *logit,
                        int64_t stride, uint8_t *from_prior, hipStream_t s);

}  // namespace fgs
