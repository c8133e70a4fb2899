// Internal declarations of the Fourier seeding kernels (seed.hip).
#pragma once

#include "fgs_internal.h"

namespace fgs {

// Longest frame line the LDS-resident FFT holds (two FP64 complex lines + twiddles < 64 KiB).
constexpr int kSeedMaxLine = 1920;

struct SeedScalars {
    double emax;     // max |I_h| (0 for a flat frame)
    int32_t thresh;  // triangle threshold (-1: no high-frequency region)
    int32_t pad;
};

struct SeedK {
    int32_t m, n, tile;
    float dmin, dmax, alpha_h, alpha_l, opacity_logit;
    float fx, fy, cx, cy;
    float R[9], t[3];  // world -> camera pose; seeds go back to world coordinates
    // missing-region check: the map rendered at the frame's pose (ra == nullptr: every pixel
    // missing) and the thresholds on opacity, depth difference and summed colour difference
    const float *ra, *rd, *rc;
    float tau_a, tau_d, tau_c;
};

struct SeedOutK {
    int64_t capacity;
    int32_t *pixel;
    uint8_t *is_high;
    float *mean, *radius, *rgb;
    int32_t *tile_count;
    int64_t *n_dev;
    GradK params;  // params.mean == nullptr: not written
    double *E;
    uint32_t *hist;
    uint8_t *missing;  // nullable: the missing-region mask, one byte per pixel
};

bool seed_size_supported(int W, int H);
size_t seed_ws_bytes(int W, int H);
// Device word holding the number of seeds found by the last launch_seed on this workspace.
uint32_t *seed_count_ptr(void *ws, int W, int H);
void launch_seed(const float *rgb, const float *depth, int W, int H, double D0, const SeedK &sk, const SeedOutK &out,
                 void *ws, SeedScalars *sc, uint32_t *status, hipStream_t s);

}  // namespace fgs
