// Structural-similarity term of the mapping loss (Sec. III-D, Eq. 16) and its gradient.
//
// The index is the standard windowed one: per channel and pixel, moments of the image x and the
// target y over an 11x11 gaussian window (sigma 1.5, normalised; zero outside the image),
// S = (2 mx my + C1)(2 (mxy - mx my) + C2) / ((mx^2 + my^2 + C1)((mxx - mx^2) + (myy - my^2) + C2)),
// averaged over the 3 P (channel, pixel) values. S depends on x only through mx, mxx and mxy, so
// d ssim / d x_q = 1/(3P) sum_p w(p - q) (A_p + 2 x_q B_p + y_q C_p) with A, B, C the partials of S
// at p with respect to those three moments (zero at pixels outside the image).
//
// Two passes, one workgroup per (channel, 32x32 tile), each with a 5-pixel halo and everything
// else in LDS, and the window applied separably (rows, then columns; explicit FMAs) with sliding
// runs in registers:
//   k_ssim_moments: the tile's 42x42 neighbourhood of x and y, the five moments at its
//     own pixels, S (summed into the tile's partial) and A, B, C, written to a workspace;
//   k_ssim_grad: the 42x42 neighbourhood of A, B and C, filtered back onto the tile,
//     combined with x and y into the gradient.
// Each pixel's moments are computed once (a single fused pass would recompute them over the halo
// of every tile that needs them); the workspace costs 36 bytes per pixel written and read.
#include "fgs_internal.h"

namespace fgs {

namespace {

constexpr int kR = 5, kK = 2 * kR + 1;  // window radius and width
constexpr int kT = 32;                  // tile edge
constexpr int kIn = kT + 2 * kR;        // 42: the pixels the tile's windows read
constexpr int kThreads = 256;
constexpr int kRowRun = 6;              // row passes: 32 columns in 6 runs (the last of 2) x 42 rows
constexpr int kColRun = 4;              // column passes: 32 rows in 8 runs x 32 columns
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct Window {
    float g[kK];  // the normalised 1D window; the 2D window is g(dx) g(dy)
};

// Loads plane over the tile's 42x42 neighbourhood (zero outside the image) into dst.
__device__ inline void load_halo(const float *__restrict__ plane, int W, int H, int ox, int oy, float (*dst)[kIn])
{
    for (int k = threadIdx.x; k < kIn * kIn; k += kThreads) {
        const int r = k / kIn, q = k % kIn;
        const int gx = ox - kR + q, gy = oy - kR + r;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        dst[r][q] = in ? plane[(int64_t)gy * W + gx] : 0.0f;
    }
}

__global__ void __launch_bounds__(kThreads)
k_ssim_moments(int W, int H, int tiles_x, int tiles, const float *__restrict__ img, const float *__restrict__ tgt, Window win,
               float *__restrict__ abc, float *__restrict__ partials)
{
    __shared__ float sx[kIn][kIn], sy[kIn][kIn];
    __shared__ float hrow[5][kIn][kT];  // the five moments summed along rows
    __shared__ float red[kThreads / kWave];
    const int tid = threadIdx.x;
    const int c = blockIdx.x / tiles, tile = blockIdx.x % tiles;  // one channel of one tile
    const int ox = (tile % tiles_x) * kT, oy = (tile / tiles_x) * kT;
    const int64_t P = (int64_t)W * H;
    float ssum = 0.0f;
    {
        load_halo(img + (int64_t)c * P, W, H, ox, oy, sx);
        load_halo(tgt + (int64_t)c * P, W, H, ox, oy, sy);
        __syncthreads();
        // rows: thread = (neighbourhood row, run of kRowRun tile columns); tile column j reads
        // neighbourhood columns j .. j + 10
        for (int k = tid; k < kIn * 6; k += kThreads) {
            const int r = k / 6, j0 = (k % 6) * kRowRun;
            float xv[kRowRun + 2 * kR], yv[kRowRun + 2 * kR], xx[kRowRun + 2 * kR], yy[kRowRun + 2 * kR],
                xy[kRowRun + 2 * kR];
#pragma unroll
            for (int t = 0; t < kRowRun + 2 * kR; ++t) {
                const bool ok = j0 + t < kIn;
                xv[t] = ok ? sx[r][j0 + t] : 0.0f;
                yv[t] = ok ? sy[r][j0 + t] : 0.0f;
                xx[t] = xv[t] * xv[t];
                yy[t] = yv[t] * yv[t];
                xy[t] = xv[t] * yv[t];
            }
#pragma unroll
            for (int u = 0; u < kRowRun; ++u) {
                float a = 0, b = 0, aa = 0, bb = 0, ab = 0;
#pragma unroll
                for (int t = 0; t < kK; ++t) {
                    const float w = win.g[t];
                    a = __builtin_fmaf(w, xv[u + t], a);
                    b = __builtin_fmaf(w, yv[u + t], b);
                    aa = __builtin_fmaf(w, xx[u + t], aa);
                    bb = __builtin_fmaf(w, yy[u + t], bb);
                    ab = __builtin_fmaf(w, xy[u + t], ab);
                }
                if (j0 + u < kT) {
                    hrow[0][r][j0 + u] = a;
                    hrow[1][r][j0 + u] = b;
                    hrow[2][r][j0 + u] = aa;
                    hrow[3][r][j0 + u] = bb;
                    hrow[4][r][j0 + u] = ab;
                }
            }
        }
        __syncthreads();
        // columns, index and partials: thread = (tile column, run of kColRun tile rows)
        {
            const int j = tid % kT, i0 = (tid / kT) * kColRun;
            float m[5][kColRun];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                float v[kColRun + 2 * kR];
#pragma unroll
                for (int t = 0; t < kColRun + 2 * kR; ++t) v[t] = hrow[q][i0 + t][j];
#pragma unroll
                for (int u = 0; u < kColRun; ++u) {
                    float s = 0;
#pragma unroll
                    for (int t = 0; t < kK; ++t) s = __builtin_fmaf(win.g[t], v[u + t], s);
                    m[q][u] = s;
                }
            }
#pragma unroll
            for (int u = 0; u < kColRun; ++u) {
                const int gx = ox + j, gy = oy + i0 + u;
                if (gx < W && gy < H) {
                    const float mx = m[0][u], my = m[1][u];
                    const float a1 = 2.0f * mx * my + kC1, a2 = 2.0f * (m[4][u] - mx * my) + kC2;
                    const float b1 = mx * mx + my * my + kC1;
                    const float b2 = (m[2][u] - mx * mx) + (m[3][u] - my * my) + kC2;
                    const float ia1 = 1.0f / a1, ia2 = 1.0f / a2, ib1 = 1.0f / b1, ib2 = 1.0f / b2;
                    const float S = (a1 * a2) * (ib1 * ib2);
                    ssum += S;
                    const int64_t p = (int64_t)gy * W + gx;
                    float *o = abc + (int64_t)c * 3 * P + p;
                    o[0] = S * (2.0f * my * ia1 - 2.0f * my * ia2 - 2.0f * mx * ib1 + 2.0f * mx * ib2);
                    o[P] = -S * ib2;
                    o[2 * P] = 2.0f * S * ia2;
                }
            }
        }
    }
    if (partials) {
        for (int o = kWave / 2; o > 0; o >>= 1) ssum += __shfl_xor(ssum, o);
        if (__lane_id() == 0) red[tid / kWave] = ssum;
        __syncthreads();
        if (tid == 0) {
            float t = 0;
            for (int w = 0; w < kThreads / kWave; ++w) t += red[w];
            partials[blockIdx.x] = t;
        }
    }
}

__global__ void __launch_bounds__(kThreads)
k_ssim_grad(int W, int H, int tiles_x, int tiles, const float *__restrict__ img, const float *__restrict__ tgt, Window win,
            const float *__restrict__ abc, float gscale, int accumulate, float *__restrict__ grad)
{
    __shared__ float sm[3][kIn][kIn];   // A, B, C over the neighbourhood
    __shared__ float hrow[3][kIn][kT];  // their row sums
    const int tid = threadIdx.x;
    const int c = blockIdx.x / tiles, tile = blockIdx.x % tiles;  // one channel of one tile
    const int ox = (tile % tiles_x) * kT, oy = (tile / tiles_x) * kT;
    const int64_t P = (int64_t)W * H;
    const float inv3P = (float)(1.0 / (3.0 * (double)P));
    {
        for (int q = 0; q < 3; ++q) load_halo(abc + ((int64_t)c * 3 + q) * P, W, H, ox, oy, sm[q]);
        __syncthreads();
        for (int k = tid; k < kIn * 6; k += kThreads) {
            const int r = k / 6, j0 = (k % 6) * kRowRun;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                float v[kRowRun + 2 * kR];
#pragma unroll
                for (int t = 0; t < kRowRun + 2 * kR; ++t) v[t] = j0 + t < kIn ? sm[q][r][j0 + t] : 0.0f;
#pragma unroll
                for (int u = 0; u < kRowRun; ++u) {
                    float s = 0;
#pragma unroll
                    for (int t = 0; t < kK; ++t) s = __builtin_fmaf(win.g[t], v[u + t], s);
                    if (j0 + u < kT) hrow[q][r][j0 + u] = s;
                }
            }
        }
        __syncthreads();
        {
            const int j = tid % kT, i0 = (tid / kT) * kColRun;
            float gsum[3][kColRun];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                float v[kColRun + 2 * kR];
#pragma unroll
                for (int t = 0; t < kColRun + 2 * kR; ++t) v[t] = hrow[q][i0 + t][j];
#pragma unroll
                for (int u = 0; u < kColRun; ++u) {
                    float s = 0;
#pragma unroll
                    for (int t = 0; t < kK; ++t) s = __builtin_fmaf(win.g[t], v[u + t], s);
                    gsum[q][u] = s;
                }
            }
#pragma unroll
            for (int u = 0; u < kColRun; ++u) {
                const int gx = ox + j, gy = oy + i0 + u;
                if (gx < W && gy < H) {
                    const int64_t p = (int64_t)c * P + (int64_t)gy * W + gx;
                    const float d = (gsum[0][u] + 2.0f * img[p] * gsum[1][u] + tgt[p] * gsum[2][u]) * inv3P;
                    grad[p] = (accumulate ? grad[p] : 0.0f) + gscale * d;
                }
            }
        }
    }
}

}  // namespace

static int64_t tiles_of(int32_t W, int32_t H) { return (int64_t)((W + kT - 1) / kT) * ((H + kT - 1) / kT); }

int64_t ssim_partials(int32_t W, int32_t H) { return 3 * tiles_of(W, H); }

int64_t ssim_ws_floats(int32_t W, int32_t H) { return 9 * (int64_t)W * H; }

void launch_ssim(int32_t W, int32_t H, const float *img, const float *tgt, float gscale, bool accumulate, float *grad,
                 float *partials, float *ws, hipStream_t s)
{
    if (W <= 0 || H <= 0) return;
    Window win;
    double g[kK], sum = 0.0;
    for (int t = 0; t < kK; ++t) {
        const double d = (double)(t - kR);
        g[t] = exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += g[t];
    }
    for (int t = 0; t < kK; ++t) win.g[t] = (float)(g[t] / sum);
    const int tiles_x = (W + kT - 1) / kT, tiles = (int)tiles_of(W, H);
    const dim3 grid((unsigned)(3 * tiles));  // (channel, tile)
    hipLaunchKernelGGL(k_ssim_moments, grid, dim3(kThreads), 0, s, W, H, tiles_x, tiles, img, tgt, win, ws, partials);
    if (grad)
        hipLaunchKernelGGL(k_ssim_grad, grid, dim3(kThreads), 0, s, W, H, tiles_x, tiles, img, tgt, win, ws, gscale,
                           accumulate ? 1 : 0, grad);
}

}  // namespace fgs
