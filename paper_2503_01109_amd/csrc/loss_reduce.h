// Device-side reduction of the mapping loss's per-tile partial sums (Eq. 16): the L1 colour and
// depth terms, PSNR, and the structural-similarity and regulariser terms, in FP64 and a fixed
// order, by one workgroup of NT threads (no float atomics: the result is deterministic). Used by
// the one-workgroup loss kernel and by the projection backward, where one extra workgroup does it
// beside the per-gaussian work.
#pragma once
#include "fgs_internal.h"

namespace fgs {

// Sum of n floats by one workgroup of NT threads in FP64 and a fixed order (every thread gets the
// sum).
template <int NT>
__device__ double block_sum(const float *__restrict__ a, int n)
{
    constexpr int NW = NT / kWave;
    __shared__ double wred[NW];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += NT) s += (double)a[k];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __syncthreads();  // wred may still be read by an earlier call
    if (__lane_id() == 0) wred[threadIdx.x / kWave] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += wred[w];
    return t;
}

// Loss and PSNR from nb per-tile partial quadruples (|C - C*|, (C - C*)^2, |D - D*| over valid
// pixels, valid pixels) by one workgroup of NT threads. A quadruple is one 16-byte load (partials
// is 16-byte aligned); each thread puts four of them in flight before adding, so the workgroup
// waits on memory about once per 4 NT tiles. ddepth_scale (nullable) receives 1/P_v, the depth
// term's normalisation.
template <int NT>
__device__ void loss_reduce(const float *__restrict__ partials, int nb, int64_t P, float lrgb, float ldepth,
                            float *__restrict__ ddepth_scale, float *__restrict__ loss, float *__restrict__ psnr,
                            const LossExtraK &extra = LossExtraK{})
{
    const double ssim_sum = extra.ssim_part ? block_sum<NT>(extra.ssim_part, extra.ssim_nb) : 0.0;
    const double reg_sum = extra.reg_part ? block_sum<NT>(extra.reg_part, extra.reg_nb) : 0.0;
    constexpr int NW = NT / kWave, U = 4;
    __shared__ double red[NW][4];
    const float4 *__restrict__ p4 = reinterpret_cast<const float4 *>(partials);
    double acc[4] = {0, 0, 0, 0};
    for (int b0 = 0; b0 < nb; b0 += U * NT) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * NT + (int)threadIdx.x;
            v[u] = b < nb ? p4[b] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc[0] += (double)v[u].x;
            acc[1] += (double)v[u].y;
            acc[2] += (double)v[u].z;
            acc[3] += (double)v[u].w;
        }
    }
    // wave sums (butterfly over the 64 lanes), then the waves' sums in order
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o);
    const int wid = threadIdx.x / kWave;
    if (__lane_id() == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wid][q] = acc[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4] = {0, 0, 0, 0};
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int q = 0; q < 4; ++q) t[q] += red[w][q];
        const double l1c = t[0], se = t[1], l1d = t[2], nv = t[3];
        const double scale = nv > 0 ? 1.0 / nv : 0.0;
        if (ddepth_scale) *ddepth_scale = (float)scale;
        double L = (double)lrgb * l1c / (3.0 * (double)P) + (double)ldepth * l1d * scale;
        if (extra.ssim_part) L += (double)extra.ssim_w * (1.0 - ssim_sum / (3.0 * (double)P));
        if (loss) *loss = (float)L;
        if (extra.reg_out) *extra.reg_out = (float)(reg_sum * (double)extra.reg_scale);
        const double mse = se / (3.0 * (double)P);
        if (psnr) *psnr = (float)(mse > 0 ? 10.0 * log10(1.0 / mse) : INFINITY);
    }
}

}  // namespace fgs
