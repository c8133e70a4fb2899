// L1 colour and depth terms of the mapping loss (Eq. 16), PSNR, and the Adam update.
//
// The loss kernel streams the rendered and target planes once: it writes the per-pixel
// gradient and per-block partial sums; a one-block kernel reduces the partials in FP64 in a
// fixed order (no float atomics, so the loss is deterministic). The depth term is a mean over
// pixels with a positive target depth, a count only known after the reduction; its gradient is
// written unscaled and the factor 1/P_v is left in device memory for the consumer.
#include "fgs_internal.h"

namespace fgs {

namespace {

constexpr int kLossThreads = 256;
constexpr int kLossItems = 4;
constexpr int kFinalThreads = 1024;  // the one-workgroup reductions of the partials

__device__ inline float sgnf(float x) { return (float)((x > 0.0f) - (x < 0.0f)); }

__global__ void __launch_bounds__(kLossThreads)
k_loss_partial(int64_t P, const float *__restrict__ rgb, const float *__restrict__ depth,
               const float *__restrict__ trgb, const float *__restrict__ tdepth, float lrgb, float ldepth,
               float *__restrict__ drgb, float *__restrict__ ddepth, float *__restrict__ partials)
{
    __shared__ float red[4][kLossThreads];
    const float inv3P = (float)(1.0 / (3.0 * (double)P));
    float l1c = 0, se = 0, l1d = 0, nv = 0;
    const int64_t base = (int64_t)blockIdx.x * kLossThreads * kLossItems;
#pragma unroll
    for (int k = 0; k < kLossItems; ++k) {
        const int64_t p = base + (int64_t)k * kLossThreads + threadIdx.x;
        if (p >= P) break;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float r = rgb[c * P + p] - trgb[c * P + p];
            l1c += fabsf(r);
            se += r * r;
            drgb[c * P + p] = lrgb * sgnf(r) * inv3P;
        }
        const float td = tdepth[p];
        const bool valid = td > 0.0f;
        const float rd = depth[p] - td;
        l1d += valid ? fabsf(rd) : 0.0f;
        nv += valid ? 1.0f : 0.0f;
        ddepth[p] = valid ? ldepth * sgnf(rd) : 0.0f;
    }
    red[0][threadIdx.x] = l1c;
    red[1][threadIdx.x] = se;
    red[2][threadIdx.x] = l1d;
    red[3][threadIdx.x] = nv;
    __syncthreads();
    for (int s = kLossThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[4 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Sum of n floats by one workgroup of kFinalThreads in FP64 and a fixed order (every thread gets
// the sum).
__device__ double block_sum(const float *__restrict__ a, int n)
{
    constexpr int NW = kFinalThreads / kWave;
    __shared__ double wred[NW];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += kFinalThreads) s += (double)a[k];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __syncthreads();  // wred may still be read by an earlier call
    if (__lane_id() == 0) wred[threadIdx.x / kWave] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += wred[w];
    return t;
}

// Loss and PSNR from nb per-tile partial quadruples (one workgroup of kFinalThreads), in FP64 and
// a fixed order. A quadruple is one 16-byte load (partials is 16-byte aligned); each thread puts
// up to four of them in flight before adding, so the kernel waits on memory about once. The
// structural-similarity and regulariser terms (extra) are reduced the same way.
__device__ void loss_reduce(const float *__restrict__ partials, int nb, int64_t P, float lrgb, float ldepth,
                            float *__restrict__ ddepth_scale, float *__restrict__ loss, float *__restrict__ psnr,
                            const LossExtraK &extra = LossExtraK{})
{
    const double ssim_sum = extra.ssim_part ? block_sum(extra.ssim_part, extra.ssim_nb) : 0.0;
    const double reg_sum = extra.reg_part ? block_sum(extra.reg_part, extra.reg_nb) : 0.0;
    constexpr int NW = kFinalThreads / kWave, U = 4;
    __shared__ double red[NW][4];
    const float4 *__restrict__ p4 = reinterpret_cast<const float4 *>(partials);
    double acc[4] = {0, 0, 0, 0};
    for (int b0 = 0; b0 < nb; b0 += U * kFinalThreads) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * kFinalThreads + (int)threadIdx.x;
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

__global__ void __launch_bounds__(kFinalThreads)
k_loss_final(const float *__restrict__ partials, int nb, int64_t P, float lrgb, float ldepth,
             float *__restrict__ ddepth_scale, float *__restrict__ loss, float *__restrict__ psnr, LossExtraK extra)
{
    loss_reduce(partials, nb, P, lrgb, ldepth, ddepth_scale, loss, psnr, extra);
}

__global__ void __launch_bounds__(kFinalThreads)
k_sum_scaled(const float *__restrict__ a, int n, double scale, float *__restrict__ out)
{
    const double t = block_sum(a, n);
    if (threadIdx.x == 0) *out = (float)(t * scale);
}

// One workgroup per view of a window: view v's tiles are window items [tile_base_v, tile_base_v+1).
__global__ void __launch_bounds__(kFinalThreads)
k_loss_final_views(const ViewK *__restrict__ views, int nv, uint32_t total_items, float *__restrict__ loss,
                   float *__restrict__ psnr)
{
    const int v = blockIdx.x;
    const ViewK &V = views[v];
    const uint32_t end = v + 1 < nv ? views[v + 1].tile_base : total_items;
    loss_reduce(V.loss.partials, (int)(end - V.tile_base), (int64_t)V.W * V.H, V.loss.lrgb, V.loss.ldepth,
                V.loss.ddepth_scale, loss ? loss + v : nullptr, psnr ? psnr + v : nullptr);
}

__device__ inline float *plane_ptr(const GradK &g, int row)
{
    const int64_t S = g.stride;
    if (row < 3) return g.mean + row * S;
    if (row < 6) return g.log_scale + (row - 3) * S;
    if (row < 10) return g.quat + (row - 6) * S;
    if (row < 11) return g.logit;
    return g.rgb + (row - 11) * S;
}

__device__ inline const float *plane_ptr(const ParamsK &g, int row)
{
    const int64_t S = g.stride;
    if (row < 3) return g.mean + row * S;
    if (row < 6) return g.log_scale + (row - 3) * S;
    if (row < 10) return g.quat + (row - 6) * S;
    if (row < 11) return g.logit;
    return g.rgb + (row - 11) * S;
}

struct Lr {
    float v[5];
};

__global__ void __launch_bounds__(256)
k_adam(GradK p, ParamsK g, GradK m, GradK v, Lr lr, float b1, float b2, float eps, float bc1, float bc2)
{
    const int row = blockIdx.y;
    const int group = row < 3 ? 0 : row < 6 ? 1 : row < 10 ? 2 : row < 11 ? 3 : 4;
    const float a = lr.v[group];
    float *pp = plane_ptr(p, row);
    const float *gg = plane_ptr(g, row);
    float *mm = plane_ptr(m, row);
    float *vv = plane_ptr(v, row);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = gg[i];
        const float mi = b1 * mm[i] + (1.0f - b1) * gi;
        const float vi = b2 * vv[i] + (1.0f - b2) * gi * gi;
        mm[i] = mi;
        vv[i] = vi;
        pp[i] -= a * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

__global__ void k_scale(float *__restrict__ x, int64_t n, const float *__restrict__ s)
{
    const float f = *s;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= f;
}

__global__ void k_step_advance(int64_t *step, const uint32_t *skip)
{
    if (threadIdx.x == 0 && !(skip && *skip)) *step += 1;
}

}  // namespace

void launch_step_advance(int64_t *step, const uint32_t *skip, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step, skip);
}

int64_t loss_partials_size(int64_t P)
{
    return 4 * ((P + kLossThreads * kLossItems - 1) / (kLossThreads * kLossItems)) + 4;
}

void launch_loss_l1(int64_t P, const float *rgb, const float *depth, const float *trgb, const float *tdepth,
                    float lrgb, float ldepth, float *drgb, float *ddepth, float *ddepth_scale, float *partials,
                    float *loss, float *psnr, hipStream_t s)
{
    const int nb = (int)((P + kLossThreads * kLossItems - 1) / (kLossThreads * kLossItems));
    hipLaunchKernelGGL(k_loss_partial, dim3(nb), dim3(kLossThreads), 0, s, P, rgb, depth, trgb, tdepth, lrgb,
                       ldepth, drgb, ddepth, partials);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kFinalThreads), 0, s, partials, nb, P, lrgb, ldepth, ddepth_scale,
                       loss, psnr, LossExtraK{});
}

void launch_loss_final(const float *partials, int nb, int64_t P, float lrgb, float ldepth, float *ddepth_scale,
                       float *loss, float *psnr, hipStream_t s, const LossExtraK &extra)
{
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kFinalThreads), 0, s, partials, nb, P, lrgb, ldepth, ddepth_scale,
                       loss, psnr, extra);
}

void launch_sum_scaled(const float *a, int n, double scale, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_scaled, dim3(1), dim3(kFinalThreads), 0, s, a, n, scale, out);
}

void launch_loss_final_views(const ViewK *views_dev, int nv, uint32_t total_items, float *loss, float *psnr,
                             hipStream_t s)
{
    if (nv <= 0) return;
    hipLaunchKernelGGL(k_loss_final_views, dim3((unsigned)nv), dim3(kFinalThreads), 0, s, views_dev, nv, total_items,
                       loss, psnr);
}

void launch_scale(float *x, int64_t n, const float *s, hipStream_t st)
{
    if (n <= 0) return;
    int64_t b = (n + 1023) / 1024;
    if (b > 2048) b = 2048;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)b), dim3(256), 0, st, x, n, s);
}

void launch_adam(const GradK &p, const ParamsK &g, const GradK &m, const GradK &v, const float lr[5], float beta1,
                 float beta2, float eps, float bc1, float bc2, hipStream_t s)
{
    if (p.n <= 0) return;
    Lr l;
    for (int k = 0; k < 5; ++k) l.v[k] = lr[k];
    int64_t bx = (p.n + 1023) / 1024;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)bx, 14), dim3(256), 0, s, p, g, m, v, l, beta1, beta2, eps, bc1, bc2);
}

}  // namespace fgs
