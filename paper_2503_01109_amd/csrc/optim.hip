// L1 colour and depth terms of the mapping loss (Eq. 16), PSNR, and the Adam update.
//
// The loss kernel streams the rendered and target planes once: it writes the per-pixel
// gradient and per-block partial sums; a one-block kernel reduces the partials in FP64 in a
// fixed order (no float atomics, so the loss is deterministic). The depth term is a mean over
// pixels with a positive target depth, a count only known after the reduction; its gradient is
// written unscaled and the factor 1/P_v is left in device memory for the consumer.
#include "fgs_internal.h"
#include "loss_reduce.h"

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

__global__ void __launch_bounds__(kFinalThreads)
k_loss_final(const float *__restrict__ partials, int nb, int64_t P, float lrgb, float ldepth,
             float *__restrict__ ddepth_scale, float *__restrict__ loss, float *__restrict__ psnr, LossExtraK extra)
{
    loss_reduce<kFinalThreads>(partials, nb, P, lrgb, ldepth, ddepth_scale, loss, psnr, extra);
}

__global__ void __launch_bounds__(kFinalThreads)
k_sum_scaled(const float *__restrict__ a, int n, double scale, float *__restrict__ out)
{
    const double t = block_sum<kFinalThreads>(a, n);
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
    loss_reduce<kFinalThreads>(V.loss.partials, (int)(end - V.tile_base), (int64_t)V.W * V.H, V.loss.lrgb, V.loss.ldepth,
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
