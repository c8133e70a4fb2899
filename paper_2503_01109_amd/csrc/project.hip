// EWA projection of 3D gaussians (Sec. III: covariance C = R S S^T R^T) and its backward.
//
// One thread per gaussian. Parameters are read as coalesced SoA planes; the arithmetic runs in
// FP64 (a few hundred flops per gaussian, far below the kernel's memory time on gfx950) and the
// outputs are rounded once to FP32. The projected mean is stored as integer pixel + FP32
// fraction so that the rasterizer can form tile-local offsets without losing the fraction to
// the magnitude of the pixel coordinate.
#include "fgs_internal.h"
#include "loss_reduce.h"

namespace fgs {

namespace {

struct Proj {
    bool valid;
    double t[3];
    double Rq[9], s[3], qn[4], qnorm;
    double Sig[9], A[6];
    double cov[3];   // Sigma'_xx, Sigma'_xy, Sigma'_yy (with low-pass)
    double conic[3];
    double m2[2];
    double opacity;
};

__device__ inline void rot_from_quat(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ inline void project_gaussian(const ParamsK &g, int64_t i, const CamK &cam, float lowpass,
                                        Proj &p)
{
    p.valid = false;
    const int64_t S = g.stride;
    const double mu[3] = {g.mean[i], g.mean[S + i], g.mean[2 * S + i]};
    const double q[4] = {g.quat[i], g.quat[S + i], g.quat[2 * S + i], g.quat[3 * S + i]};
    p.qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(p.qnorm > 0.0) || !isfinite(p.qnorm)) return;
    const double inv = 1.0 / p.qnorm;
#pragma unroll
    for (int k = 0; k < 4; ++k) p.qn[k] = q[k] * inv;
    rot_from_quat(p.qn, p.Rq);
#pragma unroll
    for (int k = 0; k < 3; ++k) p.s[k] = exp((double)g.log_scale[k * S + i]);
    // Sigma = (R S)(R S)^T
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[3 * r + c] = p.Rq[3 * r + c] * p.s[c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p.Sig[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
    const double *W = cam.R;
#pragma unroll
    for (int r = 0; r < 3; ++r)
        p.t[r] = W[3 * r] * mu[0] + W[3 * r + 1] * mu[1] + W[3 * r + 2] * mu[2] + cam.t[r];
    const double tx = p.t[0], ty = p.t[1], tz = p.t[2];
    if (!(tz > cam.z_near)) return;
    const double iz = 1.0 / tz;
    const double J00 = cam.fx * iz, J02 = -cam.fx * tx * iz * iz;
    const double J11 = cam.fy * iz, J12 = -cam.fy * ty * iz * iz;
    // A = J W (J has zeros at (0,1) and (1,0))
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        p.A[c] = J00 * W[c] + J02 * W[6 + c];
        p.A[3 + c] = J11 * W[3 + c] + J12 * W[6 + c];
    }
    double AS[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            AS[3 * r + c] = p.A[3 * r] * p.Sig[c] + p.A[3 * r + 1] * p.Sig[3 + c] + p.A[3 * r + 2] * p.Sig[6 + c];
    const double sxx = AS[0] * p.A[0] + AS[1] * p.A[1] + AS[2] * p.A[2];
    const double sxy = AS[0] * p.A[3] + AS[1] * p.A[4] + AS[2] * p.A[5];
    const double syy = AS[3] * p.A[3] + AS[4] * p.A[4] + AS[5] * p.A[5];
    p.cov[0] = sxx + lowpass;
    p.cov[1] = sxy;
    p.cov[2] = syy + lowpass;
    const double det = p.cov[0] * p.cov[2] - p.cov[1] * p.cov[1];
    if (!(det > 0.0) || !isfinite(det)) return;
    const double idet = 1.0 / det;
    p.conic[0] = p.cov[2] * idet;
    p.conic[1] = -p.cov[1] * idet;
    p.conic[2] = p.cov[0] * idet;
    p.m2[0] = cam.fx * tx * iz + cam.cx;
    p.m2[1] = cam.fy * ty * iz + cam.cy;
    p.opacity = 1.0 / (1.0 + exp(-(double)g.logit[i]));
    if (!isfinite(p.m2[0]) || !isfinite(p.m2[1]) || !isfinite(p.opacity)) return;
    p.valid = true;
}

// Pixel-index range [lo, hi] of centres x + 0.5 within [c - r, c + r], clamped to [0, size).
__device__ inline bool pixel_span(double c, double r, int32_t size, int32_t &lo, int32_t &hi)
{
    const double a = ceil(c - r - 0.5), b = floor(c + r - 0.5);
    if (!(a <= b) || b < 0.0 || a > (double)(size - 1)) return false;
    lo = a < 0.0 ? 0 : (int32_t)a;
    hi = b > (double)(size - 1) ? size - 1 : (int32_t)b;
    return true;
}

__device__ uint32_t project_one(ParamsK g, CamK cam, RasterK rk, Rec *__restrict__ rec, uint2 *__restrict__ rect,
                                uint32_t *__restrict__ count, uint32_t *__restrict__ dkey, int shift, int64_t i,
                                uint32_t &cnt, uint2 &rc);

// Projects every gaussian (one thread each): record, tile rectangle, count of covered tiles or
// super-tiles, depth key; kpart[2 b], kpart[2 b + 1] receive block b's number of (tile, gaussian)
// pairs and of gaussians that cover a tile (summed by the scan, so nothing needs zeroing first);
// csum[b] (nullable) block b's sum of the counts (the scan's block sums in gaussian order);
// shist (nullable; at most 256 super-tiles, supers_x per row): shist[s G + b], G = gridDim.x, the
// number of block b's gaussians covering super-tile s.
__global__ void __launch_bounds__(256)
k_project(ParamsK g, CamK cam, RasterK rk, Rec *__restrict__ rec, uint2 *__restrict__ rect,
          uint32_t *__restrict__ count, uint32_t *__restrict__ dkey, uint32_t *__restrict__ ids,
          uint32_t *__restrict__ n_out, int shift, uint32_t *__restrict__ kpart, uint32_t id_base,
          float *__restrict__ reg_part, uint32_t *__restrict__ csum, uint32_t *__restrict__ shist, int supers_x)
{
    __shared__ uint32_t wsum[3][4];
    __shared__ float wreg[4];
    __shared__ uint32_t lh[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *n_out = id_base + (uint32_t)g.n;
    if (shist) lh[threadIdx.x] = 0u;  // (ordered before the adds by the barrier below)
    uint32_t tiles = 0, cnt = 0;  // (tile, gaussian) pairs of this gaussian; its count
    uint2 rc = make_uint2(1u, 0u);
    if (i < g.n) {
        tiles = project_one(g, cam, rk, rec, rect, count, dkey, shift, i, cnt, rc);
        ids[i] = id_base + (uint32_t)i;
    }
    if (shist) {
        __syncthreads();
        if (cnt) {
            const uint32_t sx0 = (rc.x & 0xFFFFu) >> shift, sx1 = (rc.x >> 16) >> shift;
            const uint32_t sy0 = (rc.y & 0xFFFFu) >> shift, sy1 = (rc.y >> 16) >> shift;
            for (uint32_t sy = sy0; sy <= sy1; ++sy)
                for (uint32_t sx = sx0; sx <= sx1; ++sx) atomicAdd(&lh[sy * (uint32_t)supers_x + sx], 1u);
        }
        __syncthreads();
        shist[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = lh[threadIdx.x];
    }
    uint32_t vis = tiles != 0u;
    for (int o = 32; o > 0; o >>= 1) {
        tiles += __shfl_xor(tiles, o);
        vis += __shfl_xor(vis, o);
        cnt += __shfl_xor(cnt, o);
    }
    if ((threadIdx.x & 63) == 0) {
        wsum[0][threadIdx.x >> 6] = tiles;
        wsum[1][threadIdx.x >> 6] = vis;
        wsum[2][threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        kpart[2 * blockIdx.x + threadIdx.x] =
            wsum[threadIdx.x][0] + wsum[threadIdx.x][1] + wsum[threadIdx.x][2] + wsum[threadIdx.x][3];
    if (csum && threadIdx.x == 2) csum[blockIdx.x] = wsum[2][0] + wsum[2][1] + wsum[2][2] + wsum[2][3];
    if (reg_part) {
        // the scale regulariser's terms (Eq. 15): |s1 - s2| + s3 with s = exp(log-scale)
        float r = 0.0f;
        if (i < g.n) {
            const float s1 = expf(g.log_scale[i]), s2 = expf(g.log_scale[g.stride + i]);
            r = fabsf(s1 - s2) + expf(g.log_scale[2 * g.stride + i]);
        }
        for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o);
        if ((threadIdx.x & 63) == 0) wreg[threadIdx.x >> 6] = r;
        __syncthreads();
        if (threadIdx.x == 0) reg_part[blockIdx.x] = (wreg[0] + wreg[1]) + (wreg[2] + wreg[3]);
    }
}

__device__ uint32_t project_one(ParamsK g, CamK cam, RasterK rk, Rec *__restrict__ rec, uint2 *__restrict__ rect,
                                uint32_t *__restrict__ count, uint32_t *__restrict__ dkey, int shift, int64_t i,
                                uint32_t &cnt_out, uint2 &rc_out)
{
    Proj p;
    project_gaussian(g, i, cam, rk.lowpass, p);
    uint32_t cnt = 0, key = 0xFFFFFFFFu, tiles = 0;
    uint2 rc = make_uint2(1u, 0u);
    if (p.valid) {
        // Conservative box of the sigma_cut ellipse (its exact half-widths are
        // sigma_cut * sqrt(Sigma'_xx) and sigma_cut * sqrt(Sigma'_yy)), padded so that FP32
        // evaluation of the per-pixel test in the rasterizer can never reach outside it.
        const double rx = rk.sigma_cut * sqrt(p.cov[0]) * (1.0 + 1e-5) + 1e-3;
        const double ry = rk.sigma_cut * sqrt(p.cov[2]) * (1.0 + 1e-5) + 1e-3;
        int32_t x0, x1, y0, y1;
        if (fabs(p.m2[0]) < 1e9 && fabs(p.m2[1]) < 1e9 && pixel_span(p.m2[0], rx, cam.W, x0, x1) &&
            pixel_span(p.m2[1], ry, cam.H, y0, y1)) {
            const uint32_t tx0 = x0 / rk.tile_w, tx1 = x1 / rk.tile_w;
            const uint32_t ty0 = y0 / rk.tile_h, ty1 = y1 / rk.tile_h;
            cnt = ((tx1 >> shift) - (tx0 >> shift) + 1) * ((ty1 >> shift) - (ty0 >> shift) + 1);
            tiles = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
            rc = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
            const double fxm = floor(p.m2[0]), fym = floor(p.m2[1]);
            const float depth = (float)p.t[2];
            key = __float_as_uint(depth);
            Rec r;
            r.r0 = make_float4(__int_as_float((int)fxm), __int_as_float((int)fym), (float)(p.m2[0] - fxm),
                               (float)(p.m2[1] - fym));
            r.r1 = make_float4((float)p.conic[0], (float)p.conic[1], (float)p.conic[2], (float)p.opacity);
            const int64_t S = g.stride;
            r.r2 = make_float4(g.rgb[i], g.rgb[S + i], g.rgb[2 * S + i], depth);
            rec[i] = r;
        }
    }
    count[i] = cnt;
    dkey[i] = key;
    rect[i] = rc;
    cnt_out = cnt;
    rc_out = rc;
    return tiles;
}

// Chain rule for one gaussian: 2D gradient g2 -> 14 parameter gradients, added to out[14].
__device__ inline void chain_rule(const Proj &p, const CamK &cam, const double g2[10], double out[14])
{
    // conic = Sigma'^-1: dL/dSigma' = -X Gh X with Gh = [[ga, gb/2], [gb/2, gc]], X the conic.
    const double a = p.conic[0], b = p.conic[1], c = p.conic[2];
    const double ga = g2[2], gb = 0.5 * g2[3], gc = g2[4];
    const double XG00 = a * ga + b * gb, XG01 = a * gb + b * gc;
    const double XG10 = b * ga + c * gb, XG11 = b * gb + c * gc;
    const double d00 = -(XG00 * a + XG01 * b), d01 = -(XG00 * b + XG01 * c);
    const double d10 = -(XG10 * a + XG11 * b), d11 = -(XG10 * b + XG11 * c);
    const double D2[4] = {d00, 0.5 * (d01 + d10), 0.5 * (d01 + d10), d11};
    // Sigma' = A Sigma A^T + l I: dSigma = A^T D2 A; dA = 2 D2 A Sigma
    const double *A = p.A;
    double DA[6];  // D2 A (2x3)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        DA[k] = D2[0] * A[k] + D2[1] * A[3 + k];
        DA[3 + k] = D2[2] * A[k] + D2[3] * A[3 + k];
    }
    double dSig[9];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int v = 0; v < 3; ++v) dSig[3 * u + v] = A[u] * DA[v] + A[3 + u] * DA[3 + v];
    double dA[6];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            dA[3 * rr + k] = 2.0 * (DA[3 * rr] * p.Sig[k] + DA[3 * rr + 1] * p.Sig[3 + k] +
                                    DA[3 * rr + 2] * p.Sig[6 + k]);
    // A = J W: dJ = dA W^T; only J00, J02, J11, J12 depend on t.
    const double *W = cam.R;
    const double dJ00 = dA[0] * W[0] + dA[1] * W[1] + dA[2] * W[2];
    const double dJ02 = dA[0] * W[6] + dA[1] * W[7] + dA[2] * W[8];
    const double dJ11 = dA[3] * W[3] + dA[4] * W[4] + dA[5] * W[5];
    const double dJ12 = dA[3] * W[6] + dA[4] * W[7] + dA[5] * W[8];
    const double tx = p.t[0], ty = p.t[1], tz = p.t[2], iz = 1.0 / tz;
    const double fx = cam.fx, fy = cam.fy;
    double dtx = 0, dty = 0, dtz = 0;
    dtz += dJ00 * (-fx * iz * iz) + dJ02 * (2.0 * fx * tx * iz * iz * iz);
    dtx += dJ02 * (-fx * iz * iz);
    dtz += dJ11 * (-fy * iz * iz) + dJ12 * (2.0 * fy * ty * iz * iz * iz);
    dty += dJ12 * (-fy * iz * iz);
    dtx += g2[0] * fx * iz;
    dtz += g2[0] * (-fx * tx * iz * iz);
    dty += g2[1] * fy * iz;
    dtz += g2[1] * (-fy * ty * iz * iz);
    dtz += g2[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] += W[k] * dtx + W[3 + k] * dty + W[6 + k] * dtz;
    // Sigma = M M^T, M = R diag(s): dM = 2 dSigma M
    double M[9], dM[9];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int k = 0; k < 3; ++k) M[3 * u + k] = p.Rq[3 * u + k] * p.s[k];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            dM[3 * u + k] = 2.0 * (dSig[3 * u] * M[k] + dSig[3 * u + 1] * M[3 + k] + dSig[3 * u + 2] * M[6 + k]);
    double dR[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double ds = p.Rq[k] * dM[k] + p.Rq[3 + k] * dM[3 + k] + p.Rq[6 + k] * dM[6 + k];
        out[3 + k] += ds * p.s[k];
#pragma unroll
        for (int u = 0; u < 3; ++u) dR[3 * u + k] = dM[3 * u + k] * p.s[k];
    }
    // R(q_hat): partial derivatives of the nine entries by w, x, y, z.
    const double w = p.qn[0], x = p.qn[1], y = p.qn[2], z = p.qn[3];
    double dq[4];
    dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] +
                   w * dR[7] - 2.0 * x * dR[8]);
    dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                   z * dR[7] - 2.0 * y * dR[8]);
    dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] +
                   y * dR[5] + x * dR[6] + y * dR[7]);
    // q_hat = q/|q|: dq = (I - q_hat q_hat^T) dq_hat / |q|
    const double dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    const double iq = 1.0 / p.qnorm;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[6 + k] += (dq[k] - p.qn[k] * dot) * iq;
    out[10] += g2[5] * p.opacity * (1.0 - p.opacity);
#pragma unroll
    for (int k = 0; k < 3; ++k) out[11 + k] += g2[6 + k];
}

__device__ inline float *plane(const GradK &g, int row)
{
    const int64_t S = g.stride;
    return row < 3 ? g.mean + row * S : row < 6 ? g.log_scale + (row - 3) * S : row < 10 ? g.quat + (row - 6) * S
         : row < 11 ? g.logit : g.rgb + (row - 11) * S;
}

// The 2D gradient record of gaussian i (slots 0..9 of kG2Stride floats) into g2; returns
// whether any term is nonzero, and then clears the record (the rasterizer's next backward
// accumulates into zeros).
__device__ __forceinline__ bool take_g2(float *__restrict__ rec, double g2[10])
{
    const float4 a = reinterpret_cast<const float4 *>(rec)[0], b = reinterpret_cast<const float4 *>(rec)[1];
    const float2 c = reinterpret_cast<const float2 *>(rec)[4];
    const float v[10] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y};
    bool any = false;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        g2[k] = v[k];
        any |= v[k] != 0.0f;
    }
    if (any) {
        const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        reinterpret_cast<float4 *>(rec)[0] = z;
        reinterpret_cast<float4 *>(rec)[1] = z;
        reinterpret_cast<float2 *>(rec)[4] = make_float2(0.0f, 0.0f);
    }
    return any;
}

// Adam on the 14 parameters of gaussian i with gradient gi: update number *adam.step + 1 (device
// counter) when adam.step is set, else bias corrections adam.bc1, adam.bc2.
__device__ inline void adam_update(const AdamK &adam, const ParamsK &g, int64_t i, const float gi[14])
{
    float bc1 = adam.bc1, bc2 = adam.bc2;
    if (adam.step) {
        const int64_t s = *adam.step;
        if (s != adam.step_expect) {
            const double t = (double)(s + 1);
            bc1 = (float)(1.0 - pow((double)adam.beta1, t));
            bc2 = (float)(1.0 - pow((double)adam.beta2, t));
        }
    }
    GradK P{g.n, g.stride, (float *)g.mean, (float *)g.log_scale, (float *)g.quat, (float *)g.logit, (float *)g.rgb};
#pragma unroll
    for (int k = 0; k < 14; ++k) {
        const int group = k < 3 ? 0 : k < 6 ? 1 : k < 10 ? 2 : k < 11 ? 3 : 4;
        float *mm = plane(adam.m, k) + i, *vv = plane(adam.v, k) + i, *pp = plane(P, k) + i;
        const float mi = adam.beta1 * *mm + (1.0f - adam.beta1) * gi[k];
        const float vi = adam.beta2 * *vv + (1.0f - adam.beta2) * gi[k] * gi[k];
        *mm = mi;
        *vv = vi;
        *pp -= adam.lr[group] * (mi / bc1) / (sqrtf(vi / bc2) + adam.eps);
    }
}

// Backward of the projection, one thread per gaussian. grad2d holds one record of kG2Stride
// floats per gaussian id: d/d(mean2 x, y; conic a, b, c; opacity; r, g, b; depth); each thread
// zeroes the record it read, so grad2d is all-zero again for the next backward. The gaussian's
// 14 parameter gradients plus grad_in (nullable: gradients of earlier views) are written to
// grad_out (nullable) and, when adam.m.mean is set, applied by Adam. Every access is coalesced.
// Four waves per SIMD (at most 128 VGPRs, no spills) hide more of the memory latency than the
// three its FP64 chain rule would otherwise leave room for.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_project_bwd(ParamsK g, CamK cam, RasterK rk, float *__restrict__ grad2d, GradK grad_in, GradK grad_out, AdamK adam,
              LossFinalK lf)
{
    int64_t blk = blockIdx.x;
    if (lf.partials) {
        // the view's loss, by the first workgroup (dispatched first, so it ends well before the rest)
        if (blk == 0) {
            loss_reduce<256>(lf.partials, lf.nb, lf.P, lf.lrgb, lf.ldepth, nullptr, lf.loss, lf.psnr, lf.extra);
            return;
        }
        --blk;
    }
    const int64_t i = blk * blockDim.x + threadIdx.x;
    const int64_t n = g.n;
    if (i >= n) return;
    // an overflowed step (incomplete gradient) changes no parameter, moment or step count
    const bool skip = adam.skip && *adam.skip;
    if (i == 0 && adam.step_out) *adam.step_out = *adam.step + (skip ? 0 : 1);
    double g2[10];
    bool any = take_g2(grad2d + i * kG2Stride, g2);
    double out[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) out[k] = 0.0;
    if (any) {
        Proj p;
        project_gaussian(g, i, cam, rk.lowpass, p);
        if (p.valid) chain_rule(p, cam, g2, out);
        else any = false;
    }
    // accumulating in place with nothing to add and no update: the gradient stays as it is
    if (!any && !adam.m.mean && grad_in.mean && grad_in.mean == grad_out.mean) return;
    float gi[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) gi[k] = grad_in.mean ? plane(grad_in, k)[i] + (float)out[k] : (float)out[k];
    if (adam.reg_w != 0.0f) {
        // scale regulariser (Eq. 15), lambda_r / n (|s1 - s2| + s3): d/d log s_k = s_k d/d s_k
        const float s1 = expf(g.log_scale[i]), s2 = expf(g.log_scale[g.stride + i]);
        const float s3 = expf(g.log_scale[2 * g.stride + i]);
        const float d = (float)((s1 > s2) - (s1 < s2));
        gi[3] += adam.reg_w * d * s1;
        gi[4] -= adam.reg_w * d * s2;
        gi[5] += adam.reg_w * s3;
    }
    if (grad_out.mean)
#pragma unroll
        for (int k = 0; k < 14; ++k) plane(grad_out, k)[i] = gi[k];
    if (adam.m.mean && !skip) adam_update(adam, g, i, gi);
}

// Window backward: per gaussian, the 2D gradient records of every view (view v's at grad2d +
// v * view_stride)
// go through that view's projection; the sum is the gaussian's gradient, written to grad (if its
// pointers are set) and applied by Adam (if adam.m is set). Adam's update number is *step + 1,
// read from device memory so a captured graph can be replayed unchanged.
__global__ void __launch_bounds__(256)
k_project_bwd_window(ParamsK g, const CamK *__restrict__ cams, int nv, float lowpass, float *__restrict__ grad2d,
                     int64_t view_stride, GradK grad, AdamK adam)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = g.n;
    if (i >= n) return;
    double out[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) out[k] = 0.0;
    for (int v = 0; v < nv; ++v) {
        double g2[10];
        if (!take_g2(grad2d + v * view_stride + i * kG2Stride, g2)) continue;
        const CamK cam = cams[v];
        Proj p;
        project_gaussian(g, i, cam, lowpass, p);
        if (p.valid) chain_rule(p, cam, g2, out);
    }
    float gi[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) gi[k] = (float)out[k];
    if (grad.mean)
#pragma unroll
        for (int k = 0; k < 14; ++k) plane(grad, k)[i] = gi[k];
    if (adam.m.mean && !(adam.skip && *adam.skip)) adam_update(adam, g, i, gi);
}

}  // namespace

int64_t project_blocks(int64_t n) { return n > 0 ? (n + 255) / 256 : 1; }

void launch_project(const ParamsK &g, const CamK &cam, const RasterK &rk, Rec *rec, uint2 *rect,
                    uint32_t *count, uint32_t *dkey, uint32_t *ids, uint32_t *n_out, int shift, uint32_t *kpart,
                    hipStream_t s, uint32_t id_base, float *reg_part, uint32_t *csum, uint32_t *shist, int supers_x)
{
    hipLaunchKernelGGL(k_project, dim3((unsigned)project_blocks(g.n)), dim3(256), 0, s, g, cam, rk, rec, rect, count,
                       dkey, ids, n_out, shift, kpart, id_base, reg_part, csum, shist, supers_x);
}

void launch_project_bwd_window(const ParamsK &g, const CamK *cams_dev, int nv, float lowpass, float *grad2d,
                               int64_t view_stride, const GradK &grad, const AdamK &adam, hipStream_t s)
{
    if (g.n <= 0) return;
    const int64_t blocks = (g.n + 255) / 256;
    hipLaunchKernelGGL(k_project_bwd_window, dim3((unsigned)blocks), dim3(256), 0, s, g, cams_dev, nv, lowpass, grad2d,
                       view_stride, grad, adam);
}

void launch_project_bwd(const ParamsK &g, const CamK &cam, const RasterK &rk, float *grad2d, const GradK &grad_in,
                        const GradK &grad_out, const AdamK &adam, hipStream_t s, const LossFinalK &lf)
{
    if (g.n <= 0) return;
    const int64_t blocks = (g.n + 255) / 256 + (lf.partials ? 1 : 0);
    hipLaunchKernelGGL(k_project_bwd, dim3((unsigned)blocks), dim3(256), 0, s, g, cam, rk, grad2d, grad_in, grad_out,
                       adam, lf);
}

}  // namespace fgs
