// Learned seeding prior: tile spectral features, the GELU network on MFMA (BF16 operands, FP32
// accumulation), its backward pass and Adam.
//
// Every GEMM here has the form C[m][n] = sum_k A[m][k] B[n][k] with both operands BF16 and
// contiguous along k, so one kernel serves the forward (A = activations, B = weights), the
// input-gradient (A = output gradients, B = transposed weights) and the weight-gradient products
// (A = transposed output gradients, B = transposed activations, k running over the rows). The
// forward and input-gradient epilogues write each result twice, row-major for the next product
// and transposed for the weight gradient, so no separate transpose pass is needed.
#include <hip/hip_runtime.h>

#include <cmath>

#include "mlp_internal.h"

namespace fgs {
namespace {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (NaN kept quiet, infinities kept)
__device__ inline uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }

__device__ inline float gelu_grad(float a)
{
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * expf(-0.5f * a * a) * 0.39894228040143268f;
}

/* -------------------------------------- tile features -------------------------------------- */

__global__ void __launch_bounds__(256)
k_tile_features(const float *__restrict__ rgb, const float *__restrict__ depth, int W, int H, float dmin, float dmax,
                int64_t n_tiles, const int32_t *__restrict__ tile_ids, float *__restrict__ feat,
                int32_t *__restrict__ n_valid)
{
    __shared__ double Y[16][17];
    __shared__ double Tre[16][17], Tim[16][17];
    __shared__ double tc[16], ts[16];
    __shared__ double r_sum[4], r_sum2[4], r_min[4], r_max[4];
    __shared__ int r_cnt[4];
    const int tid = threadIdx.x, x = tid & 15, y = tid >> 4;
    const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
    const int64_t t = blockIdx.x;
    if (t >= n_tiles) return;
    const int64_t id = tile_ids ? (int64_t)tile_ids[t] : t;
    float *f = feat + t * 260;
    if (id < 0 || id >= (int64_t)tiles_x * tiles_y) {  // not a tile of this frame
        for (int k = tid; k < 260; k += 256) f[k] = 0.0f;
        if (n_valid && tid == 0) n_valid[t] = -1;
        return;
    }
    const int tx = (int)(id % tiles_x), ty = (int)(id / tiles_x);
    if (tid < 16) {
        double s, c;
        sincospi((double)tid / 8.0, &s, &c);  // angle 2 pi tid / 16
        tc[tid] = c;
        ts[tid] = s;
    }
    const int gx = tx * 16 + x, gy = ty * 16 + y;
    double lum = 0.0, d = 0.0;
    bool valid = false;
    if (gx < W && gy < H) {
        const int64_t P = (int64_t)W * H, p = (int64_t)gy * W + gx;
        lum = 0.299 * (double)rgb[p] + 0.587 * (double)rgb[P + p] + 0.114 * (double)rgb[2 * P + p];
        d = (double)depth[p];
        valid = isfinite(d) && d >= (double)dmin && d <= (double)dmax;
    }
    Y[y][x] = lum;
    // depth statistics: wave reductions, then across the four waves
    double s1 = valid ? d : 0.0, s2 = valid ? d * d : 0.0, mn = valid ? d : INFINITY, mx = valid ? d : -INFINITY;
    int cnt = valid ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
        mn = fmin(mn, __shfl_xor(mn, o));
        mx = fmax(mx, __shfl_xor(mx, o));
        cnt += __shfl_xor(cnt, o);
    }
    const int wid = tid >> 6;
    if ((tid & 63) == 0) {
        r_sum[wid] = s1;
        r_sum2[wid] = s2;
        r_min[wid] = mn;
        r_max[wid] = mx;
        r_cnt[wid] = cnt;
    }
    __syncthreads();
    // row transform: T[y][u] = sum_x Y[y][x] e^{-2 pi i u x / 16}  (thread (y, u = x))
    {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < 16; ++k) {
            const int a = (x * k) & 15;
            re += Y[y][k] * tc[a];
            im -= Y[y][k] * ts[a];
        }
        Tre[y][x] = re;
        Tim[y][x] = im;
    }
    __syncthreads();
    // column transform: F[v][u] = sum_y T[y][u] e^{-2 pi i v y / 16}  (thread (v = y, u = x))
    {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < 16; ++k) {
            const int a = (y * k) & 15;
            const double c = tc[a], s = ts[a], ar = Tre[k][x], ai = Tim[k][x];
            re += ar * c + ai * s;
            im += ai * c - ar * s;
        }
        const int i = (x + 8) & 15, j = (y + 8) & 15;  // DC at (8, 8)
        f[j * 16 + i] = (float)log1p(sqrt(re * re + im * im));
    }
    if (tid == 0) {
        double S1 = 0.0, S2 = 0.0, MN = INFINITY, MX = -INFINITY;
        int C = 0;
        for (int w = 0; w < 4; ++w) {
            S1 += r_sum[w];
            S2 += r_sum2[w];
            MN = fmin(MN, r_min[w]);
            MX = fmax(MX, r_max[w]);
            C += r_cnt[w];
        }
        if (C > 0) {
            const double mean = S1 / C, var = S2 / C - mean * mean;
            f[256] = (float)mean;
            f[257] = (float)sqrt(var > 0.0 ? var : 0.0);
            f[258] = (float)MN;
            f[259] = (float)MX;
        } else {
            f[256] = f[257] = f[258] = f[259] = 0.0f;
        }
        if (n_valid) n_valid[t] = C;
    }
}

/* ------------------------------------ operand packing ------------------------------------ */

// BF16 shadows of the packed FP32 weights: W1b [256][288], W2b [256][256], W3b [16][256],
// W2T [256][256] (W2T[k][n] = W2[n][k]), W3T [256][32] (W3T[k][o] = W3[o][k]); padding is zero.
__global__ void k_mlp_shadow(const float *__restrict__ w, uint16_t *W1b, uint16_t *W2b, uint16_t *W3b, uint16_t *W2T,
                             uint16_t *W3T)
{
    const int64_t n1 = (int64_t)kMlpHidden * kMlpInPad, n2 = (int64_t)kMlpHidden * kMlpHidden,
                  n3 = (int64_t)kMlpOutPad * kMlpHidden, n4 = (int64_t)kMlpHidden * kMlpOutK;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2 + n3 + n4;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n1) {
            const int j = (int)(i / kMlpInPad), k = (int)(i % kMlpInPad);
            W1b[i] = k < kMlpIn ? to_bf16(w[kOffW1 + (int64_t)j * kMlpIn + k]) : (uint16_t)0;
        } else if (i < n1 + n2) {
            const int64_t e = i - n1;
            const int j = (int)(e / kMlpHidden), k = (int)(e % kMlpHidden);
            const uint16_t b = to_bf16(w[kOffW2 + e]);
            W2b[e] = b;
            W2T[(int64_t)k * kMlpHidden + j] = b;
        } else if (i < n1 + n2 + n3) {
            const int64_t e = i - n1 - n2;
            const int o = (int)(e / kMlpHidden), k = (int)(e % kMlpHidden);
            W3b[e] = o < kMlpOut ? to_bf16(w[kOffW3 + (int64_t)o * kMlpHidden + k]) : (uint16_t)0;
        } else {
            const int64_t e = i - n1 - n2 - n3;
            const int k = (int)(e / kMlpOutK), o = (int)(e % kMlpOutK);
            W3T[e] = o < kMlpOut ? to_bf16(w[kOffW3 + (int64_t)o * kMlpHidden + k]) : (uint16_t)0;
        }
    }
}

// Xb [Rp][288] and (optional) XT [288][Rp] from x [rows][260]; rows >= rows and columns >= 260 zero.
__global__ void k_mlp_pack_x(const float *__restrict__ x, int64_t rows, int64_t Rp, uint16_t *__restrict__ Xb,
                             uint16_t *__restrict__ XT)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Rp * kMlpInPad;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i / kMlpInPad;
        const int k = (int)(i % kMlpInPad);
        const uint16_t b = (m < rows && k < kMlpIn) ? to_bf16(x[m * kMlpIn + k]) : (uint16_t)0;
        Xb[i] = b;
        if (XT) XT[(int64_t)k * Rp + m] = b;
    }
}

/* ------------------------------------------ GEMM ------------------------------------------ */

enum EpiKind { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DGRAD = 2, EPI_PARTIAL = 3 };

struct Epi {
    const float *bias;   // HIDDEN, OUT
    float *a_out;        // HIDDEN: pre-activation [M][N]
    const float *a_in;   // DGRAD: pre-activation [M][N] for GELU'
    uint16_t *h_out;     // HIDDEN: GELU(a) BF16 [M][N]; DGRAD: dA BF16 [M][N] (nullable)
    uint16_t *hT_out;    // transposed copy [N][ldt] (nullable)
    int64_t ldt;
    float *bias_grad;    // DGRAD: column sums of dA (atomic)
    float *y_out;        // OUT: [rows_valid][4]
    int64_t rows_valid;
    float *c_out;        // PARTIAL: [split][M][N]
};

// One workgroup: 4 waves, 64 rows x (16 JT) columns; wave w owns rows 16w..16w+15 and JT
// 16x16 MFMA accumulators. Lane l feeds row (l % 16) of A and column (l % 16) of B with 8
// consecutive k of group l / 16; the accumulator holds rows 4 (l / 16) + i of column l % 16.
// M and N are multiples of 16, K of 32; blockIdx.z takes the k range [z ksplit, (z+1) ksplit).
template <int JT, int KIND>
__global__ void __launch_bounds__(256)
k_gemm_nt(const uint16_t *__restrict__ A, int64_t lda, const uint16_t *__restrict__ B, int64_t ldb, int M, int N,
          int64_t K, int64_t ksplit, Epi e)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.y * 64 + wave * 16;
    const int n0 = blockIdx.x * (16 * JT);
    if (m0 >= M) return;
    const int64_t kb = (int64_t)blockIdx.z * ksplit;
    const int64_t ke = kb + ksplit < K ? kb + ksplit : K;
    const int r = lane & 15, g = lane >> 4;
    f32x4 acc[JT];
#pragma unroll
    for (int j = 0; j < JT; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const uint16_t *ap = A + (int64_t)(m0 + r) * lda + g * 8;
    const uint16_t *bp[JT];
    bool on[JT];
#pragma unroll
    for (int j = 0; j < JT; ++j) {
        on[j] = n0 + 16 * j < N;
        bp[j] = B + (int64_t)(on[j] ? n0 + 16 * j + r : 0) * ldb + g * 8;
    }
    for (int64_t k = kb; k < ke; k += 32) {
        const bf16x8 a = *(const bf16x8 *)(ap + k);
#pragma unroll
        for (int j = 0; j < JT; ++j)
            if (on[j]) {
                const bf16x8 b = *(const bf16x8 *)(bp[j] + k);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
            }
    }
#pragma unroll
    for (int j = 0; j < JT; ++j) {
        if (!on[j]) continue;
        const int col = n0 + 16 * j + r;
        float colsum = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = m0 + 4 * g + i;
            const float c = acc[j][i];
            const int64_t o = (int64_t)row * N + col;
            if (KIND == EPI_HIDDEN) {
                const float av = c + e.bias[col];
                if (e.a_out) e.a_out[o] = av;
                const uint16_t h = to_bf16(gelu(av));
                e.h_out[o] = h;
                if (e.hT_out) e.hT_out[(int64_t)col * e.ldt + row] = h;
            } else if (KIND == EPI_OUT) {
                if (col < kMlpOut && row < e.rows_valid) e.y_out[(int64_t)row * kMlpOut + col] = c + e.bias[col];
            } else if (KIND == EPI_DGRAD) {
                const float da = c * gelu_grad(e.a_in[o]);
                colsum += da;
                const uint16_t h = to_bf16(da);
                if (e.h_out) e.h_out[o] = h;
                if (e.hT_out) e.hT_out[(int64_t)col * e.ldt + row] = h;
            } else {
                e.c_out[((int64_t)blockIdx.z * M + row) * N + col] = c;
            }
        }
        if (KIND == EPI_DGRAD) {
            colsum += __shfl_xor(colsum, 16);
            colsum += __shfl_xor(colsum, 32);
            if (g == 0) atomicAdd(&e.bias_grad[col], colsum);
        }
    }
}

// dst[r * ld_dst + c] = sum over splits of partial[s][r][c], for r < rows, c < cols.
__global__ void k_mlp_reduce_partials(const float *__restrict__ partial, int splits, int M, int N, int rows, int cols,
                                      float *__restrict__ dst, int ld_dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)rows * cols;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int rr = (int)(i / cols), cc = (int)(i % cols);
        float s = 0.0f;
        for (int z = 0; z < splits; ++z) s += partial[((int64_t)z * M + rr) * N + cc];
        dst[(int64_t)rr * ld_dst + cc] = s;
    }
}

/* ------------------------------------ loss and update ------------------------------------ */

// dY = 2 (y - t) / (rows 4), written as BF16 row-major [Rp][32] and transposed [16][Rp], zero
// outside rows x 4.
__global__ void k_mlp_dy(const float *__restrict__ y, const float *__restrict__ t, int64_t rows, int64_t Rp,
                         uint16_t *__restrict__ dYb, uint16_t *__restrict__ dYT)
{
    const float sc = 2.0f / (float)(rows * kMlpOut);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Rp * kMlpOutK;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i / kMlpOutK;
        const int o = (int)(i % kMlpOutK);
        float d = 0.0f;
        if (m < rows && o < kMlpOut) d = (y[m * kMlpOut + o] - t[m * kMlpOut + o]) * sc;
        const uint16_t b = to_bf16(d);
        dYb[i] = b;
        if (o < kMlpOutPad) dYT[(int64_t)o * Rp + m] = b;
    }
}

// loss = mean (y - t)^2 (FP64, fixed order) and the output-bias gradient sum_m dY[m][o].
__global__ void __launch_bounds__(256)
k_mlp_loss(const float *__restrict__ y, const float *__restrict__ t, int64_t rows, double *loss, float *gb3,
           float *loss_f)
{
    __shared__ double part[5][256];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const float sc = 2.0f / (float)(rows * kMlpOut);
    for (int64_t m = threadIdx.x; m < rows; m += 256)
        for (int o = 0; o < kMlpOut; ++o) {
            const float d = y[m * kMlpOut + o] - t[m * kMlpOut + o];
            acc[0] += (double)d * (double)d;
            acc[1 + o] += (double)(d * sc);
        }
    for (int k = 0; k < 5; ++k) part[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 5; ++k) part[k][threadIdx.x] += part[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double L = part[0][0] / (double)(rows * kMlpOut);
        *loss = L;
        if (loss_f) *loss_f = (float)L;
        for (int o = 0; o < kMlpOut; ++o) gb3[o] = (float)part[1 + o][0];
    }
}

__global__ void k_mlp_zero(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_mlp_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                           float bc2, float *__restrict__ grad_out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        if (grad_out) grad_out[i] = gi;
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

/* ------------------------------------- prior on seeds ------------------------------------- */

__global__ void k_prior_apply(PriorApplyK pk, const uint32_t *__restrict__ count, int64_t capacity,
                              const int32_t *__restrict__ pixel, const float *__restrict__ y,
                              const int32_t *__restrict__ n_valid, float *__restrict__ log_scale,
                              float *__restrict__ quat, float *__restrict__ logit, int64_t S,
                              uint8_t *__restrict__ from_prior)
{
    const int64_t n = (int64_t)*count < capacity ? (int64_t)*count : capacity;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = pixel[i];
        const int px = p % pk.W, py = p / pk.W;
        const int64_t t = (int64_t)(py / 16) * pk.tiles_x + px / 16;
        bool use = n_valid[t] >= pk.min_valid;
        float o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = y[t * 4 + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) use = use && isfinite(o[k]) && fabsf(o[k]) <= pk.max_dev;
        use = use && isfinite(o[3]);
        if (use && pk.mode != 3) {
            // the radius rule's log-radius, written by the seed emission on every axis
            const float base = log_scale[i];
#pragma unroll
            for (int k = 0; k < 3; ++k) log_scale[k * S + i] = base + o[k];
#pragma unroll
            for (int k = 0; k < 4; ++k) quat[k * S + i] = pk.q[k];
        }
        if (use && pk.mode != 2) logit[i] = o[3];
        if (from_prior) from_prior[i] = use ? 1 : 0;
    }
}

unsigned grid_for(int64_t n, int64_t per = 256, int64_t cap = 2048)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

template <int JT, int KIND>
void gemm(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, int M, int N, int64_t K, int splits,
          const Epi &e, hipStream_t s)
{
    const int64_t steps = K / 32;
    const int64_t per = (steps + splits - 1) / splits;
    dim3 grid((unsigned)((N + 16 * JT - 1) / (16 * JT)), (unsigned)((M + 63) / 64), (unsigned)splits);
    hipLaunchKernelGGL((k_gemm_nt<JT, KIND>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, per * 32, e);
}

void forward(const MlpWS &ws, int64_t rows, const float *x, const float *w, float *y, bool train, hipStream_t s)
{
    const int64_t Rp = mlp_rows_padded(rows);
    const int M = (int)Rp;
    hipLaunchKernelGGL(k_mlp_shadow, dim3(592), dim3(256), 0, s, w, ws.W1b, ws.W2b, ws.W3b, ws.W2T, ws.W3T);
    hipLaunchKernelGGL(k_mlp_pack_x, dim3(grid_for(Rp * kMlpInPad)), dim3(256), 0, s, x, rows, Rp, ws.Xb,
                       train ? ws.XT : nullptr);
    Epi e = {};
    e.bias = w + kOffB1;
    e.a_out = train ? ws.a1 : nullptr;
    e.h_out = ws.h1b;
    e.hT_out = train ? ws.h1T : nullptr;
    e.ldt = Rp;
    gemm<4, EPI_HIDDEN>(ws.Xb, kMlpInPad, ws.W1b, kMlpInPad, M, kMlpHidden, kMlpInPad, 1, e, s);
    e.bias = w + kOffB2;
    e.a_out = train ? ws.a2 : nullptr;
    e.h_out = ws.h2b;
    e.hT_out = train ? ws.h2T : nullptr;
    gemm<4, EPI_HIDDEN>(ws.h1b, kMlpHidden, ws.W2b, kMlpHidden, M, kMlpHidden, kMlpHidden, 1, e, s);
    Epi eo = {};
    eo.bias = w + kOffB3;
    eo.y_out = y;
    eo.rows_valid = rows;
    gemm<1, EPI_OUT>(ws.h2b, kMlpHidden, ws.W3b, kMlpHidden, M, kMlpOutPad, kMlpHidden, 1, eo, s);
}

}  // namespace

size_t mlp_ws_bytes(int64_t rows_cap)
{
    MlpWS ws;
    mlp_ws_carve(nullptr, rows_cap, &ws);
    return (size_t)(uintptr_t)ws.loss + 64;
}

void mlp_ws_carve(void *base, int64_t rows_cap, MlpWS *ws)
{
    const int64_t Rp = mlp_rows_padded(rows_cap > 0 ? rows_cap : 1);
    char *p = (char *)base;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += (bytes + 255) / 256 * 256;
        return q;
    };
    ws->Rp = Rp;
    ws->W1b = (uint16_t *)take((size_t)kMlpHidden * kMlpInPad * 2);
    ws->W2b = (uint16_t *)take((size_t)kMlpHidden * kMlpHidden * 2);
    ws->W3b = (uint16_t *)take((size_t)kMlpOutPad * kMlpHidden * 2);
    ws->W2T = (uint16_t *)take((size_t)kMlpHidden * kMlpHidden * 2);
    ws->W3T = (uint16_t *)take((size_t)kMlpHidden * kMlpOutK * 2);
    ws->Xb = (uint16_t *)take((size_t)Rp * kMlpInPad * 2);
    ws->XT = (uint16_t *)take((size_t)Rp * kMlpInPad * 2);
    ws->a1 = (float *)take((size_t)Rp * kMlpHidden * 4);
    ws->a2 = (float *)take((size_t)Rp * kMlpHidden * 4);
    ws->h1b = (uint16_t *)take((size_t)Rp * kMlpHidden * 2);
    ws->h1T = (uint16_t *)take((size_t)Rp * kMlpHidden * 2);
    ws->h2b = (uint16_t *)take((size_t)Rp * kMlpHidden * 2);
    ws->h2T = (uint16_t *)take((size_t)Rp * kMlpHidden * 2);
    ws->dYb = (uint16_t *)take((size_t)Rp * kMlpOutK * 2);
    ws->dYT = (uint16_t *)take((size_t)Rp * kMlpOutPad * 2);
    ws->da2b = (uint16_t *)take((size_t)Rp * kMlpHidden * 2);
    ws->da2T = (uint16_t *)take((size_t)Rp * kMlpHidden * 2);
    ws->da1T = (uint16_t *)take((size_t)Rp * kMlpHidden * 2);
    ws->y = (float *)take((size_t)Rp * kMlpOut * 4);
    ws->grad = (float *)take((size_t)kMlpParams * 4);
    ws->partial = (float *)take((size_t)kMlpSplits * kMlpHidden * kMlpInPad * 4);
    ws->loss = (double *)take(8);
}

void launch_tile_features(const float *rgb, const float *depth, int W, int H, float dmin, float dmax, int64_t n_tiles,
                          const int32_t *tile_ids, float *feat, int32_t *n_valid, hipStream_t s)
{
    if (n_tiles <= 0) return;
    hipLaunchKernelGGL(k_tile_features, dim3((unsigned)n_tiles), dim3(256), 0, s, rgb, depth, W, H, dmin, dmax,
                       n_tiles, tile_ids, feat, n_valid);
}

void launch_mlp_forward(const MlpWS &ws, int64_t rows, const float *x, const float *w, float *y, bool keep,
                        hipStream_t s)
{
    if (rows <= 0) return;
    forward(ws, rows, x, w, y, keep, s);
}

void launch_mlp_train_step(const MlpWS &ws, int64_t rows, const float *x, const float *target, float *w, float *m,
                           float *v, float lr, float beta1, float beta2, float eps, float bc1, float bc2, float *loss,
                           float *grad_out, hipStream_t s)
{
    const int64_t Rp = mlp_rows_padded(rows);
    const int M = (int)Rp;
    hipLaunchKernelGGL(k_mlp_zero, dim3(grid_for(kMlpParams)), dim3(256), 0, s, ws.grad, kMlpParams);
    forward(ws, rows, x, w, ws.y, true, s);
    hipLaunchKernelGGL(k_mlp_dy, dim3(grid_for(Rp * kMlpOutK)), dim3(256), 0, s, ws.y, target, rows, Rp, ws.dYb,
                       ws.dYT);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, ws.y, target, rows, ws.loss, ws.grad + kOffB3, loss);
    // input gradients through the output and second layers (GELU' on the way), bias sums
    Epi e = {};
    e.a_in = ws.a2;
    e.h_out = ws.da2b;
    e.hT_out = ws.da2T;
    e.ldt = Rp;
    e.bias_grad = ws.grad + kOffB2;
    gemm<4, EPI_DGRAD>(ws.dYb, kMlpOutK, ws.W3T, kMlpOutK, M, kMlpHidden, kMlpOutK, 1, e, s);
    e.a_in = ws.a1;
    e.h_out = nullptr;
    e.hT_out = ws.da1T;
    e.bias_grad = ws.grad + kOffB1;
    gemm<4, EPI_DGRAD>(ws.da2b, kMlpHidden, ws.W2T, kMlpHidden, M, kMlpHidden, kMlpHidden, 1, e, s);
    // weight gradients: k runs over the rows, split over kMlpSplits workgroup slices
    Epi ep = {};
    ep.c_out = ws.partial;
    const int S = Rp / 32 >= kMlpSplits ? kMlpSplits : (int)(Rp / 32);
    gemm<4, EPI_PARTIAL>(ws.dYT, Rp, ws.h2T, Rp, kMlpOutPad, kMlpHidden, Rp, S, ep, s);
    hipLaunchKernelGGL(k_mlp_reduce_partials, dim3(grid_for(kMlpOut * kMlpHidden)), dim3(256), 0, s, ws.partial, S,
                       kMlpOutPad, kMlpHidden, kMlpOut, kMlpHidden, ws.grad + kOffW3, kMlpHidden);
    gemm<4, EPI_PARTIAL>(ws.da2T, Rp, ws.h1T, Rp, kMlpHidden, kMlpHidden, Rp, S, ep, s);
    hipLaunchKernelGGL(k_mlp_reduce_partials, dim3(grid_for(kMlpHidden * kMlpHidden)), dim3(256), 0, s, ws.partial,
                       S, kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden, ws.grad + kOffW2, kMlpHidden);
    gemm<4, EPI_PARTIAL>(ws.da1T, Rp, ws.XT, Rp, kMlpHidden, kMlpInPad, Rp, S, ep, s);
    hipLaunchKernelGGL(k_mlp_reduce_partials, dim3(grid_for(kMlpHidden * kMlpIn)), dim3(256), 0, s, ws.partial, S,
                       kMlpHidden, kMlpInPad, kMlpHidden, kMlpIn, ws.grad + kOffW1, kMlpIn);
    hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(kMlpParams)), dim3(256), 0, s, w, ws.grad, m, v, kMlpParams, lr,
                       beta1, beta2, eps, bc1, bc2, grad_out);
}

void launch_prior_apply(const PriorApplyK &pk, const uint32_t *count, int64_t capacity, const int32_t *pixel,
                        const float *y, const int32_t *n_valid, float *log_scale, float *quat, float *logit,
                        int64_t stride, uint8_t *from_prior, hipStream_t s)
{
    if (capacity <= 0) return;
    hipLaunchKernelGGL(k_prior_apply, dim3(grid_for(capacity)), dim3(256), 0, s, pk, count, capacity, pixel, y,
                       n_valid, log_scale, quat, logit, stride, from_prior);
}

}  // namespace fgs
