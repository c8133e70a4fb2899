// Fourier seeding of new gaussians (Sec. III-A, "Mapping": Eq. 2-8, the triangle threshold, Eq. 11).
//
//  1. luma of the frame (BT.601, FP64) and the 2D DFT of Eq. 2, as row transforms followed by
//     column transforms;
//  2. the Gaussian high-pass of Eq. 5 applied to the spectrum with its centre at DC (the centring
//     of Eq. 3 expressed on the unshifted spectrum, Eq. 7), and the inverse DFT of Eq. 8 with the
//     1/(HW) factor; E = |I_h|;
//  3. q = floor(255 (E / E_max)), its 256-bin histogram and the triangle threshold t; the high-
//     frequency mask is q > t, the low-frequency mask its complement;
//  4. seeds on a stride-m lattice inside the high-frequency mask and a stride-n lattice inside the
//     low-frequency mask where the depth is valid, emitted in row-major pixel order, each back-
//     projected at its pixel centre with the radius alpha d / f of Eq. 11 (alpha_h or alpha_l).
//
// The transforms are mixed-radix Stockham FFTs in FP64 with one line held in LDS; the column
// pass runs forward transform, filter and inverse transform in one kernel. Step 4's values are
// IEEE binary32 operations in a fixed order (this file is compiled without contraction), so they
// are bit-identical to any other IEEE implementation of the same sequence.
#include "fgs_internal.h"
#include "seed_internal.h"

namespace fgs {

namespace {

constexpr int kT = 256;

struct Plan {
    int32_t n, stages;
    int32_t radix[16];
};

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One Stockham pass of radix R over a line of N points (LDS in -> out).
// sign = -1 forward, +1 inverse (no scaling).
template <int R>
__device__ inline void stage_fixed(const double2 *in, double2 *out, int N, int Ns, int sign, const double2 *wR)
{
    const int M = N / R;
    for (int j = threadIdx.x; j < M; j += kT) {
        const int k = j % Ns;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r] = in[j + r * M];
            if (r && k) {
                double s, c;
                sincospi((double)(sign * 2) * (double)(k * r) / (double)(Ns * R), &s, &c);
                v[r] = cmul(v[r], make_double2(c, s));
            }
        }
        double2 V[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double2 w = wR[(q * r) % R];
                acc.x += v[q].x * w.x - v[q].y * w.y;
                acc.y += v[q].x * w.y + v[q].y * w.x;
            }
            V[r] = acc;
        }
        const int idx = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out[idx + r * Ns] = V[r];
    }
}

// Generic radix (small primes beyond 7): same pass with the butterfly in a loop.
__device__ inline void stage_generic(const double2 *in, double2 *out, int N, int Ns, int R, int sign, const double2 *wR)
{
    const int M = N / R;
    for (int j = threadIdx.x; j < M; j += kT) {
        const int k = j % Ns;
        const int idx = (j / Ns) * Ns * R + k;
        for (int r = 0; r < R; ++r) {
            double2 acc = make_double2(0.0, 0.0);
            for (int q = 0; q < R; ++q) {
                double2 x = in[j + q * M];
                if (q && k) {
                    double s, c;
                    sincospi((double)(sign * 2) * (double)(k * q) / (double)(Ns * R), &s, &c);
                    x = cmul(x, make_double2(c, s));
                }
                const double2 w = wR[(q * r) % R];
                acc.x += x.x * w.x - x.y * w.y;
                acc.y += x.x * w.y + x.y * w.x;
            }
            out[idx + r * Ns] = acc;
        }
    }
}

// Full transform of one line in LDS; returns the buffer holding the result.
__device__ double2 *fft_line(double2 *a, double2 *b, double2 *wR, const Plan &pl, int sign)
{
    int Ns = 1;
    for (int s = 0; s < pl.stages; ++s) {
        const int R = pl.radix[s];
        if (threadIdx.x < R) {
            double sn, cs;
            sincospi((double)(sign * 2) * (double)threadIdx.x / (double)R, &sn, &cs);
            wR[threadIdx.x] = make_double2(cs, sn);
        }
        __syncthreads();
        switch (R) {
        case 2: stage_fixed<2>(a, b, pl.n, Ns, sign, wR); break;
        case 3: stage_fixed<3>(a, b, pl.n, Ns, sign, wR); break;
        case 4: stage_fixed<4>(a, b, pl.n, Ns, sign, wR); break;
        case 5: stage_fixed<5>(a, b, pl.n, Ns, sign, wR); break;
        case 7: stage_fixed<7>(a, b, pl.n, Ns, sign, wR); break;
        default: stage_generic(a, b, pl.n, Ns, R, sign, wR); break;
        }
        __syncthreads();
        double2 *t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

__device__ inline double block_max(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Row transforms of the luma: one block per row. Also the row's max |luma|.
__global__ void __launch_bounds__(kT)
k_rows_fwd(const float *__restrict__ rgb, int W, int H, Plan pl, double2 *__restrict__ F, double *__restrict__ ymax)
{
    extern __shared__ double2 lds[];
    double2 *a = lds, *b = lds + W, *wR = lds + 2 * W;
    __shared__ double red[kT];
    const int y = blockIdx.x;
    const int64_t P = (int64_t)W * H;
    double m = 0.0;
    for (int x = threadIdx.x; x < W; x += kT) {
        const int64_t p = (int64_t)y * W + x;
        const double Y = 0.299 * (double)rgb[p] + 0.587 * (double)rgb[P + p] + 0.114 * (double)rgb[2 * P + p];
        a[x] = make_double2(Y, 0.0);
        m = fmax(m, fabs(Y));
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) ymax[y] = m;
    const double2 *res = fft_line(a, b, wR, pl, -1);
    for (int x = threadIdx.x; x < W; x += kT) F[(int64_t)y * W + x] = res[x];
}

// Column pass: forward transform of column u, high-pass filter, inverse transform (in place).
__global__ void __launch_bounds__(kT)
k_cols_filter(double2 *__restrict__ F, int W, int H, Plan pl, double D0)
{
    extern __shared__ double2 lds[];
    double2 *a = lds, *b = lds + H, *wR = lds + 2 * H;
    const int u = blockIdx.x;
    for (int v = threadIdx.x; v < H; v += kT) a[v] = F[(int64_t)v * W + u];
    __syncthreads();
    double2 *res = fft_line(a, b, wR, pl, -1);
    double2 *other = res == a ? b : a;
    const double ub = (double)u < W / 2.0 ? (double)u : (double)u - W;
    for (int v = threadIdx.x; v < H; v += kT) {
        const double vb = (double)v < H / 2.0 ? (double)v : (double)v - H;
        const double D2 = ub * ub + vb * vb;
        const double Hf = 1.0 - exp(-D2 / (2.0 * D0 * D0));
        res[v] = make_double2(res[v].x * Hf, res[v].y * Hf);
    }
    __syncthreads();
    res = fft_line(res, other, wR, pl, +1);
    for (int v = threadIdx.x; v < H; v += kT) F[(int64_t)v * W + u] = res[v];
}

// Inverse row transforms, 1/(WH), E = |I_h|; the row's max E.
__global__ void __launch_bounds__(kT)
k_rows_inv(const double2 *__restrict__ F, int W, int H, Plan pl, double *__restrict__ E, double *__restrict__ emax)
{
    extern __shared__ double2 lds[];
    double2 *a = lds, *b = lds + W, *wR = lds + 2 * W;
    __shared__ double red[kT];
    const int y = blockIdx.x;
    for (int x = threadIdx.x; x < W; x += kT) a[x] = F[(int64_t)y * W + x];
    __syncthreads();
    const double2 *res = fft_line(a, b, wR, pl, +1);
    const double inv = 1.0 / ((double)W * (double)H);
    double m = 0.0;
    for (int x = threadIdx.x; x < W; x += kT) {
        const double re = res[x].x * inv, im = res[x].y * inv;
        const double e = sqrt(re * re + im * im);
        E[(int64_t)y * W + x] = e;
        m = fmax(m, e);
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) emax[y] = m;
}

// E_max over rows, with the flat-frame rule (E_max <= 1e-9 max|luma| means no high-frequency
// region); clears the histogram.
__global__ void __launch_bounds__(kT)
k_emax(const double *__restrict__ emax_rows, const double *__restrict__ ymax_rows, int H, SeedScalars *__restrict__ sc,
       uint32_t *__restrict__ hist)
{
    __shared__ double red[kT];
    double e = 0.0, y = 0.0;
    for (int i = threadIdx.x; i < H; i += kT) {
        e = fmax(e, emax_rows[i]);
        y = fmax(y, ymax_rows[i]);
    }
    e = block_max(e, red);
    y = block_max(y, red);
    hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) sc->emax = e <= 1e-9 * y ? 0.0 : e;
}

__global__ void __launch_bounds__(kT)
k_hist(const double *__restrict__ E, int64_t P, const SeedScalars *__restrict__ sc, uint8_t *__restrict__ q,
       uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const double emax = sc->emax;
    for (int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x; p < P; p += (int64_t)gridDim.x * kT) {
        int v = 0;
        if (emax > 0.0) {
            v = (int)floor(255.0 * (E[p] / emax));  // the maximum maps exactly to 255
            v = v > 255 ? 255 : v;
        }
        q[p] = (uint8_t)v;
        if (emax > 0.0) atomicAdd(&h[v], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Triangle threshold over the 256 bins (one block of 256 threads): peak p = first maximum;
// endpoint e = last non-empty bin of the longer side (right on equal lengths); for bins strictly
// between p and e, the distance below the line from (p, h_p) to (e, h_e) is the integer cross
// product with the sign that makes "below" positive; the largest wins, the bin nearest the peak
// on ties. With E_max = 0 (flat frame) the threshold is -1 and every pixel is low frequency.
__global__ void __launch_bounds__(256) k_triangle(const uint32_t *__restrict__ hist, SeedScalars *__restrict__ sc)
{
    __shared__ int64_t h[256];
    __shared__ int64_t key[256];
    __shared__ int32_t sp, sa, sb;
    const int i = threadIdx.x;
    h[i] = hist[i];
    __syncthreads();
    if (i == 0) {
        int32_t a = -1, b = -1, p = 0;
        for (int k = 0; k < 256; ++k) {
            if (h[k] > 0) {
                if (a < 0) a = k;
                b = k;
            }
            if (h[k] > h[p]) p = k;
        }
        sp = p;
        sa = a;
        sb = b;
    }
    __syncthreads();
    const int32_t p = sp, a = sa, b = sb;
    const int32_t e = (b - p >= p - a) ? b : a;
    const int32_t dir = e > p ? 1 : -1;
    // key: below-distance in the high bits, closeness to the peak in the low 9 bits
    int64_t k = INT64_MIN;
    if ((i - p) * dir > 0 && (e - i) * dir > 0) {
        const int64_t cross = (int64_t)(e - p) * (h[i] - h[p]) - (h[e] - h[p]) * (int64_t)(i - p);
        const int64_t below = dir > 0 ? -cross : cross;
        k = below * 512 + (511 - (i - p) * dir);
    }
    key[i] = k;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (i < s && key[i + s] > key[i]) key[i] = key[i + s];
        __syncthreads();
    }
    if (i == 0) {
        int32_t t = p;
        if (key[0] != INT64_MIN) t = p + dir * (511 - (int32_t)(key[0] & 511));
        if (sc->emax <= 0.0 || a < 0) t = -1;
        sc->thresh = t;
    }
}

// Missing-region mask M_m (Eq. 9) at pixel p: too little rendered opacity A (M_i), or, where A > 0,
// a rendered surface depth (depth / A) far from a valid frame depth (M_d) or a rendered surface
// colour (colour / A) far from the frame's (M_c), decided in binary32 in this order of operations
// (IEEE division, no contraction).
__device__ inline bool missing_at(const SeedK &sk, int64_t p, int64_t P, const float *__restrict__ rgb, float d,
                                  bool valid)
{
    if (!sk.ra) return true;  // no map yet
    const float A = sk.ra[p];
    if (A < sk.tau_a) return true;
    if (!(A > 0.0f)) return false;
    if (valid && fabsf(sk.rd[p] / A - d) > sk.tau_d) return true;
    const float dc = (fabsf(sk.rc[p] / A - rgb[p]) + fabsf(sk.rc[P + p] / A - rgb[P + p])) +
                     fabsf(sk.rc[2 * P + p] / A - rgb[2 * P + p]);
    return dc > sk.tau_c;
}

// Whether pixel (x, y) seeds: valid depth, inside the missing region (Eq. 10 intersects both
// frequency masks with it), and on its class's lattice. miss receives M_m at the pixel.
__device__ inline bool is_seed(int x, int y, const uint8_t *q, const float *rgb, const float *depth, int W, int64_t P,
                               int thresh, const SeedK &sk, bool &high, bool &miss)
{
    const int64_t p = (int64_t)y * W + x;
    const float d = depth[p];
    high = thresh >= 0 && (int)q[p] > thresh;
    const bool valid = isfinite(d) && d >= sk.dmin && d <= sk.dmax;
    miss = missing_at(sk, p, P, rgb, d, valid);
    if (!valid || !miss) return false;
    const int s = high ? sk.m : sk.n;
    return (x % s) == 0 && (y % s) == 0;
}

// Seeds per image row, and per tile (integer atomics: the sums do not depend on their order); the
// missing-region mask when asked for.
__global__ void __launch_bounds__(kT)
k_seed_count(const uint8_t *__restrict__ q, const float *__restrict__ rgb, const float *__restrict__ depth, int W,
             int H, const SeedScalars *sc, SeedK sk, uint32_t *__restrict__ row_count, int32_t *__restrict__ tile_count,
             uint8_t *__restrict__ missing)
{
    __shared__ uint32_t cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int y = blockIdx.x, thresh = sc->thresh;
    const int tile = sk.tile;
    const int tiles_x = (W + tile - 1) / tile;
    const int64_t P = (int64_t)W * H;
    for (int x = threadIdx.x; x < W; x += kT) {
        bool high, miss;
        const bool seed = is_seed(x, y, q, rgb, depth, W, P, thresh, sk, high, miss);
        if (missing) missing[(int64_t)y * W + x] = miss ? 1 : 0;
        if (seed) {
            atomicAdd(&cnt, 1u);
            if (tile_count) atomicAdd(&tile_count[(y / tile) * tiles_x + x / tile], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) row_count[y] = cnt;
}

__global__ void __launch_bounds__(kT)
k_seed_scan(const uint32_t *__restrict__ row_count, int H, uint32_t *__restrict__ row_off, int64_t capacity,
            int64_t *__restrict__ n_dev, uint32_t *__restrict__ status)
{
    __shared__ uint32_t part[kT];
    // each thread scans a contiguous run of rows
    const int per = (H + kT - 1) / kT;
    const int r0 = threadIdx.x * per, r1 = min(H, r0 + per);
    uint32_t s = 0;
    for (int r = r0; r < r1; ++r) s += row_count[r];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int t = 0; t < kT; ++t) {
            const uint32_t v = part[t];
            part[t] = acc;
            acc += v;
        }
        row_off[H] = acc;
        if (n_dev) *n_dev = acc;
        status[ST_SEEDS] = acc;
        if ((int64_t)acc > capacity) atomicMax(&status[ST_SEED_OVF], acc);
    }
    __syncthreads();
    uint32_t off = part[threadIdx.x];
    for (int r = r0; r < r1; ++r) {
        row_off[r] = off;
        off += row_count[r];
    }
}

// Emission in row-major order: one block per row; the row's seeds are ranked by a ballot scan
// in x order. Values follow fixed binary32 operation sequences.
__global__ void __launch_bounds__(kT)
k_seed_emit(const uint8_t *__restrict__ q, const float *__restrict__ rgb, const float *__restrict__ depth, int W,
            int H, const SeedScalars *sc, SeedK sk, const uint32_t *__restrict__ row_off, SeedOutK out)
{
    __shared__ uint32_t wsum[kT / kWave];
    __shared__ uint32_t base;
    const int y = blockIdx.x, lane = __lane_id(), wid = threadIdx.x / kWave;
    const int thresh = sc->thresh;
    const int64_t P = (int64_t)W * H;
    if (threadIdx.x == 0) base = row_off[y];
    __syncthreads();
    for (int x0 = 0; x0 < W; x0 += kT) {
        const int x = x0 + threadIdx.x;
        bool high = false, miss;
        const bool s = x < W && is_seed(x, y, q, rgb, depth, W, P, thresh, sk, high, miss);
        const uint64_t bal = __ballot(s);
        if (lane == 0) wsum[wid] = __popcll(bal);
        __syncthreads();
        uint32_t off = base + __popcll(bal & ((1ull << lane) - 1ull));
        uint32_t total = 0;
        for (int w = 0; w < kT / kWave; ++w) {
            off += w < wid ? wsum[w] : 0u;
            total += wsum[w];
        }
        if (s && (int64_t)off < out.capacity) {
            const int64_t p = (int64_t)y * W + x;
            const int64_t C = out.capacity;
            const float d = depth[p];
            // back-projection at the pixel centre (binary32, this order, no contraction)
            const float X = (((float)x + 0.5f) - sk.cx) * d / sk.fx;
            const float Yc = (((float)y + 0.5f) - sk.cy) * d / sk.fy;
            const float u0 = X - sk.t[0], u1 = Yc - sk.t[1], u2 = d - sk.t[2];
            float mu[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) mu[r] = (sk.R[r] * u0 + sk.R[3 + r] * u1) + sk.R[6 + r] * u2;
            const float rad = ((high ? sk.alpha_h : sk.alpha_l) * d) / sk.fx;
            out.pixel[off] = (int32_t)p;
            out.is_high[off] = high ? 1 : 0;
#pragma unroll
            for (int r = 0; r < 3; ++r) out.mean[r * C + off] = mu[r];
            out.radius[off] = rad;
#pragma unroll
            for (int c = 0; c < 3; ++c) out.rgb[c * C + off] = rgb[c * P + p];
            if (out.params.mean) {
                // the seed as a gaussian: isotropic scale r, identity rotation, constant opacity
                const int64_t S = out.params.stride;
                const float ls = logf(rad);
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    out.params.mean[r * S + off] = mu[r];
                    out.params.log_scale[r * S + off] = ls;
                    out.params.rgb[r * S + off] = rgb[r * P + p];
                }
                out.params.quat[off] = 1.0f;
                out.params.quat[S + off] = out.params.quat[2 * S + off] = out.params.quat[3 * S + off] = 0.0f;
                out.params.logit[off] = sk.opacity_logit;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) base += total;
        __syncthreads();
    }
}

__global__ void k_fill_i32(int32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

bool make_plan(int N, Plan &pl)
{
    pl.n = N;
    pl.stages = 0;
    int n = N;
    static const int order[] = {4, 2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
    for (int p : order)
        while (n % p == 0) {
            if (pl.stages >= 16) return false;
            pl.radix[pl.stages++] = p;
            n /= p;
        }
    return n == 1;
}

}  // namespace

bool seed_size_supported(int W, int H)
{
    Plan a, b;
    return W >= 2 && H >= 2 && W <= kSeedMaxLine && H <= kSeedMaxLine && make_plan(W, a) && make_plan(H, b);
}

size_t seed_ws_bytes(int W, int H)
{
    const size_t P = (size_t)W * H;
    return P * 16 + P * 8 + P + 2 * (size_t)H * 8 + 256 * 4 + ((size_t)H + 1) * 4 * 2 + 4096;
}

uint32_t *seed_count_ptr(void *ws, int W, int H)
{
    const size_t P = (size_t)W * H;
    char *w = (char *)ws;
    w += ((P * 16 + 255) / 256) * 256;
    w += ((P * 8 + 255) / 256) * 256;
    w += ((P + 255) / 256) * 256;
    w += ((2 * (size_t)H * 8 + 255) / 256) * 256;
    w += 256 * 4;
    uint32_t *row_count = (uint32_t *)w;
    return row_count + H + H;  // row_off[H]: the total written by the seed scan
}

void launch_seed(const float *rgb, const float *depth, int W, int H, double D0, const SeedK &sk, const SeedOutK &out,
                 void *ws, SeedScalars *sc, uint32_t *status, hipStream_t s)
{
    Plan pw, ph;
    make_plan(W, pw);
    make_plan(H, ph);
    const int64_t P = (int64_t)W * H;
    char *w = (char *)ws;
    double2 *F = (double2 *)w;
    w += ((P * 16 + 255) / 256) * 256;
    double *E = (double *)w;
    w += ((P * 8 + 255) / 256) * 256;
    uint8_t *q = (uint8_t *)w;
    w += ((P + 255) / 256) * 256;
    double *ymax = (double *)w;
    double *emax = ymax + H;
    w += ((2 * H * 8 + 255) / 256) * 256;
    uint32_t *hist = (uint32_t *)w;
    w += 256 * 4;
    uint32_t *row_count = (uint32_t *)w;
    uint32_t *row_off = row_count + H;

    const size_t lds_w = (2 * (size_t)W + 32) * sizeof(double2), lds_h = (2 * (size_t)H + 32) * sizeof(double2);
    hipLaunchKernelGGL(k_rows_fwd, dim3(H), dim3(kT), lds_w, s, rgb, W, H, pw, F, ymax);
    hipLaunchKernelGGL(k_cols_filter, dim3(W), dim3(kT), lds_h, s, F, W, H, ph, D0);
    hipLaunchKernelGGL(k_rows_inv, dim3(H), dim3(kT), lds_w, s, F, W, H, pw, E, emax);
    hipLaunchKernelGGL(k_emax, dim3(1), dim3(kT), 0, s, emax, ymax, H, sc, hist);
    int64_t hb = (P + kT * 8 - 1) / (kT * 8);
    hipLaunchKernelGGL(k_hist, dim3((unsigned)(hb > 1024 ? 1024 : hb)), dim3(kT), 0, s, E, P, sc, q, hist);
    hipLaunchKernelGGL(k_triangle, dim3(1), dim3(256), 0, s, hist, sc);
    const int tiles = ((W + sk.tile - 1) / sk.tile) * ((H + sk.tile - 1) / sk.tile);
    if (out.tile_count) hipLaunchKernelGGL(k_fill_i32, dim3((tiles + 255) / 256), dim3(256), 0, s, out.tile_count, (int64_t)tiles);
    hipLaunchKernelGGL(k_seed_count, dim3(H), dim3(kT), 0, s, q, rgb, depth, W, H, sc, sk, row_count,
                       out.tile_count, out.missing);
    hipLaunchKernelGGL(k_seed_scan, dim3(1), dim3(kT), 0, s, row_count, H, row_off, out.capacity, out.n_dev, status);
    hipLaunchKernelGGL(k_seed_emit, dim3(H), dim3(kT), 0, s, q, rgb, depth, W, H, sc, sk, row_off, out);
    // diagnostics
    if (out.E) (void)hipMemcpyAsync(out.E, E, (size_t)P * 8, hipMemcpyDeviceToDevice, s);
    if (out.hist) (void)hipMemcpyAsync(out.hist, hist, 256 * 4, hipMemcpyDeviceToDevice, s);
}

}  // namespace fgs
