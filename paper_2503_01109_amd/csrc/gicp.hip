// GICP tracking (Sec. III-B "Tracking", Eq. 12-14) on the GPU.
//
//  * Frame points: one workgroup per lattice row counts the row's valid pixels; a second launch
//    (one workgroup per row again) sums the counts of the rows above its own and writes its
//    points in pixel order, placed by wave ballots.
//  * Cloud grid: the bounding box (two-stage reduction), one cell key per point, the library's
//    radix sort by key, the [start, end) range of every cell, and the points gathered in cell
//    order as float4 (x, y, z, index bits), so that a cell's points are contiguous.
//  * Neighbours and covariances: one thread per point (in cell order, so a wave's queries share
//    cells) searches rings of cells around its own: the first ring is the 3x3x3 block, later
//    ones the shell at Chebyshev distance r, until the k-th nearest found so far is closer than
//    any point outside the rings can be ((r - margin) cells). A point still unsure after
//    kKnnRings rings (an isolated one) scans the whole cloud instead: its work is then n
//    distances, where the rings could cross every empty cell of the grid. The k best are kept
//    sorted in registers by (binary32 squared distance, index): slots below KMAX - k hold -inf
//    sentinels, so the k-th entry is always the last slot and insertion is a fixed, fully
//    unrolled shift. Mean, covariance (FP64, in neighbour order), a cyclic Jacobi
//    eigen-decomposition and the plane regularisation follow in the same thread.
//  * Gauss-Newton: k_gicp_corr gives each source point 16 lanes, which split the cells of its
//    search block, keep the nearest target point within d_max, and reduce by (distance, index)
//    with shuffles; the group's first lane forms the point's 29 FP64 terms (H's upper triangle,
//    b, cost, count) and each workgroup writes the sum of its 16 points. k_gicp_solve, one
//    workgroup, sums those partials in a fixed order, solves the 6x6 system by Cholesky and
//    updates the pose in FP64, and sets a done flag that turns every later launch of the
//    iteration into a no-op.
#include "fgs_internal.h"

namespace fgs {

namespace {

constexpr int kFPThreads = 256;
constexpr int kFPWaves = kFPThreads / kWave;
constexpr int kKMax = 32;
constexpr int kKnnThreads = 128;
constexpr int kKnnRings = 4;  // rings of cells searched before a query scans the whole cloud
constexpr int kCorrThreads = 256, kCorrLanes = 16, kCorrQueries = kCorrThreads / kCorrLanes;
constexpr int kCorrBatches = 1;  // batches of kCorrQueries source points per workgroup (more serialise the
                                 // groups' latency chains: 4 batches made the launch 1.5x slower)
constexpr int kBoxBlocks = 256, kBoxThreads = 256, kBoxOut = 7;

struct PoseK {
    double R[9], t[3];
};

// ------------------------------------ frame points ------------------------------------

__device__ inline bool fp_point(const FrameK &f, int x, int y, float p[3])
{
    const float d = f.depth[(int64_t)y * f.W + x];
    if (!(isfinite(d) && d >= f.dmin && d <= f.dmax)) return false;
    const float a = (float)x + 0.5f, b = (float)y + 0.5f;
    const float X = ((a - f.cx) * d) / f.fx;
    const float Y = ((b - f.cy) * d) / f.fy;
    if (f.has_pose) {
        for (int r = 0; r < 3; ++r) {
            float w = f.R[3 * r] * X;
            w = w + f.R[3 * r + 1] * Y;
            w = w + f.R[3 * r + 2] * d;
            p[r] = w + f.t[r];
        }
    } else {
        p[0] = X;
        p[1] = Y;
        p[2] = d;
    }
    return true;
}

__global__ void __launch_bounds__(kFPThreads) k_fp_count(FrameK f, uint32_t *row_count)
{
    __shared__ uint32_t wc[kFPWaves];
    const int y = blockIdx.x * f.stride, nx = (f.W + f.stride - 1) / f.stride;
    uint32_t c = 0;
    for (int u = threadIdx.x; u < nx; u += kFPThreads) {
        float p[3];
        c += fp_point(f, u * f.stride, y, p) ? 1u : 0u;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (__lane_id() == 0) wc[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kFPWaves; ++w) t += wc[w];
        row_count[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kFPThreads)
k_fp_emit(FrameK f, const uint32_t *row_count, int rows, float *xyz, int64_t capacity, int64_t *n_dev)
{
    __shared__ uint32_t wc[kFPWaves];
    __shared__ uint32_t base_s;
    const int tid = threadIdx.x, w = tid / kWave, lane = __lane_id();
    uint32_t before = 0;
    for (int r = tid; r < (int)blockIdx.x; r += kFPThreads) before += row_count[r];
    for (int o = kWave / 2; o > 0; o >>= 1) before += __shfl_xor(before, o);
    if (lane == 0) wc[w] = before;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int q = 0; q < kFPWaves; ++q) t += wc[q];
        base_s = t;
        if ((int)blockIdx.x == rows - 1 && n_dev) *n_dev = (int64_t)t + row_count[blockIdx.x];
    }
    __syncthreads();
    uint32_t run = base_s;
    const int y = blockIdx.x * f.stride, nx = (f.W + f.stride - 1) / f.stride;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int u0 = 0; u0 < nx; u0 += kFPThreads) {
        const int u = u0 + tid;
        float p[3];
        const bool ok = u < nx && fp_point(f, u * f.stride, y, p);
        const uint64_t b = __ballot(ok);
        __syncthreads();  // wc is free again
        if (lane == 0) wc[w] = (uint32_t)__popcll(b);
        __syncthreads();
        uint32_t pos = run, all = 0;
        for (int q = 0; q < kFPWaves; ++q) {
            pos += q < w ? wc[q] : 0u;
            all += wc[q];
        }
        pos += (uint32_t)__popcll(b & below);
        if (ok && (int64_t)pos < capacity) {
            xyz[pos] = p[0];
            xyz[capacity + pos] = p[1];
            xyz[2 * capacity + pos] = p[2];
        }
        run += all;
    }
}

// --------------------------------------- grid ---------------------------------------

__global__ void __launch_bounds__(kBoxThreads)
k_bbox_part(const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z, int64_t n,
            float *__restrict__ part)
{
    __shared__ float red[kBoxOut][kBoxThreads / kWave];
    // min x, y, z, max x, y, z, and the number of points with a non-finite coordinate (fminf and
    // fmaxf pass over NaN, so those are counted apart)
    float v[kBoxOut] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0f};
    for (int64_t i = (int64_t)blockIdx.x * kBoxThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBoxThreads) {
        const float a[3] = {x[i], y[i], z[i]};
        for (int c = 0; c < 3; ++c) {
            v[c] = fminf(v[c], a[c]);
            v[3 + c] = fmaxf(v[3 + c], a[c]);
        }
        v[6] += (isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2])) ? 0.0f : 1.0f;
    }
    for (int c = 0; c < kBoxOut; ++c) {
        float t = v[c];
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const float u = __shfl_xor(t, o);
            t = c < 3 ? fminf(t, u) : (c < 6 ? fmaxf(t, u) : t + u);
        }
        if (__lane_id() == 0) red[c][threadIdx.x / kWave] = t;
    }
    __syncthreads();
    if (threadIdx.x < kBoxOut) {
        const int c = threadIdx.x;
        float t = red[c][0];
        for (int w = 1; w < kBoxThreads / kWave; ++w)
            t = c < 3 ? fminf(t, red[c][w]) : (c < 6 ? fmaxf(t, red[c][w]) : t + red[c][w]);
        part[blockIdx.x * kBoxOut + c] = t;
    }
}

__global__ void k_bbox_final(const float *__restrict__ part, int nb, float *__restrict__ out)
{
    const int c = threadIdx.x;
    if (c >= kBoxOut) return;
    float t = part[c];
    for (int b = 1; b < nb; ++b) {
        const float u = part[b * kBoxOut + c];
        t = c < 3 ? fminf(t, u) : (c < 6 ? fmaxf(t, u) : t + u);
    }
    out[c] = t;
}

__device__ inline int cell_of(float v, float o, float inv_c) { return (int)floorf((v - o) * inv_c); }

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__global__ void k_cell_keys(GridK g, const float *__restrict__ x, const float *__restrict__ y,
                            const float *__restrict__ z, int64_t n, uint32_t *__restrict__ keys,
                            uint32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cx = clampi(cell_of(x[i], g.ox, g.inv_c), 0, g.gx - 1);
    const int cy = clampi(cell_of(y[i], g.oy, g.inv_c), 0, g.gy - 1);
    const int cz = clampi(cell_of(z[i], g.oz, g.inv_c), 0, g.gz - 1);
    keys[i] = ((uint32_t)cz * (uint32_t)g.gy + (uint32_t)cy) * (uint32_t)g.gx + (uint32_t)cx;
    vals[i] = (uint32_t)i;
}

__global__ void k_gather_cells(const uint32_t *__restrict__ vals, const float *__restrict__ x,
                               const float *__restrict__ y, const float *__restrict__ z, int64_t n,
                               float4 *__restrict__ pts)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t i = vals[r];
    pts[r] = make_float4(x[i], y[i], z[i], __uint_as_float(i));
}

// ------------------------------- neighbours, covariances -------------------------------

// Squared distance from p to the box of cell (X, Y, Z) widened by the grid's margin on every side:
// every point filed in that cell lies inside the widened box (its cell index carries at most that
// much rounding), so none of them is closer than this. The box bounds' own rounding stays far
// below the margin.
__device__ inline float cell_box_d2(const GridK &g, int X, int Y, int Z, const float p[3])
{
    const float m = g.margin * g.c;
    const float lo[3] = {g.ox + (float)X * g.c - m, g.oy + (float)Y * g.c - m, g.oz + (float)Z * g.c - m};
    float d2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float e = fmaxf(0.0f, fmaxf(lo[a] - p[a], p[a] - (lo[a] + g.c + 2.0f * m)));
        d2 += e * e;
    }
    return d2;
}

// A cell whose widened box is this far cannot hold a point at squared distance `best` or less
// (the 1e-5 absorbs the binary32 rounding of both distances).
__device__ inline bool cell_beyond(float box_d2, float best) { return box_d2 > best * (1.0f + 1e-5f); }

// (d, j) comes before (e, l)
__device__ inline bool ahead(float d, uint32_t j, float e, uint32_t l) { return d < e || (d == e && j < l); }

// Smallest-eigenvalue eigenvector of the symmetric matrix (a00, a01, a02, a11, a12, a22) by
// cyclic Jacobi sweeps: each rotation in the (p, q) plane zeroes a_pq, with tan of its angle the
// root of t^2 + 2 theta t - 1 = 0 of least magnitude, theta = (a_qq - a_pp) / (2 a_pq).
__device__ void smallest_eigvec(double m[3][3], double nrm[3])
{
    double v[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = m[0][1] * m[0][1] + m[0][2] * m[0][2] + m[1][2] * m[1][2];
        const double dg = m[0][0] * m[0][0] + m[1][1] * m[1][1] + m[2][2] * m[2][2];
        if (off == 0.0 || off <= 1e-32 * dg) break;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int p = k == 2 ? 1 : 0, q = k == 0 ? 1 : 2, o = 3 - p - q;
            const double apq = m[p][q];
            if (apq == 0.0) continue;
            const double theta = (m[q][q] - m[p][p]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            m[p][p] -= t * apq;
            m[q][q] += t * apq;
            m[p][q] = m[q][p] = 0.0;
            const double aop = m[o][p], aoq = m[o][q];
            m[o][p] = m[p][o] = c * aop - s * aoq;
            m[o][q] = m[q][o] = s * aop + c * aoq;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double vp = v[r][p], vq = v[r][q];
                v[r][p] = c * vp - s * vq;
                v[r][q] = s * vp + c * vq;
            }
        }
    }
    int lo = 0;
    if (m[1][1] < m[lo][lo]) lo = 1;
    if (m[2][2] < m[lo][lo]) lo = 2;
    for (int r = 0; r < 3; ++r) nrm[r] = lo == 0 ? v[r][0] : (lo == 1 ? v[r][1] : v[r][2]);
}

// Inserts (d2, j) into the list held sorted in bd/bi when it comes before the last entry.
__device__ __attribute__((always_inline)) inline void knn_insert(float (&bd)[kKMax], uint32_t (&bi)[kKMax], float d2,
                                                                 uint32_t j)
{
    if (!ahead(d2, j, bd[kKMax - 1], bi[kKMax - 1])) return;
    bool go = true;  // the candidate still moves towards the front
#pragma unroll
    for (int s = kKMax - 1; s >= 1; --s) {
        const bool sh = go && ahead(d2, j, bd[s - 1], bi[s - 1]);
        const float nd = sh ? bd[s - 1] : (go ? d2 : bd[s]);
        const uint32_t ni = sh ? bi[s - 1] : (go ? j : bi[s]);
        bd[s] = nd;
        bi[s] = ni;
        go = sh;
    }
    // ahead of every entry: the front slot (only reachable when no sentinel holds it, k = KMAX)
    if (go) {
        bd[0] = d2;
        bi[0] = j;
    }
}

__device__ __attribute__((always_inline)) inline void knn_reset(float (&bd)[kKMax], uint32_t (&bi)[kKMax], int k)
{
#pragma unroll
    for (int s = 0; s < kKMax; ++s) {
        const bool sentinel = s < kKMax - k;  // always ahead of a real entry
        bd[s] = sentinel ? -INFINITY : INFINITY;
        bi[s] = sentinel ? 0u : 0xffffffffu;
    }
}

__global__ void __launch_bounds__(kKnnThreads)
k_knn_cov(GridK g, const uint2 *__restrict__ ranges, const float4 *__restrict__ pts, int64_t n, int k, double eps,
          const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z,
          int32_t *__restrict__ knn_out, double *__restrict__ cov)
{
    const int64_t r = (int64_t)blockIdx.x * kKnnThreads + threadIdx.x;
    if (r >= n) return;
    const float4 q = pts[r];
    const uint32_t qi = __float_as_uint(q.w);
    float bd[kKMax];
    uint32_t bi[kKMax];
    knn_reset(bd, bi, k);
    const int cx = clampi(cell_of(q.x, g.ox, g.inv_c), 0, g.gx - 1);
    const int cy = clampi(cell_of(q.y, g.oy, g.inv_c), 0, g.gy - 1);
    const int cz = clampi(cell_of(q.z, g.oz, g.inv_c), 0, g.gz - 1);
    const int rmax = max(g.gx, max(g.gy, g.gz));
    const float qp[3] = {q.x, q.y, q.z};
    auto visit = [&](int X, int Y, int Z) {
        const uint2 rg = ranges[((int64_t)Z * g.gy + Y) * g.gx + X];
        for (uint32_t p = rg.x; p < rg.y; ++p) {
            const float4 c = pts[p];
            const float ex = c.x - q.x, ey = c.y - q.y, ez = c.z - q.z;
            knn_insert(bd, bi, (ex * ex + ey * ey) + ez * ez, __float_as_uint(c.w));
        }
    };
    // the point's own cell first, so that its neighbours prune the cells around it
    visit(cx, cy, cz);
    bool found = false;
    for (int ring = 1; ring <= kKnnRings; ++ring) {
        for (int dz = -ring; dz <= ring; ++dz) {
            const int Z = cz + dz;
            if (Z < 0 || Z >= g.gz) continue;
            for (int dy = -ring; dy <= ring; ++dy) {
                const int Y = cy + dy;
                if (Y < 0 || Y >= g.gy) continue;
                const bool inner = ring > 1 && abs(dz) < ring && abs(dy) < ring;
                // on an inner (y, z) line of a shell only its two end cells are new
                for (int dx = -ring; dx <= ring; dx += inner ? 2 * ring : 1) {
                    const int X = cx + dx;
                    if (X < 0 || X >= g.gx || (dx == 0 && dy == 0 && dz == 0)) continue;
                    if (cell_beyond(cell_box_d2(g, X, Y, Z, qp), bd[kKMax - 1])) continue;
                    visit(X, Y, Z);
                }
            }
        }
        const float lim = ((float)ring - g.margin) * g.c;
        if (bd[kKMax - 1] <= lim * lim || ring >= rmax) {
            found = true;
            break;
        }
    }
    if (!found) {
        // an isolated point: beyond kKnnRings rings a scan of every point bounds the work (the
        // rings would otherwise cross all the empty cells between it and its neighbours)
        knn_reset(bd, bi, k);
        for (int64_t p = 0; p < n; ++p) {
            const float4 c = pts[p];
            const float ex = c.x - q.x, ey = c.y - q.y, ez = c.z - q.z;
            knn_insert(bd, bi, (ex * ex + ey * ey) + ez * ez, __float_as_uint(c.w));
        }
    }
    // mean and covariance of the k neighbours, in their order
    double mu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kKMax; ++s) {
        if (s < kKMax - k) continue;
        const uint32_t j = bi[s];
        mu[0] += (double)x[j];
        mu[1] += (double)y[j];
        mu[2] += (double)z[j];
    }
    for (int c = 0; c < 3; ++c) mu[c] /= (double)k;
    double C[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
    for (int s = 0; s < kKMax; ++s) {
        if (s < kKMax - k) continue;
        const uint32_t j = bi[s];
        const double e0 = (double)x[j] - mu[0], e1 = (double)y[j] - mu[1], e2 = (double)z[j] - mu[2];
        C[0][0] += e0 * e0;
        C[0][1] += e0 * e1;
        C[0][2] += e0 * e2;
        C[1][1] += e1 * e1;
        C[1][2] += e1 * e2;
        C[2][2] += e2 * e2;
        if (knn_out) knn_out[(int64_t)qi * k + (s - (kKMax - k))] = (int32_t)j;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            C[a][b] /= (double)k;
            C[b][a] = C[a][b];
        }
    double nv[3];
    smallest_eigvec(C, nv);
    const double f = 1.0 - eps;
    cov[qi] = 1.0 - f * nv[0] * nv[0];
    cov[n + qi] = -f * nv[0] * nv[1];
    cov[2 * n + qi] = -f * nv[0] * nv[2];
    cov[3 * n + qi] = 1.0 - f * nv[1] * nv[1];
    cov[4 * n + qi] = -f * nv[1] * nv[2];
    cov[5 * n + qi] = 1.0 - f * nv[2] * nv[2];
}

// ------------------------------------ Gauss-Newton ------------------------------------

constexpr int kSums = 29;  // H upper triangle (21), b (6), cost, count

// (bd, bj) <- the first by (distance, index) over the kCorrLanes lanes of a query's group
__device__ inline void group_min(float &bd, uint32_t &bj)
{
#pragma unroll
    for (int o = kCorrLanes / 2; o > 0; o >>= 1) {
        const float od = __shfl_xor(bd, o, kCorrLanes);
        const uint32_t oj = __shfl_xor(bj, o, kCorrLanes);
        if (ahead(od, oj, bd, bj)) {
            bd = od;
            bj = oj;
        }
    }
}

__global__ void __launch_bounds__(kCorrThreads)
k_gicp_corr(GridK g, const uint2 *__restrict__ ranges, const float4 *__restrict__ tpts, const float *__restrict__ tx,
            const float *__restrict__ ty, const float *__restrict__ tz, const double *__restrict__ tcov, int64_t nt,
            const float *__restrict__ sx, const float *__restrict__ sy, const float *__restrict__ sz,
            const double *__restrict__ scov, int64_t ns, float dm2, int rings, const GicpState *st,
            double *__restrict__ partials, int32_t *__restrict__ corr)
{
    __shared__ double red[kCorrQueries][kSums + 1];
    if (st->done) return;
    const int tid = threadIdx.x, ql = tid / kCorrLanes, lane = tid % kCorrLanes;
    if (lane == 0)
        for (int k = 0; k < kSums; ++k) red[ql][k] = 0.0;
    // the workgroup's kCorrBatches batches of kCorrQueries source points, one point per group
    for (int batch = 0; batch < kCorrBatches; ++batch) {
        const int64_t i = ((int64_t)blockIdx.x * kCorrBatches + batch) * kCorrQueries + ql;
        float bd = INFINITY;
        uint32_t bj = 0xffffffffu;
        float p[3] = {0.0f, 0.0f, 0.0f};
        int cx = 0, cy = 0, cz = 0;
        auto scan_point = [&](const float4 q) {
            const uint32_t j = __float_as_uint(q.w);
            const float ex = q.x - p[0], ey = q.y - p[1], ez = q.z - p[2];
            const float d2 = (ex * ex + ey * ey) + ez * ez;
            if (d2 <= dm2 && ahead(d2, j, bd, bj)) {
                bd = d2;
                bj = j;
            }
        };
        if (i < ns) {
            const float x = sx[i], y = sy[i], z = sz[i];
            for (int r = 0; r < 3; ++r) {
                float w = st->R32[3 * r] * x;
                w = w + st->R32[3 * r + 1] * y;
                w = w + st->R32[3 * r + 2] * z;
                p[r] = w + st->t32[r];
            }
            cx = cell_of(p[0], g.ox, g.inv_c);
            cy = cell_of(p[1], g.oy, g.inv_c);
            cz = cell_of(p[2], g.oz, g.inv_c);
            // the query's own cell first, its points split over the group's lanes
            if (cx >= 0 && cx < g.gx && cy >= 0 && cy < g.gy && cz >= 0 && cz < g.gz) {
                const uint2 rg = ranges[((int64_t)cz * g.gy + cy) * g.gx + cx];
                for (uint32_t k = rg.x + lane; k < rg.y; k += kCorrLanes) scan_point(tpts[k]);
            }
        }
        group_min(bd, bj);
        if (i < ns) {
            // the other cells of the search block, skipping those that cannot beat the group's best
            const int side = 2 * rings + 1, cells = side * side * side, centre = (rings * side + rings) * side + rings;
            const float best = fminf(bd, dm2);
            for (int c = lane; c < cells; c += kCorrLanes) {
                if (c == centre) continue;
                const int X = cx + c % side - rings, Y = cy + (c / side) % side - rings, Z = cz + c / (side * side) - rings;
                if (X < 0 || X >= g.gx || Y < 0 || Y >= g.gy || Z < 0 || Z >= g.gz) continue;
                if (cell_beyond(cell_box_d2(g, X, Y, Z, p), best)) continue;
                const uint2 rg = ranges[((int64_t)Z * g.gy + Y) * g.gx + X];
                for (uint32_t k = rg.x; k < rg.y; ++k) scan_point(tpts[k]);
            }
        }
        group_min(bd, bj);
        if (lane == 0) {
            double v[kSums];
            for (int k = 0; k < kSums; ++k) v[k] = 0.0;
            if (i < ns && corr) corr[i] = bj == 0xffffffffu ? -1 : (int32_t)bj;
            if (i < ns && bj != 0xffffffffu) {
                const double *R = st->R, *t = st->t;
                const double p0 = sx[i], p1 = sy[i], p2 = sz[i];
                double Tp[3], d[3];
                for (int r = 0; r < 3; ++r) Tp[r] = R[3 * r] * p0 + R[3 * r + 1] * p1 + R[3 * r + 2] * p2 + t[r];
                d[0] = (double)tx[bj] - Tp[0];
                d[1] = (double)ty[bj] - Tp[1];
                d[2] = (double)tz[bj] - Tp[2];
                // C = C_q + R C_p R^T (Eq. 13)
                const double cp[6] = {scov[i], scov[ns + i], scov[2 * ns + i], scov[3 * ns + i], scov[4 * ns + i],
                                      scov[5 * ns + i]};
                const double Cp[3][3] = {{cp[0], cp[1], cp[2]}, {cp[1], cp[3], cp[4]}, {cp[2], cp[4], cp[5]}};
                double M[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double s = 0.0;
                        for (int u = 0; u < 3; ++u) {
                            double rc = 0.0;
                            for (int w = 0; w < 3; ++w) rc += R[3 * a + w] * Cp[w][u];
                            s += rc * R[3 * b + u];
                        }
                        M[a][b] = s;
                    }
                M[0][0] += tcov[bj];
                M[0][1] += tcov[nt + bj];
                M[0][2] += tcov[2 * nt + bj];
                M[1][0] += tcov[nt + bj];
                M[1][1] += tcov[3 * nt + bj];
                M[1][2] += tcov[4 * nt + bj];
                M[2][0] += tcov[2 * nt + bj];
                M[2][1] += tcov[4 * nt + bj];
                M[2][2] += tcov[5 * nt + bj];
                // W = M^-1 from the cofactors (M is symmetric positive definite)
                const double k00 = M[1][1] * M[2][2] - M[1][2] * M[2][1], k01 = M[0][2] * M[2][1] - M[0][1] * M[2][2],
                             k02 = M[0][1] * M[1][2] - M[0][2] * M[1][1], k11 = M[0][0] * M[2][2] - M[0][2] * M[2][0],
                             k12 = M[0][2] * M[1][0] - M[0][0] * M[1][2], k22 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
                const double det = M[0][0] * k00 + M[1][0] * k01 + M[2][0] * k02;
                if (det != 0.0 && isfinite(det)) {
                    const double id = 1.0 / det;
                    const double W[3][3] = {{k00 * id, k01 * id, k02 * id},
                                            {k01 * id, k11 * id, k12 * id},
                                            {k02 * id, k12 * id, k22 * id}};
                    // J = [[Tp]_x, -I]
                    const double J[3][6] = {{0.0, -Tp[2], Tp[1], -1.0, 0.0, 0.0},
                                            {Tp[2], 0.0, -Tp[0], 0.0, -1.0, 0.0},
                                            {-Tp[1], Tp[0], 0.0, 0.0, 0.0, -1.0}};
                    double WJ[3][6], Wd[3];
                    for (int r = 0; r < 3; ++r) {
                        Wd[r] = W[r][0] * d[0] + W[r][1] * d[1] + W[r][2] * d[2];
                        for (int c = 0; c < 6; ++c) WJ[r][c] = W[r][0] * J[0][c] + W[r][1] * J[1][c] + W[r][2] * J[2][c];
                    }
                    int h = 0;
                    for (int a = 0; a < 6; ++a)
                        for (int b = a; b < 6; ++b) v[h++] = J[0][a] * WJ[0][b] + J[1][a] * WJ[1][b] + J[2][a] * WJ[2][b];
                    for (int a = 0; a < 6; ++a) v[21 + a] = J[0][a] * Wd[0] + J[1][a] * Wd[1] + J[2][a] * Wd[2];
                    v[27] = d[0] * Wd[0] + d[1] * Wd[1] + d[2] * Wd[2];
                    v[28] = 1.0;
                }
            }
            for (int k = 0; k < kSums; ++k) red[ql][k] += v[k];
        }
    }
    __syncthreads();
    if (tid < kSums) {
        double s = 0.0;
        for (int q = 0; q < kCorrQueries; ++q) s += red[q][tid];
        partials[(int64_t)blockIdx.x * kSums + tid] = s;
    }
}

// Rotation Exp(w) = I + A [w]_x + B [w]_x^2, A = sin(th) / th, B = (1 - cos(th)) / th^2.
__device__ void rot_exp(const double w[3], double E[3][3])
{
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = sqrt(th2);
    double A, B;
    if (th < 1e-5) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
    }
    const double K[3][3] = {{0.0, -w[2], w[1]}, {w[2], 0.0, -w[0]}, {-w[1], w[0], 0.0}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            const double K2 = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
            E[r][c] = (r == c ? 1.0 : 0.0) + A * K[r][c] + B * K2;
        }
}

__global__ void __launch_bounds__(1024)
k_gicp_solve(const double *__restrict__ partials, int nb, GicpState *st, int update, int max_iter, double eps_rot,
             double eps_trans, double *__restrict__ out)
{
    __shared__ double part[kSums][32];
    __shared__ double tot[kSums];
    if (st->done) return;
    const int tid = threadIdx.x;
    if (tid < kSums * 32) {
        const int v = tid / 32, s = tid % 32;
        // four loads in flight per step (the partials come from every XCD, so each is a trip to
        // memory); the order of the sums is fixed
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int b = s;
        for (; b + 96 < nb; b += 128) {
            a0 += partials[(int64_t)b * kSums + v];
            a1 += partials[(int64_t)(b + 32) * kSums + v];
            a2 += partials[(int64_t)(b + 64) * kSums + v];
            a3 += partials[(int64_t)(b + 96) * kSums + v];
        }
        for (; b < nb; b += 32) a0 += partials[(int64_t)b * kSums + v];
        part[v][s] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    if (tid < kSums) {
        double a = 0.0;
        for (int s = 0; s < 32; ++s) a += part[tid][s];
        tot[tid] = a;
        if (out) out[tid] = a;
    }
    __syncthreads();
    if (!update || tid != 0) return;
    st->cost = tot[27];
    st->count = (int64_t)tot[28];
    // Cholesky H = L L^T, then L y = -b, L^T x = y; fully unrolled so that H and L stay in
    // registers (indexed at run time they would live in scratch memory)
    double H[6][6], L[6][6], x[6], yv[6];
#pragma unroll
    for (int a = 0, h = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b, ++h) H[a][b] = H[b][a] = tot[h];
    bool ok = st->count >= 6;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            double v = H[a][b];
#pragma unroll
            for (int c = 0; c < b; ++c) v -= L[a][c] * L[b][c];
            if (a == b) {
                ok = ok && v > 0.0;
                L[a][a] = sqrt(ok ? v : 1.0);
            } else {
                L[a][b] = v / L[b][b];
            }
        }
    if (!ok) {
        st->status = 2;
        st->done = 1;
        return;
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double v = -tot[21 + a];
#pragma unroll
        for (int c = 0; c < a; ++c) v -= L[a][c] * yv[c];
        yv[a] = v / L[a][a];
    }
#pragma unroll
    for (int a = 5; a >= 0; --a) {
        double v = yv[a];
#pragma unroll
        for (int c = a + 1; c < 6; ++c) v -= L[c][a] * x[c];
        x[a] = v / L[a][a];
    }
    double E[3][3];
    rot_exp(x, E);
    double Rn[9], tn[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) Rn[3 * r + c] = E[r][0] * st->R[c] + E[r][1] * st->R[3 + c] + E[r][2] * st->R[6 + c];
        tn[r] = E[r][0] * st->t[0] + E[r][1] * st->t[1] + E[r][2] * st->t[2] + x[3 + r];
    }
    for (int q = 0; q < 9; ++q) {
        st->R[q] = Rn[q];
        st->R32[q] = (float)Rn[q];
    }
    for (int q = 0; q < 3; ++q) {
        st->t[q] = tn[q];
        st->t32[q] = (float)tn[q];
    }
    st->iters += 1;
    const double nw = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]), nv = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
    if (nw < eps_rot && nv < eps_trans) {
        st->status = 0;
        st->done = 1;
    } else if (st->iters >= max_iter) {
        st->status = 1;
        st->done = 1;
    }
}

__global__ void k_gicp_init(GicpState *st, PoseK p)
{
    if (threadIdx.x != 0) return;
    for (int q = 0; q < 9; ++q) {
        st->R[q] = p.R[q];
        st->R32[q] = (float)p.R[q];
    }
    for (int q = 0; q < 3; ++q) {
        st->t[q] = p.t[q];
        st->t32[q] = (float)p.t[q];
    }
    st->done = 0;
    st->iters = 0;
    st->status = 1;
    st->pad = 0;
    st->count = 0;
    st->cost = 0.0;
}

}  // namespace

void launch_gicp_init(GicpState *st, const double R[9], const double t[3], hipStream_t s)
{
    PoseK p;
    for (int q = 0; q < 9; ++q) p.R[q] = R[q];
    for (int q = 0; q < 3; ++q) p.t[q] = t[q];
    hipLaunchKernelGGL(k_gicp_init, dim3(1), dim3(64), 0, s, st, p);
}

void launch_frame_points(const FrameK &f, uint32_t *row_count, float *xyz, int64_t capacity, int64_t *n_dev,
                         hipStream_t s)
{
    const int rows = (f.H + f.stride - 1) / f.stride;
    hipLaunchKernelGGL(k_fp_count, dim3(rows), dim3(kFPThreads), 0, s, f, row_count);
    hipLaunchKernelGGL(k_fp_emit, dim3(rows), dim3(kFPThreads), 0, s, f, row_count, rows, xyz, capacity, n_dev);
}

int bbox_partials() { return kBoxBlocks * kBoxOut; }

void launch_bbox(const float *x, const float *y, const float *z, int64_t n, float *part, float *out, hipStream_t s)
{
    const int64_t want = (n + kBoxThreads - 1) / kBoxThreads;
    const int nb = want < 1 ? 1 : (want > kBoxBlocks ? kBoxBlocks : (int)want);
    hipLaunchKernelGGL(k_bbox_part, dim3(nb), dim3(kBoxThreads), 0, s, x, y, z, n, part);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, s, part, nb, out);
}

void launch_cell_keys(const GridK &g, const float *x, const float *y, const float *z, int64_t n, uint32_t *keys,
                      uint32_t *vals, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_cell_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, x, y, z, n, keys, vals);
}

void launch_gather_cells(const uint32_t *vals, const float *x, const float *y, const float *z, int64_t n, float4 *pts,
                         hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_cells, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vals, x, y, z, n, pts);
}

void launch_knn_cov(const GridK &g, const uint2 *ranges, const float4 *pts, int64_t n, int k, double eps,
                    const float *x, const float *y, const float *z, int32_t *knn_out, double *cov, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_knn_cov, dim3((unsigned)((n + kKnnThreads - 1) / kKnnThreads)), dim3(kKnnThreads), 0, s, g,
                       ranges, pts, n, k, eps, x, y, z, knn_out, cov);
}

int64_t gicp_partials(int64_t ns)
{
    return (ns + kCorrQueries * kCorrBatches - 1) / (kCorrQueries * kCorrBatches);
}

void launch_gicp_iteration(const GicpK &k, GicpState *st, double *partials, int32_t *corr, int update, int max_iter,
                           double eps_rot, double eps_trans, double *out, hipStream_t s)
{
    const int64_t nb = gicp_partials(k.ns);
    if (nb > 0)
        hipLaunchKernelGGL(k_gicp_corr, dim3((unsigned)nb), dim3(kCorrThreads), 0, s, k.g, k.ranges, k.tpts, k.tx,
                           k.ty, k.tz, k.tcov, k.nt, k.sx, k.sy, k.sz, k.scov, k.ns, k.dm2, k.rings, st, partials,
                           corr);
    hipLaunchKernelGGL(k_gicp_solve, dim3(1), dim3(1024), 0, s, partials, (int)nb, st, update, max_iter, eps_rot,
                       eps_trans, out);
}

}  // namespace fgs
