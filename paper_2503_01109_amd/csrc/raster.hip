// Tile rasterizer: front-to-back alpha blending of Eq. 1 (colour, depth and opacity) and its
// backward.
//
// One workgroup per screen tile, one pixel per thread. The tile's list (depth-ordered ranks of
// the gaussians whose 3-sigma box touches the tile) is walked in batches; each batch of records
// is gathered from HBM once by the whole workgroup, converted to tile-local coordinates and
// staged in LDS, then every pixel reads the records as LDS broadcasts. A pixel applies the exact
// per-pixel cutoffs (Mahalanobis distance <= sigma_cut, alpha >= alpha_min, stop before T drops
// below T_min); the workgroup leaves the list as soon as a barrier count shows every pixel done.
//
// The backward walks the same list in reverse from the last blended position of the tile,
// recovering T_i = T_{i+1}/(1 - alpha_i). Each pair yields 10 gradient terms; they are summed
// over the wave with DPP row operations, over the workgroup's waves with LDS float atomics, and
// reach HBM as one FP32 atomic per (tile, gaussian, term).
//
// The forward and the backward evaluate the cutoff decisions with the same inline functions in
// this translation unit, compiled without floating-point contraction, so both take identical
// decisions for every pair.
#include "fgs_internal.h"

namespace fgs {

namespace {

struct Pair {
    float dx, dy, Q;
};

__device__ __forceinline__ float quad_form(float ca, float cb, float cc, float dx, float dy)
{
    // Q = ca dx^2 + 2 cb dx dy + cc dy^2, fixed operation order
    const float t0 = ca * dx * dx;
    const float t1 = 2.0f * cb * dx * dy;
    const float t2 = cc * dy * dy;
    return (t0 + t1) + t2;
}

__device__ __forceinline__ void stage(const Rec &R, int x0, int y0, float4 &a, float4 &b, float4 &c)
{
    // projected mean in tile-local coordinates: integer part is exact, one rounding for the sum
    const float mx = (float)(__float_as_int(R.r0.x) - x0) + R.r0.z;
    const float my = (float)(__float_as_int(R.r0.y) - y0) + R.r0.w;
    a = make_float4(mx, my, R.r1.x, R.r1.y);          // mean2 (local), conic a, conic b
    b = make_float4(R.r1.z, R.r1.w, R.r2.w, 0.0f);    // conic c, opacity, depth
    c = make_float4(R.r2.x, R.r2.y, R.r2.z, 0.0f);    // rgb
}

// Minimum of the quadratic form Q(p - m) = a dx^2 + 2 b dx dy + c dy^2 over the rectangle
// [x0, x1] x [y0, y1] (tile-local). Q is convex, so the minimum is 0 with the centre inside,
// else on one of the four edges, where it is a 1D quadratic minimised by clamping its vertex.
__device__ __forceinline__ float rect_min_q(float a, float b, float c, float ia, float ic, float mx, float my,
                                            float x0, float x1, float y0, float y1)
{
    // ia = 1/a, ic = 1/c (precomputed by the caller)
    const float dx0 = x0 - mx, dx1 = x1 - mx, dy0 = y0 - my, dy1 = y1 - my;
    if (dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f) return 0.0f;
    float best = INFINITY;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dx = e ? dx1 : dx0;
        const float dy = fminf(fmaxf(-b * dx * ic, dy0), dy1);
        best = fminf(best, a * dx * dx + 2.0f * b * dx * dy + c * dy * dy);
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dy = e ? dy1 : dy0;
        const float dx = fminf(fmaxf(-b * dy * ia, dx0), dx1);
        best = fminf(best, a * dx * dx + 2.0f * b * dx * dy + c * dy * dy);
    }
    return best;
}

// Bit w set when the sigma_cut ellipse of a staged record can reach a pixel centre of wave w's
// strip (rows [w R, w R + R) of the tile, R = 64 / TW). Conservative by a relative 1e-3 margin:
// the per-pixel test stays the exact decision.
// Bit w set when the sigma_cut ellipse of a staged record can reach a pixel centre of wave w's
// strip (rows [w R, w R + R) of the tile, R = 64 / tw). Conservative by a relative 1e-3 margin:
// the per-pixel test stays the exact decision.
template <int NW>
__device__ __forceinline__ uint32_t strip_mask(const float4 &a4, const float4 &b4, float cut2, int tw)
{
    const int R = kWave / tw;
    uint32_t m = 0;
    const float ia = __frcp_rn(a4.z), ic = __frcp_rn(b4.x);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const float q = rect_min_q(a4.z, a4.w, b4.x, ia, ic, a4.x, a4.y, 0.5f, tw - 0.5f, w * R + 0.5f,
                                   w * R + R - 0.5f);
        if (q <= cut2 * 1.001f) m |= 1u << w;
    }
    return m;
}

// Compacts the indices k < cnt whose mask has this wave's bit into this wave's list (ascending);
// returns the list length. Wave-local: no block barrier needed.
__device__ __forceinline__ int wave_compact(const uint8_t *smask, int cnt, int wid, uint16_t *list)
{
    const int lane = __lane_id();
    int len = 0;
    for (int q = 0; q < cnt; q += kWave) {
        const int e = q + lane;
        const bool bit = e < cnt && ((smask[e] >> wid) & 1u);
        const uint64_t bal = __ballot(bit);
        if (bit) list[len + __popcll(bal & ((1ull << lane) - 1ull))] = (uint16_t)e;
        len += __popcll(bal);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return len;
}

// DPP: v + (v moved by ctrl) in the rows enabled by row_mask, v elsewhere.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v)
{
    const int t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false);
    return v + __int_as_float(t);
}

// Ten wave sums at once by a transposed butterfly: at each exchange a lane keeps half of its
// partial sums (the half its partner does not keep) and adds the partner's matching half, so
// 10 values shrink to 5, 3, 2 and 1 per lane over lane distances 1, 2, 4 and 8; two more
// exchanges add the four rows. Lane j (j < 16; every row holds the same) returns the full sum of
// term reduce_term(j), or of nothing when that is negative (padding). About 40 VALU operations
// instead of 10 separate 6-step wave sums.
__device__ __forceinline__ float reduce10(const float v[10], int lane)
{
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8;
    float a[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const float send = b0 ? v[c] : v[c + 5], mine = b0 ? v[c + 5] : v[c];
        a[c] = mine + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0xB1, 0xf, 0xf, false));
    }
    float q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float hi = c < 2 ? a[c + 3] : 0.0f, lo = a[c];
        const float send = b1 ? lo : hi, mine = b1 ? hi : lo;
        q[c] = mine + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0x4E, 0xf, 0xf, false));
    }
    float r[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const float hi = c < 1 ? q[c + 2] : 0.0f, lo = q[c];
        const float send = b2 ? lo : hi, mine = b2 ? hi : lo;
        r[c] = mine + __shfl_xor(send, 4);
    }
    const float send = b3 ? r[0] : r[1], mine = b3 ? r[1] : r[0];
    float d = mine + __shfl_xor(send, 8);
    d += __shfl_xor(d, 16);
    d += __shfl_xor(d, 32);
    return d;
}

// The term whose sum reduce10 leaves in lane j of a row (-1: padding).
__device__ __forceinline__ int reduce_term(int lane)
{
    const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
    const int i3 = b2 ? 2 + b3 : b3;  // index among the 3 values of the third exchange
    if (i3 > 2) return -1;
    const int i5 = b1 ? 3 + i3 : i3;  // among the 5 values of the second
    if (i5 > 4) return -1;
    return b0 ? 5 + i5 : i5;
}

// Sum over the 64 lanes; the total is valid in lanes 48..63.
__device__ __forceinline__ float wave_sum(float v)
{
    v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);  // row_mirror: every lane holds its row's sum
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Forward of one tile of one view by a workgroup of NT threads (one pixel each; the tile is
// tile_w x tile_h = NT pixels).
template <int NT>
__device__ void tile_fwd(const ViewK &V, int tile)
{
    constexpr int NW = NT / kWave;
    __shared__ float4 sa[NT], sb[NT], sc[NT];
    __shared__ uint8_t smask[NT];
    __shared__ uint16_t slist[NW][NT];
    __shared__ unsigned long long red[2];
    const RasterK &rk = V.rk;
    const int W = V.W, H = V.H;
    const Rec *__restrict__ rec = V.rec;
    const uint32_t *__restrict__ vals = V.vals;
    const int TW = rk.tile_w, TH = rk.tile_h;
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    const int tx = tile % rk.tiles_x, ty = tile / rk.tiles_x;
    const int x0 = tx * TW, y0 = ty * TH;
    const int lx = tid % TW, ly = tid / TW;
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < W && y < H;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint2 range = V.ranges[tile];
    const float cut2 = rk.sigma_cut * rk.sigma_cut;

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f, A = 0.0f;
    uint32_t last = 0, ntest = 0, staged = 0;
    int32_t ncon = 0;
    bool done = !inside;

    for (uint32_t b = range.x; b < range.y; b += NT) {
        if (__syncthreads_count(!done) == 0) break;
        staged += min((uint32_t)NT, range.y - b);
        const uint32_t j = b + tid;
        if (j < range.y) {
            float4 a4, b4, c4;
            stage(rec[vals[j]], x0, y0, a4, b4, c4);
            sa[tid] = a4;
            sb[tid] = b4;
            sc[tid] = c4;
            smask[tid] = (uint8_t)strip_mask<NW>(a4, b4, cut2, TW);
        }
        __syncthreads();
        const int cnt = min((uint32_t)NT, range.y - b);
        const int len = wave_compact(smask, cnt, wid, slist[wid]);
        // Branch-free per pair: every lane evaluates the entry and the decisions select what is
        // kept (the arithmetic of a kept pair is the same as with branches); the wave leaves the
        // list once all of its pixels are done.
        for (int i = 0; i < len; ++i) {
            if (__ballot(!done) == 0) break;
            const int k = slist[wid][i];
            const float4 a4 = sa[k];
            const float dx = px - a4.x, dy = py - a4.y;
            const float4 b4 = sb[k];
            const float Q = quad_form(a4.z, a4.w, b4.x, dx, dy);
            const bool near = !done && !(Q > cut2);
            const float G = __expf(-0.5f * Q);
            const float alpha = fminf(rk.alpha_max, b4.y * G);
            const float Tn = T * (1.0f - alpha);
            const bool take = near && !(alpha < rk.alpha_min);
            const bool stop = take && Tn < rk.T_min;
            const bool blend = take && !stop;
            const float w = blend ? alpha * T : 0.0f;
            const float4 c4 = sc[k];
            C0 += w * c4.x;
            C1 += w * c4.y;
            C2 += w * c4.z;
            D += w * b4.z;
            A += w;
            T = blend ? Tn : T;
            done = done || stop;
            ntest += near ? 1u : 0u;
            ncon += blend ? 1 : 0;
            last = blend ? b + k - range.x + 1 : last;
        }
    }
    if (V.counts) {
        // work counters (profiling only): block sums, one atomic per block and counter
        if (tid == 0) red[0] = red[1] = 0ull;
        __syncthreads();
        if (inside) {
            atomicAdd(&red[0], (unsigned long long)ntest);
            atomicAdd(&red[1], (unsigned long long)ncon);
        }
        __syncthreads();
        if (tid == 0) {
            atomicAdd(&V.counts[0], red[0]);
            atomicAdd(&V.counts[1], red[1]);
            atomicAdd(&V.counts[2], (unsigned long long)staged);
        }
    }
    // the next tile of a persistent workgroup restages the LDS arrays: wait for every reader
    __syncthreads();
    if (!inside) return;
    const int64_t P = (int64_t)W * H;
    const int64_t p = (int64_t)y * W + x;
    const ImageK &img = V.img;
    img.rgb[p] = C0 + T * rk.bg[0];
    img.rgb[P + p] = C1 + T * rk.bg[1];
    img.rgb[2 * P + p] = C2 + T * rk.bg[2];
    img.depth[p] = D + T * rk.bg_depth;
    if (img.alpha) img.alpha[p] = A;
    if (img.T_final) img.T_final[p] = T;
    if (img.n_contrib) img.n_contrib[p] = ncon;
    V.last[p] = last;
    V.tfinal[p] = T;
}

// Backward of one tile of one view (NT threads, one pixel each).
template <int NT>
__device__ void tile_bwd(const ViewK &V, int tile)
{
    constexpr int NW = NT / kWave;
    const RasterK &rk = V.rk;
    const int W = V.W, H = V.H;
    const Rec *__restrict__ rec = V.rec;
    const uint32_t *__restrict__ vals = V.vals;
    const uint32_t *__restrict__ ids = V.ids;
    float *__restrict__ grad2d = V.grad2d;
    const int64_t n = V.n;
    const int TW = rk.tile_w, TH = rk.tile_h;
    __shared__ float4 sa[NT], sb[NT], sc[NT];
    __shared__ uint32_t srank[NT];
    __shared__ float sacc[10][NT + 1];  // padded: the ten terms of one entry fall in different banks
    __shared__ uint32_t smax;
    __shared__ uint8_t smask[NT];
    __shared__ uint16_t slist[NW][NT];
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wid = tid / kWave;
    const int tx = tile % rk.tiles_x, ty = tile / rk.tiles_x;
    const int x0 = tx * TW, y0 = ty * TH;
    const int lx = tid % TW, ly = tid / TW;
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < W && y < H;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint2 range = V.ranges[tile];
    const float cut2 = rk.sigma_cut * rk.sigma_cut;
    const int64_t P = (int64_t)W * H;
    const int64_t p = (int64_t)y * W + x;

    uint32_t L = 0;
    float T = 1.0f, gC0 = 0, gC1 = 0, gC2 = 0, gD = 0, gA = 0;
    if (inside) {
        L = V.last[p];
        T = V.tfinal[p];
        gC0 = V.drgb[p];
        gC1 = V.drgb[P + p];
        gC2 = V.drgb[2 * P + p];
        gD = V.ddepth[p] * (V.ddepth_scale ? *V.ddepth_scale : 1.0f);
        gA = V.dalpha ? V.dalpha[p] : 0.0f;
    }
    const float Tf = T;
    float BC0 = Tf * rk.bg[0], BC1 = Tf * rk.bg[1], BC2 = Tf * rk.bg[2], BD = Tf * rk.bg_depth;

    if (tid == 0) smax = 0;
#pragma unroll
    for (int c = 0; c < 10; ++c) sacc[c][tid] = 0.0f;
    __syncthreads();
    if (L) atomicMax(&smax, L);
    __syncthreads();
    const uint32_t hi = min(range.x + smax, range.y);

    for (uint32_t bend = hi; bend > range.x; bend -= min((uint32_t)NT, bend - range.x)) {
        const uint32_t bstart = bend - min((uint32_t)NT, bend - range.x);
        const int cnt = (int)(bend - bstart);
        __syncthreads();
        if (tid < cnt) {
            const uint32_t r = vals[bstart + tid];
            float4 a4, b4, c4;
            stage(rec[r], x0, y0, a4, b4, c4);
            sa[tid] = a4;
            sb[tid] = b4;
            sc[tid] = c4;
            srank[tid] = ids[r];  // gradients are accumulated by gaussian id
            smask[tid] = (uint8_t)strip_mask<NW>(a4, b4, cut2, TW);
        }
        __syncthreads();
        const int len = wave_compact(smask, cnt, wid, slist[wid]);
        for (int i = len - 1; i >= 0; --i) {
            const int k = slist[wid][i];
            const uint32_t pos = bstart + k - range.x;  // list position of entry k
            float g[10];
            bool contrib = false;
            if (pos < L) {
                const float4 a4 = sa[k];
                const float dx = px - a4.x, dy = py - a4.y;
                const float4 b4 = sb[k];
                const float Q = quad_form(a4.z, a4.w, b4.x, dx, dy);
                if (!(Q > cut2)) {
                    const float G = __expf(-0.5f * Q);
                    const float ar = b4.y * G;
                    const float alpha = fminf(rk.alpha_max, ar);
                    if (!(alpha < rk.alpha_min)) {
                        contrib = true;
                        const float4 c4 = sc[k];
                        const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);  // 1 ulp; alpha <= alpha_max < 1
                        const float Ti = T * inv;
                        const float w = alpha * Ti;
                        const float dal = Ti * (gC0 * c4.x + gC1 * c4.y + gC2 * c4.z + gD * b4.z) -
                                          (gC0 * BC0 + gC1 * BC1 + gC2 * BC2 + gD * BD - gA * Tf) * inv;
                        g[6] = gC0 * w;
                        g[7] = gC1 * w;
                        g[8] = gC2 * w;
                        g[9] = gD * w;
                        if (ar > rk.alpha_max) {
                            g[0] = g[1] = g[2] = g[3] = g[4] = g[5] = 0.0f;
                        } else {
                            g[5] = dal * G;
                            const float dQ = -0.5f * alpha * dal;
                            g[0] = -2.0f * dQ * (a4.z * dx + a4.w * dy);
                            g[1] = -2.0f * dQ * (a4.w * dx + b4.x * dy);
                            g[2] = dQ * dx * dx;
                            g[3] = 2.0f * dQ * dx * dy;
                            g[4] = dQ * dy * dy;
                        }
                        BC0 += w * c4.x;
                        BC1 += w * c4.y;
                        BC2 += w * c4.z;
                        BD += w * b4.z;
                        T = Ti;
                    }
                }
            }
            if (!contrib) {
#pragma unroll
                for (int c = 0; c < 10; ++c) g[c] = 0.0f;
            }
            const uint64_t any = __ballot(contrib);
            if (any) {
                if ((any & (any - 1)) == 0) {
                    // a single contributing lane: no reduction needed
                    if (contrib) {
#pragma unroll
                        for (int c = 0; c < 10; ++c) atomicAdd(&sacc[c][k], g[c]);
                    }
                } else {
                    // transposed reduction: lane j of the first row ends with the wave sum of term
                    // reduce_term(j); one LDS atomic instruction adds all ten terms
                    const float t = reduce10(g, lane);
                    const int term = reduce_term(lane);
                    if (lane < 16 && term >= 0) atomicAdd(&sacc[term][k], t);
                }
            }
        }
        __syncthreads();
        if (tid < cnt) {
            const uint32_t r = srank[tid];
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                const float v = sacc[c][tid];
                if (v != 0.0f) {
                    unsafeAtomicAdd(&grad2d[c * n + r], v);
                    sacc[c][tid] = 0.0f;
                }
            }
        }
    }
    __syncthreads();  // LDS is restaged by the next tile of a persistent workgroup
}

template <int NT>
__global__ void __launch_bounds__(NT) k_raster_fwd(ViewK V) { tile_fwd<NT>(V, blockIdx.x); }

template <int NT>
__global__ void __launch_bounds__(NT) k_raster_bwd(ViewK V) { tile_bwd<NT>(V, blockIdx.x); }

__device__ inline int view_of(const ViewK *views, int nv, uint32_t g)
{
    int v = 0;
    while (v + 1 < nv && views[v + 1].tile_base <= g) ++v;
    return v;
}

// Persistent rasterizer over a window of views: workgroups pull (view, tile) items from a queue
// through an atomic counter until it runs past the last item. 256 threads per workgroup; each
// view's tile has 256 pixels in its own shape (16x16, 32x8 or 8x32).
template <bool FWD>
__global__ void __launch_bounds__(256)
k_raster_queue(const ViewK *__restrict__ views, int nv, const uint32_t *__restrict__ queue, uint32_t total,
               uint32_t *__restrict__ counter)
{
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t q = s_item;
        __syncthreads();
        if (q >= total) break;
        const uint32_t g = queue ? queue[q] : q;
        const int v = view_of(views, nv, g);
        const ViewK &V = views[v];
        if (FWD) tile_fwd<256>(V, (int)(g - V.tile_base));
        else tile_bwd<256>(V, (int)(g - V.tile_base));
    }
}

}  // namespace

bool tile_supported(int tw, int th)
{
    return (tw == 16 && th == 16) || (tw == 32 && th == 8) || (tw == 8 && th == 32) || (tw == 32 && th == 16) ||
           (tw == 16 && th == 32) || (tw == 8 && th == 8);
}

bool tile_supported_window(int tw, int th) { return tw * th == 256 && (tw == 16 || tw == 32 || tw == 8); }

static ViewK view_of_args(const RasterK &rk, int32_t W, int32_t H, const Rec *rec, const uint32_t *vals)
{
    ViewK V = {};
    V.rk = rk;
    V.W = W;
    V.H = H;
    V.rec = rec;
    V.vals = vals;
    return V;
}

static void launch_fwd_view(const ViewK &V, hipStream_t s)
{
    const unsigned tiles = (unsigned)(V.rk.tiles_x * V.rk.tiles_y);
    const int nt = V.rk.tile_w * V.rk.tile_h;
    if (nt == 256) hipLaunchKernelGGL(k_raster_fwd<256>, dim3(tiles), dim3(256), 0, s, V);
    else if (nt == 512) hipLaunchKernelGGL(k_raster_fwd<512>, dim3(tiles), dim3(512), 0, s, V);
    else hipLaunchKernelGGL(k_raster_fwd<64>, dim3(tiles), dim3(64), 0, s, V);
}

static void launch_bwd_view(const ViewK &V, hipStream_t s)
{
    const unsigned tiles = (unsigned)(V.rk.tiles_x * V.rk.tiles_y);
    const int nt = V.rk.tile_w * V.rk.tile_h;
    if (nt == 256) hipLaunchKernelGGL(k_raster_bwd<256>, dim3(tiles), dim3(256), 0, s, V);
    else if (nt == 512) hipLaunchKernelGGL(k_raster_bwd<512>, dim3(tiles), dim3(512), 0, s, V);
    else hipLaunchKernelGGL(k_raster_bwd<64>, dim3(tiles), dim3(64), 0, s, V);
}

void launch_raster_fwd(const RasterK &rk, int32_t W, int32_t H, const Rec *rec, const uint32_t *vals,
                       const uint2 *ranges, uint32_t *last, float *tfinal, const ImageK &img,
                       unsigned long long *counts, hipStream_t s)
{
    ViewK V = view_of_args(rk, W, H, rec, vals);
    V.ranges = ranges;
    V.last = last;
    V.tfinal = tfinal;
    V.img = img;
    V.counts = counts;
    launch_fwd_view(V, s);
}

void launch_raster_bwd(const RasterK &rk, int32_t W, int32_t H, const Rec *rec, const uint32_t *vals,
                       const uint32_t *ids, const uint2 *ranges, const uint32_t *last, const float *tfinal,
                       const float *drgb, const float *ddepth, const float *dalpha, const float *ddepth_scale,
                       float *grad2d, int64_t n, hipStream_t s)
{
    ViewK V = view_of_args(rk, W, H, rec, vals);
    V.ids = ids;
    V.ranges = ranges;
    V.last = (uint32_t *)last;
    V.tfinal = (float *)tfinal;
    V.drgb = drgb;
    V.ddepth = ddepth;
    V.dalpha = dalpha;
    V.ddepth_scale = ddepth_scale;
    V.grad2d = grad2d;
    V.n = n;
    launch_bwd_view(V, s);
}

void launch_raster_queue(bool fwd, const ViewK *views_dev, int nv, const uint32_t *queue, uint32_t total,
                         uint32_t *counter, int blocks, hipStream_t s)
{
    launch_zero_u32(counter, 1, s);
    if (fwd) hipLaunchKernelGGL(k_raster_queue<true>, dim3(blocks), dim3(256), 0, s, views_dev, nv, queue, total, counter);
    else hipLaunchKernelGGL(k_raster_queue<false>, dim3(blocks), dim3(256), 0, s, views_dev, nv, queue, total, counter);
}

}  // namespace fgs
