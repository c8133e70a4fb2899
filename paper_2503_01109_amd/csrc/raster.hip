// Tile rasterizer: front-to-back alpha blending of Eq. 1 (colour, depth and opacity) and its
// backward.
//
// One workgroup per screen tile, one pixel per thread. The tile's list (ids of the gaussians whose
// 3-sigma box touches the tile, in (depth, index) order) is walked in batches; each batch of records
// is gathered from HBM once by the whole workgroup, converted to tile-local coordinates and
// staged in LDS, then every pixel reads the records as LDS broadcasts. A pixel applies the exact
// per-pixel cutoffs (Mahalanobis distance <= sigma_cut, alpha >= alpha_min, stop before T drops
// below T_min); the workgroup leaves the list as soon as a barrier count shows every pixel done.
//
// The staged conic is pre-multiplied by -log2(e)/2, so a pair costs one exp2 of the scaled
// quadratic form: G = 2^(s Q) = exp(-Q/2), and the cutoff Q <= sigma_cut^2 becomes
// s Q >= s sigma_cut^2.
//
// The backward walks the same list in reverse from the last blended position of the tile,
// recovering T_i = T_{i+1}/(1 - alpha_i). The colour, depth and opacity terms behind a pair enter
// its opacity gradient only through one running sum per pixel, S = sum over later pairs of
// w_j (dL/dC . c_j + dL/dD d_j) plus the background's and the opacity output's share. Each pair
// yields 10 terms (the colour, depth and opacity gradients and five moments from which the mean
// and conic gradients follow); they are summed over the wave by a transposed butterfly, over the
// workgroup's waves with LDS float atomics, and reach HBM as FP32 atomics into the gaussian's
// 64-byte gradient record, one wave instruction covering four (tile, gaussian) entries.
//
// The forward and the backward evaluate the cutoff decisions with the same inline functions in
// this translation unit, compiled without floating-point contraction, so both take identical
// decisions for every pair.
#include "fgs_internal.h"

namespace fgs {

namespace {

// s = -log2(e)/2 scales the staged conic; 1/s = -2 ln 2 recovers the conic from it.
constexpr float kConicScale = -0.721347520444481703680f;
constexpr float kInvConicScale = -1.386294361119890618834f;

__device__ __forceinline__ float sgn(float v) { return (float)((v > 0.0f) - (v < 0.0f)); }

// Record of a list entry in tile-local coordinates: a = {mean x, mean y, s a, s b}, b = {s c,
// opacity, depth, 0}, c = {r, g, b, 0} with (a, b, c) the conic. mean and conic (unscaled) are
// returned for the strip test.
__device__ __forceinline__ void stage(const Rec &R, int x0, int y0, float4 &a, float4 &b, float4 &c, float &mx,
                                      float &my)
{
    // projected mean in tile-local coordinates: integer part is exact, one rounding for the sum
    mx = (float)(__float_as_int(R.r0.x) - x0) + R.r0.z;
    my = (float)(__float_as_int(R.r0.y) - y0) + R.r0.w;
    a = make_float4(mx, my, kConicScale * R.r1.x, (2.0f * kConicScale) * R.r1.y);  // s a, 2 s b
    b = make_float4(kConicScale * R.r1.z, R.r1.w, R.r2.w, 0.0f);
    c = make_float4(R.r2.x, R.r2.y, R.r2.z, 0.0f);
}

// One (pixel, staged record) pair: offsets from the mean, q = s Q in a fixed operation order,
// (s a dx + 2 s b dy) dx + (s c dy) dy with two FMAs, and G = 2^q = exp(-Q/2). The forward and the
// backward evaluate it identically, so they take the same decisions.
struct PairEval {
    float dx, dy, q, G;
};

__device__ __forceinline__ PairEval eval_pair(const float4 &a4, const float4 &b4, float px, float py)
{
    PairEval e;
    e.dx = px - a4.x;
    e.dy = py - a4.y;
    const float u = __builtin_fmaf(a4.w, e.dy, a4.z * e.dx);
    e.q = __builtin_fmaf(u, e.dx, (b4.x * e.dy) * e.dy);
    e.G = __builtin_amdgcn_exp2f(e.q);  // q <= 0 up to rounding, >= s sigma_cut^2 when used
    return e;
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
// strip (rows [w R, w R + R) of the tile, R = 64 / tw). Conservative by a relative 1e-3 margin:
// the per-pixel test stays the exact decision. (mx, my): tile-local mean; (ca, cb, cc): conic.
template <int NW>
__device__ __forceinline__ uint32_t strip_mask(float mx, float my, float ca, float cb, float cc, float cut2, int tw)
{
    const int R = kWave / tw;
    uint32_t m = 0;
    const float ia = __frcp_rn(ca), ic = __frcp_rn(cc);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const float q = rect_min_q(ca, cb, cc, ia, ic, mx, my, 0.5f, tw - 0.5f, w * R + 0.5f, w * R + R - 0.5f);
        if (q <= cut2 * 1.001f) m |= 1u << w;
    }
    return m;
}

// Bit w set when the sigma_cut ellipse can reach a pixel centre of wave w's 8x8 quadrant of a
// 16x16 tile (conservative by a relative 1e-3 margin).
template <int NW>
__device__ __forceinline__ uint32_t quad_mask(float mx, float my, float ca, float cb, float cc, float cut2)
{
    uint32_t m = 0;
    const float ia = __frcp_rn(ca), ic = __frcp_rn(cc);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const float x0 = 8.0f * (w & 1) + 0.5f, y0 = 8.0f * (w >> 1) + 0.5f;
        const float q = rect_min_q(ca, cb, cc, ia, ic, mx, my, x0, x0 + 7.0f, y0, y0 + 7.0f);
        if (q <= cut2 * 1.001f) m |= 1u << w;
    }
    return m;
}

// Compacts the indices k < cnt whose mask has this wave's bit into this wave's list (ascending), as
// byte offsets 16 k of the staged 16-byte records; returns the list length. Wave-local: no block
// barrier needed.
__device__ __forceinline__ int wave_compact(const uint8_t *smask, int cnt, int wid, uint16_t *list)
{
    const int lane = __lane_id();
    int len = 0;
    for (int q = 0; q < cnt; q += kWave) {
        const int e = q + lane;
        const bool bit = e < cnt && ((smask[e] >> wid) & 1u);
        const uint64_t bal = __ballot(bit);
        if (bit) list[len + __popcll(bal & ((1ull << lane) - 1ull))] = (uint16_t)(e << 4);
        len += __popcll(bal);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return len;
}

// The staged 16-byte record at byte offset o of an LDS array (the lists hold byte offsets, so a
// pair's loads take no scaling of their index).
__device__ __forceinline__ float4 rec_at(const float4 *a, int o)
{
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(a) + o);
}

// Exchange across lane distance 32 (D = 32) or 16 (D = 16) without selects: lanes whose bit D is
// clear return lo summed with the partner's lo, the others hi summed with the partner's hi
// (gfx950's row swaps: permlane32 trades the upper half of lo for the lower half of hi, permlane16
// the odd rows of lo for the even rows of hi).
template <int D>
__device__ __forceinline__ float swap_add(float lo, float hi)
{
    const auto r = D == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false)
                           : __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Exchange across lane distance 1 (PAT = quad_perm 0xB1) or 2 (0x4E): lanes with that bit clear
// return lo summed with the partner's lo, the others hi summed with the partner's hi.
template <int PAT, int BIT>
__device__ __forceinline__ float dpp_add(float lo, float hi, int lane)
{
    const bool b = lane & BIT;
    const float send = b ? lo : hi, mine = b ? hi : lo;
    return mine + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), PAT, 0xf, 0xf, false));
}

// Ten wave sums at once by a transposed butterfly: at each exchange a lane keeps the half of its
// partial sums that its partner gives away and adds the partner's matching half, so 10 values
// shrink to 5, 3, 2 and 1 per lane over lane distances 32, 16, 1 and 2 (an odd value out is summed
// by both partners); two rotations within each row of 16 add its four quads. Every lane ends with
// the full sum of one term; reduce_term names, for one lane per term, which (-1 elsewhere). The
// two widest exchanges use the row swaps, the rest DPP: about 25 VALU operations and no LDS
// traffic for ten sums.
__device__ __forceinline__ float reduce10(const float v[10], int lane)
{
    float a[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) a[c] = swap_add<32>(v[c], v[c + 5]);  // term c + 5 (lane >> 5)
    const float q0 = swap_add<16>(a[0], a[3]), q1 = swap_add<16>(a[1], a[4]), q2 = swap_add<16>(a[2], a[2]);
    const float r0 = dpp_add<0xB1, 1>(q0, q2, lane);
    const float r1 = q1 + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(q1), 0xB1, 0xf, 0xf, false));
    float d = dpp_add<0x4E, 2>(r0, r1, lane);
    d += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(d), 0x124, 0xf, 0xf, true));  // row_ror:4
    d += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(d), 0x128, 0xf, 0xf, true));  // row_ror:8
    // (kept here, where the rotation and the add fuse into one instruction, rather than moved
    // into the lanes that use the sum)
    asm volatile("" : "+v"(d));
    return d;
}

// The term whose sum reduce10 leaves in this lane, for one lane per term (-1: a copy or padding).
// Row r of 16 lanes holds terms 5 (r >> 1) + {0, 2, 1} (r even) or + {3, -, 4} (r odd) in its
// lanes 0, 1, 2.
__device__ __forceinline__ int reduce_term(int lane)
{
    const int row = lane >> 4, i = lane & 15, base = 5 * (row >> 1);
    if (i > 2) return -1;
    if ((row & 1) == 0) return base + (i == 0 ? 0 : (i == 1 ? 2 : 1));
    return i == 1 ? -1 : base + (i == 0 ? 3 : 4);
}

// Twenty wave sums at once, the ten terms of two list entries (u: the first, v: the second), by
// the same transposed butterfly: 20 values shrink to 10, 5, 3, 2 and 1 per lane over lane
// distances 32 (row swaps), 16 (row swaps), 1 and 2 (DPP) and 4 (an LDS swizzle, outside the VALU),
// and one rotation by 8 within each row adds its two halves. Every lane ends with the full sum of
// one term of one entry; reduce20_slot names, for one lane per term, which.
__device__ __forceinline__ float reduce20(const float u[10], const float v[10], int lane)
{
    float a[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) a[c] = swap_add<32>(u[c], v[c]);  // entry lane >> 5, term c
    float q[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) q[c] = swap_add<16>(a[c], a[c + 5]);
    const float r0 = dpp_add<0xB1, 1>(q[0], q[3], lane), r1 = dpp_add<0xB1, 1>(q[1], q[4], lane);
    const float r2 = q[2] + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(q[2]), 0xB1, 0xf, 0xf, false));
    const float t0 = dpp_add<0x4E, 2>(r0, r2, lane);
    const float t1 = r1 + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(r1), 0x4E, 0xf, 0xf, false));
    const bool b2 = lane & 4;
    const float send = b2 ? t0 : t1, mine = b2 ? t1 : t0;
    // ds_swizzle bitmask mode: and 0x1f, or 0, xor 4 (the partner across lane distance 4)
    float d = mine + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(send), 0x101F));
    d += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(d), 0x128, 0xf, 0xf, true));  // row_ror:8
    asm volatile("" : "+v"(d));  // (as in reduce10)
    return d;
}

// Which sum reduce20 leaves in this lane, for one lane per sum: 10 e + term for entry e (u: 0,
// v: 1), or -1 (a copy). Row r of 16 lanes holds sums 5 r + {0, 3, 2, -, 1, 4} in its lanes 0-5.
__device__ __forceinline__ int reduce20_slot(int lane)
{
    const int r = lane >> 4, i = lane & 15;
    const int off = i == 0 ? 0 : i == 1 ? 3 : i == 2 ? 2 : i == 4 ? 1 : i == 5 ? 4 : -1;
    return off < 0 ? -1 : 5 * r + off;
}

// Forward of one tile of one view by a workgroup of NT threads (one pixel each; the tile is
// tile_w x tile_h = NT pixels). COUNT: accumulate the profiling work counters; NCON: count each
// pixel's blended pairs (for the n_contrib output; implied by COUNT).
template <int NT, bool COUNT, bool NCON = COUNT, bool ALPHA = true>
__device__ void tile_fwd(const ViewK &V, int tile)
{
    constexpr int NW = NT / kWave;
    __shared__ float4 sa[NT], sb[NT], sc[NT];
    __shared__ uint8_t smask[NT];
    __shared__ uint16_t slist[NW][NT];
    __shared__ unsigned long long red[3];
    __shared__ uint32_t smx[2];
    __shared__ uint8_t sblend[NT];  // COUNT: entries of the staged batch that some pixel blended
    const RasterK &rk = V.rk;
    const int W = V.W, H = V.H;
    const Rec *__restrict__ rec = V.rec;
    const uint32_t *__restrict__ vals = V.vals;
    const int TW = rk.tile_w, TH = rk.tile_h;
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    const int sidx = tile / (kSuper * kSuper), sl = tile % (kSuper * kSuper);
    const int tx = (sidx % rk.supers_x) * kSuper + sl % kSuper, ty = (sidx / rk.supers_x) * kSuper + sl / kSuper;
    const int x0 = tx * TW, y0 = ty * TH;
    const int lx = tid % TW, ly = tid / TW;
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < W && y < H;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint2 range = V.ranges[tile];
    const float cut2 = rk.sigma_cut * rk.sigma_cut;
    const float qcut = kConicScale * cut2;
    // (canonical once here, so that the pair loop's minimum needs no canonicalising of its own)
    const float amax = __builtin_canonicalizef(rk.alpha_max);

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f, A = 0.0f;
    uint32_t last = 0, ntest = 0, staged = 0;
    int32_t ncon = 0;
    // the lane's cutoff on q: qcut while the pixel blends, +inf once it is done (outside the
    // image, or stopped before a pair that would take T below T_min), so that no pair is near
    float qc = inside ? qcut : INFINITY;
    // COUNT: list entries this pixel examines (up to the one it stops at; all if it never stops),
    // and (tile, gaussian) entries some pixel blended
    uint32_t cons = inside ? range.y - range.x : 0u, kc = 0;
    int prev_cnt = 0;
    if (COUNT) sblend[tid] = 0;  // ordered before its first use by the loop's first barrier

    for (uint32_t b = range.x; b < range.y; b += NT) {
        const int alive = __syncthreads_count(qc < INFINITY);
        if (COUNT && tid < prev_cnt) {
            kc += sblend[tid];
            sblend[tid] = 0;
        }
        if (alive == 0) break;
        staged += min((uint32_t)NT, range.y - b);
        const uint32_t j = b + tid;
        if (j < range.y) {
            const Rec R = rec[vals[j]];
            float4 a4, b4, c4;
            float mx, my;
            stage(R, x0, y0, a4, b4, c4, mx, my);
            sa[tid] = a4;
            sb[tid] = b4;
            sc[tid] = c4;
            smask[tid] = (uint8_t)strip_mask<NW>(mx, my, R.r1.x, R.r1.y, R.r1.z, cut2, TW);
        }
        __syncthreads();
        const int cnt = min((uint32_t)NT, range.y - b);
        if (COUNT) prev_cnt = cnt;
        const int len = wave_compact(smask, cnt, wid, slist[wid]);
        const uint32_t base = b - range.x + 1;
        // Branch-free per pair: every lane evaluates the entry and the decisions select what is
        // kept; T - alpha T is the new transmittance (T (1 - alpha) up to rounding). The last
        // blended entry of this chunk is kept as its byte offset and folded into `last` after it.
        int lastk = -1;
        auto pair = [&](int o) {
            const float4 a4 = rec_at(sa, o), b4 = rec_at(sb, o);
            const PairEval e = eval_pair(a4, b4, px, py);
            const bool near = !(e.q < qc);
            const float alpha = fminf(amax, b4.y * e.G);
            const bool take = near && !(alpha < rk.alpha_min);
            const float u = alpha * T, Tn = T - u;
            const bool low = Tn < rk.T_min;
            const bool blend = take && !low;
            const float w = blend ? u : 0.0f;
            const float4 c4 = rec_at(sc, o);
            C0 = __builtin_fmaf(w, c4.x, C0);
            C1 = __builtin_fmaf(w, c4.y, C1);
            C2 = __builtin_fmaf(w, c4.z, C2);
            D = __builtin_fmaf(w, b4.z, D);
            if (ALPHA) A += w;
            T = blend ? Tn : T;
            qc = take && low ? INFINITY : qc;
            if (COUNT) {
                ntest += near ? 1u : 0u;
                if (blend) sblend[o >> 4] = 1;
                if (take && low) cons = base + (uint32_t)(o >> 4);
            }
            if (COUNT || NCON) ncon += blend ? 1 : 0;
            lastk = blend ? o : lastk;
        };
        // two entries per round: the wave leaves the list once all of its pixels are done
        for (int i = 0; i < len; i += 2) {
            if (__ballot(qc < INFINITY) == 0) break;
            pair(slist[wid][i]);
            if (i + 1 < len) pair(slist[wid][i + 1]);
        }
        if (lastk >= 0) last = base + (uint32_t)(lastk >> 4);
    }
    if (COUNT) {
        // work counters (profiling only): block sums and maxima, one atomic per block and counter
        __syncthreads();
        if (tid < prev_cnt) {
            kc += sblend[tid];
            sblend[tid] = 0;
        }
        if (tid == 0) {
            red[0] = red[1] = red[2] = 0ull;
            smx[0] = smx[1] = 0u;
        }
        __syncthreads();
        if (inside) {
            atomicAdd(&red[0], (unsigned long long)ntest);
            atomicAdd(&red[1], (unsigned long long)ncon);
            atomicMax(&smx[0], cons);
            atomicMax(&smx[1], last);
        }
        if (kc) atomicAdd(&red[2], (unsigned long long)kc);
        __syncthreads();
        if (tid == 0) {
            atomicAdd(&V.counts[0], red[0]);
            atomicAdd(&V.counts[1], red[1]);
            atomicAdd(&V.counts[2], (unsigned long long)staged);
            atomicAdd(&V.counts[3], red[2]);
            atomicAdd(&V.counts[4], (unsigned long long)smx[0]);
            atomicAdd(&V.counts[5], (unsigned long long)smx[1]);
        }
    }
    // the next tile of a persistent workgroup restages the LDS arrays: wait for every reader
    __syncthreads();
    const int64_t P = (int64_t)W * H;
    const int64_t p = (int64_t)y * W + x;
    const float col[3] = {C0 + T * rk.bg[0], C1 + T * rk.bg[1], C2 + T * rk.bg[2]};
    const float dep = D + T * rk.bg_depth;
    if (inside) {
        const ImageK &img = V.img;
        if (img.rgb) {
            img.rgb[p] = col[0];
            img.rgb[P + p] = col[1];
            img.rgb[2 * P + p] = col[2];
        }
        if (img.depth) img.depth[p] = dep;
        if (ALPHA && img.alpha) img.alpha[p] = A;
        if (img.T_final) img.T_final[p] = T;
        if (img.n_contrib) img.n_contrib[p] = ncon;
        V.last[p] = last;
        V.tfinal[p] = T;
    }
    const LossK &lk = V.loss;
    if (lk.partials) {
        // the L1 terms of the mapping loss and their gradients, summed over the tile
        float q[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // |C - C*|, (C - C*)^2, |D - D*| (valid), valid
        if (inside) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float r = col[c] - lk.trgb[c * P + p];
                q[0] += fabsf(r);
                q[1] += r * r;
                lk.drgb[c * P + p] = lk.lrgb * sgn(r) * lk.inv3P;
            }
            const float td = lk.tdepth[p];
            const bool valid = td > 0.0f;
            const float rd = dep - td;
            q[2] = valid ? fabsf(rd) : 0.0f;
            q[3] = valid ? 1.0f : 0.0f;
            lk.ddepth[p] = valid ? lk.ldepth * sgn(rd) : 0.0f;
        }
        __shared__ float sred[NW][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float v = q[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (__lane_id() == 0) sred[wid][k] = v;
        }
        __syncthreads();
        if (tid < 4) {
            float t = 0.0f;
#pragma unroll
            for (int w = 0; w < NW; ++w) t += sred[w][tid];
            lk.partials[4 * (int64_t)tile + tid] = t;
        }
        __syncthreads();  // sred is reused by the next tile of a persistent workgroup
    }
}

// Backward of one (pixel, entry) pair, walking the list from the back, in two parts. bwd_decide:
// whether the forward blended it (before the pixel's last blended position, inside the cutoff,
// above alpha_min). bwd_grad: recovers T_i from T_{i+1}, writes the pair's 10 gradient terms (exact
// zeros when not taken) and advances the pixel's T and S; a lane that does not take the pair
// leaves T and S unchanged, so a wave in which no lane takes it can skip bwd_grad altogether.
struct BwdPair {
    PairEval e;
    float ar, alpha;
    bool take;
};

__device__ __forceinline__ BwdPair bwd_decide(const float4 &a4, const float4 &b4, bool before_last, float px,
                                              float py, float qcut, const RasterK &rk)
{
    BwdPair p;
    p.e = eval_pair(a4, b4, px, py);
    p.ar = b4.y * p.e.G;
    p.alpha = fminf(rk.alpha_max, p.ar);
    // before the last blended position and inside the cutoff, else -1 (below every alpha_min,
    // which is at least 0): one comparison decides, so that the wave's ballot of the decision is
    // that comparison's own lane mask
    const float a_in = before_last && !(p.e.q < qcut) ? p.alpha : -1.0f;
    p.take = !(a_in < rk.alpha_min);
    return p;
}

__device__ __forceinline__ void bwd_grad(const BwdPair &p, const float4 &b4, const float4 &c4, const RasterK &rk,
                                         float gC0, float gC1, float gC2, float gD, float &T, float &S, float g[10])
{
    const PairEval &e = p.e;
    const float alpha = p.alpha;
    const bool take = p.take;
    const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);  // 1 ulp; alpha <= alpha_max < 1
    const float Ti = T * inv;
    const float w = take ? alpha * Ti : 0.0f;
    // dL/dalpha_i = T_i X_i - S / (1 - alpha_i), X_i = dL/dC . c_i + dL/dD d_i
    const float X = __builtin_fmaf(gC0, c4.x, __builtin_fmaf(gC1, c4.y, __builtin_fmaf(gC2, c4.z, gD * b4.z)));
    const float dal = __builtin_fmaf(-S, inv, Ti * X);
    // a clamped alpha (o G > alpha_max) passes nothing to opacity, mean or conic
    const float dalg = take && !(p.ar > rk.alpha_max) ? dal : 0.0f;
    S = __builtin_fmaf(w, X, S);
    T = take ? Ti : T;
    g[6] = gC0 * w;
    g[7] = gC1 * w;
    g[8] = gC2 * w;
    g[9] = gD * w;
    g[5] = dalg * e.G;  // d alpha / d opacity = G
    // With e = alpha dL/dalpha, dL/dQ = -e/2, so the conic gradient is -(1/2) (e dx^2, 2 e dx dy,
    // e dy^2) and the mean gradient -2 dL/dQ (a dx + b dy, b dx + c dy) = (a e dx + b e dy, ...):
    // both are linear in the moments e dx, e dy, e dx^2, e dx dy, e dy^2 with coefficients of the
    // gaussian alone. The pairs leave those moments (slots 0-4), summed over the pixels; the
    // flush applies the coefficients once per (tile, gaussian).
    const float ea = alpha * dalg;
    const float edx = ea * e.dx, edy = ea * e.dy;
    g[0] = edx;
    g[1] = edy;
    g[2] = edx * e.dx;
    g[3] = edx * e.dy;
    g[4] = edy * e.dy;
}

// Backward of one tile of one view (NT threads, one pixel each). COUNT: add the backward's work
// counters to V.counts[6..9]: wave-entry evaluations (a wave evaluating one staged entry for its
// 64 pixels), those in which some pixel blended, those in which 1 to 8 pixels blended, and the
// (pixel, entry) pairs blended.
template <int NT, bool COUNT = false>
__device__ void tile_bwd(const ViewK &V, int tile)
{
    constexpr int NW = NT / kWave;
    const RasterK &rk = V.rk;
    const int W = V.W, H = V.H;
    const Rec *__restrict__ rec = V.rec;
    const uint32_t *__restrict__ vals = V.vals;
    float *__restrict__ grad2d = V.grad2d;
    const int TW = rk.tile_w, TH = rk.tile_h;
    __shared__ float4 sa[NT], sb[NT], sc[NT];
    __shared__ uint32_t sid[NT];
    __shared__ float sacc[NT][10];  // per staged entry: the ten terms summed over the workgroup
    __shared__ uint32_t smax;
    __shared__ uint8_t smask[NT];
    __shared__ uint16_t slist[NW][NT];
    __shared__ unsigned long long swork[NW][4];
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    // COUNT: this wave's wave-entry evaluations, of them with a blend, with 1-8 blending pixels,
    // and its blended pairs (wave-uniform)
    unsigned long long n_eval = 0, n_take = 0, n_few = 0, n_pairs = 0;
    auto count_entry = [&](uint64_t bal) {
        const uint32_t c = (uint32_t)__popcll(bal);
        n_eval += 1;
        n_take += c ? 1 : 0;
        n_few += (c && c <= 8) ? 1 : 0;
        n_pairs += c;
    };
    const int term = reduce_term(lane);  // the term whose wave sum this lane holds after reduce10
    const bool red_lane = term >= 0;
    const int slot20 = reduce20_slot(lane);  // the same after reduce20
    // the flush: 16 lanes per entry, lane fc adds slot fc, scaled by fscale (slots 2-9)
    const int fc = tid & 15;
    const float fscale = fc == 3 ? -1.0f : (fc == 2 || fc == 4) ? -0.5f : 1.0f;
    const int wid = tid / kWave;
    const int sidx = tile / (kSuper * kSuper), sl = tile % (kSuper * kSuper);
    const int tx = (sidx % rk.supers_x) * kSuper + sl % kSuper, ty = (sidx / rk.supers_x) * kSuper + sl / kSuper;
    const int x0 = tx * TW, y0 = ty * TH;
    // 16x16 tiles: wave w takes the 8x8 quadrant (w & 1, w >> 1), which culls partly covering
    // gaussians better than a 16x4 strip (measured faster in the backward, not the forward)
    const bool quad = TW == 16 && TH == 16;
    const int lx = quad ? 8 * (wid & 1) + (tid & 7) : tid % TW;
    const int ly = quad ? 8 * (wid >> 1) + ((tid & 63) >> 3) : tid / TW;
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < W && y < H;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint2 range = V.ranges[tile];
    const float cut2 = rk.sigma_cut * rk.sigma_cut;
    const float qcut = kConicScale * cut2;
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
    // S: what the pairs behind the current one (and the background) pass back through its
    // transmittance: dL/dC . C_behind + dL/dD D_behind - dL/dA T_final, with C_behind, D_behind
    // the colour and depth blended behind it including the background's T_final share.
    const float Tf = T;
    float S = Tf * (gC0 * rk.bg[0] + gC1 * rk.bg[1] + gC2 * rk.bg[2] + gD * rk.bg_depth - gA);

    if (tid == 0) smax = 0;
#pragma unroll
    for (int c = 0; c < 10; ++c) sacc[tid][c] = 0.0f;
    __syncthreads();
    if (L) atomicMax(&smax, L);
    // the wave's own last blended position: entries at or beyond it are blended by none of its
    // pixels and are left out of its lists before any evaluation
    uint32_t wL = L;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wL = max(wL, (uint32_t)__shfl_xor((int)wL, o));
    __syncthreads();
    const uint32_t hi = min(range.x + smax, range.y);

    for (uint32_t bend = hi; bend > range.x; bend -= min((uint32_t)NT, bend - range.x)) {
        const uint32_t bstart = bend - min((uint32_t)NT, bend - range.x);
        const int cnt = (int)(bend - bstart);
        __syncthreads();
        if (tid < cnt) {
            const uint32_t id = vals[bstart + tid];
            const Rec R = rec[id];
            float4 a4, b4, c4;
            float mx, my;
            stage(R, x0, y0, a4, b4, c4, mx, my);
            sa[tid] = a4;
            sb[tid] = b4;
            sc[tid] = c4;
            sid[tid] = id;  // gradients are accumulated by gaussian id
            smask[tid] = (uint8_t)(quad ? quad_mask<NW>(mx, my, R.r1.x, R.r1.y, R.r1.z, cut2)
                                             : strip_mask<NW>(mx, my, R.r1.x, R.r1.y, R.r1.z, cut2, TW));
        }
        __syncthreads();
        const uint32_t base = bstart - range.x;
        // this pixel's last blended position relative to the batch, clamped to [-1, NT] and as a
        // byte offset, so that an entry's test is one comparison of its list word (list positions
        // stay below 2^31)
        const int Lb = min(max((int)L - (int)base, -1), NT) * 16;
        const int len = wave_compact(smask, (int)min((uint32_t)cnt, wL > base ? wL - base : 0u), wid, slist[wid]);
        // Branch-free per pair, like the forward: the decisions select what is kept, and a lane
        // that does not take the pair contributes exact zeros. Two entries per iteration: their
        // evaluations and wave reductions are independent, only T and S pass from one to the next.
        int i = len - 1;
        for (; i >= 1; i -= 2) {
            const int k0 = slist[wid][i], k1 = slist[wid][i - 1];  // (byte offsets)
            const float4 a0 = rec_at(sa, k0), b0 = rec_at(sb, k0), a1 = rec_at(sa, k1), b1 = rec_at(sb, k1);
            const BwdPair p0 = bwd_decide(a0, b0, k0 < Lb, px, py, qcut, rk);
            const BwdPair p1 = bwd_decide(a1, b1, k1 < Lb, px, py, qcut, rk);
            // (the lane-mask ballot of the decision itself: through an int it would cost a select
            // and a compare per entry)
            const uint64_t t0 = __builtin_amdgcn_ballot_w64(p0.take), t1 = __builtin_amdgcn_ballot_w64(p1.take);
            if (COUNT) {
                count_entry(t0);
                count_entry(t1);
            }
            if (t0 && t1) {
                float g0[10], g1[10];
                bwd_grad(p0, b0, rec_at(sc, k0), rk, gC0, gC1, gC2, gD, T, S, g0);
                bwd_grad(p1, b1, rec_at(sc, k1), rk, gC0, gC1, gC2, gD, T, S, g1);
                const float t = reduce20(g0, g1, lane);
                if (slot20 >= 0) atomicAdd(&sacc[(slot20 < 10 ? k0 : k1) >> 4][slot20 % 10], t);
            } else if (t0) {
                // one entry blended by some lane: the other leaves every lane's T and S as they are
                float g[10];
                bwd_grad(p0, b0, rec_at(sc, k0), rk, gC0, gC1, gC2, gD, T, S, g);
                const float t = reduce10(g, lane);
                if (red_lane) atomicAdd(&sacc[k0 >> 4][term], t);
            } else if (t1) {
                float g[10];
                bwd_grad(p1, b1, rec_at(sc, k1), rk, gC0, gC1, gC2, gD, T, S, g);
                const float t = reduce10(g, lane);
                if (red_lane) atomicAdd(&sacc[k1 >> 4][term], t);
            }
        }
        if (i == 0) {
            const int k0 = slist[wid][0];  // (a byte offset)
            const float4 a0 = rec_at(sa, k0), b0 = rec_at(sb, k0);
            const BwdPair p0 = bwd_decide(a0, b0, k0 < Lb, px, py, qcut, rk);
            const uint64_t t0 = __builtin_amdgcn_ballot_w64(p0.take);
            if (COUNT) count_entry(t0);
            if (t0) {
                float g0[10];
                bwd_grad(p0, b0, rec_at(sc, k0), rk, gC0, gC1, gC2, gD, T, S, g0);
                const float t0 = reduce10(g0, lane);
                if (red_lane) atomicAdd(&sacc[k0 >> 4][term], t0);
            }
        }
        __syncthreads();
        // Each gaussian's ten terms form one 64-byte record of grad2d: 16 lanes per entry, lane c
        // (< 10) adds term c, so one wave instruction updates the records of four gaussians, one
        // cache line each.
        for (int e = tid >> 4; e < cnt; e += NT >> 4) {
            if (fc < 10) {
                // moments to gradients (see bwd_grad): the staged conic is s (a, 2 b, c); slots 0
                // and 1 mix the first two moments with the gaussian's conic, the rest scale theirs
                const float raw = sacc[e][fc], m0 = sacc[e][0], m1 = sacc[e][1], sbv = 0.5f * sa[e].w;
                const float P = fc == 0 ? sa[e].z : sbv, Q = fc == 0 ? sbv : sb[e].x;
                const float v = fc < 2 ? (P * m0 + Q * m1) * kInvConicScale : raw * fscale;
                if (v != 0.0f) unsafeAtomicAdd(&grad2d[(int64_t)sid[e] * kG2Stride + fc], v);
                if (raw != 0.0f) sacc[e][fc] = 0.0f;
            }
        }
    }
    if (COUNT) {
        if (lane == 0) {
            swork[wid][0] = n_eval;
            swork[wid][1] = n_take;
            swork[wid][2] = n_few;
            swork[wid][3] = n_pairs;
        }
        __syncthreads();
        if (tid < 4) {
            unsigned long long t = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) t += swork[w][tid];
            if (t) atomicAdd(&V.counts[6 + tid], t);
        }
    }
    __syncthreads();  // LDS is restaged by the next tile of a persistent workgroup
}

// eight waves per SIMD (64 VGPRs), as the window's forward
template <int NT, bool COUNT, bool NCON, bool ALPHA>
__global__ void __launch_bounds__(NT, 2048 / NT) k_raster_fwd(ViewK V) { tile_fwd<NT, COUNT, NCON, ALPHA>(V, blockIdx.x); }

template <int NT, bool COUNT>
__global__ void __launch_bounds__(NT) k_raster_bwd(ViewK V) { tile_bwd<NT, COUNT>(V, blockIdx.x); }

__device__ inline int view_of(const ViewK *views, int nv, uint32_t g)
{
    int v = 0;
    while (v + 1 < nv && views[v + 1].tile_base <= g) ++v;
    return v;
}

// Persistent rasterizer over a window of views: workgroups pull (view, tile) items through an
// atomic counter until it runs past the last item. 256 threads per workgroup; each view's tile
// has 256 pixels in its own shape (16x16, 32x8 or 8x32). The item's view descriptor is copied
// out of device memory once, so the tile code reads it from registers.
template <bool FWD, bool COUNT>
__global__ void __launch_bounds__(256)
k_raster_queue(const ViewK *__restrict__ views, int nv, uint32_t total, uint32_t *__restrict__ counter)
{
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t g = s_item;
        __syncthreads();
        if (g >= total) break;
        const ViewK V = views[view_of(views, nv, g)];
        if (FWD) tile_fwd<256, COUNT, COUNT, false>(V, (int)(g - V.tile_base));  // loss only: no image
        else tile_bwd<256>(V, (int)(g - V.tile_base));
    }
}

// The same items with one workgroup each (grid = total). The forward is held to 64 VGPRs (eight
// waves per SIMD), as the single-view forward compiles to by itself.
template <bool COUNT>
__global__ void __launch_bounds__(256, 8)
k_raster_items_fwd(const ViewK *__restrict__ views, int nv)
{
    const uint32_t g = blockIdx.x;
    const ViewK V = views[view_of(views, nv, g)];
    tile_fwd<256, COUNT, COUNT, false>(V, (int)(g - V.tile_base));  // loss only: no image
}

__global__ void __launch_bounds__(256)
k_raster_items_bwd(const ViewK *__restrict__ views, int nv)
{
    const uint32_t g = blockIdx.x;
    const ViewK V = views[view_of(views, nv, g)];
    tile_bwd<256>(V, (int)(g - V.tile_base));
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

template <bool COUNT, bool NCON, bool ALPHA>
static void launch_fwd_variant(const ViewK &V, unsigned tiles, int nt, hipStream_t s)
{
    if (nt == 256) hipLaunchKernelGGL((k_raster_fwd<256, COUNT, NCON, ALPHA>), dim3(tiles), dim3(256), 0, s, V);
    else if (nt == 512) hipLaunchKernelGGL((k_raster_fwd<512, COUNT, NCON, ALPHA>), dim3(tiles), dim3(512), 0, s, V);
    else hipLaunchKernelGGL((k_raster_fwd<64, COUNT, NCON, ALPHA>), dim3(tiles), dim3(64), 0, s, V);
}

static void launch_fwd_view(const ViewK &V, hipStream_t s)
{
    const unsigned tiles = (unsigned)tile_items(V.rk.tiles_x, V.rk.tiles_y);
    const int nt = V.rk.tile_w * V.rk.tile_h;
    // the opacity plane's running sum only when that plane is written (not by the mapping step)
    if (V.counts) launch_fwd_variant<true, true, true>(V, tiles, nt, s);
    else if (V.img.n_contrib) launch_fwd_variant<false, true, true>(V, tiles, nt, s);
    else if (V.img.alpha) launch_fwd_variant<false, false, true>(V, tiles, nt, s);
    else launch_fwd_variant<false, false, false>(V, tiles, nt, s);
}

static void launch_bwd_view(const ViewK &V, hipStream_t s)
{
    const unsigned tiles = (unsigned)tile_items(V.rk.tiles_x, V.rk.tiles_y);
    const int nt = V.rk.tile_w * V.rk.tile_h;
    if (V.counts) {
        if (nt == 256) hipLaunchKernelGGL((k_raster_bwd<256, true>), dim3(tiles), dim3(256), 0, s, V);
        else if (nt == 512) hipLaunchKernelGGL((k_raster_bwd<512, true>), dim3(tiles), dim3(512), 0, s, V);
        else hipLaunchKernelGGL((k_raster_bwd<64, true>), dim3(tiles), dim3(64), 0, s, V);
    } else {
        if (nt == 256) hipLaunchKernelGGL((k_raster_bwd<256, false>), dim3(tiles), dim3(256), 0, s, V);
        else if (nt == 512) hipLaunchKernelGGL((k_raster_bwd<512, false>), dim3(tiles), dim3(512), 0, s, V);
        else hipLaunchKernelGGL((k_raster_bwd<64, false>), dim3(tiles), dim3(64), 0, s, V);
    }
}

void launch_raster_fwd(const RasterK &rk, int32_t W, int32_t H, const Rec *rec, const uint32_t *vals,
                       const uint2 *ranges, uint32_t *last, float *tfinal, const ImageK &img, const LossK &loss,
                       unsigned long long *counts, hipStream_t s)
{
    ViewK V = view_of_args(rk, W, H, rec, vals);
    V.ranges = ranges;
    V.last = last;
    V.tfinal = tfinal;
    V.img = img;
    V.loss = loss;
    V.counts = counts;
    launch_fwd_view(V, s);
}

void launch_raster_bwd(const RasterK &rk, int32_t W, int32_t H, const Rec *rec, const uint32_t *vals,
                       const uint2 *ranges, const uint32_t *last, const float *tfinal,
                       const float *drgb, const float *ddepth, const float *dalpha, const float *ddepth_scale,
                       float *grad2d, unsigned long long *counts, hipStream_t s)
{
    ViewK V = view_of_args(rk, W, H, rec, vals);
    V.ranges = ranges;
    V.last = (uint32_t *)last;
    V.tfinal = (float *)tfinal;
    V.drgb = drgb;
    V.ddepth = ddepth;
    V.dalpha = dalpha;
    V.ddepth_scale = ddepth_scale;
    V.grad2d = grad2d;
    V.counts = counts;
    launch_bwd_view(V, s);
}

void launch_raster_window(bool fwd, bool count, const ViewK *views_dev, int nv, uint32_t total, uint32_t *counter,
                          int blocks, hipStream_t s)
{
    if (total == 0) return;
    if (blocks <= 0) {
        const dim3 grid(total);
        if (fwd && count) hipLaunchKernelGGL((k_raster_items_fwd<true>), grid, dim3(256), 0, s, views_dev, nv);
        else if (fwd) hipLaunchKernelGGL((k_raster_items_fwd<false>), grid, dim3(256), 0, s, views_dev, nv);
        else hipLaunchKernelGGL(k_raster_items_bwd, grid, dim3(256), 0, s, views_dev, nv);
        return;
    }
    launch_zero_u32(counter, 1, s);
    const dim3 grid(blocks);
    if (fwd && count)
        hipLaunchKernelGGL((k_raster_queue<true, true>), grid, dim3(256), 0, s, views_dev, nv, total, counter);
    else if (fwd)
        hipLaunchKernelGGL((k_raster_queue<true, false>), grid, dim3(256), 0, s, views_dev, nv, total, counter);
    else
        hipLaunchKernelGGL((k_raster_queue<false, false>), grid, dim3(256), 0, s, views_dev, nv, total, counter);
}

}  // namespace fgs
