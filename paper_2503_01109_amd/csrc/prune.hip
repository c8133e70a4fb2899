// Pruning of the gaussian map (Sec. III-D, "Gaussian Pruning") by stream compaction.
//
// A gaussian survives when its opacity logit is at least L_o and each of its three log-scales is
// at most L_s (the opacity and size thresholds carried into the stored values' domains on the
// host; a NaN fails its comparison). Survivors are packed in index order into the output planes,
// together with the same columns of up to three companion blocks of the same layout (the Adam
// moments).
//
// Three launches over chunks of kChunk = 2048 gaussians per 256-thread workgroup; element k of a
// thread is chunk + k * 256 + thread, so every plane is read in whole 1 KiB rows per wave:
//   k_prune_count:   the keep test, and the chunk's survivor count (wave ballots);
//   k_prune_offsets: one workgroup scans the chunk counts into exclusive offsets and the total;
//   k_prune_scatter: the keep test again (the same arithmetic, so the same answer), each
//     survivor's rank inside its chunk from the ballots, and the copy of its columns.
// The test reads 16 bytes per gaussian and the copy moves 56 bytes per plane block and survivor
// each way; the scan touches 8 bytes per chunk.
#include "fgs_internal.h"

namespace fgs {

namespace {

constexpr int kThreads = 256, kRounds = 8, kChunk = kThreads * kRounds;
constexpr int kWavesPB = kThreads / kWave;
constexpr int kScanThreads = 1024;

__device__ inline bool keep_of(const PruneK &k, int64_t i)
{
    const float *ls = k.src[0].log_scale;
    const int64_t s = k.src[0].stride;
    return k.src[0].logit[i] >= k.L_o && ls[i] <= k.L_s && ls[s + i] <= k.L_s && ls[2 * s + i] <= k.L_s;
}

// Ballots of the chunk's kRounds rounds for this wave, and the survivors in each (round, wave)
// slot written to cnt.
__device__ inline void chunk_ballots(const PruneK &k, int64_t base, uint64_t (&bal)[kRounds], uint8_t *keep_out,
                                     uint32_t (*cnt)[kWavesPB])
{
    const int tid = threadIdx.x, w = tid / kWave;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + (int64_t)r * kThreads + tid;
        const bool ok = i < k.n && keep_of(k, i);
        bal[r] = __ballot(ok);
        if (keep_out && i < k.n) keep_out[i] = ok ? 1 : 0;
        if (__lane_id() == 0) cnt[r][w] = (uint32_t)__popcll(bal[r]);
    }
}

__global__ void __launch_bounds__(kThreads) k_prune_count(PruneK k, uint32_t *chunk_count)
{
    __shared__ uint32_t cnt[kRounds][kWavesPB];
    uint64_t bal[kRounds];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    chunk_ballots(k, base, bal, k.keep, cnt);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int r = 0; r < kRounds; ++r)
            for (int w = 0; w < kWavesPB; ++w) t += cnt[r][w];
        chunk_count[blockIdx.x] = t;
    }
}

// Exclusive scan of nb chunk counts into chunk_off, and the total into *total (int64) and, when
// given, *total_out.
__global__ void __launch_bounds__(kScanThreads)
k_prune_offsets(const uint32_t *chunk_count, int64_t nb, uint32_t *chunk_off, int64_t *total, int64_t *total_out)
{
    __shared__ uint32_t wsum[kScanThreads / kWave];
    __shared__ uint32_t carry;
    const int tid = threadIdx.x, lane = __lane_id(), w = tid / kWave;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t b = b0 + tid;
        const uint32_t v = b < nb ? chunk_count[b] : 0u;
        uint32_t x = v;  // inclusive scan inside the wave
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wsum[w] = x;
        __syncthreads();
        uint32_t before = carry;
        for (int q = 0; q < w; ++q) before += wsum[q];
        if (b < nb) chunk_off[b] = before + x - v;
        __syncthreads();
        if (tid == kScanThreads - 1) carry = before + x;
        __syncthreads();
    }
    if (tid == 0) {
        *total = (int64_t)carry;
        if (total_out) *total_out = (int64_t)carry;
    }
}

__device__ inline void copy_plane(const float *src, float *dst, int64_t base, int64_t off,
                                  const uint64_t (&bal)[kRounds], const uint32_t (&rank0)[kRounds], int64_t n)
{
    const int tid = threadIdx.x;
    const uint64_t below = (1ull << __lane_id()) - 1ull;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + (int64_t)r * kThreads + tid;
        if (i < n && ((bal[r] >> __lane_id()) & 1ull))
            dst[off + rank0[r] + (uint32_t)__popcll(bal[r] & below)] = src[i];
    }
}

__global__ void __launch_bounds__(kThreads) k_prune_scatter(PruneK k, const uint32_t *chunk_off)
{
    __shared__ uint32_t cnt[kRounds][kWavesPB];
    uint64_t bal[kRounds];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    chunk_ballots(k, base, bal, nullptr, cnt);
    __syncthreads();
    // rank of this wave's first survivor in each round: the survivors of earlier rounds and of
    // earlier waves in the same round
    const int w = threadIdx.x / kWave;
    uint32_t rank0[kRounds];
    uint32_t run = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < kWavesPB; ++q) {
            const uint32_t c = cnt[r][q];
            before += q < w ? c : 0u;
            all += c;
        }
        rank0[r] = run + before;
        run += all;
    }
    const int64_t off = chunk_off[blockIdx.x];
#pragma unroll
    for (int s = 0; s < kPruneSets; ++s) {
        if (s >= k.n_sets) break;
        const ParamsK &a = k.src[s];
        const GradK &b = k.dst[s];
        const float *sp[14] = {a.mean, a.mean + a.stride, a.mean + 2 * a.stride, a.log_scale,
                               a.log_scale + a.stride, a.log_scale + 2 * a.stride, a.quat, a.quat + a.stride,
                               a.quat + 2 * a.stride, a.quat + 3 * a.stride, a.logit, a.rgb, a.rgb + a.stride,
                               a.rgb + 2 * a.stride};
        float *dp[14] = {b.mean, b.mean + b.stride, b.mean + 2 * b.stride, b.log_scale, b.log_scale + b.stride,
                         b.log_scale + 2 * b.stride, b.quat, b.quat + b.stride, b.quat + 2 * b.stride,
                         b.quat + 3 * b.stride, b.logit, b.rgb, b.rgb + b.stride, b.rgb + 2 * b.stride};
#pragma unroll
        for (int p = 0; p < 14; ++p) copy_plane(sp[p], dp[p], base, off, bal, rank0, k.n);
    }
}

}  // namespace

int64_t prune_chunks(int64_t n) { return (n + kChunk - 1) / kChunk; }

void launch_prune(const PruneK &k, uint32_t *chunk_count, uint32_t *chunk_off, int64_t *total, int64_t *total_out,
                  hipStream_t s)
{
    const int64_t nb = prune_chunks(k.n);
    if (nb > 0) hipLaunchKernelGGL(k_prune_count, dim3((unsigned)nb), dim3(kThreads), 0, s, k, chunk_count);
    hipLaunchKernelGGL(k_prune_offsets, dim3(1), dim3(kScanThreads), 0, s, chunk_count, nb, chunk_off, total,
                       total_out);
    if (nb > 0) hipLaunchKernelGGL(k_prune_scatter, dim3((unsigned)nb), dim3(kThreads), 0, s, k, chunk_off);
}

}  // namespace fgs
