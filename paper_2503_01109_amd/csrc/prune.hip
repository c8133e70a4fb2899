// Pruning of the gaussian map (Sec. III-D, "Gaussian Pruning") by stream compaction.
//
// A gaussian survives when its opacity logit is at least L_o and each of its three log-scales is
// at most L_s (the opacity and size thresholds carried into the stored values' domains on the
// host; a NaN fails its comparison). Survivors are packed in index order into the output planes:
// the 14 planes of the parameters and the same columns of up to three companion blocks of the
// same layout (the Adam moments).
//
// Gaussians are taken in chunks of kChunk = 2048 (256 threads x 8 rounds; element r of a thread
// is chunk + r * 256 + thread, so every plane is read in whole 1 KiB rows per wave). Two or three
// launches:
//   k_prune_count:   the keep test; per chunk, the 32 wave ballots and the survivor count;
//   k_prune_offsets: one workgroup scans the chunk counts into exclusive offsets and the total
//     (maps above kFoldChunks chunks; below, each scatter workgroup sums the counts before its
//     chunk itself, which saves a launch);
//   k_prune_scatter: one workgroup per (chunk, group of kGroup planes): a survivor's position is
//     its chunk's offset plus the survivors of the earlier ballots and of the lower lanes of its
//     own; every thread loads its survivors of all the group's planes before it stores any, so
//     each wave keeps up to 56 loads in flight (the copy is bound by HBM latency otherwise: a
//     500k-gaussian map gives only some 1,000 waves per plane group).
// The test reads 16 bytes per gaussian; the copy reads and writes 56 bytes per block and survivor.
#include "fgs_internal.h"

namespace fgs {

namespace {

constexpr int kThreads = 256, kRounds = 8, kChunk = kThreads * kRounds;
constexpr int kWavesPB = kThreads / kWave;
constexpr int kSlots = kChunk / kWave;      // ballots of a chunk: slot q holds elements 64 q .. 64 q + 63
constexpr int kCountThreads = 1024;
constexpr int kGroup = 7;                   // planes per scatter workgroup
constexpr int kScanThreads = 1024;
constexpr int64_t kFoldChunks = 4096;       // chunks whose offsets the scatter sums itself (8M gaussians)

// One 1024-thread workgroup per chunk, two elements per thread, so that the test's loads of a
// chunk are spread over 16 waves. Ballot slot q of a chunk holds its elements 64 q .. 64 q + 63,
// whatever the workgroup shape that computes it.
__global__ void __launch_bounds__(kCountThreads)
k_prune_count(PruneK k, uint64_t *__restrict__ ballots, uint32_t *__restrict__ chunk_count)
{
    constexpr int kR = kChunk / kCountThreads, kW = kCountThreads / kWave;
    __shared__ uint32_t wcount[kW];
    const int tid = threadIdx.x, w = tid / kWave;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    uint32_t ok = 0;  // bit r: element of round r survives
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int64_t i = base + (int64_t)r * kCountThreads + tid;
        if (i < k.n && k.logit[i] >= k.L_o && k.ls0[i] <= k.L_s && k.ls1[i] <= k.L_s && k.ls2[i] <= k.L_s)
            ok |= 1u << r;
    }
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const uint64_t b = __ballot((ok >> r) & 1u);
        c += (uint32_t)__popcll(b);
        if (__lane_id() == 0) ballots[(int64_t)blockIdx.x * kSlots + r * kW + w] = b;
        const int64_t i = base + (int64_t)r * kCountThreads + tid;
        if (k.keep && i < k.n) k.keep[i] = (uint8_t)((ok >> r) & 1u);
    }
    if (__lane_id() == 0) wcount[w] = c;
    __syncthreads();
    if (tid < kWave) {
        uint32_t t = tid < kW ? wcount[tid] : 0u;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (tid == 0) chunk_count[blockIdx.x] = t;
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

// Offset of chunk b: the sum of the counts of the chunks before it, summed by the whole workgroup
// (up to kFoldChunks chunks: 16 loads per thread from L2). The workgroup of the last chunk's first
// plane group also writes the total.
__device__ uint32_t fold_offset(const uint32_t *__restrict__ chunk_count, int64_t nb, int64_t *total,
                                int64_t *total_out)
{
    __shared__ uint32_t part[kWavesPB];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    uint32_t t = 0;
    for (int64_t q = tid; q < b; q += kThreads) t += chunk_count[q];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (__lane_id() == 0) part[tid / kWave] = t;
    __syncthreads();
    uint32_t off = 0;
#pragma unroll
    for (int q = 0; q < kWavesPB; ++q) off += part[q];
    if (b == nb - 1 && blockIdx.y == 0 && tid == 0) {
        const int64_t all = (int64_t)off + chunk_count[b];
        *total = all;
        if (total_out) *total_out = all;
    }
    return off;
}

// chunk_off: the scanned offsets, or null to sum them here from chunk_count (nb <= kFoldChunks).
__global__ void __launch_bounds__(kThreads)
k_prune_scatter(PruneK k, const uint64_t *__restrict__ ballots, const uint32_t *__restrict__ chunk_off,
                const uint32_t *__restrict__ chunk_count, int64_t nb, int64_t *total, int64_t *total_out)
{
    const int tid = threadIdx.x, w = tid / kWave, lane = __lane_id();
    const int p0 = blockIdx.y * kGroup;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    const uint64_t *B = ballots + (int64_t)blockIdx.x * kSlots;
    const uint64_t below = (1ull << lane) - 1ull;
    // destination of this thread's element in each round (kept[r]: it survives)
    uint32_t pos[kRounds];
    bool kept[kRounds];
    uint32_t run = chunk_off ? chunk_off[blockIdx.x] : fold_offset(chunk_count, nb, total, total_out);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < kWavesPB; ++q) {
            const uint32_t c = (uint32_t)__popcll(B[r * kWavesPB + q]);
            before += q < w ? c : 0u;
            all += c;
        }
        const uint64_t mine = B[r * kWavesPB + w];
        kept[r] = (mine >> lane) & 1ull;
        pos[r] = run + before + (uint32_t)__popcll(mine & below);
        run += all;
    }
    float v[kGroup][kRounds];
#pragma unroll
    for (int j = 0; j < kGroup; ++j) {
        if (p0 + j >= k.n_planes) break;
        const float *__restrict__ sp = k.src[p0 + j];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) v[j][r] = kept[r] ? sp[base + (int64_t)r * kThreads + tid] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kGroup; ++j) {
        if (p0 + j >= k.n_planes) break;
        float *__restrict__ dp = k.dst[p0 + j];
#pragma unroll
        for (int r = 0; r < kRounds; ++r)
            if (kept[r]) dp[pos[r]] = v[j][r];
    }
}

}  // namespace

int64_t prune_chunks(int64_t n) { return (n + kChunk - 1) / kChunk; }

int64_t prune_ws_words(int64_t n)
{
    const int64_t nb = prune_chunks(n);
    const int64_t a = (nb * kSlots * 2 + 63) / 64 * 64, b = (nb + 63) / 64 * 64;
    return a + 2 * b;
}

void launch_prune(const PruneK &k, uint32_t *ws, int64_t *total, int64_t *total_out, hipStream_t s)
{
    const int64_t nb = prune_chunks(k.n);
    uint64_t *ballots = (uint64_t *)ws;
    uint32_t *count = ws + (nb * kSlots * 2 + 63) / 64 * 64;
    uint32_t *off = count + (nb + 63) / 64 * 64;
    if (nb > 0) hipLaunchKernelGGL(k_prune_count, dim3((unsigned)nb), dim3(kCountThreads), 0, s, k, ballots, count);
    // up to kFoldChunks chunks the scatter sums the offsets itself; beyond, one workgroup scans them
    const bool fold = nb > 0 && nb <= kFoldChunks && k.n_planes > 0;
    if (!fold) hipLaunchKernelGGL(k_prune_offsets, dim3(1), dim3(kScanThreads), 0, s, count, nb, off, total, total_out);
    if (nb > 0 && k.n_planes > 0)
        hipLaunchKernelGGL(k_prune_scatter, dim3((unsigned)nb, (unsigned)((k.n_planes + kGroup - 1) / kGroup)),
                           dim3(kThreads), 0, s, k, ballots, fold ? nullptr : off, count, nb, total, total_out);
}

}  // namespace fgs
