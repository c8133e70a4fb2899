// Binning of projected gaussians into screen tiles and the (tile, depth) ordering of every
// tile's list.
//
// Ordering scheme: the n gaussians are first sorted by depth (32-bit keys, the bits of the
// positive FP32 depth; ids emitted in ascending order and a stable sort, so equal depths keep
// ascending index). Every gaussian then emits one (tile, depth rank) pair per covered tile, in
// depth order. A stable sort of the pairs by tile alone leaves each tile's list ordered by
// (depth, index) - the pairs never need a depth key of their own.
//
// The radix sort is an LSD sort with 8-bit digits and a fixed grid: block b handles the b-th
// contiguous chunk of the input, whose length is read from device memory, so no host round
// trip is needed between passes. Per pass: a per-block digit histogram (LDS atomics), a
// per-digit scan over blocks, and a stable scatter that ranks equal digits inside a wave with
// ballots and across the block's waves with LDS counters.
#include "fgs_internal.h"

namespace fgs {

namespace {

constexpr int kSortThreads = 256;
constexpr int kScanItems = 4;  // elements per thread in the count scan
constexpr int kScanBlock = kSortThreads * kScanItems;

__device__ inline uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Block-wide exclusive scan of one u32 per thread (256 threads). Returns the prefix; *total
// receives the block sum. Uses 8 words of LDS passed in.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *lds_w, uint32_t *total)
{
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) lds_w[wid] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) {
        const uint32_t s = lds_w[w];
        off += w < wid ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__device__ inline void chunk_of(uint32_t n, int G, int b, uint32_t &lo, uint32_t &hi)
{
    uint32_t chunk = (n + G - 1) / G;
    chunk = (chunk + kSortThreads - 1) / kSortThreads * kSortThreads;
    lo = min((uint64_t)n, (uint64_t)chunk * b);
    hi = min((uint64_t)n, (uint64_t)chunk * (b + 1));
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_hist(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ n_dev, uint32_t n_cap, int shift,
             uint32_t mask, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = min(*n_dev, n_cap);
    uint32_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, lo, hi);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kSortThreads) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
    __syncthreads();
    hist[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of the digit's row over blocks, row total to totals.
__global__ void __launch_bounds__(kSortThreads)
k_radix_rowscan(uint32_t *__restrict__ hist, int G, uint32_t *__restrict__ totals)
{
    __shared__ uint32_t w[8];
    uint32_t *row = hist + (size_t)blockIdx.x * G;
    uint32_t carry = 0;
    for (int base = 0; base < G; base += kSortThreads) {
        const int j = base + threadIdx.x;
        const uint32_t v = j < G ? row[j] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, w, &tot);
        if (j < G) row[j] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
                uint32_t *__restrict__ vout, const uint32_t *__restrict__ n_dev, uint32_t n_cap, int shift,
                uint32_t mask, int bits, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ totals)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kSortThreads / kWave][256];
    __shared__ uint32_t w8[8];
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid / kWave;
    {
        uint32_t tot;
        const uint32_t ex = block_excl_scan(totals[tid], w8, &tot);
        base[tid] = ex + hist[(size_t)tid * gridDim.x + blockIdx.x];
    }
    const uint32_t n = min(*n_dev, n_cap);
    uint32_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, lo, hi);
    for (uint32_t it = lo; it < hi; it += kSortThreads) {
#pragma unroll
        for (int w = 0; w < kSortThreads / kWave; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const uint32_t i = it + tid;
        const bool valid = i < hi;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t d = (key >> shift) & mask;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lanemask_lt());
        if (valid && rank == 0) wcnt[wid][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = base[d] + rank;
            for (int w = 0; w < wid; ++w) off += wcnt[w][d];
            kout[off] = key;
            vout[off] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortThreads / kWave; ++w) add += wcnt[w][tid];
        base[tid] += add;
        // the next iteration's clear happens after this barrier-free update: every thread only
        // touches its own digit column here, and the clear above is followed by a barrier.
        __syncthreads();
    }
}

// Per block: sum of count[ids[r]] over the block's kScanBlock ranks.
__global__ void __launch_bounds__(kSortThreads)
k_count_reduce(const uint32_t *__restrict__ ids, const uint32_t *__restrict__ count, int64_t n,
               uint32_t *__restrict__ blocksums)
{
    __shared__ uint32_t w[8];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += count[ids[base + k]];
    uint32_t tot;
    block_excl_scan(s, w, &tot);
    if (threadIdx.x == 0) blocksums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums in place; the total number of pairs goes to
// blocksums[nb] and to the status words.
__global__ void __launch_bounds__(kSortThreads)
k_scan_top(uint32_t *__restrict__ blocksums, int nb, uint32_t *__restrict__ status)
{
    __shared__ uint32_t w[8];
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kSortThreads) {
        const int j = base + threadIdx.x;
        const uint32_t v = j < nb ? blocksums[j] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, w, &tot);
        if (j < nb) blocksums[j] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        blocksums[nb] = carry;
        status[ST_PAIRS] = carry;
        status[ST_VISIBLE] = 0;
    }
}

// Per-rank exclusive offsets: offsets[r] = block offset + prefix of count[ids[.]] inside the
// block (same partition as k_count_reduce); offsets[n] = total. Also gathers the records of
// the gaussians that cover at least one tile into depth order.
__global__ void __launch_bounds__(kSortThreads)
k_scan_apply(const uint32_t *__restrict__ ids, const uint32_t *__restrict__ count, const Rec *__restrict__ rec_by_id,
             int64_t n, const uint32_t *__restrict__ blocksums, int nb, uint32_t *__restrict__ offsets,
             Rec *__restrict__ rec_sorted)
{
    __shared__ uint32_t w[8];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint32_t c[kScanItems], id[kScanItems], s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        id[k] = base + k < n ? ids[base + k] : 0u;
        c[k] = base + k < n ? count[id[k]] : 0u;
        s += c[k];
    }
    uint32_t tot;
    uint32_t off = blocksums[blockIdx.x] + block_excl_scan(s, w, &tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) {
            offsets[base + k] = off;
            if (c[k]) rec_sorted[base + k] = rec_by_id[id[k]];
        }
        off += c[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[n] = blocksums[nb];
}

// Largest r in [lo, hi] with a[r] <= v (a non-decreasing, a[lo] <= v).
__device__ inline uint32_t last_le(const uint32_t *__restrict__ a, uint32_t lo, uint32_t hi, uint32_t v)
{
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo + 1) >> 1);
        if (a[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

constexpr uint32_t kEmitChunk = 4096;  // pairs per block iteration

// Load-balanced emission: the K pairs are cut into chunks of kEmitChunk consecutive pair
// indices; a block takes a chunk, finds the depth ranks it spans by binary search over the
// per-rank offsets, and its threads write consecutive pair indices (coalesced), each finding its
// rank by a binary search inside that span. A gaussian's pairs are its tile rectangle in
// row-major order.
__global__ void __launch_bounds__(kSortThreads)
k_emit(const uint32_t *__restrict__ ids, const uint2 *__restrict__ rect, const uint32_t *__restrict__ offsets,
       int64_t n, int32_t tiles_x, int64_t cap, uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
       uint32_t *__restrict__ status, uint32_t *__restrict__ n_pairs_dev, uint32_t *__restrict__ host_status)
{
    __shared__ uint32_t span[2];
    const uint32_t K = offsets[n];
    const uint32_t limit = (int64_t)K <= cap ? K : (uint32_t)cap;
    for (uint64_t chunk = blockIdx.x; chunk * kEmitChunk < limit; chunk += gridDim.x) {
        const uint32_t j0 = (uint32_t)(chunk * kEmitChunk);
        const uint32_t j1 = min(j0 + kEmitChunk, limit);
        if (threadIdx.x == 0) {
            span[0] = last_le(offsets, 0, (uint32_t)n, j0);
            span[1] = last_le(offsets, span[0], (uint32_t)n, j1 - 1);
        }
        __syncthreads();
        const uint32_t rlo = span[0], rhi = span[1];
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += kSortThreads) {
            const uint32_t r = last_le(offsets, rlo, rhi, j);
            const uint32_t idx = j - offsets[r];
            const uint2 rc = rect[ids[r]];
            const uint32_t tx0 = rc.x & 0xFFFFu, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFFu;
            const uint32_t w = tx1 - tx0 + 1;
            const uint32_t dy = idx / w;
            keys[j] = (ty0 + dy) * (uint32_t)tiles_x + tx0 + (idx - dy * w);
            vals[j] = r;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // On overflow nothing is sorted or rendered (the pairs that were written are not a
        // complete set); the condition is recorded and reported by the next status check.
        const bool ovf = (int64_t)K > cap;
        *n_pairs_dev = ovf ? 0u : K;
        if (ovf) atomicMax(&status[ST_OVERFLOW], K);
        if (host_status) {
            host_status[0] = K;
            if (ovf) host_status[1] = 1u;
            __threadfence_system();
        }
    }
}

__global__ void __launch_bounds__(kSortThreads)
k_visible(const uint32_t *__restrict__ count, int64_t n, uint32_t *__restrict__ status)
{
    __shared__ uint32_t w[8];
    uint32_t s = 0;
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSortThreads)
        s += count[i] != 0;
    uint32_t tot;
    block_excl_scan(s, w, &tot);
    if (threadIdx.x == 0 && tot) atomicAdd(&status[ST_VISIBLE], tot);
}

__device__ inline uint32_t lower_bound_u32(const uint32_t *__restrict__ a, uint32_t n, uint32_t v)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// [start, end) of every tile's run in the sorted keys, by two binary searches per tile.
__global__ void __launch_bounds__(kSortThreads)
k_ranges(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ n_dev, uint2 *__restrict__ ranges, int64_t T)
{
    const int64_t t = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
    if (t >= T) return;
    const uint32_t K = *n_dev;
    ranges[t] = make_uint2(lower_bound_u32(keys, K, (uint32_t)t), lower_bound_u32(keys, K, (uint32_t)t + 1));
}

// Queue keys of a window: item g (tile g - tile_base of its view) gets the key 2^24 - 1 - (its list
// length, clamped), so a stable ascending sort puts the longest lists first; *n_out = total.
__global__ void __launch_bounds__(kSortThreads)
k_queue_keys(const ViewK *__restrict__ views, int nv, uint32_t total, uint32_t *__restrict__ keys,
             uint32_t *__restrict__ vals, uint32_t *__restrict__ n_out)
{
    const uint32_t g = blockIdx.x * kSortThreads + threadIdx.x;
    if (g == 0) *n_out = total;
    if (g >= total) return;
    int v = 0;
    while (v + 1 < nv && views[v + 1].tile_base <= g) ++v;
    const uint2 r = views[v].ranges[g - views[v].tile_base];
    const uint32_t len = min(r.y - r.x, 0xFFFFFFu);
    keys[g] = 0xFFFFFFu - len;
    vals[g] = g;
}

__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

void launch_queue_order(const ViewK *views_dev, int nv, uint32_t total, uint32_t *ka, uint32_t *va, uint32_t *kb,
                        uint32_t *vb, uint32_t *queue, uint32_t *n_dev, const SortWS &ws, hipStream_t s)
{
    hipLaunchKernelGGL(k_queue_keys, dim3((total + kSortThreads - 1) / kSortThreads), dim3(kSortThreads), 0, s, views_dev,
                       nv, total, ka, va, n_dev);
    launch_radix_sort(ka, va, kb, vb, queue, n_dev, total, 24, ws, s);
}

int sort_blocks(int64_t cap)
{
    int64_t G = (cap + 2047) / 2048;
    if (G < 1) G = 1;
    if (G > 4096) G = 4096;
    return (int)G;
}

static unsigned grid_for(int64_t n, int per_block, unsigned max_blocks)
{
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (unsigned)b;
}

void launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 1024, 2048)), dim3(256), 0, s, p, n);
}

void launch_zero_f32(float *p, int64_t n, hipStream_t s) { launch_zero_u32((uint32_t *)p, n, s); }

uint32_t *launch_radix_sort(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, uint32_t *v_final,
                            const uint32_t *n_dev, int64_t n_cap, int key_bits, const SortWS &ws, hipStream_t s)
{
    // Pass p reads (src) and writes (dst); src/dst alternate between the a and b buffers. The last
    // pass writes its values to v_final (which must not alias va or vb) and its keys to its usual
    // destination, which is returned.
    const int passes = key_bits <= 0 ? 1 : (key_bits + 7) / 8;
    uint32_t *sk = ka, *sv = va, *dk = kb, *dv = vb;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const int bits = key_bits - shift < 8 ? (key_bits - shift > 0 ? key_bits - shift : 1) : 8;
        const uint32_t mask = (1u << bits) - 1u;
        uint32_t *ok = dk, *ov = p == passes - 1 ? v_final : dv;
        hipLaunchKernelGGL(k_radix_hist, dim3(ws.G), dim3(kSortThreads), 0, s, sk, n_dev, (uint32_t)n_cap, shift,
                           mask, ws.hist);
        hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kSortThreads), 0, s, ws.hist, ws.G, ws.totals);
        hipLaunchKernelGGL(k_radix_scatter, dim3(ws.G), dim3(kSortThreads), 0, s, sk, sv, ok, ov, n_dev,
                           (uint32_t)n_cap, shift, mask, bits, ws.hist, ws.totals);
        if (p == passes - 1) return ok;
        sk = dk; sv = dv;
        dk = (dk == kb) ? ka : kb;
        dv = (dv == vb) ? va : vb;
    }
    return nullptr;
}

int64_t scan_blocks(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

void launch_scan_counts(const uint32_t *ids, const uint32_t *count, int64_t n, uint32_t *blocksums,
                        uint32_t *status, hipStream_t s)
{
    const int nb = (int)scan_blocks(n);
    if (nb > 0)
        hipLaunchKernelGGL(k_count_reduce, dim3(nb), dim3(kSortThreads), 0, s, ids, count, n, blocksums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kSortThreads), 0, s, blocksums, nb, status);
    hipLaunchKernelGGL(k_visible, dim3(grid_for(n, 4096, 256)), dim3(kSortThreads), 0, s, count, n, status);
}

void launch_emit(const uint32_t *ids, const uint32_t *count, const uint2 *rect, const Rec *rec_by_id,
                 const uint32_t *blocksums, uint32_t *offsets, int64_t n, int32_t tiles_x, int64_t cap, uint32_t *keys,
                 uint32_t *vals, Rec *rec_sorted, uint32_t *status, uint32_t *n_pairs_dev, uint32_t *host_status,
                 hipStream_t s)
{
    // blocksums holds the scanned per-block sums in [0, nb) and the total at [nb]
    const int nb = (int)scan_blocks(n);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb > 0 ? nb : 1), dim3(kSortThreads), 0, s, ids, count, rec_by_id, n,
                       blocksums, nb, offsets, rec_sorted);
    hipLaunchKernelGGL(k_emit, dim3(grid_for(cap, kEmitChunk, 2048)), dim3(kSortThreads), 0, s, ids, rect, offsets, n,
                       tiles_x, cap, keys, vals, status, n_pairs_dev, host_status);
}

void launch_ranges(const uint32_t *keys, const uint32_t *n_pairs_dev, int64_t cap, uint2 *ranges, int64_t T,
                   hipStream_t s)
{
    (void)cap;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((T + kSortThreads - 1) / kSortThreads)), dim3(kSortThreads), 0, s,
                       keys, n_pairs_dev, ranges, T);
}

}  // namespace fgs
