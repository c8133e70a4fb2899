// Binning of projected gaussians into screen tiles and the (tile, depth) ordering of every
// tile's list.
//
// Ordering scheme of one view: every gaussian has one (super-tile, id) pair per covered square of
// kSuper x kSuper tiles; the pairs are placed into per-super-tile lists in id order (up to 256
// super-tiles straight from the projection's per-workgroup histograms by k_super_scatter, else
// emitted in id order and sorted stably by super-tile), and each list is then put in (depth,
// index) order by a sort of its own on the depth keys (k_seg_chunk_sort, k_seg_merge: stable, so
// equal depths keep ascending index). An in-order expansion of each super-tile list into the lists of its tiles keeps
// that order. The result is exactly the stable (tile, depth, index) order of one pair per covered
// tile, while the sorts only move one pair per covered super-tile. A keyframe window orders all
// its views at once the other way round: the gaussians of every view are sorted by depth first
// (ids in ascending order and a stable sort), their pairs emitted in that order and sorted stably
// by super-tile.
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
// The count scan takes 2 ranks per thread up to 2^20 ranks (more workgroups to hide the gathers'
// latency), else 4. Each apply workgroup adds the block sums before it itself while there are at
// most kScanFold workgroups; beyond that a single-workgroup pass scans them first.
constexpr int kScanFold = 4096;
__host__ __device__ inline int scan_items(int64_t n) { return n <= ((int64_t)1 << 20) ? 2 : 4; }
constexpr uint32_t kEmitChunk = 1024;  // pairs per emission block iteration
constexpr uint32_t kEmitSpan = 2048;   // ranks of a chunk's offsets staged in LDS

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

// One block per digit: exclusive scan of the digit's row over blocks, row total to totals. Each
// thread scans a contiguous run of the row serially, so one block-wide scan covers rows of up to
// 256 x kRowRun blocks (longer rows take several rounds).
constexpr int kRowRun = 16;
__device__ inline void sum_kpart(const uint32_t *__restrict__ kpart, int npb, uint32_t *__restrict__ status,
                                 uint32_t *__restrict__ ktotal, uint32_t *w);

// kpart (nullable): block 0 also sums the projection's counts (see sum_kpart).
__global__ void __launch_bounds__(kSortThreads)
k_radix_rowscan(uint32_t *__restrict__ hist, int G, uint32_t *__restrict__ totals, const uint32_t *__restrict__ kpart,
                int npb, uint32_t *__restrict__ status, uint32_t *__restrict__ ktotal)
{
    __shared__ uint32_t w[8];
    uint32_t *row = hist + (size_t)blockIdx.x * G;
    const int per = min((G + kSortThreads - 1) / kSortThreads, kRowRun);
    uint32_t carry = 0;
    for (int base = 0; base < G; base += per * kSortThreads) {
        const int j0 = base + threadIdx.x * per;
        uint32_t v[kRowRun], sum = 0;
#pragma unroll
        for (int k = 0; k < kRowRun; ++k) {
            v[k] = k < per && j0 + k < G ? row[j0 + k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t ex = carry + block_excl_scan(sum, w, &tot);
#pragma unroll
        for (int k = 0; k < kRowRun; ++k)
            if (k < per && j0 + k < G) {
                row[j0 + k] = ex;
                ex += v[k];
            }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
    if (kpart && blockIdx.x == 0) sum_kpart(kpart, npb, status, ktotal, w);
}

// Stable scatter of the workgroup's chunk by one digit, through LDS (for digits spread over many
// values, where k_radix_scatter's stores would each hit a different line): each tile of up to
// kScatterTile keys is first ordered by digit in LDS (rounds of 256 keys in order; within a round
// each lane is ranked among the lanes of its wave holding the same digit, one ballot per digit
// bit, and the waves before it are counted through wcnt), then written out in that order, so
// that the consecutive lanes of a store land in a few runs of consecutive slots instead of one
// slot per digit.
constexpr int kScatterItems = 8, kScatterTile = kSortThreads * kScatterItems;

__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter_lds(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
                    uint32_t *__restrict__ vout, const uint32_t *__restrict__ n_dev, uint32_t n_cap, int shift,
                    uint32_t mask, int bits, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ totals)
{
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint32_t gbase[256];  // next global slot of each digit
    __shared__ uint32_t tstart[256];  // first tile slot of each digit
    __shared__ uint32_t run[256];     // digit counts of the tile, then its next tile slots
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint32_t skey[kScatterTile], sval[kScatterTile];
    __shared__ uint32_t w8[8];
    const int tid = threadIdx.x, wid = tid / kWave;
    {
        uint32_t tot;
        const uint32_t ex = block_excl_scan(totals[tid], w8, &tot);
        gbase[tid] = ex + hist[(size_t)tid * gridDim.x + blockIdx.x];
        run[tid] = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) wcnt[w][tid] = 0;
    }
    __syncthreads();
    const uint32_t n = min(*n_dev, n_cap);
    uint32_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, lo, hi);
    for (uint32_t t0 = lo; t0 < hi; t0 += kScatterTile) {
        const uint32_t nt = min((uint32_t)kScatterTile, hi - t0);
        const int rounds = (int)((nt + kSortThreads - 1) / kSortThreads);
        uint32_t key[kScatterItems], val[kScatterItems], rank[kScatterItems], cnt[kScatterItems];
        // the tile's digit counts (one add per wave and digit)
#pragma unroll
        for (int r = 0; r < kScatterItems; ++r) {
            if (r >= rounds) break;
            const uint32_t i = t0 + (uint32_t)(r * kSortThreads + tid);
            const bool valid = i < hi;
            key[r] = valid ? kin[i] : 0u;
            val[r] = valid ? vin[i] : 0u;
            const uint32_t d = (key[r] >> shift) & mask;
            uint64_t peers = __ballot(valid);
            for (int b = 0; b < bits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            rank[r] = valid ? __popcll(peers & lanemask_lt()) : kSortThreads;  // invalid: no leader
            cnt[r] = __popcll(peers);
            if (rank[r] == 0) atomicAdd(&run[d], cnt[r]);
        }
        __syncthreads();
        {
            uint32_t tot;
            const uint32_t c = run[tid];
            tstart[tid] = block_excl_scan(c, w8, &tot);  // (synchronizes the block)
            run[tid] = tstart[tid];
        }
        // local slots, round by round: the leaders publish their wave's count of their digit,
        // every lane adds the waves before it, then the leaders advance their digit's slot
#pragma unroll
        for (int r = 0; r < kScatterItems; ++r) {
            if (r >= rounds) break;
            const uint32_t d = (key[r] >> shift) & mask;
            if (rank[r] == 0) wcnt[wid][d] = cnt[r];
            __syncthreads();
            if (rank[r] < (uint32_t)kSortThreads) {
                uint32_t pos = run[d] + rank[r];
                for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
                skey[pos] = key[r];
                sval[pos] = val[r];
            }
            __syncthreads();
            if (rank[r] == 0) {
                atomicAdd(&run[d], cnt[r]);
                wcnt[wid][d] = 0;
            }
        }
        __syncthreads();
        // out in tile order: slot j of digit d goes to gbase[d] + (j - tstart[d])
        for (uint32_t j = tid; j < nt; j += kSortThreads) {
            const uint32_t k = skey[j], d = (k >> shift) & mask;
            const uint32_t g = gbase[d] + (j - tstart[d]);
            kout[g] = k;
            vout[g] = sval[j];
        }
        __syncthreads();
        gbase[tid] += run[tid] - tstart[tid];
        run[tid] = 0;
        __syncthreads();
    }
}

// Stable scatter of the workgroup's chunk by one digit, straight to memory: 256 keys per round,
// each lane ranked among the lanes of its wave holding the same digit (one ballot per digit bit),
// the waves before it counted through wcnt. Right for a digit with few distinct values (the
// keys' top bits), whose rounds already land in long runs.
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

// Per block: sum of count[ids[r]] over the block's 256 ITEMS ranks.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_count_reduce(const uint32_t *__restrict__ ids, const uint32_t *__restrict__ count, int64_t n,
               uint32_t *__restrict__ blocksums)
{
    __shared__ uint32_t w[8];
    const int64_t base = ((int64_t)blockIdx.x * kSortThreads + threadIdx.x) * ITEMS;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (base + k < n) s += count[ids[base + k]];
    uint32_t tot;
    block_excl_scan(s, w, &tot);
    if (threadIdx.x == 0) blocksums[blockIdx.x] = tot;
}


// Single block: exclusive scan of the block sums in place (the pass before k_scan_apply when there
// are more than kScanFold of them). Also sums the projection's per-block counts (kpart, npb
// blocks) into *ktotal, status[ST_PAIRS] (tile pairs) and status[ST_VISIBLE].
__device__ inline void sum_kpart(const uint32_t *__restrict__ kpart, int npb, uint32_t *__restrict__ status,
                                 uint32_t *__restrict__ ktotal, uint32_t *w)
{
    uint32_t pairs = 0, vis = 0;
    for (int j = threadIdx.x; j < npb; j += kSortThreads) {
        pairs += kpart[2 * j];
        vis += kpart[2 * j + 1];
    }
    uint32_t tp, tv;
    block_excl_scan(pairs, w, &tp);
    block_excl_scan(vis, w, &tv);
    if (threadIdx.x == 0) {
        *ktotal = tp;
        status[ST_PAIRS] = tp;
        status[ST_VISIBLE] = tv;
    }
}

__global__ void __launch_bounds__(kSortThreads)
k_scan_top(uint32_t *__restrict__ blocksums, int nb, uint32_t *__restrict__ status, const uint32_t *__restrict__ kpart,
           int npb, uint32_t *__restrict__ ktotal)
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
    sum_kpart(kpart, npb, status, ktotal, w);
}

// Per-rank exclusive offsets: offsets[r] = block offset + prefix of count[ids[.]] inside the
// block (same partition as k_count_reduce); offsets[n] = total. Also gathers the tile rectangles
// of the gaussians that cover at least one tile into rank order, and the first rank of every
// emission chunk.
// scanned: blocksums already hold exclusive prefixes (k_scan_top ran); otherwise each block adds
// the block sums before it and block 0 sums the projection's counts.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_scan_apply(const uint32_t *__restrict__ ids, const uint32_t *__restrict__ count, const uint2 *__restrict__ rect,
             int64_t n, const uint32_t *__restrict__ blocksums, bool scanned, uint32_t *__restrict__ offsets,
             uint2 *__restrict__ rect_sorted, uint32_t *__restrict__ start_rank, uint32_t max_chunks,
             uint32_t *__restrict__ status, const uint32_t *__restrict__ kpart, int npb,
             uint32_t *__restrict__ ktotal, uint32_t per)
{
    __shared__ uint32_t w[8];
    // this block's first offset: the sum of the block sums before it (per of them for each block of
    // this scan: 1 for k_count_reduce's, ITEMS for the projection's workgroups of 256 gaussians)
    uint32_t boff;
    if (scanned) {
        boff = blocksums[blockIdx.x * per];
    } else {
        uint32_t pre = 0;
        for (uint32_t j = threadIdx.x; j < blockIdx.x * per; j += kSortThreads) pre += blocksums[j];
        block_excl_scan(pre, w, &boff);
        if (blockIdx.x == 0) sum_kpart(kpart, npb, status, ktotal, w);
    }
    const int64_t base = ((int64_t)blockIdx.x * kSortThreads + threadIdx.x) * ITEMS;
    uint32_t c[ITEMS], id[ITEMS], s = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        id[k] = base + k < n ? ids[base + k] : 0u;
        c[k] = base + k < n ? count[id[k]] : 0u;
        s += c[k];
    }
    uint32_t tot;
    uint32_t off = boff + block_excl_scan(s, w, &tot);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        if (base + k < n) {
            offsets[base + k] = off;
            if (c[k]) {
                rect_sorted[base + k] = rect[id[k]];
                // emission chunks whose first pair belongs to this rank
                for (uint32_t q = (off + kEmitChunk - 1) / kEmitChunk; q < (off + c[k] + kEmitChunk - 1) / kEmitChunk &&
                                                                      q < max_chunks;
                     ++q)
                    start_rank[q] = (uint32_t)(base + k);
            }
        }
        off += c[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) offsets[n] = boff + tot;  // the last block: the total
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

// depth order inside the super-tile lists (k_seg_chunk_sort, k_seg_merge)
constexpr int kSegItems = 16;
constexpr int kChunkThreads = 512, kSegChunk = kChunkThreads * kSegItems;  // 8,192 entries per chunk
constexpr int kMergeThreads = 1024, kMergeLds = 16384;  // lists up to kMergeLds keys merge in LDS
constexpr uint32_t kBinChunk = 512;    // super-tile list entries per expansion chunk

// The tiles of super-tile (sx, sy) that a gaussian's tile rectangle rc covers, as a box of
// super-tile-local tile coordinates: lx0 | lx1 << 2 | ly0 << 4 | ly1 << 6 (never empty when the
// super-tile lies in the rectangle's super-tile range).
__device__ inline uint32_t cover_box(uint2 rc, uint32_t sx, uint32_t sy)
{
    const int x0 = (int)(sx * kSuper), y0 = (int)(sy * kSuper);
    const int lx0 = max((int)(rc.x & 0xFFFFu) - x0, 0), lx1 = min((int)(rc.x >> 16) - x0, kSuper - 1);
    const int ly0 = max((int)(rc.y & 0xFFFFu) - y0, 0), ly1 = min((int)(rc.y >> 16) - y0, kSuper - 1);
    return (uint32_t)lx0 | (uint32_t)lx1 << 2 | (uint32_t)ly0 << 4 | (uint32_t)ly1 << 6;
}

// The super-tile pairs of one view straight from the projection, for at most 256 super-tiles (one
// 8-bit digit): a workgroup per projection workgroup b of 256 gaussians generates b's pairs in
// gaussian order (per gaussian its covered super-tiles row by row, each key carrying the box of
// covered tiles above kBoxShift, the value the gaussian's id) and scatters them stably by
// super-tile, kScatterTile at a time through LDS like k_radix_scatter_lds, to the offsets of hist
// (the projection's per-workgroup super-tile counts, hist[s G + b], scanned per super-tile by
// k_radix_rowscan) after the totals of the super-tiles before. The lists come out in gaussian
// order. Nothing is written when the (tile, gaussian) pairs *ktotal exceed cap. One more
// workgroup (the last) writes the lists' ranges and chunk tables (as k_bin_chunks; empty on
// overflow).
__device__ void chunk_tables(uint2 *__restrict__ sranges, const uint32_t *__restrict__ digit_totals, int nsup,
                             uint32_t *__restrict__ cstart, uint32_t *__restrict__ csuper, uint32_t max_chunks,
                             uint32_t *__restrict__ nchunks, uint32_t *__restrict__ sstart, uint32_t smax, bool ovf,
                             uint32_t *w);

__global__ void __launch_bounds__(kSortThreads)
k_super_scatter(const uint2 *__restrict__ rect, const uint32_t *__restrict__ count, int64_t n, int32_t supers_x,
                const uint32_t *__restrict__ hist, const uint32_t *__restrict__ totals,
                const uint32_t *__restrict__ ktotal, int64_t cap, uint32_t *__restrict__ kout,
                uint32_t *__restrict__ vout, uint2 *__restrict__ sranges, int nsup, uint32_t *__restrict__ cstart,
                uint32_t *__restrict__ csuper, uint32_t max_chunks, uint32_t *__restrict__ nchunks,
                uint32_t *__restrict__ sstart, uint32_t smax)
{
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint32_t gbase[256];   // next global slot of each super-tile
    __shared__ uint32_t tstart[256];  // first tile slot of each super-tile
    __shared__ uint32_t run[256];     // super-tile counts of the tile, then its next tile slots
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint32_t skey[kScatterTile], sval[kScatterTile];
    __shared__ uint32_t soff[kSortThreads];  // the gaussians' first pair in the workgroup
    __shared__ uint2 srect[kSortThreads];
    __shared__ uint32_t w8[8];
    const int tid = threadIdx.x, wid = tid / kWave;
    const uint32_t G = gridDim.x - 1;  // the projection's workgroups; the last one writes the tables
    const bool ovf = (int64_t)*ktotal > cap;  // (uniform) overflow: nothing is placed
    if (blockIdx.x == G) {
        chunk_tables(sranges, totals, nsup, cstart, csuper, max_chunks, nchunks, sstart, smax, ovf, w8);
        return;
    }
    // every load that does not depend on another issued first
    const int64_t gi = (int64_t)blockIdx.x * kSortThreads + tid;
    const uint32_t c = gi < n ? count[gi] : 0u;
    const uint2 rc0 = gi < n ? rect[gi] : make_uint2(1u, 0u);
    const uint32_t tv = totals[tid], hv = hist[(size_t)tid * G + blockIdx.x];
    if (ovf) return;
    {
        uint32_t tot;
        const uint32_t ex = block_excl_scan(tv, w8, &tot);
        gbase[tid] = ex + hv;
        run[tid] = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) wcnt[w][tid] = 0;
    }
    uint32_t P;
    soff[tid] = block_excl_scan(c, w8, &P);  // (synchronizes the block)
    srect[tid] = rc0;
    __syncthreads();
    for (uint32_t t0 = 0; t0 < P; t0 += kScatterTile) {
        const uint32_t nt = min((uint32_t)kScatterTile, P - t0);
        const int rounds = (int)((nt + kSortThreads - 1) / kSortThreads);
        uint32_t key[kScatterItems], val[kScatterItems], rank[kScatterItems], cnt[kScatterItems];
        // the tile's pairs and their super-tile counts (one add per wave and super-tile)
#pragma unroll
        for (int r = 0; r < kScatterItems; ++r) {
            if (r >= rounds) break;
            const uint32_t j = t0 + (uint32_t)(r * kSortThreads + tid);
            const bool valid = j < t0 + nt;
            key[r] = 0u;
            val[r] = 0u;
            if (valid) {
                const uint32_t g = last_le(soff, 0, kSortThreads - 1, j);  // the gaussian holding pair j
                const uint32_t idx = j - soff[g];
                const uint2 rc = srect[g];
                const uint32_t sx0 = (rc.x & 0xFFFFu) >> kSuperShift, sx1 = (rc.x >> 16) >> kSuperShift;
                const uint32_t sy0 = (rc.y & 0xFFFFu) >> kSuperShift;
                const uint32_t wd = sx1 - sx0 + 1;
                const uint32_t dy = idx / wd;
                const uint32_t kx = sx0 + (idx - dy * wd), ky = sy0 + dy;
                key[r] = (ky * (uint32_t)supers_x + kx) | cover_box(rc, kx, ky) << kBoxShift;
                val[r] = (uint32_t)(blockIdx.x * kSortThreads) + g;
            }
            const uint32_t d = key[r] & 0xFFu;
            uint64_t peers = __ballot(valid);
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            rank[r] = valid ? __popcll(peers & lanemask_lt()) : kSortThreads;  // invalid: no leader
            cnt[r] = __popcll(peers);
            if (rank[r] == 0) atomicAdd(&run[d], cnt[r]);
        }
        __syncthreads();
        {
            uint32_t tot;
            const uint32_t c2 = run[tid];
            tstart[tid] = block_excl_scan(c2, w8, &tot);  // (synchronizes the block)
            run[tid] = tstart[tid];
        }
        // local slots, round by round: the leaders publish their wave's count of their super-tile,
        // every lane adds the waves before it, then the leaders advance their super-tile's slot
#pragma unroll
        for (int r = 0; r < kScatterItems; ++r) {
            if (r >= rounds) break;
            const uint32_t d = key[r] & 0xFFu;
            if (rank[r] == 0) wcnt[wid][d] = cnt[r];
            __syncthreads();
            if (rank[r] < (uint32_t)kSortThreads) {
                uint32_t pos = run[d] + rank[r];
                for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
                skey[pos] = key[r];
                sval[pos] = val[r];
            }
            __syncthreads();
            if (rank[r] == 0) {
                atomicAdd(&run[d], cnt[r]);
                wcnt[wid][d] = 0;
            }
        }
        __syncthreads();
        // out in tile order: slot j of super-tile d goes to gbase[d] + (j - tstart[d])
        for (uint32_t j = tid; j < nt; j += kSortThreads) {
            const uint32_t k = skey[j], d = k & 0xFFu;
            const uint32_t gpos = gbase[d] + (j - tstart[d]);
            kout[gpos] = k;
            vout[gpos] = sval[j];
        }
        __syncthreads();
        gbase[tid] += run[tid] - tstart[tid];
        run[tid] = 0;
        __syncthreads();
    }
}

// Load-balanced emission: the K pairs are cut into chunks of kEmitChunk consecutive pair
// indices; a block takes a chunk, finds the ranks it spans by binary search over the
// per-rank offsets, and its threads write consecutive pair indices (coalesced), each finding its
// rank by a binary search inside that span. A gaussian's pairs are its tile rectangle in
// row-major order; each pair carries the gaussian's id.
__global__ void __launch_bounds__(kSortThreads)
k_emit(const uint2 *__restrict__ rect_sorted, const uint32_t *__restrict__ ids, const uint32_t *__restrict__ offsets,
       const uint32_t *__restrict__ start_rank, int64_t n, int32_t tiles_x, int shift, int64_t cap,
       const uint2 *__restrict__ view_tab, uint32_t view_n, uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
       uint32_t *__restrict__ status, uint32_t *__restrict__ n_pairs_dev, uint32_t *__restrict__ host_status)
{
    __shared__ uint32_t soff[kEmitSpan];
    const uint32_t K = offsets[n];
    const uint32_t limit = (int64_t)K <= cap ? K : 0u;  // beyond the capacity nothing is emitted
    for (uint64_t chunk = blockIdx.x; chunk * kEmitChunk < limit; chunk += gridDim.x) {
        const uint32_t j0 = (uint32_t)(chunk * kEmitChunk);
        const uint32_t j1 = min(j0 + kEmitChunk, limit);
        // ranks holding pairs j0 and j1 (the table of first ranks per chunk; the last chunk ends
        // at the last rank)
        const uint32_t rlo = start_rank[chunk];
        const uint32_t rhi = j1 < K ? start_rank[chunk + 1] : (uint32_t)(n - 1);
        // the span's offsets in LDS when they fit (searched there), else searched in place
        const bool staged = rhi - rlo < kEmitSpan;
        if (staged)
            for (uint32_t k = threadIdx.x; k <= rhi - rlo; k += kSortThreads) soff[k] = offsets[rlo + k];
        __syncthreads();
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += kSortThreads) {
            uint32_t r, idx;
            if (staged) {
                const uint32_t q = last_le(soff, 0, rhi - rlo, j);
                r = rlo + q;
                idx = j - soff[q];
            } else {
                r = last_le(offsets, rlo, rhi, j);
                idx = j - offsets[r];
            }
            const uint2 rc = rect_sorted[r];
            const uint32_t tx0 = (rc.x & 0xFFFFu) >> shift, tx1 = (rc.x >> 16) >> shift, ty0 = (rc.y & 0xFFFFu) >> shift;
            const uint32_t w = tx1 - tx0 + 1;
            const uint32_t dy = idx / w;
            const uint32_t kx = tx0 + (idx - dy * w), ky = ty0 + dy;
            const uint32_t id = ids[r];
            // several views: the value is v view_n + i; keys count on from view v's first key and
            // the value emitted is i, the id within its view
            const uint32_t v = view_tab ? id / view_n : 0u;
            const uint2 vt = view_tab ? view_tab[v] : make_uint2((uint32_t)tiles_x, 0u);
            uint32_t key = vt.y + ky * vt.x + kx;
            if (shift > 0) key |= cover_box(rc, kx, ky) << kBoxShift;
            keys[j] = key;
            vals[j] = id - v * view_n;
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

/* ------------------------- tile lists from super-tile lists ------------------------- */
// A super-tile is a square of kSuper x kSuper tiles. Every gaussian first emits one pair per
// covered super-tile and the pairs are sorted by super-tile, each super-tile's list ending in
// (depth, index) order; each list is then cut into chunks of kBinChunk entries, and a workgroup
// per chunk expands its entries into the tiles they cover: a count pass, a prefix over the
// super-tile's chunks and over all tiles, and a placement pass. Entries keep the list's order
// within every tile (chunks are placed in order), so the tile lists are exactly the stable (tile,
// depth, index) order.

// Chunk table: chunk c covers entries [sranges[s].x + (c - cstart[s]) kBinChunk, ...) of
// super-tile s = csuper[c]; *nchunks = number of chunks (capped at max_chunks).
__device__ void chunk_tables(uint2 *__restrict__ sranges, const uint32_t *__restrict__ digit_totals, int nsup,
                             uint32_t *__restrict__ cstart, uint32_t *__restrict__ csuper, uint32_t max_chunks,
                             uint32_t *__restrict__ nchunks, uint32_t *__restrict__ sstart, uint32_t smax, bool ovf,
                             uint32_t *w)
{
    if (digit_totals) {
        // one radix pass sorted the super-tile keys: their ranges are the scanned digit totals
        // (empty when the pairs overflowed the capacity: nothing was placed)
        uint32_t carry = 0;
        for (int base = 0; base < nsup; base += kSortThreads) {
            const int sidx = base + threadIdx.x;
            const uint32_t v = sidx < nsup && !ovf ? digit_totals[sidx] : 0u;
            uint32_t tot;
            const uint32_t ex = carry + block_excl_scan(v, w, &tot);
            if (sidx < nsup) sranges[sidx] = make_uint2(ex, ex + v);
            carry += tot;
        }
        __syncthreads();
    }
    uint32_t carry = 0, scarry = 0;
    for (int base = 0; base < nsup; base += kSortThreads) {
        const int sidx = base + threadIdx.x;
        uint32_t nch = 0, nsc = 0;
        if (sidx < nsup) {
            const uint2 r = sranges[sidx];
            nch = (r.y - r.x + kBinChunk - 1) / kBinChunk;
            nsc = (r.y - r.x + kSegChunk - 1) / kSegChunk;
        }
        uint32_t tot;
        const uint32_t ex = carry + block_excl_scan(nch, w, &tot);
        if (sidx < nsup) {
            cstart[sidx] = ex;
            for (uint32_t c = 0; c < nch && ex + c < max_chunks; ++c) csuper[ex + c] = (uint32_t)sidx;
        }
        carry += tot;
        if (sstart) {
            // the depth-order chunks of kSegChunk entries: first chunk of every super-tile, and
            // after the nsup + 1 starts the super-tile of every chunk (at most smax chunks)
            const uint32_t sex = scarry + block_excl_scan(nsc, w, &tot);
            if (sidx < nsup) {
                sstart[sidx] = sex;
                for (uint32_t k = 0; k < nsc && sex + k < smax; ++k) sstart[nsup + 1 + sex + k] = (uint32_t)sidx;
            }
            scarry += tot;
        }
    }
    if (threadIdx.x == 0) {
        cstart[nsup] = carry;
        *nchunks = min(carry, max_chunks);
        if (sstart) sstart[nsup] = scarry;
    }
}

__global__ void __launch_bounds__(kSortThreads)
k_bin_chunks(uint2 *__restrict__ sranges, const uint32_t *__restrict__ digit_totals, int nsup,
             uint32_t *__restrict__ cstart, uint32_t *__restrict__ csuper, uint32_t max_chunks,
             uint32_t *__restrict__ nchunks, uint32_t *__restrict__ sstart, uint32_t smax,
             const uint32_t *__restrict__ ktotal, int64_t cap)
{
    __shared__ uint32_t w[8];
    chunk_tables(sranges, digit_totals, nsup, cstart, csuper, max_chunks, nchunks, sstart, smax,
                 ktotal && (int64_t)*ktotal > cap, w);
}

// Coverage of one super-tile entry from the box in its key's top byte: bit (ly * kSuper + lx)
// for each tile of the super-tile inside the box (never empty).
__device__ inline uint32_t box_bits(uint32_t key)
{
    const uint32_t b = key >> kBoxShift;
    const uint32_t lx0 = b & 3u, lx1 = (b >> 2) & 3u, ly0 = (b >> 4) & 3u, ly1 = (b >> 6) & 3u;
    const uint32_t row = ((1u << (lx1 - lx0 + 1u)) - 1u) << lx0;
    const uint32_t rows = 0x1111u & (0xFFFFu << (4u * ly0)) & (0xFFFFu >> (4u * (3u - ly1)));
    return row * rows;  // row < 16: the product places one copy of row per selected row
}

struct ChunkSpan {
    uint32_t e0, e1, s;
};

// Chunk c's entries [e0, e1) of super-tile s.
__device__ inline ChunkSpan chunk_span(uint32_t c, const uint2 *sranges, const uint32_t *cstart,
                                       const uint32_t *csuper)
{
    const uint32_t sidx = csuper[c];
    const uint2 r = sranges[sidx];
    ChunkSpan cs;
    cs.s = sidx;
    cs.e0 = r.x + (c - cstart[sidx]) * kBinChunk;
    cs.e1 = min(cs.e0 + kBinChunk, r.y);
    return cs;
}

// Per chunk: how many of its entries cover each tile of its super-tile. With tdepth set, the
// workgroups that have no chunk (or, when every workgroup has one, all of them) also count, each
// for its share of the P target depths, the positive ones (the valid pixels of the mapping loss's
// depth term) into vpart[blockIdx.x] (0 for the others).
__global__ void __launch_bounds__(kSortThreads)
k_bin_count(const uint32_t *__restrict__ skeys, const uint2 *__restrict__ sranges, const uint32_t *__restrict__ cstart,
            const uint32_t *__restrict__ csuper, const uint32_t *__restrict__ nchunks, uint32_t *__restrict__ chist,
            const float *__restrict__ tdepth, int64_t P, uint32_t *__restrict__ vpart)
{
    __shared__ uint32_t cnt[kSuper * kSuper];
    const uint32_t nc = *nchunks;
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const ChunkSpan cs = chunk_span(c, sranges, cstart, csuper);
        if (threadIdx.x < kSuper * kSuper) cnt[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t base = cs.e0; base < cs.e1; base += kSortThreads) {
            const uint32_t e = base + threadIdx.x;
            const uint32_t m = e < cs.e1 ? box_bits(skeys[e]) : 0u;
#pragma unroll
            for (int b = 0; b < kSuper * kSuper; ++b) {
                const uint64_t bal = __ballot((m >> b) & 1u);
                if (__lane_id() == 0 && bal) atomicAdd(&cnt[b], (uint32_t)__popcll(bal));
            }
        }
        __syncthreads();
        if (threadIdx.x < kSuper * kSuper) chist[(size_t)c * (kSuper * kSuper) + threadIdx.x] = cnt[threadIdx.x];
        __syncthreads();  // cnt is cleared for the next chunk
    }
    if (tdepth) {
        const uint32_t G = gridDim.x, first = nc < G ? nc : 0u;  // the counting workgroups [first, G)
        if (blockIdx.x < first) {
            if (threadIdx.x == 0) vpart[blockIdx.x] = 0u;
            return;
        }
        __shared__ uint32_t wv[kSortThreads / kWave];
        const int64_t per = (P + (G - first) - 1) / (G - first), p0 = (int64_t)(blockIdx.x - first) * per;
        const int64_t p1 = min(P, p0 + per);
        uint32_t v = 0;
        for (int64_t p = p0 + threadIdx.x; p < p1; p += kSortThreads) v += tdepth[p] > 0.0f ? 1u : 0u;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (__lane_id() == 0) wv[threadIdx.x / kWave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < kSortThreads / kWave; ++w) t += wv[w];
            vpart[blockIdx.x] = t;
        }
    }
}

// Per super-tile (kSuper^2 threads): exclusive prefix of each tile's counts over the super-tile's
// chunks (in place) and the tile's total.
__global__ void k_bin_prefix(const uint32_t *__restrict__ cstart, uint32_t *__restrict__ chist,
                             uint32_t *__restrict__ tile_total)
{
    constexpr int NB = kSuper * kSuper, U = 8;
    const int sidx = blockIdx.x, b = threadIdx.x;
    const uint32_t c0 = cstart[sidx], c1 = cstart[sidx + 1];
    uint32_t run = 0;
    for (uint32_t c = c0; c < c1; c += U) {
        // U chunks' counts in flight at once (loads clamped to the last chunk), then their prefixes
        uint32_t v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = chist[(size_t)min(c + j, c1 - 1u) * NB + b];
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (c + j < c1) {
                chist[(size_t)(c + j) * NB + b] = run;
                run += v[j];
            }
    }
    tile_total[(size_t)sidx * NB + b] = run;  // zero for tiles beyond the image
}

// Single block: tile ranges from the tile totals (super-tile-major items: each thread takes one
// super-tile's 16 tiles, the block scans the super-tile sums), the pair count K, and the capacity
// check; on overflow every range is empty and the condition is recorded. With dscale set, also
// 1/P_v from the nv valid-pixel counts vpart (0 when no pixel is valid), as the loss reduction
// computes it.
__global__ void __launch_bounds__(kSortThreads)
k_bin_tiles(const uint32_t *__restrict__ tile_total, int nsup, int64_t cap, const uint32_t *__restrict__ ktotal,
            uint2 *__restrict__ ranges, uint32_t *__restrict__ status, uint32_t *__restrict__ n_pairs_dev,
            uint32_t *__restrict__ host_status, uint32_t *__restrict__ ok, uint32_t *__restrict__ step_ovf,
            int first_of_step, const uint32_t *__restrict__ vpart, int nv, float *__restrict__ dscale)
{
    constexpr int NB = kSuper * kSuper, R = kBinGrid / kSortThreads;
    __shared__ uint32_t w[8];
    // the valid-pixel counts (nv <= kBinGrid), loaded together with the tile totals below and
    // summed after them
    uint32_t vc[R];
    if (dscale)
#pragma unroll
        for (int r = 0; r < R; ++r) vc[r] = vpart[min((int)threadIdx.x + r * kSortThreads, nv - 1)];
    // K counted by the projection equals the sum of the tile totals whenever the super-tile pairs
    // fit (they are at most K); beyond the capacity nothing is placed
    const uint32_t K = *ktotal;
    const bool ovf = (int64_t)K > cap;
    uint32_t carry = 0;
    for (int base = 0; base < nsup; base += kSortThreads) {
        const int sidx = base + threadIdx.x;
        uint32_t v[NB], sum = 0;
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            v[l] = sidx < nsup ? tile_total[(size_t)sidx * NB + l] : 0u;
            sum += v[l];
        }
        uint32_t tot;
        uint32_t at = carry + block_excl_scan(sum, w, &tot);
        if (sidx < nsup)
#pragma unroll
            for (int l = 0; l < NB; ++l) {
                ranges[(size_t)sidx * NB + l] = ovf ? make_uint2(0u, 0u) : make_uint2(at, at + v[l]);
                at += v[l];
            }
        carry += tot;
    }
    if (dscale) {
        uint32_t v = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) v += (int)threadIdx.x + r * kSortThreads < nv ? vc[r] : 0u;
        uint32_t tot;
        block_excl_scan(v, w, &tot);
        if (threadIdx.x == 0) *dscale = tot > 0 ? (float)(1.0 / (double)tot) : 0.0f;
    }
    if (threadIdx.x == 0) {
        status[ST_PAIRS] = K;
        *n_pairs_dev = ovf ? 0u : K;
        *ok = ovf ? 0u : 1u;
        // the step's overflow word: set by the first binning of a step, or-ed by the others
        if (step_ovf && (first_of_step || ovf)) *step_ovf = ovf ? 1u : 0u;
        if (ovf) atomicMax(&status[ST_OVERFLOW], K);
        if (host_status) {
            host_status[0] = K;
            if (ovf) host_status[1] = 1u;
            __threadfence_system();
        }
    }
}

// Per chunk: writes each entry's gaussian id into the lists of the tiles it covers, in order.
__global__ void __launch_bounds__(kSortThreads)
k_bin_place(const uint32_t *__restrict__ skeys, const uint32_t *__restrict__ svals, const uint2 *__restrict__ sranges,
            const uint32_t *__restrict__ cstart, const uint32_t *__restrict__ csuper,
            const uint32_t *__restrict__ nchunks, const uint32_t *__restrict__ chist,
            const uint2 *__restrict__ ranges, const uint32_t *__restrict__ ok, uint32_t *__restrict__ vals)
{
    constexpr int NB = kSuper * kSuper, NW = kSortThreads / kWave;
    __shared__ uint32_t run[NB];
    __shared__ uint32_t wtot[NW][NB];
    const uint32_t nc = *ok ? *nchunks : 0u;
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid / kWave;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const ChunkSpan cs = chunk_span(c, sranges, cstart, csuper);
        if (tid < NB) run[tid] = ranges[(size_t)cs.s * NB + tid].x + chist[(size_t)c * NB + tid];
        for (uint32_t base = cs.e0; base < cs.e1; base += kSortThreads) {
            const uint32_t e = base + tid;
            uint32_t id = 0, m = 0;
            if (e < cs.e1) {
                id = svals[e];
                m = box_bits(skeys[e]);
            }
            uint64_t bal[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) bal[b] = __ballot((m >> b) & 1u);
            if (lane < NB) wtot[wid][lane] = (uint32_t)__popcll(bal[lane]);
            __syncthreads();
            if (m) {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if ((m >> b) & 1u) {
                        uint32_t pos = run[b] + (uint32_t)__popcll(bal[b] & lt);
                        for (int w2 = 0; w2 < wid; ++w2) pos += wtot[w2][b];
                        vals[pos] = id;
                    }
                }
            }
            __syncthreads();
            if (tid < NB) {
                uint32_t add = 0;
#pragma unroll
                for (int w2 = 0; w2 < NW; ++w2) add += wtot[w2][tid];
                run[tid] += add;
            }
            __syncthreads();
        }
    }
}

__device__ inline uint32_t lower_bound_u32(const uint32_t *__restrict__ a, uint32_t n, uint32_t v, uint32_t mask)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((a[mid] & mask) < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// [start, end) of every key's run in the sorted keys (compared under mask), by two binary
// searches per key.
__global__ void __launch_bounds__(kSortThreads)
k_ranges(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ n_dev, uint2 *__restrict__ ranges, int64_t T,
         uint32_t mask)
{
    const int64_t t = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
    if (t >= T) return;
    const uint32_t K = *n_dev;
    ranges[t] = make_uint2(lower_bound_u32(keys, K, (uint32_t)t, mask), lower_bound_u32(keys, K, (uint32_t)t + 1, mask));
}

/* ------------------------- depth order inside every super-tile list ------------------------- */
// Each super-tile list arrives in ascending gaussian id (the pairs are emitted in id order and
// the super-tile sort is stable) and is reordered, stably, by the gaussian's depth key, so that it
// ends in (depth, index) order. Two launches:
//  - k_seg_chunk_sort: every list is cut into chunks of kSegChunk consecutive entries, and each
//    chunk is sorted in LDS by a workgroup: 16 consecutive entries per thread in registers, an LSD
//    radix sort over 4-bit digits of only the bits that differ within the chunk (key - min, whose
//    bits above those of max - min are zero), each entry ranked by its thread's own digit counts
//    and a scan of those counts over the workgroup, the permuted (key, position) pairs written to
//    LDS and read back. A list of one chunk is then written out whole; the chunks of a longer
//    list go to scratch as sorted runs (depth key, gaussian id, super-tile key).
//  - k_seg_merge: the runs of a list are merged stably (the earlier run first on equal keys, which
//    keeps equal keys in index order) by merge path. A list of two chunks is merged in LDS by
//    kMergeParts workgroups, each staging both runs and writing its part of the list; a longer
//    list is merged by one workgroup, level by level through global memory.

template <int NW>
struct SegShared {
    uint32_t wtot[NW][8];  // per wave: digit counts (two 16-bit fields per word), then their prefix
    uint32_t tot[8];       // the workgroup's digit counts
};

// Inclusive sum over the wave's lanes by DPP: shifts by 1, 2, 4 and 8 within each row of 16 lanes
// (lanes shifted in from outside the row add 0), then the last lane of row 0 broadcast into row 1
// and row 2's into row 3, then lane 31 into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false); // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false); // row_bcast:31
    return x;
}

// Ranks the workgroup's NT * 16 elements (thread t holds elements 16 t .. 16 t + 15) by the 4-bit
// digit at `shift`. Element j of this thread goes to off(d) + lr(j), d its digit: off(d) (written
// to toff, 16-bit fields, two per word, by digit pair then thread) counts every element of a
// smaller digit and the elements of digit d in earlier threads; lr(j) = the elements of digit d
// among this thread's before j (byte j & 3 of lr[j >> 2]). The thread's digit counts are 4-bit
// fields of one 64-bit word (a count reaches 16 only when all 16 elements share a digit, which is
// caught separately); the scans run on two 16-bit fields per word, which add without carries
// since every sum stays below 2^16.
template <int NT>
__device__ __forceinline__ void seg_rank(const uint32_t (&k)[kSegItems], int shift, uint32_t (&lr)[kSegItems / 4],
                                         uint32_t *toff, SegShared<NT / kWave> &S)
{
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid / kWave;
    uint64_t c = 0;
    uint32_t r = 0, d = 0;
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        d = (k[j] >> shift) & 15u;
        const uint32_t s4 = d << 2;
        r = (uint32_t)(c >> s4) & 15u;
        lr[j >> 2] = (j & 3) ? (lr[j >> 2] | (r << ((j & 3) * 8))) : r;
        c += 1ull << s4;
    }
    // the local ranks are final here: keep them in their four registers rather than have the
    // compiler recompute them after the scan
#pragma unroll
    for (int q = 0; q < kSegItems / 4; ++q) asm volatile("" : "+v"(lr[q]));
    const bool all_same = r == kSegItems - 1;  // the last element has 15 of its digit before it
    const uint32_t lo = (uint32_t)c, hi = (uint32_t)(c >> 32);
    uint32_t p[8], s[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t w = q < 4 ? lo : hi, b = (q & 3) * 8;
        p[q] = all_same ? (q == (int)(d >> 1) ? (uint32_t)kSegItems << ((d & 1u) << 4) : 0u)
                        : (((w >> b) & 15u) | (((w >> (b + 4)) & 15u) << 16));
        s[q] = wave_incl_sum(p[q]);
    }
    if (lane == kWave - 1)
#pragma unroll
        for (int q = 0; q < 8; ++q) S.wtot[wid][q] = s[q];
    __syncthreads();
    if (tid < 8 * NW) {
        // NW lanes per register q, lane w holding wave w's count: a scan over the NW lanes
        const int q = tid / NW, w = tid % NW;
        const uint32_t v = S.wtot[w][q];
        uint32_t incl = v;
#pragma unroll
        for (int o = 1; o < NW; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, NW);
            incl += w >= o ? y : 0u;
        }
        S.wtot[w][q] = incl - v;
        if (w == NW - 1) S.tot[q] = incl;
    }
    __syncthreads();
    uint32_t acc = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t t = S.tot[q], tlo = t & 0xFFFFu;
        const uint32_t dig = acc | ((acc + tlo) << 16);
        acc += tlo + (t >> 16);
        toff[q * NT + tid] = dig + S.wtot[wid][q] + (s[q] - p[q]);  // smaller digits, earlier waves, earlier lanes
    }
}

// This thread's element j: its digit's offset plus its local rank.
template <int NT>
__device__ __forceinline__ uint32_t seg_slot(const uint32_t *toff, uint32_t d, const uint32_t (&lr)[kSegItems / 4],
                                             int j)
{
    const uint32_t w = toff[(d >> 1) * NT + threadIdx.x];
    return ((w >> ((d & 1u) << 4)) & 0xFFFFu) + ((lr[j >> 2] >> ((j & 3) * 8)) & 0xFFu);
}

// LDS word of key slot r: bits 2-3 of r flipped by bits 5-6, so that the 16-byte reads of the
// 16 consecutive keys of neighbouring threads spread over all banks (a bijection on each aligned
// run of 128 slots that keeps every aligned group of four slots together).
__device__ __forceinline__ uint32_t seg_swz(uint32_t r) { return r ^ (((r >> 5) & 3u) << 2); }

// Number of 4-bit passes that order keys in [mn, mx] once mn is subtracted from them.
__device__ __forceinline__ int seg_passes(uint32_t mn, uint32_t mx)
{
    const uint32_t x = mx - mn;
    return x ? (32 - __clz(x) + 3) / 4 : 0;
}

__global__ void __launch_bounds__(kChunkThreads)
k_seg_chunk_sort(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
                 uint32_t *__restrict__ vout, const uint2 *__restrict__ sranges, const uint32_t *__restrict__ sstart,
                 int nsup, const uint32_t *__restrict__ dkey, uint32_t *__restrict__ tkey, uint32_t *__restrict__ tids,
                 uint32_t *__restrict__ tsk)
{
    constexpr int NT = kChunkThreads, NW = NT / kWave;
    __shared__ __align__(16) uint32_t lkey[kSegChunk];
    __shared__ __align__(16) uint16_t lpos[kSegChunk];
    __shared__ uint32_t toff[8 * NT];
    __shared__ uint32_t lid[kSegChunk];  // the entries' gaussian ids and coverage boxes (a one-chunk
    __shared__ uint8_t lbox[kSegChunk];  // list is written out from LDS)
    __shared__ SegShared<NW> S;
    __shared__ uint32_t red[2 * NW];
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid / kWave;
    const uint32_t c = blockIdx.x;  // (< the chunks sstart has room for: the grid)
    const uint32_t nchunk = sstart[nsup], ssup = sstart[nsup + 1 + c];
    if (c >= nchunk) return;
    const int sidx = (int)ssup;
    const uint2 rg = sranges[sidx];
    const uint32_t x0 = rg.x + (c - sstart[sidx]) * (uint32_t)kSegChunk;  // the chunk's first entry
    const uint32_t n = min((uint32_t)kSegChunk, rg.y - x0);
    const bool single = rg.y - rg.x <= (uint32_t)kSegChunk;
    // the chunk's depth keys in LDS (coalesced reads of the ids, all issued before the gathers that
    // depend on them), padded with all ones; the chunk's smallest and largest key
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    {
        // (loads at clamped indices, n >= 1, and the results masked: no branch per element, so
        // the compiler keeps all of them in flight)
        uint32_t id[kSegItems], bx[kSegItems];
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            const uint32_t i = x0 + min((uint32_t)(tid + j * NT), n - 1);
            id[j] = vin[i];
            bx[j] = kin[i] >> kBoxShift;
        }
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            const uint32_t i = tid + j * NT;
            const uint32_t key = i < n ? dkey[id[j]] : 0xFFFFFFFFu;
            mn = min(mn, key);
            mx = max(mx, i < n ? key : 0u);
            lkey[seg_swz(i)] = key;
            lpos[i] = (uint16_t)i;
            lid[i] = id[j];
            lbox[i] = (uint8_t)bx[j];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = min(mn, (uint32_t)__shfl_xor(mn, o));
        mx = max(mx, (uint32_t)__shfl_xor(mx, o));
    }
    if (lane == 0) {
        red[2 * wid] = mn;
        red[2 * wid + 1] = mx;
    }
    __syncthreads();  // (also orders the stores above before the reads below)
    mn = 0xFFFFFFFFu;
    mx = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        mn = min(mn, red[2 * w]);
        mx = max(mx, red[2 * w + 1]);
    }
    // The passes sort key - mn (order-preserving for keys >= mn) on its low 4 passes bits; the
    // first pass reads the keys and subtracts, later passes read the differences. Depth keys are
    // the bits of finite positive floats, below 2^31, so the padding keys (all ones) are told apart
    // and stay all ones: at least as large as every difference in the sorted bits, and after the
    // chunk's entries, so a stable sort keeps them last.
    const int passes = seg_passes(mn, mx);
    uint32_t k[kSegItems], lr[kSegItems / 4];
    for (int pass = 0; pass < passes; ++pass) {
        uint32_t pos2[kSegItems / 2];  // positions, two 16-bit fields per word
        const uint4 *p4 = reinterpret_cast<const uint4 *>(lpos + kSegItems * tid);
#pragma unroll
        for (int j = 0; j < kSegItems / 4; ++j) {
            // four consecutive slots stay together under the swizzle
            const uint4 v = *reinterpret_cast<const uint4 *>(lkey + seg_swz(kSegItems * tid + 4 * j));
            k[4 * j] = v.x;
            k[4 * j + 1] = v.y;
            k[4 * j + 2] = v.z;
            k[4 * j + 3] = v.w;
        }
#pragma unroll
        for (int j = 0; j < kSegItems / 8; ++j) {
            const uint4 v = p4[j];
            pos2[4 * j] = v.x;
            pos2[4 * j + 1] = v.y;
            pos2[4 * j + 2] = v.z;
            pos2[4 * j + 3] = v.w;
        }
        if (pass == 0)
#pragma unroll
            for (int j = 0; j < kSegItems; ++j) k[j] = k[j] == 0xFFFFFFFFu ? k[j] : k[j] - mn;
        const int shift = 4 * pass;
        seg_rank<NT>(k, shift, lr, toff, S);  // (its barriers order the reads above before the writes below)
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            const uint32_t r = seg_slot<NT>(toff, (k[j] >> shift) & 15u, lr, j);
            lkey[seg_swz(r)] = k[j];
            lpos[r] = (uint16_t)(pos2[j >> 1] >> ((j & 1) * 16));
        }
        __syncthreads();
    }
    // out: a one-chunk list in its final place, else the sorted run (the keys themselves, restored
    // from key - mn, the gaussian ids and the super-tile keys) for the merge. Every key of a
    // super-tile list holds the same super-tile below kBoxShift. (Every load at an index inside
    // the chunk; the stores without a branch per element when all of this thread's outputs are
    // inside it.)
    const uint32_t add = passes > 0 ? mn : 0u;
    const bool full = tid + (kSegItems - 1) * NT < n;
    const uint32_t sid = kin[x0] & kSuperKeyMask;
    uint32_t kk[kSegItems], vv[kSegItems], dk[kSegItems];
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        const uint32_t r = min((uint32_t)(tid + j * NT), n - 1);
        const uint32_t q = lpos[r];
        dk[j] = lkey[seg_swz(r)] + add;
        kk[j] = sid | (uint32_t)lbox[q] << kBoxShift;
        vv[j] = lid[q];
    }
    uint32_t *ok = single ? kout : tsk, *ov = single ? vout : tids;
    if (full) {
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            ok[x0 + tid + j * NT] = kk[j];
            ov[x0 + tid + j * NT] = vv[j];
            if (!single) tkey[x0 + tid + j * NT] = dk[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < kSegItems; ++j)
            if (tid + j * NT < n) {
                ok[x0 + tid + j * NT] = kk[j];
                ov[x0 + tid + j * NT] = vv[j];
                if (!single) tkey[x0 + tid + j * NT] = dk[j];
            }
    }
}

// Reads of the keys being merged: straight from global memory, or from LDS at the swizzled slot
// i + i / 64 (one spare word per 64 entries), so that the merge's reads, which step about four
// entries from lane to lane, fall into distinct banks.
struct GlobalKeys {
    const uint32_t *k;
    __device__ uint32_t operator()(uint32_t i) const { return k[i]; }
};
__device__ __forceinline__ uint32_t lds_slot(uint32_t i) { return i + (i >> 6); }
struct LdsKeys {
    const uint32_t *k;
    __device__ uint32_t operator()(uint32_t i) const { return k[lds_slot(i)]; }
};

// Merge path of output index o when merging sorted runs a = key[a0, a0 + la) and b = key[b0,
// b0 + lb) stably (a first on equal keys): the number of elements of a among the first o outputs.
template <class Keys>
__device__ __forceinline__ uint32_t merge_split(Keys key, uint32_t a0, uint32_t la, uint32_t b0, uint32_t lb,
                                                uint32_t o)
{
    uint32_t lo = o > lb ? o - lb : 0u, hi = min(o, la);
    while (lo < hi) {
        const uint32_t i = (lo + hi) >> 1;  // a[i] is taken before b[o - 1 - i] iff a[i] <= b[o - 1 - i]
        if (key(a0 + i) <= key(b0 + o - 1 - i)) lo = i + 1;
        else hi = i;
    }
    return lo;
}

// One thread's kMergeItems consecutive outputs o0 .. of a merge level: runs of L entries of the
// keys [0, n) merged pairwise, stably (the earlier run first on equal keys). Found from the
// thread's start on the merge path, then branch-free (the heads of both runs are loaded at clamped
// indices every step, both loads issued together; an exhausted run's head reads as all ones). src:
// each output's index in the keys, key: its key. Outputs past n get src = n - 1.
constexpr int kMergeItems = 8;
template <class Keys>
__device__ __forceinline__ void merge_round(Keys keys, uint32_t n, uint32_t L, uint32_t o0,
                                            uint32_t (&src)[kMergeItems], uint32_t (&key)[kMergeItems])
{
    // the pair of runs holding outputs o0 .. o0 + 7 (a pair spans 2 L >= 8 outputs)
    const uint32_t base = o0 / (2 * L) * (2 * L);
    const uint32_t la = min(L, n - base), lb = min(L, n - base - la);
    const uint32_t o = o0 - base;
    uint32_t i = merge_split(keys, base, la, base + la, lb, o), j = o - i;
    // the second run's reads stay inside the pair's entries (la >= 1; with lb = 0 they read the
    // first run's head and are not used)
    const uint32_t b0 = lb ? base + la : base, bl = lb ? lb - 1u : 0u;
#pragma unroll
    for (int t = 0; t < kMergeItems; ++t) {
        const uint32_t va = keys(base + min(i, la - 1u)), vb = keys(b0 + min(j, bl));
        const uint32_t ha = i < la ? va : 0xFFFFFFFFu, hb = j < lb ? vb : 0xFFFFFFFFu;
        const bool takeA = i < la && (j >= lb || ha <= hb);
        src[t] = min(takeA ? base + i : base + la + j, n - 1);
        key[t] = takeA ? ha : hb;
        i += takeA ? 1u : 0u;
        j += takeA ? 0u : 1u;
    }
}

// A list of two chunks (kSegChunk < n <= kMergeLds): one merge level in LDS, the runs' keys, ids
// and coverage boxes staged first (keys and ids at their swizzled slots), the outputs read from
// LDS. The workgroup writes the outputs [part P, (part + 1) P) of the list, P = kMergeLds /
// kMergeParts (its first P / kMergeItems threads).
constexpr int kMergeParts = 4;
__device__ __forceinline__ void merge_staged(uint32_t *lk, uint32_t *lid, uint8_t *lbox, uint32_t n, uint32_t x,
                                             uint32_t part,
                                             const uint32_t *__restrict__ tkey, const uint32_t *__restrict__ tid,
                                             const uint32_t *__restrict__ tsk, uint32_t *__restrict__ kout,
                                             uint32_t *__restrict__ vout)
{
    constexpr int J = kMergeLds / kMergeThreads;
    {
        uint32_t k[J], v[J], b[J];  // all of a thread's loads in flight at once
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t i = x + min((uint32_t)(threadIdx.x + j * kMergeThreads), n - 1);
            k[j] = tkey[i];
            v[j] = tid[i];
            b[j] = tsk[i] >> kBoxShift;
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t i = threadIdx.x + j * kMergeThreads;
            if (i < n) {
                lk[lds_slot(i)] = k[j];
                lid[lds_slot(i)] = v[j];
                lbox[i] = (uint8_t)b[j];
            }
        }
    }
    __syncthreads();
    const uint32_t sid = tsk[x] & kSuperKeyMask;  // the super-tile of every key of the list
    constexpr uint32_t P = kMergeLds / kMergeParts;
    static_assert(P <= kMergeThreads * kMergeItems, "a workgroup's part is one round of its threads");
    const uint32_t o0 = part * P + threadIdx.x * kMergeItems;
    if (threadIdx.x * kMergeItems < P && o0 < n) {
        uint32_t src[kMergeItems], key[kMergeItems];
        merge_round(LdsKeys{lk}, n, kSegChunk, o0, src, key);
        uint32_t kk[kMergeItems], vv[kMergeItems];
#pragma unroll
        for (int t = 0; t < kMergeItems; ++t) {
            kk[t] = sid | (uint32_t)lbox[src[t]] << kBoxShift;
            vv[t] = lid[lds_slot(src[t])];
        }
        if (o0 + kMergeItems <= n) {
#pragma unroll
            for (int t = 0; t < kMergeItems; ++t) {
                kout[x + o0 + t] = kk[t];
                vout[x + o0 + t] = vv[t];
            }
        } else {
#pragma unroll
            for (int t = 0; t < kMergeItems; ++t)
                if (o0 + t < n) {
                    kout[x + o0 + t] = kk[t];
                    vout[x + o0 + t] = vv[t];
                }
        }
    }
}

// A longer list: merge levels through global memory, (key, id, super-tile key) moving from the
// arrays a to the arrays b and back, the last level writing the outputs.
__device__ void merge_global(uint32_t *ka, uint32_t *ia, uint32_t *sa, uint32_t *kb, uint32_t *ib, uint32_t *sb,
                             uint32_t n, uint32_t *__restrict__ kout, uint32_t *__restrict__ vout)
{
    for (uint32_t L = kSegChunk; L < n; L *= 2) {
        const bool last = 2 * L >= n;
        for (uint32_t o0 = threadIdx.x * kMergeItems; o0 < n; o0 += kMergeThreads * kMergeItems) {
            uint32_t src[kMergeItems], key[kMergeItems];
            merge_round(GlobalKeys{ka}, n, L, o0, src, key);
            uint32_t iv[kMergeItems], sv[kMergeItems];
#pragma unroll
            for (int t = 0; t < kMergeItems; ++t) {
                iv[t] = ia[src[t]];
                sv[t] = sa[src[t]];
            }
#pragma unroll
            for (int t = 0; t < kMergeItems; ++t)
                if (o0 + t < n) {
                    if (last) {
                        kout[o0 + t] = sv[t];
                        vout[o0 + t] = iv[t];
                    } else {
                        kb[o0 + t] = key[t];
                        ib[o0 + t] = iv[t];
                        sb[o0 + t] = sv[t];
                    }
                }
        }
        __syncthreads();  // the level's outputs are the next level's runs
        uint32_t *t;
        t = ka; ka = kb; kb = t;
        t = ia; ia = ib; ib = t;
        t = sa; sa = sb; sb = t;
    }
}

// Every list of several chunks, kMergeParts workgroups per list (blockIdx.x = kMergeParts list +
// part): a list of two chunks is merged by all of them, each writing its part; a longer one by
// the first (the sorted runs in (tkey, tid, tsk); tkey2, tid2 and tsk2 are scratch for lists
// longer than kMergeLds).
__global__ void __launch_bounds__(kMergeThreads)
k_seg_merge(uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, const uint2 *__restrict__ sranges,
            uint32_t *__restrict__ tkey, uint32_t *__restrict__ tid, uint32_t *__restrict__ tsk,
            uint32_t *__restrict__ tkey2, uint32_t *__restrict__ tid2, uint32_t *__restrict__ tsk2)
{
    static_assert(2 * kSegChunk == kMergeLds, "a list that fits in LDS has two chunks: one merge level");
    __shared__ uint32_t lk[kMergeLds + kMergeLds / 64], lid[kMergeLds + kMergeLds / 64];
    __shared__ uint8_t lbox[kMergeLds];
    const uint32_t part = blockIdx.x % kMergeParts;
    const uint2 rg = sranges[blockIdx.x / kMergeParts];
    const uint32_t x = rg.x, n = rg.y - rg.x;
    if (n <= (uint32_t)kSegChunk) return;  // one chunk: already in place
    if (n <= (uint32_t)kMergeLds) {
        if (part * (kMergeLds / kMergeParts) < n) merge_staged(lk, lid, lbox, n, x, part, tkey, tid, tsk, kout, vout);
    } else if (part == 0)
        merge_global(tkey + x, tid + x, tsk + x, tkey2 + x, tid2 + x, tsk2 + x, n, kout + x, vout + x);
}

__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

int sort_blocks(int64_t cap, int per_block)
{
    int64_t G = (cap + per_block - 1) / per_block;
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
        hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kSortThreads), 0, s, ws.hist, ws.G, ws.totals, nullptr, 0,
                           nullptr, nullptr);
        // the last pass of several sorts the top bits, whose few values already give long runs
        if (p == passes - 1 && passes > 1)
            hipLaunchKernelGGL(k_radix_scatter, dim3(ws.G), dim3(kSortThreads), 0, s, sk, sv, ok, ov, n_dev,
                               (uint32_t)n_cap, shift, mask, bits, ws.hist, ws.totals);
        else
            hipLaunchKernelGGL(k_radix_scatter_lds, dim3(ws.G), dim3(kSortThreads), 0, s, sk, sv, ok, ov, n_dev,
                               (uint32_t)n_cap, shift, mask, bits, ws.hist, ws.totals);
        if (p == passes - 1) return ok;
        sk = dk; sv = dv;
        dk = (dk == kb) ? ka : kb;
        dv = (dv == vb) ? va : vb;
    }
    return nullptr;
}

int64_t scan_blocks(int64_t n)
{
    const int64_t per = (int64_t)kSortThreads * scan_items(n);
    return (n + per - 1) / per;
}

int64_t scan_blocks_cap(int64_t n) { return (n + 2 * kSortThreads - 1) / (2 * kSortThreads) + 1; }

void launch_scan_counts(const uint32_t *ids, const uint32_t *count, int64_t n, uint32_t *blocksums, hipStream_t s)
{
    const int nb = (int)scan_blocks(n);
    if (nb <= 0) return;
    if (scan_items(n) == 2)
        hipLaunchKernelGGL(k_count_reduce<2>, dim3(nb), dim3(kSortThreads), 0, s, ids, count, n, blocksums);
    else
        hipLaunchKernelGGL(k_count_reduce<4>, dim3(nb), dim3(kSortThreads), 0, s, ids, count, n, blocksums);
}

int64_t emit_chunks(int64_t cap) { return (cap + kEmitChunk - 1) / kEmitChunk + 1; }

void launch_emit(const uint32_t *ids, const uint32_t *count, const uint2 *rect, uint32_t *blocksums,
                 uint32_t *offsets, int64_t n, int32_t keys_x, int shift, int64_t cap, uint32_t *keys, uint32_t *vals,
                 uint2 *rect_sorted, uint32_t *start_rank, uint32_t *status, uint32_t *n_pairs_dev,
                 uint32_t *host_status, const uint32_t *kpart, int64_t proj_blocks, uint32_t *ktotal, hipStream_t s,
                 const uint2 *view_tab, uint32_t view_n, uint32_t *csum)
{
    // the block sums: blocksums (launch_scan_counts, one per scan block in [0, nb)) or csum (the
    // projection's, one per 256 ranks, so scan_items(n) per scan block)
    const int nb = (int)scan_blocks(n);
    const bool scanned = nb > kScanFold;
    uint32_t *sums = csum ? csum : blocksums;
    const uint32_t per = csum ? (uint32_t)scan_items(n) : 1u;
    const int nsums = csum ? (int)project_blocks(n) : nb;
    if (scanned)
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kSortThreads), 0, s, sums, nsums, status, kpart,
                           (int)proj_blocks, ktotal);
    const dim3 grid(nb > 0 ? nb : 1);
    if (scan_items(n) == 2)
        hipLaunchKernelGGL(k_scan_apply<2>, grid, dim3(kSortThreads), 0, s, ids, count, rect, n, sums, scanned,
                           offsets, rect_sorted, start_rank, (uint32_t)emit_chunks(cap), status, kpart,
                           (int)proj_blocks, ktotal, per);
    else
        hipLaunchKernelGGL(k_scan_apply<4>, grid, dim3(kSortThreads), 0, s, ids, count, rect, n, sums, scanned,
                           offsets, rect_sorted, start_rank, (uint32_t)emit_chunks(cap), status, kpart,
                           (int)proj_blocks, ktotal, per);
    hipLaunchKernelGGL(k_emit, dim3(grid_for(cap, kEmitChunk, 2048)), dim3(kSortThreads), 0, s, rect_sorted, ids,
                       offsets, start_rank, n, keys_x, shift, cap, view_tab, view_n, keys, vals, status, n_pairs_dev,
                       host_status);
}

void launch_super_scan(int64_t n, uint32_t *hist, uint32_t *totals, const uint32_t *kpart, uint32_t *status,
                       uint32_t *ktotal, hipStream_t s)
{
    const int G = (int)project_blocks(n);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kSortThreads), 0, s, hist, G, totals, kpart, G, status, ktotal);
}

void launch_super_scatter(const uint2 *rect, const uint32_t *count, int64_t n, int32_t supers_x, const uint32_t *hist,
                          const uint32_t *totals, const uint32_t *ktotal, int64_t cap, uint32_t *keys, uint32_t *vals,
                          const BinWS &b, uint2 *sranges, int nsup, uint32_t *sstart, int64_t smax, hipStream_t s)
{
    const int G = (int)project_blocks(n);  // (and one more workgroup for the chunk tables)
    hipLaunchKernelGGL(k_super_scatter, dim3((unsigned)G + 1u), dim3(kSortThreads), 0, s, rect, count, n, supers_x, hist,
                       totals, ktotal, cap, keys, vals, sranges, nsup, b.cstart, b.csuper, (uint32_t)b.max_chunks,
                       b.nchunks, sstart, (uint32_t)smax);
}

int64_t bin_max_chunks(int64_t cap, int64_t nsup) { return (cap + kBinChunk - 1) / kBinChunk + nsup; }

void launch_bin_chunks(const BinWS &b, uint2 *sranges, const uint32_t *digit_totals, int nsup, hipStream_t s,
                       uint32_t *sstart, int64_t smax, const uint32_t *ktotal, int64_t cap)
{
    hipLaunchKernelGGL(k_bin_chunks, dim3(1), dim3(kSortThreads), 0, s, sranges, digit_totals, nsup, b.cstart,
                       b.csuper, (uint32_t)b.max_chunks, b.nchunks, sstart, (uint32_t)smax, ktotal, cap);
}

void launch_bin_count(const BinWS &b, const uint32_t *skeys, const uint2 *sranges, hipStream_t s,
                      const float *tdepth, int64_t P)
{
    hipLaunchKernelGGL(k_bin_count, dim3(grid_for(b.max_chunks, 1, kBinGrid)), dim3(kSortThreads), 0, s, skeys, sranges,
                       b.cstart, b.csuper, b.nchunks, b.chist, tdepth, P, b.vpart);
}

void launch_bin_counts(const BinWS &b, const uint32_t *skeys, uint2 *sranges, const uint32_t *digit_totals, int nsup,
                       hipStream_t s)
{
    launch_bin_chunks(b, sranges, digit_totals, nsup, s);
    launch_bin_count(b, skeys, sranges, s);
}

int64_t seg_max_chunks(int64_t cap, int64_t nsup) { return (cap + kSegChunk - 1) / kSegChunk + nsup; }

void launch_seg_sort(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, const uint2 *sranges,
                     const uint32_t *sstart, int nsup, int64_t max_chunks, const uint32_t *dkey, uint32_t *const t[6],
                     hipStream_t s)
{
    if (nsup <= 0 || max_chunks <= 0) return;
    hipLaunchKernelGGL(k_seg_chunk_sort, dim3((unsigned)max_chunks), dim3(kChunkThreads), 0, s, kin, vin, kout, vout,
                       sranges, sstart, nsup, dkey, t[0], t[1], t[2]);
    hipLaunchKernelGGL(k_seg_merge, dim3((unsigned)(kMergeParts * nsup)), dim3(kMergeThreads), 0, s, kout, vout, sranges,
                       t[0], t[1], t[2], t[3], t[4], t[5]);
}

void launch_bin_tiles(const BinWS &b, int nsup, int64_t cap, const uint32_t *ktotal, uint2 *ranges, uint32_t *status,
                      uint32_t *n_pairs_dev, uint32_t *host_status, uint32_t *step_ovf, bool first_of_step,
                      hipStream_t s, float *dscale)
{
    hipLaunchKernelGGL(k_bin_prefix, dim3((unsigned)nsup), dim3(kSuper * kSuper), 0, s, b.cstart, b.chist,
                       b.tile_total);
    hipLaunchKernelGGL(k_bin_tiles, dim3(1), dim3(kSortThreads), 0, s, b.tile_total, nsup, cap, ktotal, ranges, status,
                       n_pairs_dev, host_status, b.ok, step_ovf, first_of_step ? 1 : 0, b.vpart,
                       (int)grid_for(b.max_chunks, 1, kBinGrid), dscale);
}

void launch_bin_place(const BinWS &b, const uint32_t *skeys, const uint32_t *svals, const uint2 *sranges,
                      const uint2 *ranges, uint32_t *vals, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_place, dim3(grid_for(b.max_chunks, 1, kBinGrid)), dim3(kSortThreads), 0, s, skeys, svals,
                       sranges, b.cstart, b.csuper, b.nchunks, b.chist, ranges, b.ok, vals);
}

void launch_ranges(const uint32_t *keys, const uint32_t *n_dev, uint2 *ranges, int64_t T, uint32_t mask,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((T + kSortThreads - 1) / kSortThreads)), dim3(kSortThreads), 0, s,
                       keys, n_dev, ranges, T, mask);
}

}  // namespace fgs
