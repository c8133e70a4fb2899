// Binning of projected gaussians into screen tiles and the (tile, depth) ordering of every
// tile's list.
//
// Ordering scheme: the n gaussians are first sorted by depth (32-bit keys, the bits of the
// positive FP32 depth; ids emitted in ascending order and a stable sort, so equal depths keep
// ascending index). Every gaussian then emits one (super-tile, depth rank) pair per covered
// square of kSuper x kSuper tiles, in depth order; a stable sort of those pairs by super-tile
// alone leaves each super-tile's list in (depth, index) order, and an in-order expansion of each
// super-tile list into the lists of its tiles keeps that order. The result is exactly the stable
// (tile, depth rank) order of one pair per covered tile, while the sort only moves one pair per
// covered super-tile; no pair ever carries a depth key of its own.
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
__global__ void __launch_bounds__(kSortThreads)
k_radix_rowscan(uint32_t *__restrict__ hist, int G, uint32_t *__restrict__ totals)
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
// of the gaussians that cover at least one tile into depth order, and the first rank of every
// emission chunk.
// scanned: blocksums already hold exclusive prefixes (k_scan_top ran); otherwise each block adds
// the block sums before it and block 0 sums the projection's counts.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_scan_apply(const uint32_t *__restrict__ ids, const uint32_t *__restrict__ count, const uint2 *__restrict__ rect,
             int64_t n, const uint32_t *__restrict__ blocksums, bool scanned, uint32_t *__restrict__ offsets,
             uint2 *__restrict__ rect_sorted, uint32_t *__restrict__ start_rank, uint32_t max_chunks,
             uint32_t *__restrict__ status, const uint32_t *__restrict__ kpart, int npb,
             uint32_t *__restrict__ ktotal)
{
    __shared__ uint32_t w[8];
    // this block's first offset: the sum of the block sums before it
    uint32_t boff;
    if (scanned) {
        boff = blocksums[blockIdx.x];
    } else {
        uint32_t pre = 0;
        for (uint32_t j = threadIdx.x; j < blockIdx.x; j += kSortThreads) pre += blocksums[j];
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

constexpr uint32_t kBinChunk = 512;    // super-tile list entries per expansion chunk
constexpr int kBinGrid = 4096;         // workgroups of the expansion kernels (each loops over chunks)

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

// Load-balanced emission: the K pairs are cut into chunks of kEmitChunk consecutive pair
// indices; a block takes a chunk, finds the depth ranks it spans by binary search over the
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
// covered super-tile (in depth order) and the pairs are sorted by super-tile; each super-tile's
// list is then cut into chunks of kBinChunk entries, and a workgroup per chunk expands its
// entries into the tiles they cover: a count pass, a prefix over the super-tile's chunks and
// over all tiles, and a placement pass. Entries stay in depth order within every tile (the
// super-tile sort is stable and chunks are placed in order), so the tile lists are exactly the
// stable (tile, depth rank) order.

// Chunk table: chunk c covers entries [sranges[s].x + (c - cstart[s]) kBinChunk, ...) of
// super-tile s = csuper[c]; *nchunks = number of chunks (capped at max_chunks).
__global__ void __launch_bounds__(kSortThreads)
k_bin_chunks(uint2 *__restrict__ sranges, const uint32_t *__restrict__ digit_totals, int nsup,
             uint32_t *__restrict__ cstart, uint32_t *__restrict__ csuper, uint32_t max_chunks,
             uint32_t *__restrict__ nchunks)
{
    __shared__ uint32_t w[8];
    if (digit_totals) {
        // one radix pass sorted the super-tile keys: their ranges are the scanned digit totals
        uint32_t carry = 0;
        for (int base = 0; base < nsup; base += kSortThreads) {
            const int sidx = base + threadIdx.x;
            const uint32_t v = sidx < nsup ? digit_totals[sidx] : 0u;
            uint32_t tot;
            const uint32_t ex = carry + block_excl_scan(v, w, &tot);
            if (sidx < nsup) sranges[sidx] = make_uint2(ex, ex + v);
            carry += tot;
        }
        __syncthreads();
    }
    uint32_t carry = 0;
    for (int base = 0; base < nsup; base += kSortThreads) {
        const int sidx = base + threadIdx.x;
        uint32_t nch = 0;
        if (sidx < nsup) {
            const uint2 r = sranges[sidx];
            nch = (r.y - r.x + kBinChunk - 1) / kBinChunk;
        }
        uint32_t tot;
        const uint32_t ex = carry + block_excl_scan(nch, w, &tot);
        if (sidx < nsup) {
            cstart[sidx] = ex;
            for (uint32_t c = 0; c < nch && ex + c < max_chunks; ++c) csuper[ex + c] = (uint32_t)sidx;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        cstart[nsup] = carry;
        *nchunks = min(carry, max_chunks);
    }
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

// Per chunk: how many of its entries cover each tile of its super-tile.
__global__ void __launch_bounds__(kSortThreads)
k_bin_count(const uint32_t *__restrict__ skeys, const uint2 *__restrict__ sranges, const uint32_t *__restrict__ cstart,
            const uint32_t *__restrict__ csuper, const uint32_t *__restrict__ nchunks, uint32_t *__restrict__ chist)
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
}

// Per super-tile (kSuper^2 threads): exclusive prefix of each tile's counts over the super-tile's
// chunks (in place) and the tile's total.
__global__ void k_bin_prefix(const uint32_t *__restrict__ cstart, uint32_t *__restrict__ chist,
                             uint32_t *__restrict__ tile_total)
{
    const int sidx = blockIdx.x, b = threadIdx.x;
    uint32_t run = 0;
    for (uint32_t c = cstart[sidx]; c < cstart[sidx + 1]; ++c) {
        uint32_t *h = chist + (size_t)c * (kSuper * kSuper) + b;
        const uint32_t v = *h;
        *h = run;
        run += v;
    }
    tile_total[(size_t)sidx * (kSuper * kSuper) + b] = run;  // zero for tiles beyond the image
}

// Single block: tile ranges from the tile totals (super-tile-major items: each thread takes one
// super-tile's 16 tiles, the block scans the super-tile sums), the pair count K, and the capacity
// check; on overflow every range is empty and the condition is recorded.
__global__ void __launch_bounds__(kSortThreads)
k_bin_tiles(const uint32_t *__restrict__ tile_total, int nsup, int64_t cap, const uint32_t *__restrict__ ktotal,
            uint2 *__restrict__ ranges, uint32_t *__restrict__ status, uint32_t *__restrict__ n_pairs_dev,
            uint32_t *__restrict__ host_status, uint32_t *__restrict__ ok, uint32_t *__restrict__ step_ovf,
            int first_of_step)
{
    constexpr int NB = kSuper * kSuper;
    __shared__ uint32_t w[8];
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
        hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kSortThreads), 0, s, ws.hist, ws.G, ws.totals);
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
                 const uint2 *view_tab, uint32_t view_n)
{
    // blocksums holds the per-block sums of the counts in [0, nb)
    const int nb = (int)scan_blocks(n);
    const bool scanned = nb > kScanFold;
    if (scanned)
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kSortThreads), 0, s, blocksums, nb, status, kpart,
                           (int)proj_blocks, ktotal);
    const dim3 grid(nb > 0 ? nb : 1);
    if (scan_items(n) == 2)
        hipLaunchKernelGGL(k_scan_apply<2>, grid, dim3(kSortThreads), 0, s, ids, count, rect, n, blocksums, scanned,
                           offsets, rect_sorted, start_rank, (uint32_t)emit_chunks(cap), status, kpart,
                           (int)proj_blocks, ktotal);
    else
        hipLaunchKernelGGL(k_scan_apply<4>, grid, dim3(kSortThreads), 0, s, ids, count, rect, n, blocksums, scanned,
                           offsets, rect_sorted, start_rank, (uint32_t)emit_chunks(cap), status, kpart,
                           (int)proj_blocks, ktotal);
    hipLaunchKernelGGL(k_emit, dim3(grid_for(cap, kEmitChunk, 2048)), dim3(kSortThreads), 0, s, rect_sorted, ids,
                       offsets, start_rank, n, keys_x, shift, cap, view_tab, view_n, keys, vals, status, n_pairs_dev,
                       host_status);
}

int64_t bin_max_chunks(int64_t cap, int64_t nsup) { return (cap + kBinChunk - 1) / kBinChunk + nsup; }

void launch_bin_counts(const BinWS &b, const uint32_t *skeys, uint2 *sranges, const uint32_t *digit_totals, int nsup,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_chunks, dim3(1), dim3(kSortThreads), 0, s, sranges, digit_totals, nsup, b.cstart,
                       b.csuper, (uint32_t)b.max_chunks, b.nchunks);
    hipLaunchKernelGGL(k_bin_count, dim3(grid_for(b.max_chunks, 1, kBinGrid)), dim3(kSortThreads), 0, s, skeys, sranges,
                       b.cstart, b.csuper, b.nchunks, b.chist);
}

void launch_bin_tiles(const BinWS &b, int nsup, int64_t cap, const uint32_t *ktotal, uint2 *ranges, uint32_t *status,
                      uint32_t *n_pairs_dev, uint32_t *host_status, uint32_t *step_ovf, bool first_of_step,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_prefix, dim3((unsigned)nsup), dim3(kSuper * kSuper), 0, s, b.cstart, b.chist,
                       b.tile_total);
    hipLaunchKernelGGL(k_bin_tiles, dim3(1), dim3(kSortThreads), 0, s, b.tile_total, nsup, cap, ktotal, ranges, status,
                       n_pairs_dev, host_status, b.ok, step_ovf, first_of_step ? 1 : 0);
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
