// K4: stable LSD radix sort of (uint64 key, uint32 value) pairs with 8-bit
// digits, K5: per-tile [start, end) ranges of the sorted keys, and the
// exclusive scan shared with the instantiation stage.
//
// Two kernels first count the digits of every pass at once (the digit
// totals do not depend on the order of the keys).  Each pass is then
// reduce-then-scan: (1) every block counts the digits of its 2048-key tile
// in LDS, (2) one block per digit scans that digit's row of the digit-major
// [256][blocks] histogram and adds the totals of the smaller digits, giving
// every (digit, block) its output offset,
// (3) every block ranks its keys stably -- each wave owns a contiguous
// 512-key slice, ranks within a 64-key step by matching digits with
// ballots, and the per-wave digit counts are prefix-summed across waves --
// and scatters them.  No inter-block waiting, so passes are deterministic
// and need no forward-progress assumptions.  Pair counts are read on the
// device, so the grid covers `capacity` and surplus blocks only contribute
// zero counts.
//
// The first pass can drop dead keys (all ones): instantiation writes one for
// every candidate tile that fails the tile test, and they never reach the
// later passes.
#include "vrs_internal.h"

namespace vrs {

constexpr int kSortWaves = kSortThreads / 64;
constexpr uint64_t kDeadKey = ~0ull;
static_assert(kSortThreads == kRadix, "one thread per digit in the count kernels");

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 (per-block scan, scan of block sums, add-back).
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Exclusive scan over the block (kScanThreads threads): an inclusive scan
// within each wave by lane shuffles, then the wave totals through LDS.  The
// closing barrier lets the caller scan again with the same `sh`.
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t* sh, uint32_t& total) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t v = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(v, off);
        if (lane >= off) v += y;
    }
    if (lane == 63) sh[w] = v;
    __syncthreads();
    uint32_t below = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        const uint32_t s = sh[k];
        below += k < w ? s : 0u;
        all += s;
    }
    total = all;
    __syncthreads();
    return below + v - x;
}

// Sum of a uint64 over the block (every thread gets it).
__device__ inline uint64_t block_sum_u64(uint64_t x, uint64_t* sh) {
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) t += sh[k];
    __syncthreads();
    return t;
}

// in and out may alias: every thread reads its items before writing them.
// A block whose items sum to 2^32 - 1 or more stores that saturated value as
// its sum, which k_scan_sums reports as an overflow.
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const uint32_t* in, uint32_t* out,
                                                             uint32_t* __restrict__ sums, size_t n) {
    __shared__ uint32_t sh[kScanThreads];
    __shared__ uint64_t sh64[kScanThreads / 64];
    const size_t base = size_t(blockIdx.x) * kScanTile + size_t(threadIdx.x) * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    uint64_t s64 = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
        s64 += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(s, sh, tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    const uint64_t t64 = block_sum_u64(s64, sh64);
    if (threadIdx.x == 0) sums[blockIdx.x] = t64 >= 0xFFFFFFFFull ? 0xFFFFFFFFu : tot;
}

// Single block: exclusive scan of the block sums in chunks with a carry.
// The grand total is also summed in 64 bits: if it (or a saturated block
// sum) reaches 2^32 - 1 the offsets are unrepresentable, so the total is
// set to 0 (nothing downstream reads an offset) and the overflow reported.
__global__ void __launch_bounds__(kScanThreads) k_scan_sums(uint32_t* __restrict__ sums, size_t nb,
                                                            uint32_t* __restrict__ total, int* status) {
    __shared__ uint32_t sh[kScanThreads];
    __shared__ uint64_t sh64[kScanThreads / 64];
    uint32_t carry = 0;
    uint64_t carry64 = 0;
    for (size_t c0 = 0; c0 < nb; c0 += kScanTile) {
        const size_t base = c0 + size_t(threadIdx.x) * kScanItems;
        uint32_t v[kScanItems];
        uint32_t s = 0;
        uint64_t s64 = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < nb ? sums[base + k] : 0u;
            s += v[k];
            s64 += v[k];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(s, sh, tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < nb) sums[base + k] = ex;
            ex += v[k];
        }
        carry += tot;
        carry64 += block_sum_u64(s64, sh64);
    }
    if (threadIdx.x == 0) {
        const bool over = carry64 >= 0xFFFFFFFFull;
        if (over) set_status(status, VRS_ERR_UNSUPPORTED);
        if (total) *total = over ? 0u : carry;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(uint32_t* __restrict__ out,
                                                           const uint32_t* __restrict__ sums, size_t n) {
    const uint32_t add = sums[blockIdx.x];
    const size_t base = size_t(blockIdx.x) * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
        if (base + k < n) out[base + k] += add;
}

// The second half of a scan of at most kScanFusedTiles tiles in one launch,
// fused with instantiation's set-up: every block sums the tile sums before
// its own (in 64 bits, from L2) and adds that to its tile; block 0 stores the
// grand total in n_inst[0] -- 0, with the overflow reported, when it reaches
// 2^32 - 1 (a saturated tile sum does) -- zeroes n_inst[1] and reports a
// total above `capacity`; every block clears a share of `clear`.
constexpr size_t kScanFusedTiles = 4096;
__global__ void __launch_bounds__(kScanThreads) k_scan_add_setup(uint32_t* __restrict__ out,
                                                                 const uint32_t* __restrict__ sums, size_t n,
                                                                 size_t nb, uint32_t* __restrict__ n_inst,
                                                                 size_t capacity, int* status,
                                                                 uint32_t* __restrict__ clear, size_t n_clear) {
    __shared__ uint64_t sh64[kScanThreads / 64];
    uint64_t before = 0, all = 0;
    for (size_t k = threadIdx.x; k < nb; k += kScanThreads) {
        const uint32_t v = sums[k];
        all += v;
        before += k < size_t(blockIdx.x) ? v : 0u;
    }
    before = block_sum_u64(before, sh64);
    all = block_sum_u64(all, sh64);
    const uint32_t add = uint32_t(before);
    const size_t base = size_t(blockIdx.x) * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
        if (base + k < n) out[base + k] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const bool over = all >= 0xFFFFFFFFull;
        if (over) set_status(status, VRS_ERR_UNSUPPORTED);
        const uint32_t tot = over ? 0u : uint32_t(all);
        n_inst[0] = tot;
        n_inst[1] = 0;
        if (size_t(tot) > capacity) set_status(status, VRS_ERR_CAPACITY);
    }
    for (size_t i = size_t(blockIdx.x) * kScanThreads + threadIdx.x; i < n_clear; i += size_t(gridDim.x) * kScanThreads)
        clear[i] = 0u;
}

// Exclusive scan of n > 0 words in two launches when it spans at most
// kScanFusedTiles tiles, with instantiation's set-up (see k_scan_add_setup);
// returns VRS_ERR_UNSUPPORTED without launching anything otherwise.
int launch_scan_with_setup(const uint32_t* in, uint32_t* out, size_t n, uint32_t* n_inst, uint32_t* tmp,
                           size_t capacity, int* status, uint32_t* clear, size_t n_clear, hipStream_t s) {
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    if (n == 0 || nb > kScanFusedTiles) return VRS_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kScanThreads), 0, s, in, out, tmp, n);
    hipLaunchKernelGGL(k_scan_add_setup, dim3(nb), dim3(kScanThreads), 0, s, out, tmp, n, nb, n_inst, capacity, status,
                       clear, n_clear);
    return launch_status(hipGetLastError());
}

__global__ void k_store_zero(uint32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

size_t scan_tmp_words(size_t n) { return (n + kScanTile - 1) / kScanTile + 64; }

int launch_exclusive_scan(const uint32_t* in, uint32_t* out, size_t n, uint32_t* total, uint32_t* tmp,
                          int* status, hipStream_t s) {
    if (n == 0) {
        if (total) hipLaunchKernelGGL(k_store_zero, dim3(1), dim3(64), 0, s, total);
        return launch_status(hipGetLastError());
    }
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kScanThreads), 0, s, in, out, tmp, n);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tmp, nb, total, status);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanThreads), 0, s, out, tmp, n);
    return launch_status(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Radix sort.
// ---------------------------------------------------------------------------
__device__ inline size_t n_eff(const uint32_t* n_dev, size_t capacity) {
    const size_t n = size_t(*n_dev);
    return n < capacity ? n : capacity;
}

// Digit counts go to kSubHist copies of the histogram by lane (lane mod
// kSubHist), summed at the end: a byte that takes few values (the top byte of
// the depths, the high byte of the tiles) would otherwise put many lanes of
// one atomic instruction on the same LDS word, which serializes them.
constexpr int kSubHist = 4;

__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint64_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ n_dev,
                                                             size_t capacity, int shift, int drop,
                                                             uint32_t* __restrict__ hist, int nblocks) {
    __shared__ uint32_t cnt[kSubHist][kRadix];
#pragma unroll
    for (int c = 0; c < kSubHist; ++c) cnt[c][threadIdx.x] = 0;
    __syncthreads();
    const int sub = threadIdx.x % kSubHist;
    const size_t n = n_eff(n_dev, capacity);
    const size_t base = size_t(blockIdx.x) * kSortTile;
    // Every load is issued before the first count, so the wave waits for
    // memory once rather than once per key.
    uint64_t key[kSortItemsPerLane];
#pragma unroll
    for (int k = 0; k < kSortItemsPerLane; ++k) {
        const size_t idx = base + size_t(k) * kSortThreads + threadIdx.x;
        key[k] = idx < n ? keys[idx] : kDeadKey;
    }
#pragma unroll
    for (int k = 0; k < kSortItemsPerLane; ++k) {
        const size_t idx = base + size_t(k) * kSortThreads + threadIdx.x;
        if (idx < n && !(drop && key[k] == kDeadKey)) atomicAdd(&cnt[sub][uint32_t(key[k] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int s = 0; s < kSubHist; ++s) c += cnt[s][threadIdx.x];
    hist[size_t(threadIdx.x) * nblocks + blockIdx.x] = c;
}

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Rank the block's keys stably, place them in LDS in (digit, rank) order,
// then write each digit's run to its global offset: consecutive threads
// write consecutive addresses within a run.
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, size_t capacity, int shift, int drop,
    const uint32_t* __restrict__ hist, int sd, int sb) {
    __shared__ uint32_t wcnt[kSortWaves][kRadix];
    __shared__ uint32_t goff[kRadix];     // global offset of each digit's run
    __shared__ uint32_t loff[kRadix];     // start of each digit's run in the block
    __shared__ uint32_t scan_sh[kSortThreads];
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int lane = t & 63;
    for (int k = 0; k < kSortWaves; ++k) wcnt[k][t] = 0;
    goff[t] = hist[size_t(t) * sd + size_t(blockIdx.x) * sb];
    __syncthreads();
    const size_t n = n_eff(n_dev, capacity);
    if (size_t(blockIdx.x) * kSortTile >= n) return;  // whole block empty (uniform)
    const size_t base = size_t(blockIdx.x) * kSortTile + size_t(w) * (kSortTile / kSortWaves);

    uint64_t key[kSortItemsPerLane];
    uint32_t val[kSortItemsPerLane];
    uint32_t rank[kSortItemsPerLane];
    bool live[kSortItemsPerLane];
    const uint64_t lt = lanemask_lt();
    // All loads first (the ranking below orders LDS accesses with wave
    // fences, which would otherwise hold each load until the previous step).
#pragma unroll
    for (int it = 0; it < kSortItemsPerLane; ++it) {
        const size_t idx = base + size_t(it) * 64 + lane;
        const bool in = idx < n;
        key[it] = in ? kin[idx] : 0ull;
        val[it] = in ? vin[idx] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kSortItemsPerLane; ++it) {
        const size_t idx = base + size_t(it) * 64 + lane;
        const bool in = idx < n;
        const bool ok = in && !(drop && key[it] == kDeadKey);
        live[it] = ok;
        const uint32_t d = uint32_t(key[it] >> shift) & 0xFFu;
        // Lanes holding the same digit: intersect the ballots of each bit.
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t before = __popcll(m & lt);
        const uint32_t c0 = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        rank[it] = c0 + before;
        if (ok && before == 0) wcnt[w][d] = c0 + __popcll(m);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    // Exclusive prefix over waves for every digit (thread t owns digit t),
    // then over digits: the start of each digit's run in the block.
    uint32_t cnt = 0;
    for (int k = 0; k < kSortWaves; ++k) {
        const uint32_t c = wcnt[k][t];
        wcnt[k][t] = cnt;
        cnt += c;
    }
    uint32_t live_total;
    loff[t] = block_exclusive_scan(cnt, scan_sh, live_total);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItemsPerLane; ++it) {
        if (live[it]) {
            const uint32_t d = uint32_t(key[it] >> shift) & 0xFFu;
            const uint32_t lp = loff[d] + wcnt[w][d] + rank[it];
            skey[lp] = key[it];
            sval[lp] = val[it];
        }
    }
    __syncthreads();
    for (uint32_t i = uint32_t(t); i < live_total; i += kSortThreads) {
        const uint64_t k = skey[i];
        const uint32_t d = uint32_t(k >> shift) & 0xFFu;
        const size_t pos = size_t(goff[d]) + (i - loff[d]);
        kout[pos] = k;
        vout[pos] = sval[i];
    }
}

// Digit counts of every pass for one 2048-key tile: block b writes
// counts[p][b][d], and hist0[d][b] for the first pass.
__global__ void __launch_bounds__(kSortThreads) k_digit_counts(const uint64_t* __restrict__ keys,
                                                               const uint32_t* __restrict__ n_dev, size_t capacity,
                                                               int passes, int drop,
                                                               uint32_t* __restrict__ counts, int nblocks,
                                                               uint32_t* __restrict__ live_out,
                                                               uint32_t* __restrict__ totals,
                                                               uint32_t* __restrict__ hist0) {
    __shared__ uint32_t cnt[kMaxPasses][kSubHist][kRadix];
    __shared__ uint32_t wlive[kSortWaves];
    const int sub = threadIdx.x % kSubHist;
    for (int p = 0; p < passes; ++p)
        for (int s = 0; s < kSubHist; ++s) cnt[p][s][threadIdx.x] = 0;
    // The digit totals that k_digit_totals adds up next start at zero.
    if (blockIdx.x == 0)
        for (int p = 0; p < passes; ++p) totals[p * kRadix + threadIdx.x] = 0;
    __syncthreads();
    const size_t n = n_eff(n_dev, capacity);
    const size_t base = size_t(blockIdx.x) * kSortTile;
    uint32_t live = 0;
    uint64_t key[kSortItemsPerLane];
#pragma unroll
    for (int k = 0; k < kSortItemsPerLane; ++k) {  // all loads first
        const size_t idx = base + size_t(k) * kSortThreads + threadIdx.x;
        key[k] = idx < n ? keys[idx] : kDeadKey;
    }
#pragma unroll
    for (int k = 0; k < kSortItemsPerLane; ++k) {
        const size_t idx = base + size_t(k) * kSortThreads + threadIdx.x;
        if (idx < n && !(drop && key[k] == kDeadKey)) {
            ++live;
            for (int p = 0; p < passes; ++p) atomicAdd(&cnt[p][sub][uint32_t(key[k] >> (8 * p)) & 0xFFu], 1u);
        }
    }
    if (live_out) {  // uniform
        for (int off = 32; off >= 1; off >>= 1) live += __shfl_xor(live, off);
        if ((threadIdx.x & 63) == 0) wlive[threadIdx.x >> 6] = live;
    }
    __syncthreads();
    if (live_out && threadIdx.x == 0) {
        uint32_t b = 0;
        for (int w = 0; w < kSortWaves; ++w) b += wlive[w];
        if (b) atomicAdd(live_out, b);
    }
    uint32_t c0 = 0;
    for (int p = 0; p < passes; ++p) {
        uint32_t c = 0;
#pragma unroll
        for (int s = 0; s < kSubHist; ++s) c += cnt[p][s][threadIdx.x];
        counts[(size_t(p) * nblocks + blockIdx.x) * kRadix + threadIdx.x] = c;
        if (p == 0) c0 = c;
    }
    // The first pass's counts once more, digit-major as the later passes'
    // histograms are, so that its row scan reads whole rows.
    hist0[size_t(threadIdx.x) * nblocks + blockIdx.x] = c0;
}

// Digit totals of every pass: block (r, p) adds rows [32r, 32r + 32) of
// pass p's counts, one thread per digit, so every load reads a whole
// 1 KB row; the partial sums go to totals (zeroed by k_digit_counts) with
// integer atomics, which are exact in any order.
constexpr int kTotalRows = 32;
__global__ void __launch_bounds__(kRadix) k_digit_totals(const uint32_t* __restrict__ counts, int nblocks,
                                                         uint32_t* __restrict__ totals) {
    const int p = blockIdx.y, d = threadIdx.x, b0 = blockIdx.x * kTotalRows;
    const int rows = min(kTotalRows, nblocks - b0);
    const uint32_t* c = counts + (size_t(p) * nblocks + b0) * kRadix + d;
    uint32_t tot = 0;
#pragma unroll 8
    for (int r = 0; r < rows; ++r) tot += c[size_t(r) * kRadix];
    if (tot) atomicAdd(&totals[p * kRadix + d], tot);
}

// One block per digit d: exclusive scan of the digit's per-block counts,
// plus the digit's offset (the totals of the smaller digits), in place.
__global__ void __launch_bounds__(kScanThreads) k_digit_row_scan(uint32_t* __restrict__ hist, int nblocks,
                                                                 int sd, int sb,
                                                                 const uint32_t* __restrict__ totals) {
    __shared__ uint32_t sh[kScanThreads];
    const int d = blockIdx.x;
    uint32_t tot;
    block_exclusive_scan(int(threadIdx.x) < d ? totals[threadIdx.x] : 0u, sh, tot);
    uint32_t carry = tot;  // sum of the totals of digits < d
    uint32_t* row = hist + size_t(d) * sd;
    for (int c0 = 0; c0 < nblocks; c0 += kScanTile) {
        const int base = c0 + int(threadIdx.x) * kScanItems;
        uint32_t v[kScanItems];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < nblocks ? row[size_t(base + k) * sb] : 0u;
            sum += v[k];
        }
        uint32_t t2;
        uint32_t ex = block_exclusive_scan(sum, sh, t2) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < nblocks) row[size_t(base + k) * sb] = ex;
            ex += v[k];
        }
        carry += t2;
    }
}

__global__ void k_copy_pairs(const uint64_t* __restrict__ ks, const uint32_t* __restrict__ vs,
                             uint64_t* __restrict__ kd, uint32_t* __restrict__ vd,
                             const uint32_t* __restrict__ n_dev, size_t capacity) {
    const size_t n = n_eff(n_dev, capacity);
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_tile_ranges(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
                              size_t capacity, uint32_t tiles_total, uint32_t* __restrict__ ranges) {
    const size_t n = n_eff(n_dev, capacity);
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
        const uint32_t tile = uint32_t(keys[i] >> 32);
        if (tile >= tiles_total) continue;
        if (i == 0 || uint32_t(keys[i - 1] >> 32) != tile) ranges[2 * size_t(tile)] = uint32_t(i);
        if (i + 1 == n || uint32_t(keys[i + 1] >> 32) != tile) ranges[2 * size_t(tile) + 1] = uint32_t(i + 1);
    }
}

// ---------------------------------------------------------------------------
static size_t sort_blocks(size_t capacity) { return (capacity + kSortTile - 1) / kSortTile; }

size_t sort_ws_bytes(size_t capacity) { return sort_ws_layout_bytes(capacity); }

int launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return VRS_OK;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks < 4096 ? blocks : 4096), dim3(256), 0, s, p, n, v);
    return launch_status(hipGetLastError());
}

// Sort min(*n_first, capacity) pairs; with drop_first the first pass drops
// dead keys and the remaining passes sort min(*n_rest, capacity) pairs.
// With drop_first and a non-null `live_out` (zeroed by the caller), the
// number of live keys is added to *live_out before the first pass, so
// n_rest may point at it.
int launch_sort_pairs_ex(uint64_t* keys, uint32_t* vals, const uint32_t* n_first, const uint32_t* n_rest,
                         bool drop_first, size_t capacity, int key_bits, void* ws, int* err, hipStream_t s,
                         uint32_t* live_out) {
    (void)err;  // no pass waits on another block, so nothing can time out
    if (capacity == 0 || key_bits <= 0) return VRS_OK;
    const int nb = int(sort_blocks(capacity));
    uint64_t* k2 = static_cast<uint64_t*>(ws);
    uint32_t* v2 = reinterpret_cast<uint32_t*>(k2 + capacity);
    size_t off = capacity * (sizeof(uint64_t) + sizeof(uint32_t));
    off = (off + 255) & ~size_t(255);
    uint32_t* hist = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + off);
    const size_t hist_len = size_t(kRadix) * nb;
    uint32_t* totals = hist + ((hist_len + 63) & ~size_t(63));
    uint32_t* counts = totals + size_t(kMaxPasses) * kRadix;
    const int passes = (key_bits + 7) / 8;
    // Digit totals of every pass (the live keys are the same in every pass;
    // the first pass drops the dead ones).
    hipLaunchKernelGGL(k_digit_counts, dim3(nb), dim3(kSortThreads), 0, s, keys, n_first, capacity, passes,
                       drop_first ? 1 : 0, counts, nb, drop_first ? live_out : nullptr, totals, hist);
    hipLaunchKernelGGL(k_digit_totals, dim3((nb + kTotalRows - 1) / kTotalRows, passes), dim3(kRadix), 0, s, counts,
                       nb, totals);
    uint64_t *ka = keys, *kb = k2;
    uint32_t *va = vals, *vb = v2;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const int drop = (p == 0 && drop_first) ? 1 : 0;
        const uint32_t* n_dev = (p == 0 || !drop_first) ? n_first : n_rest;
        // The first pass's per-block counts are those k_digit_counts wrote
        // to hist (same keys, same order).  Element (digit d, block b) at
        // d * sd + b * sb.
        uint32_t* h = hist;
        const int sd = nb, sb = 1;
        if (p > 0) {
            hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortThreads), 0, s, ka, n_dev, capacity, shift, drop,
                               hist, nb);
        }
        hipLaunchKernelGGL(k_digit_row_scan, dim3(kRadix), dim3(kScanThreads), 0, s, h, nb, sd, sb,
                           totals + p * kRadix);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortThreads), 0, s, ka, va, kb, vb, n_dev, capacity,
                           shift, drop, h, sd, sb);
        uint64_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        const size_t blocks = (capacity + 255) / 256;
        hipLaunchKernelGGL(k_copy_pairs, dim3(blocks < 4096 ? blocks : 4096), dim3(256), 0, s, ka, va, keys, vals,
                           drop_first ? n_rest : n_first, capacity);
    }
    return launch_status(hipGetLastError());
}

int launch_sort_pairs(uint64_t* keys, uint32_t* vals, const uint32_t* n_dev, size_t capacity, int key_bits,
                      void* ws, int* err, hipStream_t s) {
    return launch_sort_pairs_ex(keys, vals, n_dev, n_dev, false, capacity, key_bits, ws, err, s, nullptr);
}

// With clear false the caller has zeroed `ranges` already.
int launch_tile_ranges(const uint64_t* keys, const uint32_t* n_dev, size_t capacity, uint32_t tiles_total,
                       uint32_t* ranges, hipStream_t s, bool clear) {
    if (clear) {
        const int rc = launch_fill_u32(ranges, size_t(tiles_total) * 2, 0u, s);
        if (rc != VRS_OK) return rc;
    }
    if (capacity == 0) return VRS_OK;
    const size_t blocks = (capacity + 255) / 256;
    hipLaunchKernelGGL(k_tile_ranges, dim3(blocks < 8192 ? blocks : 8192), dim3(256), 0, s, keys, n_dev, capacity,
                       tiles_total, ranges);
    return launch_status(hipGetLastError());
}

}  // namespace vrs
