// K4: stable LSD radix sort of (uint64 key, uint32 value) pairs with 8-bit
// digits, and K5: per-tile [start, end) ranges of the sorted keys.
//
// Each pass is reduce-then-scan: (1) every block counts the digits of its
// 4096-key tile in LDS, (2) one block scans the digit-major [256][blocks]
// histogram, (3) every block ranks its keys stably -- each wave owns a
// contiguous 1024-key slice, ranks within a 64-key step by matching digits
// with ballots, and the per-wave digit counts are prefix-summed across waves
// -- and scatters to its global offsets.  No inter-block waiting, so the
// passes are deterministic and need no forward-progress assumptions.  The
// number of pairs is read on the device, so the grid covers `capacity` and
// surplus blocks only contribute zero counts.
#include "vrs_internal.h"

namespace vrs {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItemsPerLane = 16;
constexpr int kSortTile = kSortThreads * kSortItemsPerLane;  // 4096
constexpr int kRadix = 256;

__device__ inline size_t n_eff(const uint32_t* n_dev, size_t capacity) {
    const size_t n = size_t(*n_dev);
    return n < capacity ? n : capacity;
}

__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint64_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ n_dev,
                                                             size_t capacity, int shift,
                                                             uint32_t* __restrict__ hist, int nblocks) {
    __shared__ uint32_t cnt[kRadix];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const size_t n = n_eff(n_dev, capacity);
    const size_t base = size_t(blockIdx.x) * kSortTile;
    for (int k = 0; k < kSortItemsPerLane; ++k) {
        const size_t idx = base + size_t(k) * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[uint32_t(keys[idx] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    hist[size_t(threadIdx.x) * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Single block exclusive scan of `len` words in chunks with a carry.
constexpr int kHistScanThreads = 1024;
__global__ void __launch_bounds__(kHistScanThreads) k_hist_scan(uint32_t* __restrict__ h, size_t len) {
    __shared__ uint32_t sh[kHistScanThreads];
    constexpr int kItems = 8;
    uint32_t carry = 0;
    const int t = threadIdx.x;
    for (size_t c0 = 0; c0 < len; c0 += size_t(kHistScanThreads) * kItems) {
        const size_t b = c0 + size_t(t) * kItems;
        uint32_t v[kItems];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            v[k] = b + k < len ? h[b + k] : 0u;
            s += v[k];
        }
        sh[t] = s;
        __syncthreads();
        for (int off = 1; off < kHistScanThreads; off <<= 1) {
            const uint32_t y = t >= off ? sh[t - off] : 0u;
            __syncthreads();
            sh[t] += y;
            __syncthreads();
        }
        uint32_t ex = sh[t] - s + carry;
        const uint32_t tot = sh[kHistScanThreads - 1];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (b + k < len) h[b + k] = ex;
            ex += v[k];
        }
        carry += tot;
    }
}

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, size_t capacity, int shift,
    const uint32_t* __restrict__ hist, int nblocks) {
    __shared__ uint32_t wcnt[kSortWaves][kRadix];
    __shared__ uint32_t goff[kRadix];
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int lane = t & 63;
    for (int k = 0; k < kSortWaves; ++k) wcnt[k][t] = 0;
    goff[t] = hist[size_t(t) * nblocks + blockIdx.x];
    __syncthreads();
    const size_t n = n_eff(n_dev, capacity);
    const size_t base = size_t(blockIdx.x) * kSortTile + size_t(w) * (kSortTile / kSortWaves);
    if (size_t(blockIdx.x) * kSortTile >= n) return;  // whole block empty (uniform)

    uint64_t key[kSortItemsPerLane];
    uint32_t val[kSortItemsPerLane];
    uint32_t rank[kSortItemsPerLane];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int it = 0; it < kSortItemsPerLane; ++it) {
        const size_t idx = base + size_t(it) * 64 + lane;
        const bool ok = idx < n;
        key[it] = ok ? kin[idx] : 0ull;
        val[it] = ok ? vin[idx] : 0u;
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
    // Exclusive prefix over waves for every digit (thread t owns digit t).
    {
        uint32_t acc = 0;
        for (int k = 0; k < kSortWaves; ++k) {
            const uint32_t c = wcnt[k][t];
            wcnt[k][t] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItemsPerLane; ++it) {
        const size_t idx = base + size_t(it) * 64 + lane;
        if (idx < n) {
            const uint32_t d = uint32_t(key[it] >> shift) & 0xFFu;
            const size_t pos = size_t(goff[d]) + wcnt[w][d] + rank[it];
            kout[pos] = key[it];
            vout[pos] = val[it];
        }
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
size_t sort_ws_bytes(size_t capacity) {
    const size_t nb = (capacity + kSortTile - 1) / kSortTile;
    size_t b = capacity * (sizeof(uint64_t) + sizeof(uint32_t));  // ping-pong buffers
    b = (b + 255) & ~size_t(255);
    b += (size_t(kRadix) * (nb ? nb : 1) + 64) * sizeof(uint32_t);   // histogram
    return b;
}

int launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return VRS_OK;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks < 4096 ? blocks : 4096), dim3(256), 0, s, p, n, v);
    return launch_status(hipGetLastError());
}

int launch_sort_pairs(uint64_t* keys, uint32_t* vals, const uint32_t* n_dev, size_t capacity,
                      int key_bits, void* ws, hipStream_t s) {
    if (capacity == 0 || key_bits <= 0) return VRS_OK;
    const int nb = int((capacity + kSortTile - 1) / kSortTile);
    uint64_t* k2 = static_cast<uint64_t*>(ws);
    uint32_t* v2 = reinterpret_cast<uint32_t*>(k2 + capacity);
    size_t off = capacity * (sizeof(uint64_t) + sizeof(uint32_t));
    off = (off + 255) & ~size_t(255);
    uint32_t* hist = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + off);
    const int passes = (key_bits + 7) / 8;
    uint64_t *ka = keys, *kb = k2;
    uint32_t *va = vals, *vb = v2;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortThreads), 0, s, ka, n_dev, capacity, shift, hist, nb);
        hipLaunchKernelGGL(k_hist_scan, dim3(1), dim3(kHistScanThreads), 0, s, hist, size_t(kRadix) * nb);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortThreads), 0, s, ka, va, kb, vb, n_dev, capacity,
                           shift, hist, nb);
        uint64_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        const size_t blocks = (capacity + 255) / 256;
        hipLaunchKernelGGL(k_copy_pairs, dim3(blocks < 4096 ? blocks : 4096), dim3(256), 0, s, ka, va, keys, vals,
                           n_dev, capacity);
    }
    return launch_status(hipGetLastError());
}

int launch_tile_ranges(const uint64_t* keys, const uint32_t* n_dev, size_t capacity, uint32_t tiles_total,
                       uint32_t* ranges, hipStream_t s) {
    int rc = launch_fill_u32(ranges, size_t(tiles_total) * 2, 0u, s);
    if (rc != VRS_OK) return rc;
    if (capacity == 0) return VRS_OK;
    const size_t blocks = (capacity + 255) / 256;
    hipLaunchKernelGGL(k_tile_ranges, dim3(blocks < 8192 ? blocks : 8192), dim3(256), 0, s, keys, n_dev, capacity,
                       tiles_total, ranges);
    return launch_status(hipGetLastError());
}

}  // namespace vrs
