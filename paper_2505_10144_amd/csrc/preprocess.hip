// K1 (per-Gaussian preprocessing + exact instance count) and K3 (instance
// keys), plus the exclusive scan that places each Gaussian's instances.
//
// One thread per Gaussian loops over all views, so the 236 bytes of
// parameters are read from HBM once per batch of views (coalesced SoA loads)
// and each view's 128-byte record is written with vector stores.
#include "geom.h"

namespace vrs {

// Real spherical harmonics (orthonormal, Condon-Shortley phase) up to degree
// 3 written as polynomials of the unit direction (x, y, z), k = l^2 + l + m.
__device__ inline void sh_eval(const GaussPtrs& g, int i, const double v[3], double rgb[3]) {
    const int n = g.n;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    const double x = v[0], y = v[1], z = v[2];
    const double pi = M_PI;
    double Y[16];
    Y[0] = 0.5 / sqrt(pi);
    if (K > 1) {
        const double c1 = sqrt(3.0 / (4.0 * pi));
        Y[1] = -c1 * y;
        Y[2] = c1 * z;
        Y[3] = -c1 * x;
    }
    if (K > 4) {
        const double c2a = sqrt(15.0 / (4.0 * pi));   // xy, yz, xz terms
        const double c2b = sqrt(5.0 / (16.0 * pi));   // 3z^2 - 1
        const double c2c = sqrt(15.0 / (16.0 * pi));  // x^2 - y^2
        Y[4] = c2a * x * y;
        Y[5] = -c2a * y * z;
        Y[6] = c2b * (3.0 * z * z - 1.0);
        Y[7] = -c2a * x * z;
        Y[8] = c2c * (x * x - y * y);
    }
    if (K > 9) {
        const double c3a = sqrt(35.0 / (32.0 * pi));   // |m| = 3
        const double c3b = sqrt(105.0 / (4.0 * pi));   // m = -2: xyz
        const double c3c = sqrt(21.0 / (32.0 * pi));   // |m| = 1
        const double c3d = sqrt(7.0 / (16.0 * pi));    // m = 0
        const double c3e = sqrt(105.0 / (16.0 * pi));  // m = 2
        Y[9] = -c3a * y * (3.0 * x * x - y * y);
        Y[10] = c3b * x * y * z;
        Y[11] = -c3c * y * (5.0 * z * z - 1.0);
        Y[12] = c3d * z * (5.0 * z * z - 3.0);
        Y[13] = -c3c * x * (5.0 * z * z - 1.0);
        Y[14] = c3e * z * (x * x - y * y);
        Y[15] = -c3a * x * (x * x - 3.0 * y * y);
    }
    for (int c = 0; c < 3; ++c) {
        double acc = 0.5;
        for (int k = 0; k < K; ++k) acc += double(g.sh[(k * 3 + c) * n + i]) * Y[k];
        rgb[c] = fmax(acc, 0.0);
    }
}

__global__ void __launch_bounds__(256) k_preprocess(GaussPtrs g, GeoViews views, Knobs kn,
                                                    float* __restrict__ proj,
                                                    uint32_t* __restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const GaussLocal G = load_gaussian(g, i);
    for (int v = 0; v < views.n; ++v) {
        const GeoView& V = views.v[v];
        Geo geo;
        uint32_t cnt = 0;
        const size_t row = (size_t(v) * size_t(g.n) + size_t(i)) * kRec;
        if (!make_geo(G, V, kn, geo)) {
            counts[size_t(v) * g.n + i] = 0;
            continue;
        }
        int tx0, tx1, ty0, ty1;
        cone_tiles(geo, V, tx0, tx1, ty0, ty1);
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                double bx0, by0, bx1, by1;
                tile_box(V, tx, ty, bx0, by0, bx1, by1);
                cnt += tile_test(geo, V, bx0, by0, bx1, by1, nullptr) ? 1u : 0u;
            }
        counts[size_t(v) * g.n + i] = cnt;
        // Colour from the eye centre o = -R^T t.
        double eye[3];
        for (int c = 0; c < 3; ++c)
            eye[c] = -(double(V.R[c]) * V.t[0] + double(V.R[3 + c]) * V.t[1] + double(V.R[6 + c]) * V.t[2]);
        double dir[3] = {G.mu[0] - eye[0], G.mu[1] - eye[1], G.mu[2] - eye[2]};
        const double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        for (int c = 0; c < 3; ++c) dir[c] /= dn;
        double rgb[3];
        sh_eval(g, i, dir, rgb);
        // Record.
        float rec[kRec];
        const double xi = floor(geo.x0), yi = floor(geo.y0);
        rec[R_X0I] = float(xi);
        rec[R_Y0I] = float(yi);
        rec[R_X0F] = float(geo.x0 - xi);
        rec[R_Y0F] = float(geo.y0 - yi);
        // Scale so that |z|^2 = (log2 e / 2) D^2 and alpha = opacity * 2^-|z|^2.
        const double zs = sqrt(0.5 / M_LN2);
        for (int k = 0; k < 4; ++k) rec[R_M00 + k] = float(geo.M[k] * zs);
        rec[R_A3X] = float(geo.a3x);
        rec[R_A3Y] = float(geo.a3y);
        const double l2s = log2(geo.sigma);
        rec[R_L2S] = float(l2s);
        rec[R_KAP] = float(l2s - log2(double(kn.alpha_min)));
        // Depth along the pixel ray d = (x0 + dx - cx, y0 + dy - cy, f) / f:
        // w(delta) = W3 d = w0 + dx wx + dy wy, t = (w . m) / |w|^2.
        const double iz = 1.0 / geo.muc[2];
        double w0[3], wx[3], wy[3];
        for (int r = 0; r < 3; ++r) {
            w0[r] = (geo.W3[3 * r] * geo.muc[0] + geo.W3[3 * r + 1] * geo.muc[1] + geo.W3[3 * r + 2] * geo.muc[2]) * iz;
            wx[r] = geo.W3[3 * r] / V.f;
            wy[r] = geo.W3[3 * r + 1] / V.f;
        }
        rec[R_N0] = float(w0[0] * geo.m[0] + w0[1] * geo.m[1] + w0[2] * geo.m[2]);
        rec[R_NX] = float(wx[0] * geo.m[0] + wx[1] * geo.m[1] + wx[2] * geo.m[2]);
        rec[R_NY] = float(wy[0] * geo.m[0] + wy[1] * geo.m[1] + wy[2] * geo.m[2]);
        rec[R_SPARE0] = 0.f;
        for (int r = 0; r < 3; ++r) {
            rec[R_W0 + r] = float(w0[r]);
            rec[R_WX + r] = float(wx[r]);
            rec[R_WY + r] = float(wy[r]);
            rec[R_RGB + r] = float(rgb[r]);
        }
        rec[R_SIG] = float(geo.sigma);
        rec[R_SPARE1] = 0.f;
        rec[R_SPARE2] = 0.f;
        rec[R_SPARE3] = 0.f;
        float4* dst = reinterpret_cast<float4*>(proj + row);
#pragma unroll
        for (int k = 0; k < kRec / 4; ++k)
            dst[k] = make_float4(rec[4 * k], rec[4 * k + 1], rec[4 * k + 2], rec[4 * k + 3]);
    }
}

__global__ void __launch_bounds__(256) k_duplicate(GaussPtrs g, GeoViews views, Knobs kn,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint32_t* __restrict__ counts,
                                                   uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ gids, size_t capacity) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    bool loaded = false;
    GaussLocal G;
    for (int v = 0; v < views.n; ++v) {
        const size_t slot = size_t(v) * g.n + i;
        if (counts[slot] == 0) continue;
        if (!loaded) { G = load_gaussian(g, i); loaded = true; }
        const GeoView& V = views.v[v];
        Geo geo;
        if (!make_geo(G, V, kn, geo)) continue;
        size_t off = offsets[slot];
        int tx0, tx1, ty0, ty1;
        cone_tiles(geo, V, tx0, tx1, ty0, ty1);
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                double bx0, by0, bx1, by1, depth;
                tile_box(V, tx, ty, bx0, by0, bx1, by1);
                if (!tile_test(geo, V, bx0, by0, bx1, by1, &depth)) continue;
                if (off < capacity) {
                    const uint64_t tile = uint64_t(V.tile_off) + uint64_t(ty) * V.ntx + tx;
                    keys[off] = (tile << 32) | uint64_t(ord_f32(float(depth)));
                    gids[off] = uint32_t(i);
                }
                ++off;
            }
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 counts (three phases: per-block scan, scan of the
// block sums, add-back).  The total goes to *total.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t* sh, uint32_t& total) {
    // sh: kScanThreads words.
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t y = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    total = sh[kScanThreads - 1];
    const uint32_t incl = sh[t];
    __syncthreads();
    return incl - x;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out,
                                                             uint32_t* __restrict__ sums, size_t n) {
    __shared__ uint32_t sh[kScanThreads];
    const size_t base = size_t(blockIdx.x) * kScanTile + size_t(threadIdx.x) * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(s, sh, tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums in chunks with a carry.
__global__ void __launch_bounds__(kScanThreads) k_scan_sums(uint32_t* __restrict__ sums, size_t nb,
                                                            uint32_t* __restrict__ total) {
    __shared__ uint32_t sh[kScanThreads];
    uint32_t carry = 0;
    for (size_t c0 = 0; c0 < nb; c0 += kScanTile) {
        const size_t base = c0 + size_t(threadIdx.x) * kScanItems;
        uint32_t v[kScanItems];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < nb ? sums[base + k] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(s, sh, tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < nb) sums[base + k] = ex;
            ex += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(uint32_t* __restrict__ out,
                                                           const uint32_t* __restrict__ sums, size_t n) {
    const uint32_t add = sums[blockIdx.x];
    const size_t base = size_t(blockIdx.x) * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
        if (base + k < n) out[base + k] += add;
}

__global__ void k_check_capacity(const uint32_t* n_inst, size_t capacity, int* status) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && size_t(*n_inst) > capacity)
        set_status(status, VRS_ERR_CAPACITY);
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
size_t scan_ws_bytes(size_t n) {
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    return (n + nb + 64) * sizeof(uint32_t);
}

int launch_preprocess(const GaussPtrs& g, const GeoViews& views, const Knobs& kn, float* proj,
                      uint32_t* counts, hipStream_t s) {
    if (g.n == 0) return VRS_OK;
    const int blocks = (g.n + 255) / 256;
    hipLaunchKernelGGL(k_preprocess, dim3(blocks), dim3(256), 0, s, g, views, kn, proj, counts);
    return launch_status(hipGetLastError());
}

int launch_duplicate(const GaussPtrs& g, const GeoViews& views, const Knobs& kn,
                     const uint32_t* counts, uint64_t* keys, uint32_t* gids, size_t capacity,
                     uint32_t* n_inst, void* ws, int* status, hipStream_t s) {
    const size_t n = size_t(g.n) * size_t(views.n);
    uint32_t* offsets = static_cast<uint32_t*>(ws);
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    uint32_t* sums = offsets + n;
    if (n == 0) {
        hipError_t e = hipMemsetAsync(n_inst, 0, sizeof(uint32_t), s);
        return launch_status(e);
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kScanThreads), 0, s, counts, offsets, sums, n);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, sums, nb, n_inst);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanThreads), 0, s, offsets, sums, n);
    hipLaunchKernelGGL(k_check_capacity, dim3(1), dim3(64), 0, s, n_inst, capacity, status);
    const int blocks = (g.n + 255) / 256;
    hipLaunchKernelGGL(k_duplicate, dim3(blocks), dim3(256), 0, s, g, views, kn, offsets, counts, keys,
                       gids, capacity);
    return launch_status(hipGetLastError());
}

}  // namespace vrs
