// K1: per-Gaussian preprocessing (Optimal-Projection render records, the FP64
// tile-test records and candidate-tile counts) and K3: Gaussian/tile
// instantiation with the exact tangent-plane tile test (Eq. 4).
//
// K1 runs one thread per Gaussian and loops over the views, so the 236 bytes
// of parameters are read from HBM once per batch of views with coalesced SoA
// loads.  It does no tile tests: the count it writes is the number of
// candidate tiles under the cone bound.  K3 then runs one thread per
// candidate (Gaussian, tile) -- no per-thread loops, hence no divergence
// between Gaussians with few and many tiles -- and writes the key of a kept
// instance or a dead key (all ones) that the first radix pass drops.
#include "geom.h"

namespace vrs {

// Real spherical harmonics (orthonormal, Condon-Shortley phase) up to degree
// 3 written as polynomials of the unit direction (x, y, z), k = l^2 + l + m.
__device__ inline void sh_basis(const float v[3], float Y[16]) {
#pragma clang fp contract(off)
    const float x = v[0], y = v[1], z = v[2];
    constexpr double pi = M_PI;
    const float c0 = float(0.5 / sqrt(pi));
    const float c1 = float(sqrt(3.0 / (4.0 * pi)));
    const float c2a = float(sqrt(15.0 / (4.0 * pi)));   // xy, yz, xz terms
    const float c2b = float(sqrt(5.0 / (16.0 * pi)));   // 3z^2 - 1
    const float c2c = float(sqrt(15.0 / (16.0 * pi)));  // x^2 - y^2
    const float c3a = float(sqrt(35.0 / (32.0 * pi)));   // |m| = 3
    const float c3b = float(sqrt(105.0 / (4.0 * pi)));   // m = -2: xyz
    const float c3c = float(sqrt(21.0 / (32.0 * pi)));   // |m| = 1
    const float c3d = float(sqrt(7.0 / (16.0 * pi)));    // m = 0
    const float c3e = float(sqrt(105.0 / (16.0 * pi)));  // m = 2
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (3.f * z * z - 1.f);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (x * x - y * y);
    Y[9] = -c3a * y * (3.f * x * x - y * y);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (5.f * z * z - 1.f);
    Y[12] = c3d * z * (5.f * z * z - 3.f);
    Y[13] = -c3c * x * (5.f * z * z - 1.f);
    Y[14] = c3e * z * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3.f * y * y);
}

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The render records of a wave's 64 consecutive Gaussians are staged in LDS
// and written out as contiguous 1 KB pieces (a record per lane would make
// every store instruction touch 64 different lines).  In LDS, field f of
// record r sits at r * 8 + (f ^ (r & 7)), so the 64 lanes writing one field
// of their records spread over all banks (a record-major layout puts every
// lane of such a store in the same four banks), and the write-out still
// reads each record's eight fields as one contiguous 128-byte run.
__device__ inline int stage_slot(int r, int f) { return r * 8 + (f ^ (r & 7)); }

__global__ void __launch_bounds__(256) k_preprocess(GaussPtrs g, GeoViews views, Knobs kn,
                                                    float* __restrict__ proj, TileRect* __restrict__ rects,
                                                    uint32_t* __restrict__ counts, int* status) {
    __shared__ float4 stage[4][64 * 8];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wave_i0 = i - lane;
    if (wave_i0 >= g.n) return;  // whole wave past the end
    const bool inb = i < g.n;
    const GaussLocal G = load_gaussian(g, inb ? i : wave_i0);
    // A Gaussian with a NaN or infinite parameter is culled from every view
    // and reported (once per wave).
    if (__ballot(inb && G.nonfinite) != 0ull && lane == 0) set_status(status, VRS_ERR_NONFINITE);
    for (int v = 0; v < views.n; ++v) {
        const GeoView& V = views.v[v];
        const size_t slot = size_t(v) * size_t(g.n) + size_t(i);
        Geo geo;
        const bool ok = inb && make_geo(G, V, kn, views.ln_amin, geo);
        if (inb && !ok) counts[slot] = 0;
        if (ok) {
            int tx0, tx1, ty0, ty1;
            float bbox[4];
            cone_tiles(geo, V, tx0, tx1, ty0, ty1, bbox);
            const int ncx = max(tx1 - tx0 + 1, 0), ncy = max(ty1 - ty0 + 1, 0);
            const TileGeo& t = geo.tg;
            TileRect rc;
            rc.tx0 = tx0;
            rc.ty0 = ty0;
            rc.ncx = uint16_t(ncx);
            rc.ncy = uint16_t(ncy);
            // With visibility culling, only the visible tiles of the
            // rectangle: four reads of the summed-area table (Fig. 5b).
            const int cnt = (V.sat && ncx > 0 && ncy > 0) ? int(sat_count(V.sat, V.ntx, tx0, tx1, ty0, ty1))
                                                         : ncx * ncy;
            rc.count = cnt;
            counts[slot] = uint32_t(cnt);
            rects[slot] = rc;
            // Render record (field map in vrs_internal.h); the colour goes to
            // the colour array (k_color).
            const double xi = floor(t.x0), yi = floor(t.y0);
            const float zs = float(sqrt(0.5 / M_LN2));  // |z|^2 = (log2 e / 2) D^2
            float4* st = stage[w];
            st[stage_slot(lane, 0)] = make_float4(float(xi), float(yi), float(t.x0 - xi), float(t.y0 - yi));
            st[stage_slot(lane, 1)] =
                make_float4(float(t.M[0]) * zs, float(t.M[1]) * zs, float(t.M[2]) * zs, float(t.M[3]) * zs);
            st[stage_slot(lane, 2)] =
                make_float4(float(t.a3x), float(t.a3y), float(geo.l2s), float(t.kappa * (0.5 * M_LOG2E)));
            st[stage_slot(lane, 3)] = make_float4(float(t.n0), float(t.nx), float(t.ny), float(G.sigma));
            st[stage_slot(lane, 4)] = make_float4(float(t.w0[0]), float(t.w0[1]), float(t.w0[2]), float(t.wx[0]));
            st[stage_slot(lane, 5)] = make_float4(float(t.wx[1]), float(t.wx[2]), float(t.wy[0]), float(t.wy[1]));
            st[stage_slot(lane, 6)] = make_float4(float(t.wy[2]), 0.f, 0.f, 0.f);
            st[stage_slot(lane, 7)] = make_float4(bbox[0], bbox[1], bbox[2], bbox[3]);
        }
        const uint64_t okm = __ballot(ok);
        wave_sync_lds();
        // Piece q = 64 c + lane of the wave's records: record q / 8, field q % 8.
        float4* dst = reinterpret_cast<float4*>(proj + (size_t(v) * size_t(g.n) + size_t(wave_i0)) * kRec);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int q = c * 64 + lane;
            if ((okm >> (q >> 3)) & 1ull) dst[q] = stage[w][stage_slot(q >> 3, q & 7)];
        }
        wave_sync_lds();
    }
}

// View-dependent colour of every Gaussian in every view from its SH
// coefficients, written to the colour array as one float4 per slot (kept
// apart from k_preprocess so that the 48 coefficients do not occupy
// registers across the FP64 set-up).  The SH degree is a template
// parameter: the coefficients are loaded once per Gaussian, all at a time,
// and applied to every view; views go in groups (two for a stereo pair,
// else four) that bound the registers their basis values take.  Culled
// Gaussian-views get a colour too; no list refers to them.
template <int kColorViews, int kDeg>
__global__ void __launch_bounds__(256) k_color(GaussPtrs g, GeoViews views, float* __restrict__ proj, int* status) {
    // No implicit multiply-add contraction: every rounding is the one the
    // source states (the explicit fmaf calls), so a view's colour is the
    // same bits whichever instantiation and view slot computes it.
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int n = g.n;
    constexpr int K = (kDeg + 1) * (kDeg + 1);
    // All coefficients are loaded up front, so their loads are in flight
    // together rather than one coefficient's three at a time.
    float sh[K * 3];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) sh[k] = g.sh[k * n + i];
    float4* cols = const_cast<float4*>(colour_array(proj, size_t(views.n) * size_t(n)));
    const double mu[3] = {double(g.means[i]), double(g.means[n + i]), double(g.means[2 * n + i])};
    for (int v0 = 0; v0 < views.n; v0 += kColorViews) {
        float Y[kColorViews][16];
        float rgb[kColorViews][3];
#pragma unroll
        for (int j = 0; j < kColorViews; ++j) {
            const int v = min(v0 + j, views.n - 1);
            const GeoView& V = views.v[v];
            // Direction from the eye centre o = -R^T t to the mean.
            double dir[3];
            for (int c = 0; c < 3; ++c)
                dir[c] = mu[c] + (double(V.R[c]) * V.t[0] + double(V.R[3 + c]) * V.t[1] + double(V.R[6 + c]) * V.t[2]);
            const double idn = 1.0 / sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
            const float fd[3] = {float(dir[0] * idn), float(dir[1] * idn), float(dir[2] * idn)};
            sh_basis(fd, Y[j]);
            rgb[j][0] = rgb[j][1] = rgb[j][2] = 0.5f;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int j = 0; j < kColorViews; ++j) rgb[j][c] = fmaf(sh[k * 3 + c], Y[j][k], rgb[j][c]);
            }
        }
#pragma unroll
        for (int j = 0; j < kColorViews; ++j) {
            if (v0 + j < views.n) {
                // A colour made non-finite by NaN or infinite coefficients is
                // taken as black and reported.
                const bool fin = isfinite(rgb[j][0]) && isfinite(rgb[j][1]) && isfinite(rgb[j][2]);
                if (!fin) set_status(status, VRS_ERR_NONFINITE);
                cols[size_t(v0 + j) * size_t(n) + size_t(i)] =
                    fin ? make_float4(fmaxf(rgb[j][0], 0.f), fmaxf(rgb[j][1], 0.f), fmaxf(rgb[j][2], 0.f), 0.f)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    }
}


// The k-th candidate tile of a Gaussian: the k-th tile of its rectangle in
// row-major order, or, when some of the rectangle is invisible, the k-th
// visible one -- rows are skipped by their visible counts and the column is
// found by a binary search of the row's counts, all from the summed-area
// table.
__device__ inline void kth_tile(const GeoView& V, const TileRect& tg, int k, int& tx, int& ty) {
    const int ncx = tg.ncx;
    if (!V.sat || tg.count == ncx * int(tg.ncy)) {
        tx = tg.tx0 + k % ncx;
        ty = tg.ty0 + k / ncx;
        return;
    }
    const int x0 = tg.tx0, x1 = tg.tx0 + ncx - 1;
    int y = tg.ty0;
    for (;;) {
        const int rc = int(sat_count(V.sat, V.ntx, x0, x1, y, y));
        if (k < rc) break;
        k -= rc;
        ++y;
    }
    int lo = x0, hi = x1;  // smallest x with more than k visible tiles in [x0, x]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (int(sat_count(V.sat, V.ntx, x0, mid, y, y)) > k) hi = mid;
        else lo = mid + 1;
    }
    tx = lo;
    ty = y;
}

// One wave per block owns 64 consecutive (view, Gaussian) slots and deals
// their candidates out to its lanes 64 at a time, so every lane tests one
// candidate per step whatever the spread of per-Gaussian counts.  First each
// lane derives its own slot's FP64 set-up from the Gaussian's parameters
// into LDS (44 bytes read per Gaussian-view instead of a 176-byte record
// written by K1 and read back here).  The owner of candidate j of the wave
// is found by a 6-step search of the wave's count prefix in LDS; the lane
// then reads the owner's set-up from LDS and its rectangle from K1.  n_inst[0]: candidates (from the scan),
// n_inst[1]: kept instances.

template <int kViews>
__global__ void __launch_bounds__(64) k_duplicate(GaussPtrs g, GeoViews views, Knobs kn, int n,
                                                  const TileRect* __restrict__ rects,
                                                  const uint32_t* __restrict__ offsets,
                                                  const uint32_t* __restrict__ counts, size_t nslots,
                                                  uint32_t* __restrict__ n_inst, uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ gids, size_t capacity) {
    __shared__ uint32_t pre[65];
    __shared__ GeoView vw[kViews];  // the views the block's slots fall in, from v_lo
    __shared__ TileGeo tgl[64];
    __shared__ int mark[64];
    // No candidates, or more than the 32-bit offsets can address (the scan
    // then reports the overflow and leaves a total of 0): nothing to write.
    if (n_inst[0] == 0u) return;
    const int lane = threadIdx.x;
    const size_t s0 = size_t(blockIdx.x) * 64;
    const size_t nown = min(size_t(64), nslots - s0);
    const int v_lo = int(s0 / size_t(n)), v_hi = int((s0 + nown - 1) / size_t(n));
    for (int v = v_lo; v <= v_hi; ++v)
        if (lane == 0) vw[v - v_lo] = views.v[v];
    const size_t s = s0 + lane;
    const uint32_t c = s < nslots ? counts[s] : 0u;
    // This slot's tile rectangle, as four words that the candidates' lanes
    // fetch from the owner's lane.
    uint4 myrc = make_uint4(0u, 0u, 0u, 0u);
    if (c > 0) myrc = reinterpret_cast<const uint4*>(rects)[s];
    uint32_t incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    pre[lane] = incl - c;
    if (lane == 63) pre[64] = incl;
    __syncthreads();
    if (c > 0) {  // K1 counted candidates: the set-up succeeds as it did there
        const int v = int(s / size_t(n));
        Geo geo;
        if (make_geo(load_gaussian(g, int(s - size_t(v) * size_t(n))), vw[v - v_lo], kn, views.ln_amin, geo)) {
            // Per-Gaussian key depths (view z, distance) replace the per-tile
            // depth: r then holds the key of every tile of the Gaussian.
            if (kn.depth_mode == VRS_DEPTH_VIEW_Z) geo.tg.r = geo.muc[2];
        } else {
            // (Not reached.)  Every tile test then fails: dead keys.
            geo.tg.x0 = geo.tg.y0 = __builtin_nan("");
            geo.tg.kappa = -1.0;
        }
        tgl[lane] = geo.tg;
    }
    __syncthreads();
    const uint32_t total = pre[64];
    const uint32_t my0 = incl - c;  // this slot's first candidate in the block
    const size_t base = offsets[s0];
    for (uint32_t j0 = 0; j0 < total; j0 += 64) {
        // Owner of candidate j0 + lane: every slot with candidates in this
        // window marks where its run enters it; the owner is the last mark at
        // or before the lane (a running maximum, the slots being in order).
        mark[lane] = -1;
        __syncthreads();
        if (c > 0 && my0 < j0 + 64u && my0 + c > j0) mark[(my0 > j0 ? my0 : j0) - j0] = lane;
        __syncthreads();
        int ow = mark[lane];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(ow, d);
            if (lane >= d) ow = max(ow, y);
        }
        __syncthreads();  // (the marks are read before the next window's reset)
        TileRect rc;
        {
            const uint4 r4 = make_uint4(__shfl(myrc.x, ow), __shfl(myrc.y, ow), __shfl(myrc.z, ow), __shfl(myrc.w, ow));
            memcpy(&rc, &r4, sizeof(rc));
        }
        const uint32_t j = j0 + lane;
        bool kept;
        const size_t cg = base + j;
        if (j < total && cg < capacity) {
            const size_t o = s0 + ow;
            const int v = int(o / size_t(n));
            const int i = int(o - size_t(v) * size_t(n));
            const GeoView& V = vw[v - v_lo];
            const TileGeo& tg = tgl[ow];
            const int k = int(j - pre[ow]);
            int tx, ty;
            kth_tile(V, rc, k, tx, ty);
            double bx0, by0, bx1, by1, depth;
            tile_box(V, tx, ty, bx0, by0, bx1, by1);
            kept = tile_test(tg, V, bx0, by0, bx1, by1, &depth);
            if (kn.depth_mode != VRS_DEPTH_TILE_MAX) depth = tg.r;
            const uint64_t tile = uint64_t(V.tile_off) + uint64_t(ty) * V.ntx + tx;
            keys[cg] = kept ? ((tile << 32) | uint64_t(ord_f32(float(depth)))) : ~0ull;
            gids[cg] = uint32_t(i);
        }
    }
}

// n_inst[1] = number of live (non-dead) keys among the candidates: per-thread
// counts, one block reduction, one atomic per block.
__global__ void __launch_bounds__(256) k_count_live(const uint64_t* __restrict__ keys, uint32_t* n_inst,
                                                    size_t capacity) {
    __shared__ uint32_t part[4];
    const size_t total = min(size_t(n_inst[0]), capacity);
    uint32_t cnt = 0;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x)
        cnt += keys[i] != ~0ull ? 1u : 0u;
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t b = part[0] + part[1] + part[2] + part[3];
        if (b) atomicAdd(&n_inst[1], b);
    }
}

// Also clears `clear` (n_clear words: the tile ranges the sort fills in
// later, when the caller passes them), saving that launch.
__global__ void k_dup_init(uint32_t* n_inst, size_t capacity, int* status, uint32_t* __restrict__ clear,
                           size_t n_clear) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        n_inst[1] = 0;
        if (size_t(n_inst[0]) > capacity) set_status(status, VRS_ERR_CAPACITY);
    }
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_clear; i += size_t(gridDim.x) * blockDim.x)
        clear[i] = 0u;
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------

template <int kColorViews>
void launch_color(const GaussPtrs& g, const GeoViews& views, float* proj, int* status, int blocks, hipStream_t s) {
    switch (g.sh_degree) {
        case 0: hipLaunchKernelGGL((k_color<kColorViews, 0>), dim3(blocks), dim3(256), 0, s, g, views, proj, status); break;
        case 1: hipLaunchKernelGGL((k_color<kColorViews, 1>), dim3(blocks), dim3(256), 0, s, g, views, proj, status); break;
        case 2: hipLaunchKernelGGL((k_color<kColorViews, 2>), dim3(blocks), dim3(256), 0, s, g, views, proj, status); break;
        default: hipLaunchKernelGGL((k_color<kColorViews, 3>), dim3(blocks), dim3(256), 0, s, g, views, proj, status); break;
    }
}

int launch_preprocess(const GaussPtrs& g, const GeoViews& views, const Knobs& kn, float* proj,
                      uint32_t* counts, int* status, hipStream_t s) {
    if (g.n == 0) return VRS_OK;
    const size_t nslots = size_t(g.n) * views.n;
    TileRect* rects = reinterpret_cast<TileRect*>(reinterpret_cast<char*>(proj) + rect_offset_bytes(nslots));
    const int blocks = (g.n + 255) / 256;
    hipLaunchKernelGGL(k_preprocess, dim3(blocks), dim3(256), 0, s, g, views, kn, proj, rects, counts, status);
    // Groups of two views for a stereo pair (no work on padding views),
    // else four.
    if (views.n <= 2)
        launch_color<2>(g, views, proj, status, blocks, s);
    else
        launch_color<4>(g, views, proj, status, blocks, s);
    return launch_status(hipGetLastError());
}

// With count_live false n_inst[1] is left at zero for the caller to fill
// (the sort's first kernel counts the live keys anyway).
int launch_duplicate(const GaussPtrs& g, const GeoViews& views, const Knobs& kn, const float* proj,
                     const uint32_t* counts, uint64_t* keys, uint32_t* gids, size_t capacity,
                     uint32_t* n_inst, void* ws, int* status, hipStream_t s, bool count_live, uint32_t* clear,
                     size_t n_clear) {
    const size_t nslots = size_t(g.n) * size_t(views.n);
    uint32_t* offsets = static_cast<uint32_t*>(ws);
    uint32_t* tmp = offsets + nslots;
    // Candidate offsets, the candidate total in n_inst[0], and the set-up
    // below, in two launches where the scan is small enough.
    int rc = launch_scan_with_setup(counts, offsets, nslots, n_inst, tmp, capacity, status, clear, n_clear, s);
    if (rc == VRS_ERR_UNSUPPORTED) {
        rc = launch_exclusive_scan(counts, offsets, nslots, n_inst, tmp, status, s);
        if (rc != VRS_OK) return rc;
        const size_t clear_blocks = (n_clear + 255) / 256;
        hipLaunchKernelGGL(k_dup_init, dim3(clear_blocks == 0 ? 1 : (clear_blocks < 1024 ? clear_blocks : 1024)),
                           dim3(256), 0, s, n_inst, capacity, status, clear, n_clear);
    } else if (rc != VRS_OK) {
        return rc;
    }
    if (nslots == 0 || capacity == 0) return launch_status(hipGetLastError());
    const TileRect* rects =
        reinterpret_cast<const TileRect*>(reinterpret_cast<const char*>(proj) + rect_offset_bytes(nslots));
    const size_t blocks = (nslots + 63) / 64;
    // 64 consecutive slots fall in at most two views when a view has 64
    // Gaussians or more.
    if (g.n >= 64)
        hipLaunchKernelGGL(k_duplicate<2>, dim3(blocks), dim3(64), 0, s, g, views, kn, g.n, rects, offsets, counts,
                           nslots, n_inst, keys, gids, capacity);
    else
        hipLaunchKernelGGL(k_duplicate<VRS_MAX_VIEWS>, dim3(blocks), dim3(64), 0, s, g, views, kn, g.n, rects,
                           offsets, counts, nslots, n_inst, keys, gids, capacity);
    if (count_live) hipLaunchKernelGGL(k_count_live, dim3(256), dim3(256), 0, s, keys, n_inst, capacity);
    return launch_status(hipGetLastError());
}

}  // namespace vrs
