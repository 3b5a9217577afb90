// K2: single-pass foveation map (Sec. 4.3, Fig. 5a).  For every 32x32 tile of
// a foveated view, decide from the continuous mask at its pixel centres
// whether it is a LOW periphery tile or is split into four 16x16 subtiles,
// and whether each subtile is HIGH (mask 1 everywhere) or HYBRID.  Then build
// the compact list of render work items, whose length is the exact number of
// blocks the render launch needs.
//
// Disc fovea: the mask depends on the angle e between a pixel's ray and the
// fovea-centre ray: w = 0 iff e >= rho (1 + b), w = 1 iff e <= rho.  Both
// tests are made on cos(e) in FP64 against host-computed cosines, so classes
// are decided far more precisely than the float32 inputs.  Rectangle fovea
// (the paper's layout): the weight itself is evaluated in FP64, operation by
// operation as the definition writes it.
//
// Visibility culling (Sec. 4.3, Fig. 5b): per view, the bitfield of sort
// tiles holding a visible pixel of the headset's mask, stored as its
// summed-area table.
#include "vrs_internal.h"

namespace vrs {

constexpr uint8_t kSubNone = 255;

// Rectangle mask weight (FP64): per axis clamp((h (1 + b) - |p - c|) / (h b), 0, 1),
// the smaller of the two; the indicator of the closed rectangle without a band.
__device__ inline double rect_weight(const FovView& V, double px, double py) {
#pragma clang fp contract(off)
    double w = 1.0;
    const double p[2] = {px, py};
    for (int a = 0; a < 2; ++a) {
        const double d = fabs(p[a] - V.fc[a]);
        const double h = V.half[a];
        double u;
        if (!(h > 0.0)) u = 0.0;
        else if (!(V.band > 0.0)) u = d <= h ? 1.0 : 0.0;
        else u = fmin(fmax((h * (1.0 + V.band) - d) / (h * V.band), 0.0), 1.0);
        w = fmin(w, u);
    }
    return w;
}

// One block per 32x32 tile of a foveated view: 256 threads x 4 pixels.
__global__ void __launch_bounds__(256) k_fovea_classes(FovView V, uint8_t* __restrict__ cls) {
    const int tile = blockIdx.x;
    const int tx = tile % V.ntx32, ty = tile / V.ntx32;
    __shared__ int any_pos;          // some pixel has w > 0
    __shared__ int not_one[4];       // subtile has a pixel with w < 1
    __shared__ int present[4];       // subtile has an in-image pixel
    if (threadIdx.x == 0) any_pos = 0;
    if (threadIdx.x < 4) { not_one[threadIdx.x] = 0; present[threadIdx.x] = 0; }
    __syncthreads();
    for (int k = 0; k < 4; ++k) {
        const int p = threadIdx.x + 256 * k;  // 0..1023
        const int lx = p & 31, ly = p >> 5;
        const int x = tx * 32 + lx, y = ty * 32 + ly;
        if (x >= V.W || y >= V.H) continue;
        const int sub = (lx >> 4) + 2 * (ly >> 4);
        bool pos, one;
        if (V.shape == VRS_FOVEA_RECT) {
            const double w = rect_weight(V, double(x) + 0.5, double(y) + 0.5);
            pos = w > 0.0;
            one = w >= 1.0;
        } else {
            const double d0 = (double(x) + 0.5 - V.cx) / V.f;
            const double d1 = (double(y) + 0.5 - V.cy) / V.f;
            const double dn = sqrt(d0 * d0 + d1 * d1 + 1.0);
            double c = (d0 * V.dc[0] + d1 * V.dc[1] + V.dc[2]) / (dn * V.dcn);
            c = fmin(fmax(c, -1.0), 1.0);
            pos = !V.all_low && !(c <= V.cos_low);
            one = !V.all_low && (c >= V.cos_high);
        }
        if (pos) atomicOr(&any_pos, 1);
        if (!one) atomicOr(&not_one[sub], 1);
        atomicOr(&present[sub], 1);
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int s = threadIdx.x;
        const int sx = 2 * tx + (s & 1), sy = 2 * ty + (s >> 1);
        uint8_t c;
        if (!present[s]) c = kSubNone;
        else if (!any_pos) c = VRS_CLASS_LOW;
        else c = not_one[s] ? VRS_CLASS_HYBRID : VRS_CLASS_HIGH;
        cls[V.cls_off + size_t(sy) * V.ntx16 + sx] = c;
    }
}

// Single block: count work items per tile, scan, and write them in order
// (view, tile, subtile).
__global__ void __launch_bounds__(1024) k_fovea_items(ItemViews views, const uint8_t* __restrict__ cls,
                                                     uint32_t* __restrict__ count,
                                                     uint32_t* __restrict__ items) {
    __shared__ uint32_t sh[1024];
    uint32_t carry = 0;
    const int t = threadIdx.x;
    for (int v = 0; v < views.n; ++v) {
        const ItemView& V = views.v[v];
        const int ntiles = V.ntiles;
        for (int c0 = 0; c0 < ntiles; c0 += 1024) {
            const int tile = c0 + t;
            uint32_t nit = 0;
            uint8_t sc[4] = {kSubNone, kSubNone, kSubNone, kSubNone};
            if (tile < ntiles) {
                const int tx = tile % V.ntx, ty = tile / V.ntx;
                if (!V.foveated && V.T == 16) {
                    nit = 1;
                } else if (!V.foveated) {
                    // Plain view with 32x32 sort tiles: one item per in-image subtile.
                    for (int s = 0; s < 4; ++s) {
                        const bool in = tx * 32 + (s & 1) * 16 < V.W && ty * 32 + (s >> 1) * 16 < V.H;
                        sc[s] = in ? VRS_CLASS_PLAIN : kSubNone;
                        nit += in ? 1u : 0u;
                    }
                } else {
                    for (int s = 0; s < 4; ++s)
                        sc[s] = cls[V.cls_off + size_t(2 * ty + (s >> 1)) * V.ntx16 + 2 * tx + (s & 1)];
                    if (sc[0] == VRS_CLASS_LOW) nit = 1;
                    else
                        for (int s = 0; s < 4; ++s) nit += sc[s] != kSubNone ? 1u : 0u;
                }
            }
            sh[t] = nit;
            __syncthreads();
            for (int off = 1; off < 1024; off <<= 1) {
                const uint32_t y = t >= off ? sh[t - off] : 0u;
                __syncthreads();
                sh[t] += y;
                __syncthreads();
            }
            uint32_t pos = carry + sh[t] - nit;
            const uint32_t tot = sh[1023];
            __syncthreads();
            if (tile < ntiles) {
                if (!V.foveated && V.T == 16) {
                    items[pos] = item_pack(v, VRS_CLASS_PLAIN, 0, uint32_t(tile));
                } else if (V.foveated && sc[0] == VRS_CLASS_LOW) {
                    items[pos] = item_pack(v, VRS_CLASS_LOW, 0, uint32_t(tile));
                } else {
                    for (int s = 0; s < 4; ++s)
                        if (sc[s] != kSubNone) items[pos++] = item_pack(v, sc[s], s, uint32_t(tile));
                }
            }
            carry += tot;
        }
    }
    if (t == 0) *count = carry;
}

// One block per sort tile of a view: the tile's bit (some pixel visible, or
// no mask) goes to the interior of the summed-area table, S[ty + 1][tx + 1].
__global__ void __launch_bounds__(256) k_vis_tiles(VisView V) {
    const int tile = blockIdx.x;
    const int tx = tile % V.ntx, ty = tile / V.ntx;
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (!V.mask) {
        if (threadIdx.x == 0) any = 1;
    } else {
        for (int p = threadIdx.x; p < V.T * V.T; p += 256) {
            const int x = tx * V.T + p % V.T, y = ty * V.T + p / V.T;
            if (x < V.W && y < V.H && V.mask[size_t(y) * V.W + x] != 0) any = 1;  // benign race: all write 1
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) V.sat[size_t(ty + 1) * (V.ntx + 1) + tx + 1] = any ? 1u : 0u;
}

// One block per view: zero the table's first row and column, then prefix
// sums along the rows, then along the columns.
__global__ void __launch_bounds__(1024) k_vis_sat(VisViews views) {
    const VisView& V = views.v[blockIdx.x];
    const int st = V.ntx + 1;
    for (int x = threadIdx.x; x < st; x += blockDim.x) V.sat[x] = 0u;
    for (int y = threadIdx.x; y < V.nty + 1; y += blockDim.x) V.sat[size_t(y) * st] = 0u;
    __syncthreads();
    for (int y = 1 + threadIdx.x; y <= V.nty; y += blockDim.x) {
        uint32_t run = 0;
        for (int x = 1; x <= V.ntx; ++x) {
            run += V.sat[size_t(y) * st + x];
            V.sat[size_t(y) * st + x] = run;
        }
    }
    __syncthreads();
    for (int x = 1 + threadIdx.x; x <= V.ntx; x += blockDim.x) {
        uint32_t run = 0;
        for (int y = 1; y <= V.nty; ++y) {
            run += V.sat[size_t(y) * st + x];
            V.sat[size_t(y) * st + x] = run;
        }
    }
}

int launch_fovea_plan(const FovView* fviews, const ItemViews& iviews, const VisViews& vis, void* plan,
                      size_t items_max, hipStream_t s) {
    uint32_t* count = static_cast<uint32_t*>(plan);
    uint32_t* items = reinterpret_cast<uint32_t*>(static_cast<char*>(plan) + kPlanItemsOff);
    uint8_t* cls = reinterpret_cast<uint8_t*>(items + items_max);
    for (int v = 0; v < iviews.n; ++v) {
        if (!iviews.v[v].foveated) continue;
        const FovView& V = fviews[v];
        hipLaunchKernelGGL(k_fovea_classes, dim3(V.ntx32 * V.nty32), dim3(256), 0, s, V, cls);
    }
    hipLaunchKernelGGL(k_fovea_items, dim3(1), dim3(1024), 0, s, iviews, cls, count, items);
    for (int v = 0; v < vis.n; ++v)
        hipLaunchKernelGGL(k_vis_tiles, dim3(vis.v[v].ntx * vis.v[v].nty), dim3(256), 0, s, vis.v[v]);
    hipLaunchKernelGGL(k_vis_sat, dim3(vis.n), dim3(1024), 0, s, vis);
    return launch_status(hipGetLastError());
}

}  // namespace vrs
