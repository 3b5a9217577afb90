// Internal declarations shared by the HIP translation units of libvrs.
// Kernels take compact per-view tables by value (kernel arguments stay well
// under 4 KB for VRS_MAX_VIEWS views), so calls on different streams never
// share mutable state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vrs.h"

namespace vrs {

constexpr int kRec = VRS_RECORD_FLOATS;

// Radix sort geometry (K4): 256-thread blocks each ranking a 2048-key tile
// (twice the blocks of 4096-key tiles: better latency hiding, 3 % faster
// sort), 8-bit digits, at most 8 passes.
constexpr int kSortThreads = 256;
constexpr int kSortItemsPerLane = 12;
constexpr int kSortTile = kSortThreads * kSortItemsPerLane;
constexpr int kRadix = 256;
constexpr int kMaxPasses = 8;

// Sort workspace for `capacity` pairs: ping-pong pairs, the [256][blocks]
// histogram of one pass, the digit offsets of every pass, and the per-tile
// digit counts of every pass.
constexpr size_t sort_ws_layout_bytes(size_t capacity) {
    const size_t nb = capacity ? (capacity + kSortTile - 1) / kSortTile : 1;
    return ((capacity * (sizeof(uint64_t) + sizeof(uint32_t)) + 255) & ~size_t(255)) +
           ((size_t(kRadix) * nb + 63) & ~size_t(63)) * sizeof(uint32_t) +
           size_t(kMaxPasses) * kRadix * sizeof(uint32_t) +
           size_t(kMaxPasses) * nb * kRadix * sizeof(uint32_t);
}

// Record layout (floats) of one projected Gaussian in one view.  The render
// kernel stages fields [4, 28) plus the tile-relative mean offset; the per-pair
// arithmetic it needs is described next to each group.
enum RecField : int {
    R_X0I = 0, R_Y0I = 1,    // integer part of the mean's image point (pixels)
    R_X0F = 2, R_Y0F = 3,    // fractional part in [0, 1)
    R_M00 = 4, R_M01 = 5,    // z = M delta / h: whitened tangent-plane coords,
    R_M10 = 6, R_M11 = 7,    //   scaled so that |z|^2 = log2(e) D^2 / 2
    R_A3X = 8, R_A3Y = 9,    // h = 1 + a3 . delta  (> 0 iff the ray is in front)
    R_L2S = 10,              // log2(opacity)
    R_KAP = 11,              // log2(opacity) - log2(alpha_min): pass iff |z|^2 <= KAP
    R_N0 = 12, R_NX = 13, R_NY = 14,  // depth numerator  n0 + nx dx + ny dy
    R_SIG = 15,              // opacity
    R_W0 = 16,               // depth denominator |w0 + dx wx + dy wy|^2 (w0: 16..18,
    R_WX = 19, R_WY = 22,    //   wx: 19..21, wy: 22..24)
    R_FREE = 25,             // 25..27 unused (colours are in the colour array)
    R_BOX = 28,              // pixel box (x0, y0, x1, y1) holding every sample
                             //   where alpha can reach alpha_min
};

// Layout of the `proj` buffer for nslots = n_views * n (view-major) slots:
// the FP32 render records, then the candidate tile rectangles (16 bytes
// each), then one float4 colour (r, g, b, 0) per slot.
constexpr size_t kTileRectBytes = 16;
__host__ __device__ inline size_t rect_offset_bytes(size_t nslots) { return nslots * kRec * sizeof(float); }
__host__ __device__ inline size_t colour_offset_bytes(size_t nslots) {
    return nslots * (kRec * sizeof(float) + kTileRectBytes);
}
__host__ __device__ inline const float4* colour_array(const float* proj, size_t nslots) {
    return reinterpret_cast<const float4*>(reinterpret_cast<const char*>(proj) + colour_offset_bytes(nslots));
}

struct GaussPtrs {
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opac;
    const float* sh;
    int n;
    int sh_degree;
};

// Geometry of one view for the per-Gaussian kernels.
struct GeoView {
    double f;
    double inv_f;
    float R[9];
    float t[3];
    float cx, cy;
    int W, H;
    int T;        // sort tile size (16 or 32)
    int ntx, nty; // sort grid
    uint32_t tile_off;
    const uint32_t* sat;  // summed-area table of visible sort tiles [nty+1][ntx+1], or null (all visible)
};

// Visible tiles inside the inclusive tile rectangle [tx0, tx1] x [ty0, ty1]
// from the summed-area table's four corners.
__host__ __device__ inline uint32_t sat_count(const uint32_t* S, int ntx, int tx0, int tx1, int ty0, int ty1) {
    const size_t st = size_t(ntx) + 1;
    return (S[size_t(ty1 + 1) * st + tx1 + 1] - S[size_t(ty0) * st + tx1 + 1]) -
           (S[size_t(ty1 + 1) * st + tx0] - S[size_t(ty0) * st + tx0]);
}

struct GeoViews {
    int n;
    double ln_amin;  // ln(alpha_min)
    GeoView v[VRS_MAX_VIEWS];
};

struct Knobs {
    float z_near, alpha_min, alpha_max, t_min, dilation;
    float bg[3];
    int window;  // resort window W (the insertion network may have more slots)
    int depth_mode;  // VRS_DEPTH_*: the sort key depth
};

// The instantiated insertion networks; a window W runs on the smallest one
// with at least W slots (the surplus slots hold placeholders that are never
// emitted before the final flush, so the network behaves as a W-window).
// W = 0 (no resort) runs on the one-slot network with its slot a
// placeholder: every entry is emitted as it arrives.
__host__ __device__ inline int window_network(int w) {
    return w <= 1 ? 1 : w <= 4 ? w : w <= 6 ? 6 : w <= 8 ? 8 : w <= 12 ? 12 : w <= 16 ? 16 : w <= 24 ? 24 : 32;
}

// Alpha of a (sample, entry) pair that passed the alpha_min test: opacity
// 2^(-q / h^2) with q = |M delta|^2 and h = 1 + a3 . delta, clamped to
// alpha_max.  One definition for the forward blend and the backward replay,
// so that both take the same roundings.  The hardware exp2 has no denormal
// range handling; a passing pair's exponent is at least log2(alpha_min),
// far inside the normal range, where it equals exp2f.
__device__ inline float splat_alpha(float l2s, float q, float h2, float amax) {
    return fminf(amax, __builtin_amdgcn_exp2f(fmaf(-q, __builtin_amdgcn_rcpf(h2), l2s)));
}

// Per-view data for the render and compose kernels.
// The continuous foveation mask in FP32 (HYBRID blending, two-pass blend).
struct FovMaskF {
    int shape;          // VRS_FOVEA_DISC or VRS_FOVEA_RECT
    float f, cx, cy;    // camera focal length and principal point (pixels)
    float fdir[3];      // disc: unit ray of the fovea centre (camera frame)
    float rho, band;    // disc radius (rad); band fraction
    float fc[2], half[2];  // rectangle: centre and half-extents (pixels)
};

// Mask weight at the centre of pixel (x, y).
__device__ inline float fovea_weight(const FovMaskF& M, int x, int y) {
    const float px = float(x) + 0.5f, py = float(y) + 0.5f;
    if (M.shape == VRS_FOVEA_RECT) {
        float w = 1.f;
        const float p[2] = {px, py};
        for (int a = 0; a < 2; ++a) {
            const float d = fabsf(p[a] - M.fc[a]);
            const float h = M.half[a];
            float u;
            if (!(h > 0.f)) u = 0.f;
            else if (!(M.band > 0.f)) u = d <= h ? 1.f : 0.f;
            else u = fminf(fmaxf((h * (1.f + M.band) - d) / (h * M.band), 0.f), 1.f);
            w = fminf(w, u);
        }
        return w;
    }
    if (!(M.rho > 0.f)) return 0.f;
    // Angle between the pixel's ray and the fovea-centre ray.
    const float d0 = (px - M.cx) / M.f, d1 = (py - M.cy) / M.f;
    const float cx_ = d1 * M.fdir[2] - M.fdir[1];
    const float cy_ = M.fdir[0] - d0 * M.fdir[2];
    const float cz_ = d0 * M.fdir[1] - d1 * M.fdir[0];
    const float dotp = d0 * M.fdir[0] + d1 * M.fdir[1] + M.fdir[2];
    const float e = atan2f(sqrtf(cx_ * cx_ + cy_ * cy_ + cz_ * cz_), dotp);
    if (!(M.band > 0.f)) return e <= M.rho ? 1.f : 0.f;
    return fminf(fmaxf((M.rho * (1.f + M.band) - e) / (M.rho * M.band), 0.f), 1.f);
}

// The FP32 mask parameters of a view (host side).
inline FovMaskF make_fov_mask(const vrs_camera& c, const vrs_fovea& fv) {
    FovMaskF m;
    const double f = (double(c.width) / 2.0) / tan(double(c.fov_x_deg) * (M_PI / 180.0) / 2.0);
    m.shape = fv.shape;
    m.f = float(f);
    m.cx = c.cx;
    m.cy = c.cy;
    const double d0 = (double(fv.center_px[0]) - double(c.cx)) / f;
    const double d1 = (double(fv.center_px[1]) - double(c.cy)) / f;
    const double dn = sqrt(d0 * d0 + d1 * d1 + 1.0);
    m.fdir[0] = float(d0 / dn);
    m.fdir[1] = float(d1 / dn);
    m.fdir[2] = float(1.0 / dn);
    m.rho = float(double(fv.radius_deg) * (M_PI / 180.0));
    m.band = fv.band_frac;
    m.fc[0] = fv.center_px[0];
    m.fc[1] = fv.center_px[1];
    m.half[0] = fv.half_px[0];
    m.half[1] = fv.half_px[1];
    return m;
}

struct RenderView {
    float* out;         // final rgba [4][H][W]
    float* pre;         // pre-compose image (foveated views), else == out
    FovMaskF mask;      // foveation mask (foveated views)
    int W, H;
    int T;              // sort tile size (16 or 32)
    int ntx;            // sort grid width
    int ntx16;          // 16x16 subtile grid width (class map row)
    uint32_t tile_off;
    uint32_t cls_off;   // offset of this view's class map in the plan
    uint8_t foveated;
    uint8_t nomix;      // write HYBRID samples unmixed (the backward's re-render)
    uint8_t skip;       // render nothing for this view's items
    uint8_t pad_;
};

struct RenderViews {
    int n;
    RenderView v[VRS_MAX_VIEWS];
};
static_assert(sizeof(RenderViews) < 3584, "render kernel arguments stay under 4 KB");

struct FovView {  // FP64 class decision of one foveated view
    double f, cx, cy;
    double dc[3];      // fovea-centre ray (unnormalised)
    double dcn;        // |dc|
    double cos_low;    // LOW iff cos(e) <= cos_low at every pixel
    double cos_high;   // HIGH iff cos(e) >= cos_high at every pixel
    int all_low;       // rho <= 0
    int shape;         // VRS_FOVEA_DISC or VRS_FOVEA_RECT
    double band;       // band fraction
    double fc[2];      // rectangle: centre (pixels)
    double half[2];    // rectangle: half-extents (pixels)
    int W, H, ntx32, nty32, ntx16, nty16;
    uint32_t cls_off;
};

// Visibility culling input of one view: the per-pixel mask (or null) and
// where its sort tiles' summed-area table goes.
struct VisView {
    const uint8_t* mask;
    int W, H, T, ntx, nty;
    uint32_t* sat;
};

struct VisViews {
    int n;
    VisView v[VRS_MAX_VIEWS];
};

// What the item builder needs of every view.
struct ItemView {
    int foveated;
    int T;          // sort tile size
    int ntx;        // sort grid width
    int ntx16;      // class-map row length
    int ntiles;     // sort-grid tiles of the view
    int W, H;
    uint32_t cls_off;
};

struct ItemViews {
    int n;
    ItemView v[VRS_MAX_VIEWS];
};

// Plain views of a backward launch.  Block b belongs to the view v with
// item_off[v] <= b < item_off[v + 1]; a 16x16 sort tile is one item, a
// 32x32 tile four (its 16x16 subtiles, row-major).
// A view of a backward launch.  Plain views: rgba and grad are the forward
// output and dL/d(output).  Foveated views: per-sample buffers in the
// pre-compose layout (a pixel's own sample, a LOW group's at its top-left
// pixel): rgba the samples' forward colour and alpha before the HYBRID mix,
// grad dL/d(sample).
struct BwdView {
    const float* rgba;  // [4][H][W]
    const float* grad;  // [4][H][W]
    int W, H, T, ntx;
    uint32_t tile_off;
};

struct BwdViews {
    int n;
    BwdView v[VRS_MAX_VIEWS];
};

// Chain of dL/d(final image) of a foveated view back to its samples.
struct FovGradView {
    const float* gout;    // dL/d(final)   [4][H][W]
    float* gpre;          // dL/d(pre-compose image)
    float* gsamp;         // dL/d(sample), pre-compose layout
    const uint8_t* cls;   // this view's class map (16x16 subtiles)
    int W, H, ntx16;
    FovMaskF mask;
};

// Gradient outputs, the layouts of GaussPtrs.
struct GradPtrs {
    float* means;
    float* log_scales;
    float* quats;
    float* opac;
    float* sh;
};

// Work items: view (5 bits) | class (2) | subtile (2) | sort-grid tile (23).
__host__ __device__ inline uint32_t item_pack(int view, int cls, int sub, uint32_t tile) {
    return (uint32_t(view) << 27) | (uint32_t(cls) << 25) | (uint32_t(sub) << 23) | tile;
}
__host__ __device__ inline int item_view(uint32_t it) { return int(it >> 27); }
__host__ __device__ inline int item_class(uint32_t it) { return int((it >> 25) & 3u); }
__host__ __device__ inline int item_sub(uint32_t it) { return int((it >> 23) & 3u); }
__host__ __device__ inline uint32_t item_tile(uint32_t it) { return it & 0x7FFFFFu; }

// Status helper: the first error written wins.
__device__ inline void set_status(int* status, int code) {
    if (status) atomicCAS(status, 0, code);
}

// Plan layout (bytes): [0, 4) item count, [256, 256 + 4 * items_max) items,
// then the u8 class maps of all views (16x16 subtile grids).
constexpr size_t kPlanItemsOff = 256;

// Launch helpers (host).
int launch_status(hipError_t e);
size_t scan_tmp_words(size_t n);
// Exclusive scan of n uint32 (in may equal out); *total (if non-null) gets
// the sum; tmp holds scan_tmp_words(n) words.  A sum of 2^32 - 1 or more
// sets *total to 0 and writes VRS_ERR_UNSUPPORTED to *status (if non-null).
int launch_exclusive_scan(const uint32_t* in, uint32_t* out, size_t n, uint32_t* total, uint32_t* tmp,
                          int* status, hipStream_t s);
// The same scan in two launches for 0 < n <= 4096 tiles of 2048 words (else
// VRS_ERR_UNSUPPORTED and nothing launched), fused with instantiation's
// set-up: the total goes to n_inst[0] (0 on overflow, as above), n_inst[1]
// is zeroed, a total above `capacity` writes VRS_ERR_CAPACITY to *status,
// and clear[0, n_clear) is zeroed.
int launch_scan_with_setup(const uint32_t* in, uint32_t* out, size_t n, uint32_t* n_inst, uint32_t* tmp,
                           size_t capacity, int* status, uint32_t* clear, size_t n_clear, hipStream_t s);

}  // namespace vrs
