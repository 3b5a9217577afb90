// Two-pass foveated rendering, the comparison baseline of App. A: a centre
// pass at full resolution through a tight frustum, a periphery pass at half
// resolution, and one kernel that upsamples the periphery bilinearly and
// blends it with the centre by the continuous foveation mask.  The passes
// themselves are ordinary plain renders (vrs_preprocess, vrs_sort,
// vrs_render_foveated) of the cameras vrs_two_pass_views derives.
#include <math.h>
#include <string.h>

#include "vrs_internal.h"

namespace vrs {

struct TwoPassView {
    float* out;               // [4][H][W]
    const float* centre;      // [4][y1-y0][x1-x0], or null
    const float* low;         // [4][hl][wl]
    int W, H, wl, hl;
    int x0, y0, x1, y1;       // centre box
    FovMaskF mask;            // foveation mask of the full-resolution view
};

// One thread per output pixel of one view.
__global__ void __launch_bounds__(256) k_two_pass_compose(TwoPassView V) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= V.W || y >= V.H) return;
    // Bilinear sample of the half-resolution image: its pixel centres sit at
    // full-resolution 2i + 1, so pixel centre x + 1/2 is at (x + 1/2)/2 - 1/2.
    const float sx = (float(x) + 0.5f) * 0.5f - 0.5f, sy = (float(y) + 0.5f) * 0.5f - 0.5f;
    const float fx0 = floorf(sx), fy0 = floorf(sy);
    const float ax = sx - fx0, ay = sy - fy0;
    const int ix = int(fx0), iy = int(fy0);
    const int xa = min(max(ix, 0), V.wl - 1), xb = min(max(ix + 1, 0), V.wl - 1);
    const int ya = min(max(iy, 0), V.hl - 1), yb = min(max(iy + 1, 0), V.hl - 1);
    const size_t lplane = size_t(V.wl) * V.hl, plane = size_t(V.W) * V.H;
    const bool in_box = x >= V.x0 && x < V.x1 && y >= V.y0 && y < V.y1;
    const float wm = in_box ? fovea_weight(V.mask, x, y) : 0.f;
    const int cw = V.x1 - V.x0;
    const size_t cplane = size_t(cw) * size_t(V.y1 - V.y0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float* L = V.low + c * lplane;
        const float top = fmaf(ax, L[size_t(ya) * V.wl + xb] - L[size_t(ya) * V.wl + xa], L[size_t(ya) * V.wl + xa]);
        const float bot = fmaf(ax, L[size_t(yb) * V.wl + xb] - L[size_t(yb) * V.wl + xa], L[size_t(yb) * V.wl + xa]);
        float o = fmaf(ay, bot - top, top);
        if (in_box) {
            const float cv = V.centre[c * cplane + size_t(y - V.y0) * cw + (x - V.x0)];
            o = fmaf(wm, cv - o, o);
        }
        V.out[c * plane + size_t(y) * V.W + x] = o;
    }
}

}  // namespace vrs

using namespace vrs;

namespace {

float derive_fov(int width, double f) { return float(2.0 * atan(double(width) / 2.0 / f) * (180.0 / M_PI)); }

double focal_of(const vrs_camera& c) {
    return (double(c.width) / 2.0) / tan(double(c.fov_x_deg) * (M_PI / 180.0) / 2.0);
}

}  // namespace

extern "C" {

int vrs_two_pass_views(const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views, const vrs_params* p,
                       const void* plan, vrs_camera* centre_cams, int32_t* centre_boxes, vrs_camera* low_cams,
                       vrs_stream_t stream) {
    if (!cams || !foveas || !p || !plan || !centre_cams || !centre_boxes || !low_cams) return VRS_ERR_INVALID_ARG;
    if (n_views < 1 || n_views > VRS_MAX_VIEWS) return VRS_ERR_INVALID_ARG;
    vrs_sizes sz;
    int rc = vrs_workspace_size(0, cams, foveas, n_views, p, 0, &sz);
    if (rc != VRS_OK) return rc;
    // The class maps of the plan, to the host.
    const size_t cls_off = kPlanItemsOff + size_t(sz.items_max) * 4;
    const size_t cls_bytes = sz.plan_bytes - cls_off;
    uint8_t* cls = static_cast<uint8_t*>(malloc(cls_bytes ? cls_bytes : 1));
    if (!cls) return VRS_ERR_HIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(cls, static_cast<const char*>(plan) + cls_off, cls_bytes, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        free(cls);
        return VRS_ERR_HIP;
    }
    size_t off = 0;
    for (int v = 0; v < n_views; ++v) {
        const vrs_camera& c = cams[v];
        const double f = focal_of(c);
        int32_t* b = centre_boxes + 4 * v;
        b[0] = b[1] = b[2] = b[3] = 0;
        if (foveas[v].enabled) {
            // Bounding box of the split 32x32 tiles (a pixel centre with w > 0).
            const int nt32x = (c.width + 31) / 32, nt32y = (c.height + 31) / 32;
            const int ntx16 = 2 * nt32x;
            int tx0 = nt32x, ty0 = nt32y, tx1 = -1, ty1 = -1;
            for (int ty = 0; ty < nt32y; ++ty)
                for (int tx = 0; tx < nt32x; ++tx) {
                    const uint8_t k = cls[off + size_t(2 * ty) * ntx16 + 2 * tx];
                    if (k == VRS_CLASS_HIGH || k == VRS_CLASS_HYBRID) {
                        tx0 = tx < tx0 ? tx : tx0;
                        ty0 = ty < ty0 ? ty : ty0;
                        tx1 = tx > tx1 ? tx : tx1;
                        ty1 = ty > ty1 ? ty : ty1;
                    }
                }
            off += size_t(ntx16) * size_t(2 * nt32y);
            if (tx1 >= 0) {
                b[0] = tx0 * 32;
                b[1] = ty0 * 32;
                b[2] = (tx1 + 1) * 32 < c.width ? (tx1 + 1) * 32 : c.width;
                b[3] = (ty1 + 1) * 32 < c.height ? (ty1 + 1) * 32 : c.height;
            }
        }
        vrs_camera& cc = centre_cams[v];
        cc = c;
        if (b[2] > b[0]) {
            cc.width = b[2] - b[0];
            cc.height = b[3] - b[1];
            cc.fov_x_deg = derive_fov(cc.width, f);
            cc.cx = float(double(c.cx) - b[0]);
            cc.cy = float(double(c.cy) - b[1]);
        }
        vrs_camera& lc = low_cams[v];
        lc = c;
        lc.width = (c.width + 1) / 2;
        lc.height = (c.height + 1) / 2;
        lc.fov_x_deg = derive_fov(lc.width, f / 2.0);
        lc.cx = float(double(c.cx) / 2.0);
        lc.cy = float(double(c.cy) / 2.0);
    }
    free(cls);
    return VRS_OK;
}

int vrs_two_pass_compose(const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                         const int32_t* centre_boxes, const float* const* centre_rgba,
                         const float* const* low_rgba, float* const* out_rgba, vrs_stream_t stream) {
    if (!cams || !foveas || !centre_boxes || !low_rgba || !out_rgba) return VRS_ERR_INVALID_ARG;
    if (n_views < 1 || n_views > VRS_MAX_VIEWS) return VRS_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (int v = 0; v < n_views; ++v) {
        const vrs_camera& c = cams[v];
        const vrs_fovea& fv = foveas[v];
        const int32_t* b = centre_boxes + 4 * v;
        if (c.width < 1 || c.height < 1 || !low_rgba[v] || !out_rgba[v]) return VRS_ERR_INVALID_ARG;
        const bool has_box = b[2] > b[0] && b[3] > b[1];
        if (has_box && (b[0] < 0 || b[1] < 0 || b[2] > c.width || b[3] > c.height || !centre_rgba ||
                        !centre_rgba[v] || !fv.enabled))
            return VRS_ERR_INVALID_ARG;
        TwoPassView V;
        memset(&V, 0, sizeof(V));
        V.out = out_rgba[v];
        V.centre = has_box ? centre_rgba[v] : nullptr;
        V.low = low_rgba[v];
        V.W = c.width;
        V.H = c.height;
        V.wl = (c.width + 1) / 2;
        V.hl = (c.height + 1) / 2;
        if (has_box) {
            V.x0 = b[0]; V.y0 = b[1]; V.x1 = b[2]; V.y1 = b[3];
        }
        V.mask = make_fov_mask(c, fv);
        hipLaunchKernelGGL(k_two_pass_compose, dim3((c.width + 63) / 64, (c.height + 3) / 4), dim3(256), 0, s, V);
    }
    return launch_status(hipGetLastError());
}

}  // extern "C"
