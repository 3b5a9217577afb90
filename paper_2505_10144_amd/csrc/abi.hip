// The extern "C" entry points declared in include/vrs.h: argument
// validation, per-view tables, buffer layouts and kernel launches.
#include <math.h>
#include <string.h>

#include "vrs_internal.h"

namespace vrs {

int launch_status(hipError_t e) { return e == hipSuccess ? VRS_OK : VRS_ERR_HIP; }

// Launchers defined in the kernel translation units.
int launch_preprocess(const GaussPtrs&, const GeoViews&, const Knobs&, float*, uint32_t*, int*, hipStream_t);
int launch_duplicate(const GaussPtrs&, const GeoViews&, const Knobs&, const float*, const uint32_t*, uint64_t*,
                     uint32_t*, size_t, uint32_t*, void*, int*, hipStream_t, bool, uint32_t*, size_t);
size_t sort_ws_bytes(size_t capacity);
int launch_sort_pairs(uint64_t*, uint32_t*, const uint32_t*, size_t, int, void*, int*, hipStream_t);
int launch_sort_pairs_ex(uint64_t*, uint32_t*, const uint32_t*, const uint32_t*, bool, size_t, int, void*, int*,
                         hipStream_t, uint32_t*);

// Bytes per Gaussian and view in `proj`: the FP32 render record plus the FP64
// tile-test record (TileGeo, 192 bytes) that instantiation reads.
constexpr size_t kProjBytesPerSlot = kRec * sizeof(float) + kTileRectBytes + 4 * sizeof(float);
size_t dup_ws_bytes(size_t nslots) { return (nslots + scan_tmp_words(nslots) + 64) * sizeof(uint32_t); }
int launch_tile_ranges(const uint64_t*, const uint32_t*, size_t, uint32_t, uint32_t*, hipStream_t, bool = true);
int launch_blend(const float*, uint32_t, const uint32_t*, const uint32_t*, const uint32_t*, uint32_t, uint32_t*, int,
                 int, const RenderViews&, const Knobs&, int, unsigned long long*, hipStream_t);
uint32_t* order_counter(void* ws);
int launch_compose(const RenderViews&, const uint8_t*, hipStream_t);
size_t order_ws_bytes(size_t items_max);
const uint32_t* launch_order_items(const uint32_t* items, uint32_t n_items, const uint32_t* count_dev,
                                   size_t items_max, const uint32_t* ranges, const RenderViews& views, void* ws,
                                   int* err, hipStream_t s);

int launch_fovea_plan(const FovView* fviews, const ItemViews& iviews, const VisViews& vis, void* plan,
                      size_t items_max, hipStream_t s);
}  // namespace vrs

namespace {

using namespace vrs;

struct ViewLayout {
    double f;
    int foveated;
    int T, ntx, nty;
    int ntx16, nty16;
    uint32_t tile_off;
    uint32_t cls_off;
    size_t pre_off;  // float offset into the render workspace
    size_t sat_off;  // byte offset of the view's summed-area table in the plan
};

struct Layout {
    int n_views;
    ViewLayout v[VRS_MAX_VIEWS];
    uint32_t tiles_total;
    uint32_t items_max;
    size_t cls_bytes;
    size_t plan_bytes;
    size_t render_ws_floats;  // pre-compose images of foveated views
    size_t order_off;         // bytes: the work-item ordering area after them
    size_t render_ws_bytes;
};

bool finite_f(float x) { return isfinite(x); }

int check_params(const vrs_params* p) {
    if (!p) return VRS_ERR_INVALID_ARG;
    if (p->tile != 16 && p->tile != 32) return VRS_ERR_INVALID_ARG;
    if (p->window < 0 || p->window > VRS_MAX_WINDOW) return VRS_ERR_INVALID_ARG;
    if (p->depth_mode < VRS_DEPTH_TILE_MAX || p->depth_mode > VRS_DEPTH_DISTANCE) return VRS_ERR_INVALID_ARG;
    if (p->blend_batch != 16 && p->blend_batch != 32 && p->blend_batch != 64) return VRS_ERR_UNSUPPORTED;
    if (p->schedule != VRS_SCHEDULE_ONESHOT && p->schedule != VRS_SCHEDULE_PERSISTENT) return VRS_ERR_INVALID_ARG;
    if (!(p->z_near > 0.f) || !finite_f(p->z_near)) return VRS_ERR_INVALID_ARG;
    if (!(p->alpha_min > 0.f && p->alpha_min < 1.f)) return VRS_ERR_INVALID_ARG;
    if (!(p->alpha_max >= p->alpha_min && p->alpha_max <= 1.f)) return VRS_ERR_INVALID_ARG;
    if (!(p->t_min > 0.f && p->t_min < 1.f)) return VRS_ERR_INVALID_ARG;
    if (!(p->dilation >= 0.f) || !finite_f(p->dilation)) return VRS_ERR_INVALID_ARG;
    for (int c = 0; c < 3; ++c)
        if (!finite_f(p->background[c])) return VRS_ERR_INVALID_ARG;
    return VRS_OK;
}

int make_layout(const vrs_camera* cams, const vrs_fovea* foveas, int n_views, const vrs_params* p, Layout& L) {
    if (!cams || !foveas || n_views < 1 || n_views > VRS_MAX_VIEWS) return VRS_ERR_INVALID_ARG;
    int rc = check_params(p);
    if (rc != VRS_OK) return rc;
    L.n_views = n_views;
    uint64_t tiles = 0, items = 0, cls = 0, pre = 0;
    for (int v = 0; v < n_views; ++v) {
        const vrs_camera& c = cams[v];
        const vrs_fovea& fv = foveas[v];
        if (c.width < 1 || c.height < 1 || c.width > (1 << 16) || c.height > (1 << 16)) return VRS_ERR_INVALID_ARG;
        if (!(c.fov_x_deg > 0.f && c.fov_x_deg < 180.f)) return VRS_ERR_INVALID_ARG;
        for (int k = 0; k < 12; ++k)
            if (!finite_f(c.world_to_cam[k])) return VRS_ERR_INVALID_ARG;
        if (!finite_f(c.cx) || !finite_f(c.cy)) return VRS_ERR_INVALID_ARG;
        if (fv.enabled) {
            if (!finite_f(fv.center_px[0]) || !finite_f(fv.center_px[1])) return VRS_ERR_INVALID_ARG;
            if (!(fv.band_frac >= 0.f) || !finite_f(fv.band_frac)) return VRS_ERR_INVALID_ARG;
            if (fv.shape == VRS_FOVEA_DISC) {
                if (!(fv.radius_deg >= 0.f && fv.radius_deg <= 180.f)) return VRS_ERR_INVALID_ARG;
            } else if (fv.shape == VRS_FOVEA_RECT) {
                if (!(fv.half_px[0] >= 0.f) || !(fv.half_px[1] >= 0.f) || !finite_f(fv.half_px[0]) ||
                    !finite_f(fv.half_px[1]))
                    return VRS_ERR_INVALID_ARG;
            } else {
                return VRS_ERR_INVALID_ARG;
            }
        }
        ViewLayout& V = L.v[v];
        V.f = (double(c.width) / 2.0) / tan(double(c.fov_x_deg) * (M_PI / 180.0) / 2.0);
        V.foveated = fv.enabled ? 1 : 0;
        V.T = V.foveated ? 32 : p->tile;
        V.ntx = (c.width + V.T - 1) / V.T;
        V.nty = (c.height + V.T - 1) / V.T;
        const int nt32x = (c.width + 31) / 32, nt32y = (c.height + 31) / 32;
        V.ntx16 = 2 * nt32x;
        V.nty16 = 2 * nt32y;
        V.tile_off = uint32_t(tiles);
        tiles += uint64_t(V.ntx) * V.nty;
        items += (V.T == 32) ? 4ull * V.ntx * V.nty : uint64_t(V.ntx) * V.nty;
        V.cls_off = uint32_t(cls);
        if (V.foveated) cls += uint64_t(V.ntx16) * V.nty16;
        V.pre_off = size_t(pre);
        if (V.foveated) pre += 4ull * c.width * c.height;
    }
    if (tiles >= (1ull << 31) || items >= (1ull << 23)) return VRS_ERR_UNSUPPORTED;
    L.tiles_total = uint32_t(tiles);
    L.items_max = uint32_t(items);
    L.cls_bytes = size_t(cls);
    // Then, per view, the summed-area table of its visible sort tiles.
    size_t sat = kPlanItemsOff + size_t(items) * 4 + ((size_t(cls) + 255) & ~size_t(255));
    for (int v = 0; v < n_views; ++v) {
        L.v[v].sat_off = sat;
        sat += ((size_t(L.v[v].ntx + 1) * size_t(L.v[v].nty + 1) * sizeof(uint32_t)) + 255) & ~size_t(255);
    }
    L.plan_bytes = sat;
    L.render_ws_floats = size_t(pre);
    L.order_off = ((size_t(pre) * sizeof(float)) + 255) & ~size_t(255);
    L.render_ws_bytes = L.order_off + order_ws_bytes(size_t(items));
    return VRS_OK;
}

int check_gaussians(const vrs_gaussians* g) {
    if (!g || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return VRS_ERR_INVALID_ARG;
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
        return VRS_ERR_INVALID_ARG;
    return VRS_OK;
}

GaussPtrs gauss_ptrs(const vrs_gaussians* g) {
    GaussPtrs p;
    p.means = g->means;
    p.log_scales = g->log_scales;
    p.quats = g->quats;
    p.opac = g->opacity_logits;
    p.sh = g->sh;
    p.n = g->n;
    p.sh_degree = g->sh_degree;
    return p;
}

Knobs knobs(const vrs_params* p) {
    Knobs k;
    k.z_near = p->z_near;
    k.alpha_min = p->alpha_min;
    k.alpha_max = p->alpha_max;
    k.t_min = p->t_min;
    k.dilation = p->dilation;
    for (int c = 0; c < 3; ++c) k.bg[c] = p->background[c];
    k.window = p->window;
    k.depth_mode = p->depth_mode;
    return k;
}

GeoViews geo_views(const vrs_camera* cams, const Layout& L, const vrs_params* p, const void* plan) {
    GeoViews G;
    memset(&G, 0, sizeof(G));
    G.n = L.n_views;
    G.ln_amin = log(double(p->alpha_min));
    for (int v = 0; v < L.n_views; ++v) {
        GeoView& o = G.v[v];
        const ViewLayout& V = L.v[v];
        o.f = V.f;
        o.inv_f = 1.0 / V.f;
        for (int k = 0; k < 3; ++k) {
            for (int j = 0; j < 3; ++j) o.R[3 * k + j] = cams[v].world_to_cam[4 * k + j];
            o.t[k] = cams[v].world_to_cam[4 * k + 3];
        }
        o.cx = cams[v].cx;
        o.cy = cams[v].cy;
        o.W = cams[v].width;
        o.H = cams[v].height;
        o.T = V.T;
        o.ntx = V.ntx;
        o.nty = V.nty;
        o.tile_off = V.tile_off;
        o.sat = plan ? reinterpret_cast<const uint32_t*>(static_cast<const char*>(plan) + V.sat_off) : nullptr;
    }
    return G;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int key_bits_for(uint32_t tiles_total) {
    int b = 0;
    while (b < 32 && (uint64_t(1) << b) < uint64_t(tiles_total)) ++b;
    return 32 + b;
}

}  // namespace

static int duplicate_impl(const vrs_gaussians* g, const vrs_camera* cams, const vrs_fovea* foveas,
                          int32_t n_views, const vrs_params* p, const void* plan, const void* proj,
                          const uint32_t* counts,
                          uint64_t* keys, uint32_t* gids, size_t capacity, uint32_t* n_inst_dev, void* ws,
                          size_t ws_bytes, int32_t* status_dev, vrs_stream_t stream, bool count_live,
                          uint32_t* clear = nullptr, size_t n_clear = 0) {
    int rc = check_gaussians(g);
    if (rc != VRS_OK) return rc;
    Layout L;
    rc = make_layout(cams, foveas, n_views, p, L);
    if (rc != VRS_OK) return rc;
    const size_t nv = size_t(n_views) * size_t(g->n);
    if (!n_inst_dev || (nv > 0 && (!counts || !ws || !proj)) || (capacity > 0 && (!keys || !gids)))
        return VRS_ERR_INVALID_ARG;
    if (capacity > 0xFFFFFFFFull || nv > 0xFFFFFFFFull) return VRS_ERR_UNSUPPORTED;
    if (ws_bytes < dup_ws_bytes(nv) || !aligned(keys, 8) || !aligned(ws, 16) || !aligned(proj, 16))
        return VRS_ERR_INVALID_ARG;
    if (plan && !aligned(plan, 256)) return VRS_ERR_INVALID_ARG;
    return launch_duplicate(gauss_ptrs(g), geo_views(cams, L, p, plan), knobs(p), static_cast<const float*>(proj), counts,
                            keys, gids, capacity, n_inst_dev, ws, status_dev, reinterpret_cast<hipStream_t>(stream),
                            count_live, clear, n_clear);
}

extern "C" {

const char* vrs_status_string(int code) {
    switch (code) {
        case VRS_OK: return "VRS_OK";
        case VRS_ERR_INVALID_ARG: return "VRS_ERR_INVALID_ARG";
        case VRS_ERR_CAPACITY: return "VRS_ERR_CAPACITY";
        case VRS_ERR_HIP: return "VRS_ERR_HIP";
        case VRS_ERR_UNSUPPORTED: return "VRS_ERR_UNSUPPORTED";
        case VRS_ERR_SCRATCH: return "VRS_ERR_SCRATCH";
        case VRS_ERR_NONFINITE: return "VRS_ERR_NONFINITE";
        default: return "VRS_ERR_UNKNOWN";
    }
}

const char* vrs_version(void) { return "vrs 0.1 gfx950"; }

int vrs_workspace_size(int32_t n, const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                       const vrs_params* p, size_t capacity, vrs_sizes* out) {
    if (!out || n < 0) return VRS_ERR_INVALID_ARG;
    Layout L;
    const int rc = make_layout(cams, foveas, n_views, p, L);
    if (rc != VRS_OK) return rc;
    const size_t nv = size_t(n_views) * size_t(n);
    out->proj_bytes = nv * kProjBytesPerSlot;
    out->counts_bytes = nv * sizeof(uint32_t);
    out->tiles_total = L.tiles_total;
    out->items_max = L.items_max;
    out->plan_bytes = L.plan_bytes;
    const size_t a = dup_ws_bytes(nv), b = sort_ws_bytes(capacity);
    out->sort_ws_bytes = a > b ? a : b;
    out->render_ws_bytes = L.render_ws_bytes;
    return VRS_OK;
}

int vrs_fovea_plan(const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views, const vrs_params* p,
                   const uint8_t* const* vis_masks, void* plan, size_t plan_bytes, uint32_t* n_items,
                   vrs_stream_t stream) {
    Layout L;
    int rc = make_layout(cams, foveas, n_views, p, L);
    if (rc != VRS_OK) return rc;
    if (!plan || !n_items || plan_bytes < L.plan_bytes || !aligned(plan, 256)) return VRS_ERR_INVALID_ARG;
    FovView fv[VRS_MAX_VIEWS];
    ItemViews iv;
    VisViews vis;
    memset(fv, 0, sizeof(fv));
    memset(&iv, 0, sizeof(iv));
    memset(&vis, 0, sizeof(vis));
    iv.n = n_views;
    vis.n = n_views;
    for (int v = 0; v < n_views; ++v) {
        const ViewLayout& V = L.v[v];
        const vrs_camera& c = cams[v];
        const vrs_fovea& f = foveas[v];
        FovView& o = fv[v];
        o.f = V.f;
        o.cx = c.cx;
        o.cy = c.cy;
        o.dc[0] = (double(f.center_px[0]) - double(c.cx)) / V.f;
        o.dc[1] = (double(f.center_px[1]) - double(c.cy)) / V.f;
        o.dc[2] = 1.0;
        o.dcn = sqrt(o.dc[0] * o.dc[0] + o.dc[1] * o.dc[1] + 1.0);
        const double rho = double(f.radius_deg) * (M_PI / 180.0);
        const double b = double(f.band_frac);
        o.all_low = rho <= 0.0 ? 1 : 0;
        const double outer = rho * (1.0 + b);
        o.cos_low = outer >= M_PI ? -2.0 : cos(outer);
        o.cos_high = rho >= M_PI ? -2.0 : cos(rho);
        o.shape = f.shape;
        o.band = b;
        o.fc[0] = double(f.center_px[0]);
        o.fc[1] = double(f.center_px[1]);
        o.half[0] = double(f.half_px[0]);
        o.half[1] = double(f.half_px[1]);
        o.W = c.width;
        o.H = c.height;
        o.ntx32 = (c.width + 31) / 32;
        o.nty32 = (c.height + 31) / 32;
        o.ntx16 = V.ntx16;
        o.nty16 = V.nty16;
        o.cls_off = V.cls_off;
        ItemView& it = iv.v[v];
        it.foveated = V.foveated;
        it.T = V.T;
        it.ntx = V.ntx;
        it.ntx16 = V.ntx16;
        it.ntiles = V.ntx * V.nty;
        it.W = c.width;
        it.H = c.height;
        it.cls_off = V.cls_off;
        VisView& vv = vis.v[v];
        vv.mask = vis_masks ? vis_masks[v] : nullptr;
        vv.W = c.width;
        vv.H = c.height;
        vv.T = V.T;
        vv.ntx = V.ntx;
        vv.nty = V.nty;
        vv.sat = reinterpret_cast<uint32_t*>(static_cast<char*>(plan) + V.sat_off);
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rc = launch_fovea_plan(fv, iv, vis, plan, L.items_max, s);
    if (rc != VRS_OK) return rc;
    uint32_t cnt = 0;
    if (hipMemcpyAsync(&cnt, plan, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return VRS_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return VRS_ERR_HIP;
    *n_items = cnt;
    return VRS_OK;
}

int vrs_preprocess(const vrs_gaussians* g, const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                   const vrs_params* p, const void* plan, void* proj, uint32_t* counts, int32_t* status_dev,
                   vrs_stream_t stream) {
    int rc = check_gaussians(g);
    if (rc != VRS_OK) return rc;
    Layout L;
    rc = make_layout(cams, foveas, n_views, p, L);
    if (rc != VRS_OK) return rc;
    if (g->n > 0 && (!proj || !counts || !aligned(proj, 16))) return VRS_ERR_INVALID_ARG;
    if (plan && !aligned(plan, 256)) return VRS_ERR_INVALID_ARG;
    return launch_preprocess(gauss_ptrs(g), geo_views(cams, L, p, plan), knobs(p), static_cast<float*>(proj), counts,
                             status_dev, reinterpret_cast<hipStream_t>(stream));
}

int vrs_duplicate(const vrs_gaussians* g, const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                  const vrs_params* p, const void* plan, const void* proj, const uint32_t* counts, uint64_t* keys,
                  uint32_t* gids, size_t capacity, uint32_t* n_inst_dev, void* ws, size_t ws_bytes,
                  int32_t* status_dev, vrs_stream_t stream) {
    return duplicate_impl(g, cams, foveas, n_views, p, plan, proj, counts, keys, gids, capacity, n_inst_dev, ws,
                          ws_bytes, status_dev, stream, true);
}

size_t vrs_sort_pairs_workspace_size(size_t capacity) { return sort_ws_bytes(capacity); }

int vrs_sort_pairs(uint64_t* keys, uint32_t* vals, const uint32_t* n_dev, size_t capacity, int32_t key_bits,
                   void* ws, size_t ws_bytes, int32_t* status_dev, vrs_stream_t stream) {
    if (key_bits < 0 || key_bits > 64 || !n_dev) return VRS_ERR_INVALID_ARG;
    if (capacity > 0xFFFFFFFFull) return VRS_ERR_UNSUPPORTED;
    if (capacity > 0 && (!keys || !vals || !ws || ws_bytes < sort_ws_bytes(capacity) || !aligned(keys, 8) ||
                         !aligned(ws, 16)))
        return VRS_ERR_INVALID_ARG;
    return launch_sort_pairs(keys, vals, n_dev, capacity, key_bits, ws, status_dev,
                             reinterpret_cast<hipStream_t>(stream));
}

int vrs_tile_ranges(const uint64_t* keys, const uint32_t* n_dev, size_t capacity, uint32_t tiles_total,
                    uint32_t* ranges, vrs_stream_t stream) {
    if (!n_dev || (tiles_total > 0 && !ranges) || (capacity > 0 && !keys)) return VRS_ERR_INVALID_ARG;
    return launch_tile_ranges(keys, n_dev, capacity, tiles_total, ranges, reinterpret_cast<hipStream_t>(stream));
}

int vrs_sort(const vrs_gaussians* g, const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
             const vrs_params* p, const void* plan, const void* proj, const uint32_t* counts, uint64_t* keys,
             uint32_t* gids, size_t capacity, uint32_t* n_inst_dev, uint32_t* ranges, void* ws, size_t ws_bytes,
             int32_t* status_dev, vrs_stream_t stream) {
    Layout L;
    int rc = make_layout(cams, foveas, n_views, p, L);
    if (rc != VRS_OK) return rc;
    if (!ranges && L.tiles_total > 0) return VRS_ERR_INVALID_ARG;
    if (capacity > 0 && ws_bytes < sort_ws_bytes(capacity)) return VRS_ERR_INVALID_ARG;
    // The sort's first kernel counts the kept instances into n_inst_dev[1].
    // Instantiation also clears the tile ranges that the sort fills in.
    rc = duplicate_impl(g, cams, foveas, n_views, p, plan, proj, counts, keys, gids, capacity, n_inst_dev, ws,
                        ws_bytes, status_dev, stream, false, ranges, size_t(L.tiles_total) * 2);
    if (rc != VRS_OK) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (capacity > 0) {
        // The first pass drops the dead keys of culled candidates.
        rc = launch_sort_pairs_ex(keys, gids, n_inst_dev, n_inst_dev + 1, true, capacity,
                                  key_bits_for(L.tiles_total), ws, status_dev, s, n_inst_dev + 1);
        if (rc != VRS_OK) return rc;
    }
    return launch_tile_ranges(keys, n_inst_dev + 1, capacity, L.tiles_total, ranges, s, false);
}

}  // extern "C"

namespace {

// One view's table for the render kernels.
void fill_render_view(RenderView& o, const ViewLayout& V, const vrs_camera& c, const vrs_fovea& f, float* out,
                      float* pre) {
    memset(&o, 0, sizeof(o));
    o.out = out;
    o.pre = pre;
    o.mask = make_fov_mask(c, f);
    o.W = c.width;
    o.H = c.height;
    o.T = V.T;
    o.ntx = V.ntx;
    o.ntx16 = V.ntx16;
    o.tile_off = V.tile_off;
    o.cls_off = V.cls_off;
    o.foveated = uint8_t(V.foveated);
}

// Shared argument checks and tables of the render entry points.
int render_setup(int32_t n, const void* proj, const uint32_t* gids, const uint32_t* ranges, const vrs_camera* cams,
                 const vrs_fovea* foveas, int32_t n_views, const vrs_params* p, const void* plan, uint32_t n_items,
                 float* const* rgba, void* ws, size_t ws_bytes, RenderViews& R, Layout& L) {
    int rc = make_layout(cams, foveas, n_views, p, L);
    if (rc != VRS_OK) return rc;
    if (n < 0 || !plan || !rgba || n_items > L.items_max) return VRS_ERR_INVALID_ARG;
    if (n_items > 0 && (!proj || !gids || !ranges || !aligned(proj, 16))) return VRS_ERR_INVALID_ARG;
    if (L.render_ws_floats > 0 && (!ws || ws_bytes < L.render_ws_floats * sizeof(float)))
        return VRS_ERR_INVALID_ARG;
    if (n_items > 0 && (!ws || ws_bytes < L.render_ws_bytes || !aligned(ws, 256))) return VRS_ERR_INVALID_ARG;
    memset(&R, 0, sizeof(R));
    R.n = n_views;
    for (int v = 0; v < n_views; ++v) {
        const ViewLayout& V = L.v[v];
        if (!rgba[v]) return VRS_ERR_INVALID_ARG;
        fill_render_view(R.v[v], V, cams[v], foveas[v], rgba[v],
                         V.foveated ? static_cast<float*>(ws) + V.pre_off : rgba[v]);
    }
    return VRS_OK;
}

const uint32_t* plan_items(const void* plan) {
    return reinterpret_cast<const uint32_t*>(static_cast<const char*>(plan) + kPlanItemsOff);
}
const uint8_t* plan_classes(const void* plan, const Layout& L) {
    return static_cast<const uint8_t*>(plan) + kPlanItemsOff + size_t(L.items_max) * 4;
}

}  // namespace

extern "C" {

int vrs_blend(const void* proj, int32_t n, const uint32_t* gids, const uint32_t* ranges, const vrs_camera* cams,
              const vrs_fovea* foveas, int32_t n_views, const vrs_params* p, const void* plan, uint32_t n_items,
              float* const* rgba, void* ws, size_t ws_bytes, int32_t* status_dev, vrs_stream_t stream) {
    (void)status_dev;
    RenderViews R;
    Layout L;
    int rc = render_setup(n, proj, gids, ranges, cams, foveas, n_views, p, plan, n_items, rgba, ws, ws_bytes, R, L);
    if (rc != VRS_OK) return rc;
    if (n_items == 0) return VRS_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint32_t* items = launch_order_items(plan_items(plan), n_items, static_cast<const uint32_t*>(plan),
                                               L.items_max, ranges, R, static_cast<char*>(ws) + L.order_off,
                                               status_dev, s);
    if (!items) return VRS_ERR_HIP;
    return launch_blend(static_cast<const float*>(proj), uint32_t(n), gids, ranges, items, n_items,
                        order_counter(static_cast<char*>(ws) + L.order_off), p->blend_batch, p->schedule, R, knobs(p),
                        p->window, nullptr, s);
}

int vrs_blend_stats(const void* proj, int32_t n, const uint32_t* gids, const uint32_t* ranges,
                    const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views, const vrs_params* p,
                    const void* plan, uint32_t n_items, float* const* rgba, void* ws, size_t ws_bytes,
                    uint64_t* counters_dev, vrs_stream_t stream) {
    RenderViews R;
    Layout L;
    if (!counters_dev) return VRS_ERR_INVALID_ARG;
    int rc = render_setup(n, proj, gids, ranges, cams, foveas, n_views, p, plan, n_items, rgba, ws, ws_bytes, R, L);
    if (rc != VRS_OK) return rc;
    if (n_items == 0) return VRS_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint32_t* items = launch_order_items(plan_items(plan), n_items, static_cast<const uint32_t*>(plan),
                                               L.items_max, ranges, R, static_cast<char*>(ws) + L.order_off,
                                               nullptr, s);
    if (!items) return VRS_ERR_HIP;
    return launch_blend(static_cast<const float*>(proj), uint32_t(n), gids, ranges, items, n_items,
                        order_counter(static_cast<char*>(ws) + L.order_off), p->blend_batch, p->schedule, R, knobs(p),
                        p->window, reinterpret_cast<unsigned long long*>(counters_dev), s);
}

int vrs_compose(const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views, const vrs_params* p,
                const void* plan, float* const* rgba, void* ws, size_t ws_bytes, vrs_stream_t stream) {
    RenderViews R;
    Layout L;
    int rc = render_setup(0, nullptr, nullptr, nullptr, cams, foveas, n_views, p, plan, 0, rgba, ws, ws_bytes, R, L);
    if (rc != VRS_OK) return rc;
    return launch_compose(R, plan_classes(plan, L), reinterpret_cast<hipStream_t>(stream));
}

int vrs_render_foveated(const void* proj, int32_t n, const uint32_t* gids, const uint32_t* ranges,
                        const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views, const vrs_params* p,
                        const void* plan, uint32_t n_items, float* const* rgba, void* ws, size_t ws_bytes,
                        int32_t* status_dev, vrs_stream_t stream) {
    int rc = vrs_blend(proj, n, gids, ranges, cams, foveas, n_views, p, plan, n_items, rgba, ws, ws_bytes,
                       status_dev, stream);
    if (rc != VRS_OK) return rc;
    return vrs_compose(cams, foveas, n_views, p, plan, rgba, ws, ws_bytes, stream);
}

}  // extern "C"

namespace vrs {
size_t backward_ws_bytes(size_t n, int n_views);
int launch_backward(const GaussPtrs&, const GeoViews&, const float*, const uint32_t*, const uint32_t*,
                    const uint32_t*, uint32_t, const BwdViews&, const Knobs&, int, float*, const GradPtrs&,
                    hipStream_t);
int launch_fov_grads(const FovGradView& V, hipStream_t s);
}  // namespace vrs

namespace {

// Backward workspace: the per-view render-record gradients, then for every
// foveated view three [4][H][W] float planes: its samples' forward values
// (HYBRID unmixed), dL/d(pre-compose image) and dL/d(sample).
size_t bwd_fov_off(size_t n, int n_views) { return (backward_ws_bytes(n, n_views) + 255) & ~size_t(255); }

// Then the work items in longest-first order (the ordering area of the blend).
size_t bwd_order_off(size_t n, const vrs_camera* cams, const vrs_fovea* foveas, int n_views) {
    size_t b = bwd_fov_off(n, n_views);
    for (int v = 0; v < n_views; ++v)
        if (foveas[v].enabled) b += 3 * 4 * size_t(cams[v].width) * size_t(cams[v].height) * sizeof(float);
    return (b + 255) & ~size_t(255);
}

size_t bwd_ws_total(size_t n, const vrs_camera* cams, const vrs_fovea* foveas, int n_views, size_t items_max) {
    return bwd_order_off(n, cams, foveas, n_views) + order_ws_bytes(items_max);
}

}  // namespace

extern "C" {

size_t vrs_backward_workspace_size(int32_t n, const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                                   const vrs_params* p) {
    Layout L;
    if (n < 0 || make_layout(cams, foveas, n_views, p, L) != VRS_OK) return 0;
    return bwd_ws_total(size_t(n), cams, foveas, n_views, size_t(L.items_max));
}

int vrs_render_backward(const vrs_gaussians* g, const void* proj, const uint32_t* gids, const uint32_t* ranges,
                        const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views, const vrs_params* p,
                        const void* plan, uint32_t n_items, const float* const* rgba,
                        const float* const* grad_rgba, const vrs_gaussian_grads* out, void* ws, size_t ws_bytes,
                        int32_t* status_dev, vrs_stream_t stream) {
    (void)status_dev;
    int rc = check_gaussians(g);
    if (rc != VRS_OK) return rc;
    Layout L;
    rc = make_layout(cams, foveas, n_views, p, L);
    if (rc != VRS_OK) return rc;
    if (!rgba || !grad_rgba || !out || !plan || !aligned(plan, 256) || n_items > L.items_max)
        return VRS_ERR_INVALID_ARG;
    bool any_fov = false;
    for (int v = 0; v < n_views; ++v) any_fov = any_fov || foveas[v].enabled;
    if (g->n > 0) {
        if (!proj || !gids || !ranges || !aligned(proj, 16)) return VRS_ERR_INVALID_ARG;
        if (!out->means || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh)
            return VRS_ERR_INVALID_ARG;
        if (!ws || !aligned(ws, 256) || ws_bytes < bwd_ws_total(size_t(g->n), cams, foveas, n_views, L.items_max))
            return VRS_ERR_INVALID_ARG;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint32_t* items = plan_items(plan);  // longest first once ordered below
    BwdViews B;
    memset(&B, 0, sizeof(B));
    B.n = n_views;
    RenderViews R;
    memset(&R, 0, sizeof(R));
    R.n = n_views;
    float* fov_ws = reinterpret_cast<float*>(static_cast<char*>(ws) + bwd_fov_off(size_t(g->n), n_views));
    for (int v = 0; v < n_views; ++v) {
        if (!grad_rgba[v] || (!foveas[v].enabled && !rgba[v])) return VRS_ERR_INVALID_ARG;
        const ViewLayout& V = L.v[v];
        BwdView& o = B.v[v];
        o.W = cams[v].width;
        o.H = cams[v].height;
        o.T = V.T;
        o.ntx = V.ntx;
        o.tile_off = V.tile_off;
        RenderView& r = R.v[v];
        fill_render_view(r, V, cams[v], foveas[v], nullptr, nullptr);
        if (!foveas[v].enabled || g->n == 0) {
            o.rgba = rgba[v];
            o.grad = grad_rgba[v];
            r.skip = 1;
            continue;
        }
        const size_t plane = size_t(o.W) * size_t(o.H);
        float* cfin = fov_ws;
        float* gpre = cfin + 4 * plane;
        float* gsamp = gpre + 4 * plane;
        fov_ws = gsamp + 4 * plane;
        o.rgba = cfin;
        o.grad = gsamp;
        r.out = cfin;
        r.pre = cfin;
        r.nomix = 1;
        FovGradView F;
        F.gout = grad_rgba[v];
        F.gpre = gpre;
        F.gsamp = gsamp;
        F.cls = plan_classes(plan, L) + V.cls_off;
        F.W = o.W;
        F.H = o.H;
        F.ntx16 = V.ntx16;
        F.mask = make_fov_mask(cams[v], foveas[v]);
        rc = launch_fov_grads(F, s);
        if (rc != VRS_OK) return rc;
    }
    if (g->n > 0 && n_items > 0) {
        // The same longest-first order as the forward's: the replay blocks
        // are long, and the longest last would extend the launch.
        items = launch_order_items(plan_items(plan), n_items, static_cast<const uint32_t*>(plan), L.items_max, ranges,
                                   R, static_cast<char*>(ws) + bwd_order_off(size_t(g->n), cams, foveas, n_views),
                                   nullptr, s);
        if (!items) return VRS_ERR_HIP;
    }
    if (any_fov && g->n > 0 && n_items > 0) {
        // The foveated views' samples as the forward blended them (HYBRID
        // samples unmixed), into the workspace; plain views are skipped.
        rc = launch_blend(static_cast<const float*>(proj), uint32_t(g->n), gids, ranges, items, n_items, nullptr,
                          p->blend_batch, VRS_SCHEDULE_ONESHOT, R, knobs(p), p->window, nullptr, s);
        if (rc != VRS_OK) return rc;
    }
    GradPtrs G;
    G.means = out->means;
    G.log_scales = out->log_scales;
    G.quats = out->quats;
    G.opac = out->opacity_logits;
    G.sh = out->sh;
    return launch_backward(gauss_ptrs(g), geo_views(cams, L, p, nullptr), static_cast<const float*>(proj), gids,
                           ranges, items, n_items, B, knobs(p), p->window, static_cast<float*>(ws), G, s);
}

}  // extern "C"
