/*
 * vrs.h -- C ABI of the MI355X (gfx950) foveated Gaussian-splat rasterizer.
 *
 * The library implements the rendering path of VRSplat (arXiv 2505.10144):
 * Optimal-Projection preprocessing of 3D Gaussians (Sec. 3 end, Sec. 4.2),
 * Gaussian/tile instantiation with tangent-plane tile culling (Eq. 4), a
 * radix sort of tile|depth keys (Sec. 3 tile binning), and per-tile
 * front-to-back blending (Eq. 2) with per-sample depth resorting (Sec. 4.1)
 * in which full-resolution fovea tiles and half-resolution periphery tiles
 * run in one launch (Sec. 4.3, Fig. 5a).
 *
 * Conventions shared by every entry point
 *  - Every array argument is device memory owned by the caller (for example a
 *    torch tensor).  The library never allocates, frees or retains caller
 *    memory and keeps no global mutable state; calls on different streams are
 *    independent.  Structs passed by pointer are host memory, read during
 *    the call only.
 *  - All work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 *    the null stream).  The only entry point that synchronises is
 *    vrs_fovea_plan, which returns the exact work-item count to the host.
 *  - The return value reports argument errors and launch errors
 *    (VRS_ERR_INVALID_ARG, VRS_ERR_UNSUPPORTED, VRS_ERR_HIP).  Conditions
 *    only the device can see are written to *status_dev, an int32 that the
 *    caller zeroes beforehand; the first error written wins.
 *  - Floats are IEEE binary32; all per-pair arithmetic is FP32, per-Gaussian
 *    set-up geometry and the tile test run in FP64 and are rounded once.
 */
#ifndef VRS_H
#define VRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* vrs_stream_t; /* hipStream_t */

/* Status codes (return values and *status_dev). */
#define VRS_OK 0
#define VRS_ERR_INVALID_ARG (-1)
#define VRS_ERR_CAPACITY (-2)
#define VRS_ERR_HIP (-3)
#define VRS_ERR_UNSUPPORTED (-4)
#define VRS_ERR_SCRATCH (-5) /* request larger than the fixed scratch of a no-allocation entry point */
#define VRS_ERR_NONFINITE (-6) /* (device) a Gaussian parameter was NaN or infinite; see vrs_preprocess */

/* Limits. */
#define VRS_MAX_VIEWS 32
#define VRS_MAX_WINDOW 32
#define VRS_RECORD_FLOATS 32 /* floats per projected Gaussian record (128 B) */

/* Render work-item classes (Sec. 4.3): LOW = 32x32 periphery tile shaded as
 * 16x16 samples at 2x2-group centres; HIGH = 16x16 fovea subtile at full
 * resolution; HYBRID = transitional subtile (full resolution blended with its
 * 2x2-group mean by the continuous mask); PLAIN = 16x16 tile of a
 * non-foveated view. */
#define VRS_CLASS_LOW 0
#define VRS_CLASS_HIGH 1
#define VRS_CLASS_HYBRID 2
#define VRS_CLASS_PLAIN 3

/* Gaussians (Sec. 3 Eq. 1; optimised parameters of Sec. 4.1), structure of
 * arrays, FP32, device memory:
 *   means[3][n]          world-space mean
 *   log_scales[3][n]     natural log of the per-axis standard deviation
 *   quats[4][n]          rotation (w, x, y, z), any non-zero length
 *   opacity_logits[n]    opacity = 1 / (1 + exp(-o))
 *   sh[K][3][n]          real SH coefficients, K = (sh_degree+1)^2, index
 *                        k = l^2 + l + m, Condon-Shortley phase; colour =
 *                        max(0, sum_k sh_k Y_k(v) + 0.5), v = unit vector from
 *                        the eye centre to the mean. */
typedef struct {
    int32_t n;
    int32_t sh_degree; /* 0..3 */
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opacity_logits;
    const float* sh;
} vrs_gaussians;

/* Pinhole camera (Sec. 5; App. D varies focal length and resolution).
 * x_cam = R x_world + t with world_to_cam = [R | t] row-major 3x4; camera
 * axes x right, y down, z forward; square pixels with focal length
 * f = (width/2) / tan(fov_x/2) pixels; principal point (cx, cy) in pixels;
 * pixel (i, j) is sampled at (i + 0.5, j + 0.5). */
typedef struct {
    float world_to_cam[12];
    float fov_x_deg;
    float cx, cy;
    int32_t width, height;
} vrs_camera;

/* Fovea (Sec. 4.3): the continuous mask w of the full-resolution centre
 * region, with band fraction b = band_frac (the paper uses a 10 % linear
 * band).
 *   shape VRS_FOVEA_DISC: w = clamp((rho (1 + b) - e) / (rho b), 0, 1) of
 *     the angle e between a pixel's ray and the ray through center_px, rho =
 *     radius_deg.
 *   shape VRS_FOVEA_RECT (the paper's layout, Sec. 5: a centre region of
 *     half the image with 10 % padding): per axis
 *     u = clamp((h (1 + b) - |p - c|) / (h b), 0, 1) with half-extent
 *     h = half_px[axis] and c = center_px[axis], w = min(u_x, u_y).
 *   Without a band (b = 0) w is the indicator of the disc or rectangle.
 * enabled = 0 renders the view plainly. */
#define VRS_FOVEA_DISC 0
#define VRS_FOVEA_RECT 1
typedef struct {
    int32_t enabled;
    float center_px[2];
    float radius_deg;
    float band_frac;
    int32_t shape;
    float half_px[2];
} vrs_fovea;

/* Blend schedules (performance only; the output is identical). */
#define VRS_SCHEDULE_ONESHOT 0    /* one block per work item, longest first        */
#define VRS_SCHEDULE_PERSISTENT 1 /* a chip-filling grid whose waves draw (item,    \
                                     quadrant) units longest first from an atomic
                                     counter                                        */

/* Sort key depth (depth_mode). */
#define VRS_DEPTH_TILE_MAX 0 /* per-tile depth at the splat's maximum point (Sec. 4.2) */
#define VRS_DEPTH_VIEW_Z 1   /* view-space z of the mean (one depth per Gaussian)    */
#define VRS_DEPTH_DISTANCE 2 /* distance from the eye to the mean (per Gaussian)     */

/* Renderer knobs.  tile: 16 or 32 for plain views (a 32x32 tile is rendered
 * as four 16x16 subtiles) -- foveated views always use 32x32 sort tiles;
 * window: per-sample resort window length W, 0..32 (Sec. 4.1; 0 blends in
 * key order without resorting, like the global-sort comparison renderers of
 * Sec. 5); depth_mode: one of VRS_DEPTH_* (the key depth); blend_batch:
 * list entries staged per wave and batch, 16, 32 or 64 (the forward blend
 * stages at most 56 at a time), and schedule, one of VRS_SCHEDULE_* (both
 * performance only, never changing the output).
 * z_near: near cull on camera z; alpha_min: culling and skip threshold
 * (1/255, Sec. 4.2); alpha_max: alpha clamp (0.99); t_min: transmittance at
 * which a sample stops (1e-4); dilation: px^2 added to the 2D covariance
 * (App. D); background: RGB composited behind. */
typedef struct {
    int32_t tile;
    int32_t window;
    int32_t blend_batch;
    int32_t schedule;
    float z_near;
    float alpha_min;
    float alpha_max;
    float t_min;
    float dilation;
    float background[3];
    int32_t depth_mode;
} vrs_params;

/* Buffer sizes for one configuration (all bytes unless noted). */
typedef struct {
    size_t proj_bytes;       /* per view and Gaussian: a 128-byte FP32 render record
                                ([n_views][n][32] floats); after all of them a
                                16-byte candidate tile rectangle each; after those a
                                float4 colour (r, g, b, 0) each                      */
    size_t counts_bytes;     /* uint32 counts[n_views][n]                         */
    uint32_t tiles_total;    /* sum over views of sort-grid tiles (ranges rows)    */
    uint32_t items_max;      /* upper bound on render work items                   */
    size_t plan_bytes;       /* work list + per-view subtile class maps            */
    size_t sort_ws_bytes;    /* vrs_duplicate/vrs_sort workspace for `capacity`    */
    size_t render_ws_bytes;  /* vrs_render_foveated workspace: pre-compose images of
                                foveated views, then the work-item ordering        */
} vrs_sizes;

/* Sizes of every buffer the other entry points need.  `capacity` is the
 * instance capacity the caller intends to pass to vrs_sort.  Host-only, no
 * device work.  Returns VRS_ERR_INVALID_ARG for bad arguments. */
int vrs_workspace_size(int32_t n, const vrs_camera* cams, const vrs_fovea* foveas,
                       int32_t n_views, const vrs_params* p, size_t capacity,
                       vrs_sizes* out);

/* Foveation map (Sec. 4.3: the tile-to-class mapping is cheap to build at
 * the start of a frame and gives the exact block count of the single
 * launch; it is built once per eye configuration and reused).  Writes into
 * `plan` (plan_bytes from vrs_workspace_size) the class of every 16x16
 * subtile of every view and a compact list of render work items: per
 * foveated view, one LOW item per periphery 32x32 tile and one HIGH/HYBRID
 * item per in-image subtile of a split tile; per plain view, one PLAIN item
 * per 16x16 tile.  Synchronises `stream` and returns the exact item count in
 * *n_items.  Classes are decided in FP64.
 * Visibility culling (Sec. 4.3, Fig. 5b): vis_masks (may be null) holds per
 * view a device pointer to a uint8 [height][width] mask (nonzero = visible
 * through the headset's lens) or null (all visible).  The plan then also
 * holds, per view, the bitfield of sort tiles with a visible pixel as its
 * summed-area table (uint32 [nty + 1][ntx + 1]), from which vrs_preprocess
 * counts and vrs_duplicate enumerates only the visible tiles a splat
 * covers.  Tiles without a visible pixel get no instances; their pixels are
 * rendered as background (alpha 0).  The masks are read during the call
 * only. */
int vrs_fovea_plan(const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                   const vrs_params* p, const uint8_t* const* vis_masks, void* plan,
                   size_t plan_bytes, uint32_t* n_items, vrs_stream_t stream);

/* Per-Gaussian preprocessing (Sec. 3 Eq. 1, Optimal Projection of Sec. 3 end
 * and Sec. 4.2, SH colour; one thread per Gaussian covering every view).
 * Writes into `proj` (proj_bytes, 16-byte aligned) each Gaussian's FP32
 * render record per view -- rows [n_views][n][VRS_RECORD_FLOATS] -- its
 * candidate tile rectangle and its colour, and into counts[n_views][n] the number of candidate
 * tiles: the tiles meeting the image of the cone of directions in which the
 * splat can reach alpha_min (a conservative bound; the exact tile test of
 * Eq. 4 runs in vrs_duplicate, which derives the FP64 set-up again from `g`).  With a plan (from vrs_fovea_plan with the
 * same cameras, foveas and params; may be null) only the visible tiles of
 * that rectangle are counted, exactly, from the plan's summed-area table at
 * the rectangle's corners (Sec. 4.3, Fig. 5b).  Culled Gaussians (camera z <= z_near,
 * opacity < alpha_min, non-finite parameters) get 0.  Sort grids: 32x32 for
 * foveated views, p->tile otherwise.  A Gaussian with a NaN or infinite
 * mean, log-scale, quaternion or opacity logit is culled from every view,
 * and one with a NaN or infinite SH coefficient is coloured black; either
 * writes VRS_ERR_NONFINITE to *status_dev (if status_dev is not null) while
 * the frame is still rendered from the other Gaussians. */
int vrs_preprocess(const vrs_gaussians* g, const vrs_camera* cams, const vrs_fovea* foveas,
                   int32_t n_views, const vrs_params* p, const void* plan, void* proj,
                   uint32_t* counts, int32_t* status_dev, vrs_stream_t stream);

/* Gaussian/tile instantiation (Sec. 3 tile binning; Eq. 4 culling; per-tile
 * depth at the back-projected maximum point, Sec. 4.2).  Exclusive scan of
 * the candidate counts, then one thread per candidate (Gaussian, tile) runs
 * the exact tangent-plane tile test in FP64 and writes, at the candidate's
 * slot (order: view, Gaussian, tile; with a plan, the k-th candidate of a
 * Gaussian is the k-th visible tile of its rectangle in row-major order,
 * found from the summed-area table; pass the plan given to vrs_preprocess),
 *   keys[c] = (global_tile << 32) | ord(float32(depth)),  gids[c] = Gaussian
 * for a kept instance, or keys[c] = UINT64_MAX (dead) for a culled one;
 * global_tile = view offset + ty*ntx + tx and ord maps float order to
 * unsigned order.  n_inst_dev[0] receives the number of candidates (the
 * capacity needed) and n_inst_dev[1] the number of kept instances.  If the
 * candidates exceed `capacity`, *status_dev = VRS_ERR_CAPACITY and only the
 * first `capacity` slots are written.  If there are 2^32 - 1 candidates or
 * more (beyond the 32-bit instance offsets), *status_dev =
 * VRS_ERR_UNSUPPORTED, n_inst_dev[0] = n_inst_dev[1] = 0 and nothing is
 * written.  `proj`/`counts` come from vrs_preprocess with the same `g`,
 * cameras and params (the FP64 tile-test set-up of each counted Gaussian
 * is derived again here from `g`, by the code vrs_preprocess ran); `ws`
 * must hold sort_ws_bytes. */
int vrs_duplicate(const vrs_gaussians* g, const vrs_camera* cams, const vrs_fovea* foveas,
                  int32_t n_views, const vrs_params* p, const void* plan, const void* proj,
                  const uint32_t* counts, uint64_t* keys, uint32_t* gids, size_t capacity,
                  uint32_t* n_inst_dev, void* ws, size_t ws_bytes, int32_t* status_dev,
                  vrs_stream_t stream);

/* Stable LSD radix sort of (keys, vals) by the low `key_bits` bits of the
 * key (Sec. 3: the instances are sorted).  Equal keys keep their input order,
 * so instances written in Gaussian order come out ordered by (key, gid).
 * Sorts min(*n_dev, capacity) pairs in place; `ws` must hold
 * vrs_sort_pairs_workspace_size(capacity) bytes.  Each 8-bit digit pass is
 * reduce-then-scan (per-block digit counts, a multi-block scan, a stable
 * scatter); no block waits on another.  status_dev (may be null) is the
 * device status word of the other entry points; the sort itself reports no
 * device-side condition. */
int vrs_sort_pairs(uint64_t* keys, uint32_t* vals, const uint32_t* n_dev, size_t capacity,
                   int32_t key_bits, void* ws, size_t ws_bytes, int32_t* status_dev,
                   vrs_stream_t stream);
size_t vrs_sort_pairs_workspace_size(size_t capacity);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sort as vrs_sort_pairs, same arguments and result, but its workspace is a
 * fixed device array inside the library instead of caller memory, so the
 * call allocates nothing.  Each GPU the library runs on holds its own array
 * of vrs_sort_pairs_workspace_size(VRS_SORT_NOALLOC_MAX_PAIRS) bytes (about
 * 30 MiB) until the process ends.  capacity > VRS_SORT_NOALLOC_MAX_PAIRS
 * returns VRS_ERR_SCRATCH with nothing enqueued.  Every call on one GPU uses
 * that GPU's one array: calls that may overlap on the same GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * Nothing in the array needs to be cleared between calls. */
#define VRS_SORT_NOALLOC_MAX_PAIRS 2097152u
int vrs_sort_pairs_noalloc(uint64_t* keys, uint32_t* vals, const uint32_t* n_dev, size_t capacity,
                           int32_t key_bits, int32_t* status_dev, vrs_stream_t stream);

/* Tile ranges of sorted keys: ranges[t] = {first, last + 1} of global tile t,
 * {0, 0} for empty tiles.  ranges has tiles_total rows of two uint32. */
int vrs_tile_ranges(const uint64_t* keys, const uint32_t* n_dev, size_t capacity,
                    uint32_t tiles_total, uint32_t* ranges, vrs_stream_t stream);

/* vrs_duplicate, then the radix sort by (key, gid) whose first pass drops the
 * dead keys, so the first n_inst_dev[1] entries of keys/gids are the sorted
 * instances, then vrs_tile_ranges over them. */
int vrs_sort(const vrs_gaussians* g, const vrs_camera* cams, const vrs_fovea* foveas,
             int32_t n_views, const vrs_params* p, const void* plan, const void* proj,
             const uint32_t* counts, uint64_t* keys, uint32_t* gids, size_t capacity,
             uint32_t* n_inst_dev, uint32_t* ranges, void* ws, size_t ws_bytes,
             int32_t* status_dev, vrs_stream_t stream);

/* Per-tile blending in one launch over every work item of every view (Eq. 2;
 * Sec. 4.1 per-sample resorting with a window of p->window entries; Sec. 4.3
 * LOW/HIGH/HYBRID items), followed by the periphery reconstruction of
 * foveated views (nearest-neighbour upsampling and a 3x3 binomial blur of
 * LOW pixels, Sec. 4.3).  proj/n: the records written by vrs_preprocess
 * for n Gaussians; gids/ranges: the sorted instances of vrs_sort.  rgba[v]
 * is a device pointer to view v's output, planar float [4][height][width]
 * (R, G, B, alpha = 1 - T).  `plan` and n_items come from vrs_fovea_plan for
 * the same cameras/foveas/params; `ws` (256-byte aligned) must hold
 * render_ws_bytes.  The work items run longest first: before the blend, a
 * one-block counting sort orders them by the length of their tile's list
 * on a log scale (the order within a key is unspecified), which changes the
 * scheduling only, never the output. */
int vrs_render_foveated(const void* proj, int32_t n, const uint32_t* gids, const uint32_t* ranges,
                        const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                        const vrs_params* p, const void* plan, uint32_t n_items,
                        float* const* rgba, void* ws, size_t ws_bytes,
                        int32_t* status_dev, vrs_stream_t stream);

/* The two halves of vrs_render_foveated, for callers that time or schedule
 * them separately: vrs_blend runs the single-launch per-tile blending (LOW
 * items write their 2x2 groups, foveated views write into `ws`, plain views
 * straight into rgba); vrs_compose then writes the final image of every
 * foveated view from `ws` (nothing to do for plain views). */
int vrs_blend(const void* proj, int32_t n, const uint32_t* gids, const uint32_t* ranges,
              const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
              const vrs_params* p, const void* plan, uint32_t n_items,
              float* const* rgba, void* ws, size_t ws_bytes, int32_t* status_dev,
              vrs_stream_t stream);
int vrs_compose(const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                const vrs_params* p, const void* plan, float* const* rgba, void* ws,
                size_t ws_bytes, vrs_stream_t stream);

/* Instrumented vrs_blend (same output) that also adds to counters_dev[6]
 * (uint64, caller-zeroed): [0] evaluated (sample, list entry) pairs, [1]
 * pairs whose alpha reaches alpha_min, [2] in-image samples, [3] samples
 * stopped by t_min, [4] list entries staged by the waves, [5] wave-level
 * window insertion steps (each runs the insertion network on all 64
 * lanes).  These are the work units of the blending roofline; it runs
 * slower than vrs_blend. */
int vrs_blend_stats(const void* proj, int32_t n, const uint32_t* gids, const uint32_t* ranges,
                    const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                    const vrs_params* p, const void* plan, uint32_t n_items,
                    float* const* rgba, void* ws, size_t ws_bytes, uint64_t* counters_dev,
                    vrs_stream_t stream);

/* Gradients of a scalar loss with respect to the Gaussian parameters, in the
 * layouts of vrs_gaussians (device memory, FP32, overwritten):
 *   means[3][n], log_scales[3][n], quats[4][n], opacity_logits[n],
 *   sh[K][3][n] with K = (sh_degree+1)^2. */
typedef struct {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
} vrs_gaussian_grads;

/* Workspace bytes of vrs_render_backward: per view and Gaussian, 12 FP32
 * gradients of the render record, per foveated view three [4][H][W] FP32
 * planes (its samples' forward values, dL/d(pre-compose image),
 * dL/d(sample)), and the work items in longest-first order.  0 for invalid
 * arguments. */
size_t vrs_backward_workspace_size(int32_t n, const vrs_camera* cams, const vrs_fovea* foveas,
                                   int32_t n_views, const vrs_params* p);

/* Gradients of the rendered images (Sec. 4.1 fine-tunes position, rotation,
 * scale, opacity and SH coefficients by backpropagation through the
 * renderer with StopThePop ordering and Optimal Projection), for plain and
 * foveated views.  Inputs: the Gaussians `g`; proj/gids/ranges, the plan
 * with its n_items and rgba[v] from the forward pass (vrs_fovea_plan,
 * vrs_preprocess, vrs_sort, vrs_render_foveated) with the same cameras,
 * foveas and params; grad_rgba[v] = dL/d(rgba[v]), planar
 * [4][height][width].  Foveated views (rgba[v] is not read): dL/d(rgba) is
 * carried back through the periphery's blur and nearest-neighbour
 * upsampling and through the HYBRID mix to the samples, whose blends are
 * first re-rendered into the workspace (HYBRID samples unmixed).  The per-sample blending state is recomputed by
 * replaying the forward (same entries in the same order, same FP32
 * arithmetic), not stored; a sample's final colour and alpha are read from
 * rgba[v].  Gradients pass through the windowed order as a fixed
 * permutation (a discrete decision), and are zero through a clamped alpha
 * (alpha_max) or a clamped colour (negative SH sum).  Writes every array of
 * `out` (n Gaussians).  `ws` (256-byte aligned) must hold
 * vrs_backward_workspace_size(n, cams, foveas, n_views, p) bytes.
 * Asynchronous on `stream`. */
int vrs_render_backward(const vrs_gaussians* g, const void* proj, const uint32_t* gids,
                        const uint32_t* ranges, const vrs_camera* cams, const vrs_fovea* foveas,
                        int32_t n_views, const vrs_params* p, const void* plan, uint32_t n_items,
                        const float* const* rgba, const float* const* grad_rgba,
                        const vrs_gaussian_grads* out, void* ws, size_t ws_bytes,
                        int32_t* status_dev, vrs_stream_t stream);

/* Two-pass foveated rendering, the comparison baseline of App. A: a centre
 * pass at full resolution through a tight frustum, a periphery pass at half
 * resolution, then one blend.  Set-up (host, once per eye configuration):
 * from the plan that vrs_fovea_plan built for these cameras, foveas and
 * params, writes per view
 *   centre_boxes[4v..4v+3] = (x0, y0, x1, y1): the bounding box of the 32x32
 *     tiles holding a pixel centre with mask w > 0 (x1 == x0: none);
 *   centre_cams[v]: same pose and focal length, image = that box (principal
 *     point shifted, horizontal FoV re-derived from the box width);
 *   low_cams[v]: ceil(W/2) x ceil(H/2), focal length f/2, principal point
 *     halved, so that low-resolution pixel (i, j) looks along the ray of the
 *     full-resolution point (2i+1, 2j+1).
 * The passes are plain renders (fovea disabled, tile 16) of these cameras;
 * render the periphery with p->dilation / 4 (the same splats in angle).
 * Copies the class maps to the host: synchronises `stream`. */
int vrs_two_pass_views(const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                       const vrs_params* p, const void* plan, vrs_camera* centre_cams,
                       int32_t* centre_boxes, vrs_camera* low_cams, vrs_stream_t stream);

/* The blend of the two passes (App. A): per output pixel, the periphery
 * image upsampled bilinearly between its pixel centres (edge-clamped), and
 * inside the centre box out = w c + (1 - w) up(low) with the continuous
 * mask w of the fovea (Sec. 4.3); RGBA alike.  centre_rgba[v] is the centre
 * pass's [4][y1-y0][x1-x0] image (may be null for views without a box),
 * low_rgba[v] the periphery pass's [4][ceil(H/2)][ceil(W/2)], out_rgba[v]
 * [4][H][W].  Asynchronous on `stream`. */
int vrs_two_pass_compose(const vrs_camera* cams, const vrs_fovea* foveas, int32_t n_views,
                         const int32_t* centre_boxes, const float* const* centre_rgba,
                         const float* const* low_rgba, float* const* out_rgba, vrs_stream_t stream);

/* Fine-tuning (Sec. 4.1 fine-tunes a converged model by backpropagation;
 * Sec. 5: 5K further iterations).  The image loss, read as L1 + L2:
 *   L = mean |I - I*| + 0.2 mean (I - I*)^2 over the RGB channels of every
 *   pixel of every view,
 * written to *loss_dev (device double), and grad_rgba[v] = dL/d(rgba[v])
 * (RGB (sign(I - I*) + 0.4 (I - I*)) / n, alpha 0), all [4][H][W] planar.
 * The value is reduced in a fixed order (deterministic).  `ws` (8-byte
 * aligned) holds vrs_loss_workspace_size(n_views) bytes.  Asynchronous. */
size_t vrs_loss_workspace_size(int32_t n_views);
int vrs_loss_l1l2(const vrs_camera* cams, int32_t n_views, const float* const* rgba,
                  const float* const* target, float* const* grad_rgba, double* loss_dev, void* ws,
                  size_t ws_bytes, vrs_stream_t stream);

/* One Adam step (bias-corrected, step >= 1) over `count` parameters:
 * m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
 * param <- param - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * m and v start at zero for step 1.  Asynchronous. */
int vrs_adam_step(float* param, const float* grad, float* m, float* v, size_t count, float lr,
                  float beta1, float beta2, float eps, int32_t step, vrs_stream_t stream);

/* Human-readable name of a status code. */
const char* vrs_status_string(int code);

/* Library version string ("vrs <major>.<minor> gfx950"). */
const char* vrs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VRS_H */
