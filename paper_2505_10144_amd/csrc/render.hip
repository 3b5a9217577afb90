// K6: per-tile blending in one launch over the work items of every view, and
// K7: periphery reconstruction of foveated views.
//
// K6 (Eq. 2; Sec. 4.1 per-pixel resorting; Sec. 4.3 single-pass foveation).
// One 256-thread block per work item.  Each thread owns one sample: a pixel
// of a 16x16 tile/subtile, or the centre of a 2x2 group of a 32x32 LOW tile
// (half resolution).  The four waves of a block walk the tile's sorted list
// independently: each wave stages 64 list entries at a time in its own LDS
// slice (one record per lane, so there is no block barrier) and then every
// lane evaluates the splat for its sample from broadcast LDS reads.  Entries
// whose alpha reaches alpha_min go into a per-sample window of W entries kept
// sorted in registers; when it overflows the entry with the smallest depth is
// blended.  A wave stops as soon as all of its samples have stopped.
//
// Per-pair arithmetic (pixel offset delta = sample - mean image point):
//   z = M delta / h, h = 1 + a3 . delta;  alpha = opacity * 2^(-|z|^2 / h^2)
//   (M carries the factor that turns e^(-D^2/2) into a power of two);
//   the pass test |z|^2 <= KAP h^2 needs no division;
//   depth t = (n0 + nx dx + ny dy) / |w0 + dx wx + dy wy|^2 (ray depth of
//   maximum density, ordered identically to the unit-ray depth).
#include <float.h>

#include "vrs_internal.h"

namespace vrs {

int launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);

constexpr int kRenderThreads = 256;
constexpr int kBatch = 56;      // entries staged per wave and batch, at most
constexpr int kStage = 6;       // float4 per staged entry
constexpr int kInbox = 6;       // entries a lane collects before the wave drains

// A window entry: depth, alpha and the Gaussian's index; its colour is
// fetched from the render record when the entry is blended.
struct Slot {
    float t, a;
    uint32_t id;
};

template <int W>
struct Window {
    float t[W], a[W];
    uint32_t id[W];

    // A window of w <= W entries: w placeholders at -FLT_MAX, which the
    // first w insertions emit (blending them is a no-op, alpha 0), and W - w
    // at +FLT_MAX, which no finite depth displaces, so an insertion emits
    // the smallest of the w real entries and the new one; the final flush
    // reaches them last, after every real entry.
    __device__ inline void init(int w) {
#pragma unroll
        for (int i = 0; i < W; ++i) {
            t[i] = i < w ? -FLT_MAX : FLT_MAX;
            a[i] = 0.f; id[i] = 0u;
        }
    }

    // Insert x, then remove and return the entry with the smallest depth.
    // With c[i] = (t[i] <= x.t) (a prefix of the sorted window), the result
    // is: emitted = c[0] ? slot 0 : x, and slot i becomes slot i+1 if
    // c[i+1], else x if c[i], else stays -- so a window entry wins ties (it
    // arrived earlier).  For the depths that is the median of t[i], x.t and
    // t[i+1] (one instruction); alpha and index follow the masks.  Slots are
    // rewritten in ascending order, each from itself and its not-yet-
    // rewritten neighbour, so the update is in place.
    // Pushing an entry with t = -inf and alpha = 0 leaves the window
    // unchanged and returns that entry, whose blend is a no-op: lanes with
    // nothing to insert run the same instructions as the others.
    __device__ inline Slot push(const Slot& x) {
        bool c[W];
#pragma unroll
        for (int i = 0; i < W; ++i) c[i] = t[i] <= x.t;
        Slot e;
        e.t = c[0] ? t[0] : x.t;
        e.a = c[0] ? a[0] : x.a;
        e.id = c[0] ? id[0] : x.id;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            a[i] = c[i] ? x.a : a[i];
            id[i] = c[i] ? x.id : id[i];
            if (i + 1 < W) {
                t[i] = __builtin_amdgcn_fmed3f(t[i], x.t, t[i + 1]);
                a[i] = c[i + 1] ? a[i + 1] : a[i];
                id[i] = c[i + 1] ? id[i + 1] : id[i];
            } else {
                t[i] = c[i] ? x.t : t[i];
            }
            // Keep each slot's update together so that it can be done in
            // the slot's own registers (no rotation copies at the loop edge).
            __builtin_amdgcn_sched_barrier(0);
        }
        return e;
    }
};

struct Accum {
    float T, cr, cg, cb;
    bool alive;

    // Front-to-back blending of one entry, split in two: weight() takes the
    // entry's alpha, advances the transmittance and returns the entry's
    // weight T alpha (zero when it is not blended: the entry that would take
    // T below t_min stops the sample); add() accumulates weight x colour.
    // Colours are added in the order of the weights, so deferring add() does
    // not change the result.  Branch-free so that the window state never
    // merges across divergent paths.
    __device__ inline float weight(float a, float t_min) {
        const float Tn = T * (1.f - a);
        const bool stop = Tn < t_min;
        const bool ok = alive && !stop;
        const float w = ok ? T * a : 0.f;
        T = ok ? Tn : T;
        alive = ok;
        return w;
    }
    __device__ inline void add(float w, float r, float g, float b) {
        cr = fmaf(w, r, cr);
        cg = fmaf(w, g, cg);
        cb = fmaf(w, b, cb);
    }
};

// Colour (x, y, z) of Gaussian `gid` in a view's slice of the colour array.
__device__ inline float4 gauss_colour(const float4* __restrict__ vcol, uint32_t gid) { return vcol[gid]; }

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave's share of a work item: the 8x8 quadrant wv of the item's 16x16
// samples (pixels of a 16x16 (sub)tile, or the half-resolution samples of a
// LOW tile).  A square quadrant rather than a 16x4 strip: its pixel box
// meets fewer splat boxes, and its samples see more similar lists, so the
// insertion network idles less (blend 0.70 -> 0.66 ms).  `st` is
// the wave's own LDS slice; min(batch, kBatch) list entries are staged at a
// time.  STATS = true is the instrumented variant: it also counts evaluated
// (sample, entry) pairs, pairs that reach alpha_min, in-image samples,
// samples stopped by t_min and list entries staged.
//
// Window insertions are batched per lane: an entry that reaches alpha_min at
// a sample goes into the lane's inbox (LDS, its own column), and when some
// lane's inbox is full the wave drains every lane's inbox through the
// window in arrival order.  Each lane therefore pushes exactly the entries,
// in exactly the order, of an immediate insertion -- the output is the same
// bit for bit -- but the insertion network, which runs on all 64 lanes
// whenever any lane inserts, runs about as often as the busiest lane
// inserts rather than once per entry that any lane inserts.  A lane whose
// transmittance has fallen below t_min is only found to have stopped at the
// next drain; the entries it collects meanwhile are then skipped.  The
// instrumented variant inserts immediately (an inbox of one), so that its
// counters measure the algorithm's work.
template <int W, bool STATS>
__device__ inline void render_unit(uint32_t item, int wv, float4 (*st)[kStage], float2 (*ib)[64], uint32_t (*ibg)[64],
                                   const float* __restrict__ proj, uint32_t n_gauss,
                                   const uint32_t* __restrict__ gids, const uint32_t* __restrict__ ranges,
                                   const RenderViews& views, const Knobs& kn, int batch,
                                   unsigned long long* __restrict__ stats) {
    constexpr int kCap = STATS ? 1 : kInbox;
    batch = min(batch, kBatch);
    const int v = item_view(item);
    const int cls = item_class(item);
    const int sub = item_sub(item);
    const uint32_t tile = item_tile(item);
    const RenderView& V = views.v[v];
    if (V.skip) return;  // (waves never wait on each other: the whole wave leaves)
    const int T = V.foveated ? 32 : V.T;
    const int tx = int(tile % uint32_t(V.ntx)), ty = int(tile / uint32_t(V.ntx));
    const int ox = tx * T, oy = ty * T;  // sort-tile origin (pixels)
    const int lane = int(threadIdx.x) & 63;

    // Sample of this thread, relative to the tile origin.
    int px, py;      // first pixel covered
    float sx, sy;    // sample position relative to (ox, oy)
    // Wave wv owns the 8x8 quadrant (qx, qy) of the item's 16x16 samples.
    const int qx = wv & 1, qy = wv >> 1;
    if (cls == VRS_CLASS_LOW) {
        const int gx = 8 * qx + (lane & 7), gy = 8 * qy + (lane >> 3);
        px = ox + 2 * gx;
        py = oy + 2 * gy;
        sx = float(2 * gx + 1);
        sy = float(2 * gy + 1);
    } else {
        // Quad-major layout: lanes 4q..4q+3 hold one aligned 2x2 group.
        const int q = lane >> 2, k = lane & 3;
        const int lx = 8 * qx + 2 * (q & 3) + (k & 1), ly = 8 * qy + 2 * (q >> 2) + (k >> 1);
        const int bx = (T == 32) ? (sub & 1) * 16 : 0, by = (T == 32) ? (sub >> 1) * 16 : 0;
        px = ox + bx + lx;
        py = oy + by + ly;
        sx = float(bx + lx) + 0.5f;
        sy = float(by + ly) + 0.5f;
    }
    const bool inimg = px < V.W && py < V.H;

    Accum acc;
    acc.T = 1.f; acc.cr = 0.f; acc.cg = 0.f; acc.cb = 0.f;
    acc.alive = inimg;
    Window<W> win;
    win.init(kn.window);

    const uint2 rg = reinterpret_cast<const uint2*>(ranges)[V.tile_off + tile];
    const float* vproj = proj + size_t(v) * size_t(n_gauss) * kRec;
    const float4* vcol = colour_array(proj, size_t(views.n) * size_t(n_gauss)) + size_t(v) * size_t(n_gauss);
    const float amax = kn.alpha_max, tmin = kn.t_min;
    uint32_t n_pairs = 0, n_contrib = 0, n_staged = 0, n_push = 0;
    int cnt = 0;  // entries in this lane's inbox
    float pw = 0.f;                                 // weight of the last emission
    float4 pc = make_float4(0.f, 0.f, 0.f, 0.f);   // its colour (x, y, z)

    // This wave's samples lie in a pixel rectangle; list entries whose box
    // misses it cannot reach alpha_min at any of them and are skipped for
    // the whole wave (hierarchical culling of 16x16 subtiles against their
    // parent's 32x32 list, generalised to every wave).
    float rx0, ry0, rx1, ry1;
    if (cls == VRS_CLASS_LOW) {
        rx0 = float(ox + 16 * qx + 1); rx1 = float(ox + 16 * qx + 15);
        ry0 = float(oy + 16 * qy + 1); ry1 = float(oy + 16 * qy + 15);
    } else {
        const int bx = (T == 32) ? (sub & 1) * 16 : 0, by = (T == 32) ? (sub >> 1) * 16 : 0;
        rx0 = float(ox + bx + 8 * qx) + 0.5f; rx1 = float(ox + bx + 8 * qx) + 7.5f;
        ry0 = float(oy + by + 8 * qy) + 0.5f; ry1 = float(oy + by + 8 * qy) + 7.5f;
    }

    // Collect entries into the inboxes until some lane's inbox is full or the
    // list ends, then push every lane's inbox through its window in arrival
    // order; repeat.  A single drain site keeps the window's registers apart
    // from the collecting loop's.
    // One push of every lane's inbox entry i (a placeholder where the lane
    // has fewer) through its window, blending the entry that leaves.
    auto drain_step = [&](int i) {
        const bool has = i < cnt;
        if (STATS) ++n_push;
        Slot x;
        x.t = -INFINITY; x.a = 0.f; x.id = 0u;
        if (has) {
            const float2 v2 = ib[i][lane];
            x.t = v2.x; x.a = v2.y; x.id = ibg[i][lane];
        }
        const Slot e = win.push(x);
        const float w = acc.weight(e.a, tmin);
        // Add the previous emission, whose colour load was issued one step
        // earlier (a zero weight adds nothing: colours are finite), then
        // issue this one's.  The load is unconditional so that it lands
        // straight in the registers the next step reads: e.id is a list
        // entry's Gaussian or the placeholder 0, and the wave has list
        // entries, so the record exists.
        acc.add(pw, pc.x, pc.y, pc.z);
        pw = w;
        pc = gauss_colour(vcol, e.id);
    };

    uint32_t b0 = rg.x;          // first list entry of the staged batch
    uint64_t todo = 0;           // staged entries of the batch still to test
    bool staged = false;         // a batch is staged in this wave's slice
    for (;;) {
        bool full = false;
        for (;;) {
            if (todo == 0ull) {
                if (staged) {
                    wave_sync_lds();
                    b0 += uint32_t(batch);
                }
                if (b0 >= rg.y || __ballot(acc.alive) == 0ull) break;
                const int nb = int(min(uint32_t(batch), rg.y - b0));
                bool rel = false;
                if (lane < nb) {
                    const uint32_t gid = gids[b0 + lane];
                    const float4* rec = reinterpret_cast<const float4*>(vproj + size_t(gid) * kRec);
                    const float4 p7 = rec[7];
                    rel = (p7.z >= rx0) & (p7.x <= rx1) & (p7.w >= ry0) & (p7.y <= ry1);
                    if (rel) {
                        const float4 p0 = rec[0], p1 = rec[1], p2 = rec[2], p3 = rec[3];
                        const float4 p4 = rec[4], p5 = rec[5];
                        const float wy2 = vproj[size_t(gid) * kRec + 24];
                        // Mean offset relative to the tile origin, split so that
                        // the integer part is exact: (ox - x0i) - x0f.
                        const float ex = float(ox - int(p0.x)) - p0.z;
                        const float ey = float(oy - int(p0.y)) - p0.w;
                        st[lane][0] = make_float4(ex, ey, p1.x, p1.y);          // M00 M01
                        st[lane][1] = make_float4(p1.z, p1.w, p2.x, p2.y);      // M10 M11 a3x a3y
                        st[lane][2] = make_float4(p2.z, p2.w, p3.x, p3.y);      // l2s kap n0 nx
                        st[lane][3] = make_float4(p3.z, p4.x, p4.y, p4.z);      // ny w0
                        st[lane][4] = make_float4(p4.w, p5.x, p5.y, p5.z);      // wx wy.x
                        st[lane][5] = make_float4(p5.w, wy2, __uint_as_float(gid), 0.f);  // wy.yz gid
                    }
                }
                todo = __ballot(rel);
                staged = true;
                if (STATS) n_staged += uint32_t(__popcll(todo));
                wave_sync_lds();
                continue;
            }
            const int j = __builtin_ctzll(todo);
            todo &= todo - 1;
            const float4 f0 = st[j][0], f1 = st[j][1], f2 = st[j][2];
            const float dx = f0.x + sx, dy = f0.y + sy;
            const float z1 = fmaf(f0.z, dx, f0.w * dy);
            const float z2 = fmaf(f1.x, dx, f1.y * dy);
            const float h = fmaf(f1.z, dx, fmaf(f1.w, dy, 1.f));
            const float q = fmaf(z1, z1, z2 * z2);
            const float h2 = h * h;
            const bool pass = acc.alive && (h > 0.f) && (q <= f2.y * h2);
            if (STATS) {
                n_pairs += acc.alive ? 1u : 0u;
                n_contrib += pass ? 1u : 0u;
            }
            if (pass) {
                const float4 f3 = st[j][3], f4 = st[j][4], f5 = st[j][5];
                const float a = splat_alpha(f2.x, q, h2, amax);
                const float num = fmaf(f2.w, dx, fmaf(f3.x, dy, f2.z));
                const float w0 = fmaf(f4.x, dx, fmaf(f4.w, dy, f3.y));
                const float w1 = fmaf(f4.y, dx, fmaf(f5.x, dy, f3.z));
                const float w2 = fmaf(f4.z, dx, fmaf(f5.y, dy, f3.w));
                const float den = fmaf(w0, w0, fmaf(w1, w1, w2 * w2));
                const float t = num * __builtin_amdgcn_rcpf(den);
                ib[cnt][lane] = make_float2(t, a);
                ibg[cnt][lane] = __float_as_uint(f5.z);
                ++cnt;
            }
            if (__ballot(cnt >= kCap) != 0ull) {  // wave-uniform
                full = true;
                break;
            }
        }
        if (!full) break;
        // Drain: every lane pushes its inbox through its window in order.
        // Some lane's inbox is full, so every step is needed; the steps are
        // unrolled and unconditional, so the window stays in the same
        // registers from step to step.
#pragma unroll
        for (int i = 0; i < kCap; ++i) drain_step(i);
        cnt = 0;
        if (__ballot(acc.alive) == 0ull) break;
    }
    // The list ended (or every sample stopped): drain what is left.
#pragma unroll 1
    for (int i = 0; i < kCap; ++i) {
        if (__ballot(i < cnt) == 0ull) break;  // wave-uniform
        drain_step(i);
    }
    acc.add(pw, pc.x, pc.y, pc.z);
    // Flush the window in ascending depth order: weights first (they chain
    // through T), then the colours, four loads in flight at a time (which
    // keeps the register peak down).
    float wf[W];
#pragma unroll
    for (int i = 0; i < W; ++i) wf[i] = acc.weight(win.a[i], tmin);
#pragma unroll
    for (int i0 = 0; i0 < W; i0 += 4) {
        float4 c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (i0 + k < W && wf[i0 + k] != 0.f) c[k] = gauss_colour(vcol, win.id[i0 + k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k < W) acc.add(wf[i0 + k], c[k].x, c[k].y, c[k].z);
        __builtin_amdgcn_sched_barrier(0);
    }

    if (STATS) {
        // Wave sums, then one atomic per counter and wave (staged entries are
        // counted once per wave already).
        unsigned long long c[4] = {n_pairs, n_contrib, inimg ? 1ull : 0ull, (inimg && !acc.alive) ? 1ull : 0ull};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            for (int d = 32; d >= 1; d >>= 1) c[k] += __shfl_xor(c[k], d);
        if (lane == 0) {
            for (int k = 0; k < 4; ++k) atomicAdd(&stats[k], c[k]);
            atomicAdd(&stats[4], (unsigned long long)n_staged);
            atomicAdd(&stats[5], (unsigned long long)n_push);
        }
    }
    float o[4] = {acc.cr + acc.T * kn.bg[0], acc.cg + acc.T * kn.bg[1], acc.cb + acc.T * kn.bg[2], 1.f - acc.T};
    float* dst = V.foveated ? V.pre : V.out;
    const size_t plane = size_t(V.W) * size_t(V.H);
    if (cls == VRS_CLASS_LOW) {
        for (int c = 0; c < 4; ++c) {
            float* pl = dst + c * plane;
            for (int yy = 0; yy < 2; ++yy)
                for (int xx = 0; xx < 2; ++xx)
                    if (px + xx < V.W && py + yy < V.H) pl[size_t(py + yy) * V.W + px + xx] = o[c];
        }
        return;
    }
    if (cls == VRS_CLASS_HYBRID && !V.nomix) {
        // The continuous foveation mask at this pixel.
        const float wm = fovea_weight(V.mask, px, py);
        // Mean of the aligned 2x2 group over its in-image pixels.
        const float cnt0 = inimg ? 1.f : 0.f;
        float cnt = cnt0 + __shfl_xor(cnt0, 1);
        cnt = cnt + __shfl_xor(cnt, 2);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float mine = inimg ? o[c] : 0.f;
            float s = mine + __shfl_xor(mine, 1);
            s = s + __shfl_xor(s, 2);
            o[c] = wm * o[c] + (1.f - wm) * (s / cnt);
        }
    }
    if (inimg) {
        const size_t off = size_t(py) * V.W + px;
#pragma unroll
        for (int c = 0; c < 4; ++c) dst[c * plane + off] = o[c];
    }
}

// K6 launch.  One-shot schedule (PERSIST = false): one block per work item,
// in the given (longest-first) order.  Persistent schedule: a grid that
// fills the chip once, whose waves take (item, quadrant) units in order from
// an atomic counter until none are left, so a wave that finishes early
// starts new work at once instead of idling until its block's slowest wave
// ends.  The counter must be zero at launch; every wave exits after drawing
// a unit past the end.
//
// LDS per block: the four waves' staging slices (21 KB) and inboxes (18 KB),
// so that four blocks fit a CU; with W <= 16 the kernel is held to 128 VGPRs,
// which makes that four waves per SIMD.  The blend is bound by instruction
// issue, and the fourth wave hides the latency of LDS reads and of the
// record loads better than a larger inbox would save drains; within that
// budget a 6-entry inbox with 56-entry batches drains less often than a
// 5-entry one with 64-entry batches (0.624 -> 0.615 ms on the stereo frame).
template <int W, bool STATS, bool PERSIST>
__global__ void __launch_bounds__(kRenderThreads) __attribute__((amdgpu_waves_per_eu(W <= 16 ? 4 : 1)))
k_render(const float* __restrict__ proj, uint32_t n_gauss, const uint32_t* __restrict__ gids,
         const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ items, uint32_t n_items,
         uint32_t* __restrict__ counter, int batch, RenderViews views, Knobs kn,
         unsigned long long* __restrict__ stats) {
    __shared__ float4 stage[kRenderThreads / 64][kBatch][kStage];
    __shared__ float2 inbox[kRenderThreads / 64][kInbox][64];
    __shared__ uint32_t inbox_id[kRenderThreads / 64][kInbox][64];
    // Wave index, known to the compiler as wave-uniform (scalar registers).
    const int slot = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    if (!PERSIST) {
        render_unit<W, STATS>(items[blockIdx.x], slot, stage[slot], inbox[slot], inbox_id[slot], proj, n_gauss, gids,
                              ranges, views, kn, batch, stats);
        return;
    }
    const int lane = int(threadIdx.x) & 63;
    const uint32_t n_units = 4u * n_items;
    for (;;) {
        uint32_t u = 0;
        if (lane == 0) u = atomicAdd(counter, 1u);
        u = __builtin_amdgcn_readfirstlane(u);
        if (u >= n_units) break;
        render_unit<W, STATS>(items[u >> 2], int(u & 3u), stage[slot], inbox[slot], inbox_id[slot], proj, n_gauss,
                              gids, ranges, views, kn, batch, stats);
    }
}

// K7: LOW pixels of a foveated view take the 3x3 binomial blur of the
// nearest-neighbour-upsampled image (coordinates clamped to the image); other
// pixels are copied.  One block per 64x16 tile: a thread owns a column of
// four output pixels and reads the six rows their windows span once each (a
// wave reads whole 256-byte row segments of each plane).  Workgroups are dealt to the
// eight XCDs round-robin, and each XCD has its own L2; the block index is
// remapped so that every XCD gets a contiguous band of tile rows, whose
// blur halos then hit in that XCD's L2 instead of being fetched again by a
// neighbour XCD.
constexpr uint32_t kXcds = 8;

constexpr int kComposeRows = 4;  // output rows per thread

__global__ void __launch_bounds__(256) k_compose(RenderView V, const uint8_t* __restrict__ cls, uint32_t ntiles,
                                                 uint32_t per_xcd) {
    const uint32_t tid = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (tid >= ntiles) return;
    const uint32_t ntx = uint32_t(V.W + 63) / 64;
    const int x = int(tid % ntx) * 64 + int(threadIdx.x & 63);
    const int y0 = (int(tid / ntx) * 4 + int(threadIdx.x >> 6)) * kComposeRows;
    if (x >= V.W || y0 >= V.H) return;
    const size_t plane = size_t(V.W) * size_t(V.H);
    const int xs[3] = {max(x - 1, 0), x, min(x + 1, V.W - 1)};
    // Rows y0 - 1 .. y0 + kComposeRows (clamped): each is read once and
    // serves the three outputs whose window holds it.
    int ry[kComposeRows + 2];
#pragma unroll
    for (int r = 0; r < kComposeRows + 2; ++r) ry[r] = min(max(y0 - 1 + r, 0), V.H - 1);
    uint8_t c[kComposeRows];
#pragma unroll
    for (int r = 0; r < kComposeRows; ++r)
        c[r] = cls[V.cls_off + size_t(min(y0 + r, V.H - 1) >> 4) * V.ntx16 + (x >> 4)];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float* p = V.pre + k * plane;
        float h[kComposeRows + 2], mid[kComposeRows + 2];
#pragma unroll
        for (int r = 0; r < kComposeRows + 2; ++r) {
            const float* row = p + size_t(ry[r]) * V.W;
            const float a = row[xs[0]], b = row[xs[1]], d = row[xs[2]];
            h[r] = fmaf(1.f, a, fmaf(2.f, b, d));  // horizontal 1-2-1
            mid[r] = b;
        }
#pragma unroll
        for (int r = 0; r < kComposeRows; ++r) {
            if (y0 + r >= V.H) break;
            const float s = fmaf(1.f, h[r + 2], fmaf(2.f, h[r + 1], h[r]));
            V.out[k * plane + size_t(y0 + r) * V.W + x] = c[r] == VRS_CLASS_LOW ? s * (1.f / 16.f) : mid[r + 1];
        }
    }
}

// K7 with 16-byte accesses, for views whose width is a multiple of 4: a
// thread owns a 4x4 pixel block (one 16x16 subtile, so one class decides
// it).  Per row and plane it loads one float4 and takes the pixels left and
// right of it from the neighbouring lanes (loading them only at the wave's
// two ends).  One block covers 256x16 pixels: 64 lanes x 4 columns, 4 waves
// x 4 rows, with the same XCD-aware block order as k_compose.  In a LOW
// block the blend wrote each value to a 2x2 pixel group, so the block's
// second and fourth rows repeat its first and third and are not loaded.  The
// arithmetic is k_compose's, term for term.
__global__ void __launch_bounds__(256) k_compose4(RenderView V, const uint8_t* __restrict__ cls, uint32_t ntiles,
                                                  uint32_t per_xcd) {
    const uint32_t tid = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (tid >= ntiles) return;
    const uint32_t ntx = uint32_t(V.W + 255) / 256;
    const int lane = int(threadIdx.x & 63);
    const int x = int(tid % ntx) * 256 + 4 * lane;
    const int y0 = (int(tid / ntx) * 4 + int(threadIdx.x >> 6)) * 4;
    if (y0 >= V.H) return;  // whole wave
    const bool act = x < V.W;
    const int xc = act ? x : V.W - 4;  // lanes past the edge load in bounds, store nothing
    const size_t plane = size_t(V.W) * size_t(V.H);
    const int xl = max(xc - 1, 0), xr = min(xc + 4, V.W - 1);
    int ry[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) ry[r] = min(max(y0 - 1 + r, 0), V.H - 1);
    const uint8_t c = cls[V.cls_off + size_t(y0 >> 4) * V.ntx16 + (xc >> 4)];
    const bool low = c == VRS_CLASS_LOW;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float* p = V.pre + k * plane;
        float4 h[6], mid[6];
        float4 vprev = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const float* row = p + size_t(ry[r]) * V.W;
            float4 v = vprev;
            if (!low || r == 0 || r == 1 || r == 3 || r == 5) v = *reinterpret_cast<const float4*>(row + xc);
            vprev = v;
            // Left neighbour: lane - 1's last pixel (or the clamped pixel at
            // the image edge, or a load at the wave's first lane).
            const float up = __shfl_up(v.w, 1);
            const float dn = __shfl_down(v.x, 1);
            float left = lane > 0 ? up : row[xl];
            if (xc == 0) left = v.x;
            float right = (lane < 63 && xc + 4 < V.W) ? dn : row[xr];
            if (!act) right = v.w;
            h[r].x = fmaf(1.f, left, fmaf(2.f, v.x, v.y));
            h[r].y = fmaf(1.f, v.x, fmaf(2.f, v.y, v.z));
            h[r].z = fmaf(1.f, v.y, fmaf(2.f, v.z, v.w));
            h[r].w = fmaf(1.f, v.z, fmaf(2.f, v.w, right));
            mid[r] = v;
        }
        if (!act) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (y0 + r >= V.H) break;
            float4 o = mid[r + 1];
            if (low) {
                o.x = fmaf(1.f, h[r + 2].x, fmaf(2.f, h[r + 1].x, h[r].x)) * (1.f / 16.f);
                o.y = fmaf(1.f, h[r + 2].y, fmaf(2.f, h[r + 1].y, h[r].y)) * (1.f / 16.f);
                o.z = fmaf(1.f, h[r + 2].z, fmaf(2.f, h[r + 1].z, h[r].z)) * (1.f / 16.f);
                o.w = fmaf(1.f, h[r + 2].w, fmaf(2.f, h[r + 1].w, h[r].w)) * (1.f / 16.f);
            }
            *reinterpret_cast<float4*>(V.out + k * plane + size_t(y0 + r) * V.W + x) = o;
        }
    }
}

// Blocks of a persistent launch: enough to fill every CU at the kernel's
// occupancy, never more than the work items.
template <typename K>
static uint32_t persistent_blocks(K kernel, uint32_t n_items) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kRenderThreads, 0) != hipSuccess ||
        cus <= 0 || per_cu <= 0)
        return n_items;
    const uint64_t b = uint64_t(cus) * uint64_t(per_cu);
    return uint32_t(b < n_items ? b : n_items);
}

template <int W, bool STATS>
static void launch_render_ws(const float* proj, uint32_t n_gauss, const uint32_t* gids, const uint32_t* ranges,
                             const uint32_t* items, uint32_t n_items, uint32_t* counter, int batch, int schedule,
                             const RenderViews& views, const Knobs& kn, unsigned long long* stats, hipStream_t s) {
    if (schedule == VRS_SCHEDULE_PERSISTENT) {
        const uint32_t blocks = persistent_blocks(k_render<W, STATS, true>, n_items);
        hipLaunchKernelGGL((k_render<W, STATS, true>), dim3(blocks), dim3(kRenderThreads), 0, s, proj, n_gauss, gids,
                           ranges, items, n_items, counter, batch, views, kn, stats);
    } else {
        hipLaunchKernelGGL((k_render<W, STATS, false>), dim3(n_items), dim3(kRenderThreads), 0, s, proj, n_gauss,
                           gids, ranges, items, n_items, counter, batch, views, kn, stats);
    }
}

template <int W>
static void launch_render_w(const float* proj, uint32_t n_gauss, const uint32_t* gids, const uint32_t* ranges,
                            const uint32_t* items, uint32_t n_items, uint32_t* counter, int batch, int schedule,
                            const RenderViews& views, const Knobs& kn, unsigned long long* stats, hipStream_t s) {
    if (stats)
        launch_render_ws<W, true>(proj, n_gauss, gids, ranges, items, n_items, counter, batch, schedule, views, kn,
                                  stats, s);
    else
        launch_render_ws<W, false>(proj, n_gauss, gids, ranges, items, n_items, counter, batch, schedule, views, kn,
                                   stats, s);
}

int launch_blend(const float* proj, uint32_t n_gauss, const uint32_t* gids, const uint32_t* ranges,
                 const uint32_t* items, uint32_t n_items, uint32_t* counter, int batch, int schedule,
                 const RenderViews& views, const Knobs& kn, int window, unsigned long long* stats, hipStream_t s) {
    if (n_items == 0) return VRS_OK;
    if (schedule == VRS_SCHEDULE_PERSISTENT) {
        const int rc = launch_fill_u32(counter, 1, 0u, s);
        if (rc != VRS_OK) return rc;
    }
#define VRS_W(w)                                                                                                  \
    case w:                                                                                                       \
        launch_render_w<w>(proj, n_gauss, gids, ranges, items, n_items, counter, batch, schedule, views, kn, stats, \
                           s);                                                                                    \
        break;
    switch (window_network(window)) {
        VRS_W(1) VRS_W(2) VRS_W(3) VRS_W(4) VRS_W(6) VRS_W(8) VRS_W(12) VRS_W(16) VRS_W(24) VRS_W(32)
        default: return VRS_ERR_UNSUPPORTED;
    }
#undef VRS_W
    return launch_status(hipGetLastError());
}

// Longest-first order of the work items (list scheduling: the blocks that
// take longest start first, so they do not extend the end of the launch).
// The cost of an item is the length of its sort tile's list (halved for a
// subtile, see cost_key); the key is that cost on a log scale with 16 steps
// per octave.  One block does a
// counting sort by that key, longest first: an LDS histogram, its scan,
// then every item takes the next slot of its key's run with an LDS atomic.
// Each key's run is split into kOrderSub parts by thread (thread mod
// kOrderSub), with a counter each, so that the many items of a popular key
// do not all update one LDS word.  The order within a run depends on
// timing, which does not matter: every item writes only its own pixels.
constexpr int kOrderThreads = 1024;
constexpr int kOrderPer = 16;  // items a thread has in flight
constexpr int kOrderSub = 4;
static_assert(256 * kOrderSub == kOrderThreads, "one (key, part) counter per thread in the scan");

// `sub`: a 16x16 subtile of a 32x32 sort tile, whose waves cull its list to
// 8x8-pixel rectangles and so evaluate about half the entries a LOW item of
// the same list does; its cost is taken as half its list length.
__device__ inline uint32_t cost_key(uint2 rg, bool sub) {
    const uint32_t c = sub ? (rg.y - rg.x) >> 1 : rg.y - rg.x;
    uint32_t b = 0;
    if (c != 0) {
        const int e = 31 - __clz(int(c));
        const uint32_t m = e >= 4 ? (c >> (e - 4)) & 15u : (c << (4 - e)) & 15u;
        b = min(255u, uint32_t(e) * 16u + m + 1u);
    }
    return 255u - b;  // ascending key = descending cost
}

__global__ void __launch_bounds__(kOrderThreads) k_order_items(const uint32_t* __restrict__ items,
                                                               const uint32_t* __restrict__ count_dev,
                                                               uint32_t n_max, const uint32_t* __restrict__ ranges,
                                                               RenderViews views, uint32_t* __restrict__ out) {
    __shared__ uint32_t cnt[256 * kOrderSub];  // (key, part), key-major
    __shared__ uint32_t wsum[kOrderThreads / 64];
    __shared__ uint32_t toff[VRS_MAX_VIEWS];  // each view's first global tile
    const int t = threadIdx.x;
    const uint32_t part = uint32_t(t % kOrderSub);
    const uint32_t n = min(*count_dev, n_max);
    constexpr uint32_t kChunk = uint32_t(kOrderThreads * kOrderPer);
    cnt[t] = 0;
    if (t < views.n) toff[t] = views.v[t].tile_off;
    __syncthreads();
    const uint2* rgs = reinterpret_cast<const uint2*>(ranges);
    // A chunk's items, then their list ranges, each as one batch of loads.
    auto keys_of = [&](uint32_t c0, const uint32_t (&it)[kOrderPer], uint32_t (&key)[kOrderPer]) {
        uint2 rg[kOrderPer];
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j) {
            rg[j] = make_uint2(0u, 0u);
            if (c0 + uint32_t(j * kOrderThreads + t) < n) rg[j] = rgs[toff[item_view(it[j])] + item_tile(it[j])];
        }
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j) {
            const RenderView& V = views.v[item_view(it[j])];
            key[j] = cost_key(rg[j], item_class(it[j]) != VRS_CLASS_LOW && (V.foveated || V.T == 32));
        }
    };
    // Each thread keeps kOrderPer items (and their list-range loads) in
    // flight at a time.  The first chunk's items and keys stay in registers
    // for the scatter (the only chunk when there are at most kChunk items);
    // later chunks are loaded again.
    uint32_t it0[kOrderPer], key0[kOrderPer];
#pragma unroll
    for (int j = 0; j < kOrderPer; ++j) {
        const uint32_t i = uint32_t(j * kOrderThreads + t);
        it0[j] = i < n ? items[i] : 0u;
    }
    keys_of(0u, it0, key0);
#pragma unroll
    for (int j = 0; j < kOrderPer; ++j)
        if (uint32_t(j * kOrderThreads + t) < n) atomicAdd(&cnt[key0[j] * kOrderSub + part], 1u);
    for (uint32_t c0 = kChunk; c0 < n; c0 += kChunk) {
        uint32_t it[kOrderPer], key[kOrderPer];
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j) {
            const uint32_t i = c0 + uint32_t(j * kOrderThreads + t);
            it[j] = i < n ? items[i] : 0u;
        }
        keys_of(c0, it, key);
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j)
            if (c0 + uint32_t(j * kOrderThreads + t) < n) atomicAdd(&cnt[key[j] * kOrderSub + part], 1u);
    }
    __syncthreads();
    // Exclusive scan of the (key, part) counts, one per thread.
    const uint32_t x = cnt[t];
    uint32_t v = x;
    {
        const int lane = t & 63;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(v, o);
            if (lane >= o) v += y;
        }
        if (lane == 63) wsum[t >> 6] = v;
    }
    __syncthreads();
    {
        uint32_t pre = 0;
        for (int k = 0; k < (t >> 6); ++k) pre += wsum[k];
        cnt[t] = pre + v - x;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kOrderPer; ++j)
        if (uint32_t(j * kOrderThreads + t) < n) out[atomicAdd(&cnt[key0[j] * kOrderSub + part], 1u)] = it0[j];
    for (uint32_t c0 = kChunk; c0 < n; c0 += kChunk) {
        uint32_t it[kOrderPer], key[kOrderPer];
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j) {
            const uint32_t i = c0 + uint32_t(j * kOrderThreads + t);
            it[j] = i < n ? items[i] : 0u;
        }
        keys_of(c0, it, key);
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j)
            if (c0 + uint32_t(j * kOrderThreads + t) < n) out[atomicAdd(&cnt[key[j] * kOrderSub + part], 1u)] = it[j];
    }
}

// Ordering area: [0, 256) the persistent schedule's unit counter, then the
// ordered items.
size_t order_ws_bytes(size_t items_max) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    return 256 + al(items_max * 4);
}

uint32_t* order_counter(void* ws) { return static_cast<uint32_t*>(ws); }

// Writes the ordered items into the ordering area `ws` and returns them.
const uint32_t* launch_order_items(const uint32_t* items, uint32_t n_items, const uint32_t* count_dev,
                                   size_t items_max, const uint32_t* ranges, const RenderViews& views, void* ws,
                                   int* err, hipStream_t s) {
    (void)err;
    (void)items_max;
    uint32_t* out = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + 256);
    if (n_items == 0) return out;
    hipLaunchKernelGGL(k_order_items, dim3(1), dim3(kOrderThreads), 0, s, items, count_dev, n_items, ranges, views,
                       out);
    if (hipGetLastError() != hipSuccess) return nullptr;
    return out;
}

int launch_compose(const RenderViews& views, const uint8_t* cls, hipStream_t s) {
    for (int v = 0; v < views.n; ++v) {
        const RenderView& V = views.v[v];
        if (!V.foveated) continue;
        if (V.W % 4 == 0 && (reinterpret_cast<uintptr_t>(V.pre) & 15u) == 0 &&
            (reinterpret_cast<uintptr_t>(V.out) & 15u) == 0) {
            const uint32_t ntiles = uint32_t((V.W + 255) / 256) * uint32_t((V.H + 15) / 16);
            const uint32_t per = (ntiles + kXcds - 1) / kXcds;
            hipLaunchKernelGGL(k_compose4, dim3(per * kXcds), dim3(256), 0, s, V, cls, ntiles, per);
            continue;
        }
        const uint32_t ntiles = uint32_t((V.W + 63) / 64) * uint32_t((V.H + 4 * kComposeRows - 1) / (4 * kComposeRows));
        const uint32_t per = (ntiles + kXcds - 1) / kXcds;
        hipLaunchKernelGGL(k_compose, dim3(per * kXcds), dim3(256), 0, s, V, cls, ntiles, per);
    }
    return launch_status(hipGetLastError());
}

}  // namespace vrs
