// K8: gradients of the rendered images with respect to the Gaussian
// parameters (Sec. 4.1: the Gaussians are fine-tuned by backpropagation
// through the StopThePop-ordered, Optimal-Projection renderer), for plain
// (non-foveated) views.
//
// K8a (k_render_bwd) replays, per sample, the forward blending of k_render:
// the same list order, box culling, alpha test, resort window and stop rule
// in the same FP32 arithmetic, so it emits the same entries in the same
// order.  Nothing per sample is stored by the forward pass; the replay needs
// only the forward's final colour and transmittance (read back from the
// output image).  For the i-th blended entry of a sample it forms
//   dL/dc_i     = g_rgb alpha_i T_i
//   dL/dalpha_i = g_rgb . (c_i T_i - S_i / (1 - alpha_i)) + g_a T_fin / (1 - alpha_i),
//   S_i         = (C_fin - C_<=i) + background T_fin   (the colour behind i),
// where only the scalar g_rgb . C_<=i of the running colour is needed, then
// chains dL/dalpha through alpha = opacity 2^(-|z|^2 / h^2) to the 12
// per-view splat parameters of the render record (M, a3, mean image point,
// opacity, RGB).  The window holds (depth, alpha, arrival index).  Emitted
// pairs are queued per wave and their gradients computed a wave-full at a
// time (see the kernel).  The records of the last three staged batches stay
// in a block-shared LDS ring beside their gradient accumulators; a batch's
// sums go to the per-view [Gaussian][12] buffer with one global atomic per
// value when the batch leaves the ring.  A window entry emitted after its
// batch left the ring is re-read from HBM and accumulated with global
// atomics.
//
// The LDS accumulators are 64-bit fixed point, added with integer atomics:
// on gfx950, LDS float atomics run far below the rate of LDS integer
// atomics, and the lanes of a wave mostly emit different entries (their
// windows differ), so the adds cannot be combined across lanes first.  Each
// (entry, value) accumulator takes its binary scale from its first nonzero
// contribution g0: units of 2^(e0 + 20 - 54) with |g0| < 2^e0, so
// contributions up to 2^20 |g0| are exact to 2^-34 |g0| and 256 of them
// cannot overflow.  A larger contribution bypasses the accumulator and is
// added to the global buffer directly (float atomic).
//
// K8b (k_color_bwd, k_geom_bwd) chains the per-view splat gradients to the
// raw parameters (means, log-scales, quaternions, opacity logits, SH), one
// thread per Gaussian.  The set-up geometry of K1 is re-evaluated in FP64
// forward-mode dual numbers, one pass per geometric parameter, which gives
// exact derivatives of the formulas K1 uses; the SH colour is differentiated
// with the basis polynomials' analytic gradients.
#include <float.h>

#include "geom.h"

namespace vrs {

constexpr int kBwdThreads = 256;
constexpr int kBwdBatch = 64;  // entries staged per batch (one per lane of a wave)
constexpr int kRingBatches = 3;
constexpr int kRing = kBwdBatch * kRingBatches;
constexpr int kG = 12;  // gradient values per (view, Gaussian)
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kUnset = -0x7FFFFFFF;   // accumulator scale not chosen yet
constexpr int kHead = 20;             // headroom bits over the first contribution

// Gradient slots of one (view, Gaussian).
enum GradField : int {
    G_M = 0,    // dL/dM00, M01, M10, M11 of the render record
    G_A3 = 4,   // dL/da3x, a3y
    G_XY = 6,   // dL/d(mean image point x, y)
    G_SIG = 8,  // dL/dopacity
    G_RGB = 9,  // dL/dcolour r, g, b
};

template <int W>
struct BWindow {
    float t[W], a[W];
    uint32_t k[W];

    // w <= W real slots, as the forward window (k_render's Window::init).
    __device__ inline void init(int w) {
#pragma unroll
        for (int i = 0; i < W; ++i) {
            t[i] = i < w ? -FLT_MAX : FLT_MAX;
            a[i] = 0.f;
            k[i] = kNone;
        }
    }
    // The forward window's insertion network (see k_render): inserts x and
    // returns the entry with the smallest depth among the window and x.
    __device__ inline void push(float xt, float xa, uint32_t xk, float& ea, uint32_t& ek) {
        bool c[W];
#pragma unroll
        for (int i = 0; i < W; ++i) c[i] = t[i] <= xt;
        ea = c[0] ? a[0] : xa;
        ek = c[0] ? k[0] : xk;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            a[i] = c[i] ? xa : a[i];
            k[i] = c[i] ? xk : k[i];
            if (i + 1 < W) {
                t[i] = __builtin_amdgcn_fmed3f(t[i], xt, t[i + 1]);  // as in k_render
                a[i] = c[i + 1] ? a[i + 1] : a[i];
                k[i] = c[i + 1] ? k[i + 1] : k[i];
            } else {
                t[i] = c[i] ? xt : t[i];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // Remove slot 0 (the smallest depth); the last slot becomes empty.
    __device__ inline void shift() {
#pragma unroll
        for (int i = 0; i + 1 < W; ++i) {
            t[i] = t[i + 1];
            a[i] = a[i + 1];
            k[i] = k[i + 1];
        }
        t[W - 1] = -FLT_MAX;
        a[W - 1] = 0.f;
        k[W - 1] = kNone;
    }
};

// Fixed-point accumulation of one contribution (see above).  Returns false
// when it does not fit the accumulator's range; the caller adds it elsewhere.
// `e` is the scale as read before (a scale, once set, never changes while
// its entry is in the ring; if it was still unset the compare-and-swap
// below returns whichever scale won).
__device__ inline bool fixed_add(unsigned long long* acc, int* scale, int e, float g) {
    if (e == kUnset) {
        int fe;
        frexpf(g, &fe);  // |g| < 2^fe
        const int want = fe + kHead;
        const int old = atomicCAS(scale, kUnset, want);
        e = old == kUnset ? want : old;
    }
    const float x = ldexpf(g, 30 - e);  // exact power-of-two scaling
    if (!(fabsf(x) < 1073741824.f)) return false;
    const int hi = int(x);  // x - hi is exact, and so is its product with 2^24
    const int lo = __float2int_rn((x - float(hi)) * 16777216.f);
    const long long v = (static_cast<long long>(hi) << 24) + lo;
    atomicAdd(acc, static_cast<unsigned long long>(v));
    return true;
}

__device__ inline float fixed_value(unsigned long long acc, int scale) {
    return float(ldexp(double(static_cast<long long>(acc)), scale - 54));
}

// Staged form of one list entry (6 float4): tile-relative mean offset, M,
// a3, log2 opacity, KAP, the depth coefficients and the Gaussian's index.
// The colour stays in the colour array.
__device__ inline void stage_entry(const float4* rec, uint32_t gid, int ox, int oy, float4 out[6]) {
    const float4 p0 = rec[0], p1 = rec[1], p2 = rec[2], p3 = rec[3];
    const float4 p4 = rec[4], p5 = rec[5];
    const float wy2 = reinterpret_cast<const float*>(rec)[24];
    out[0] = make_float4(float(ox - int(p0.x)) - p0.z, float(oy - int(p0.y)) - p0.w, p1.x, p1.y);
    out[1] = make_float4(p1.z, p1.w, p2.x, p2.y);
    out[2] = make_float4(p2.z, p2.w, p3.x, p3.y);
    out[3] = make_float4(p3.z, p4.x, p4.y, p4.z);
    out[4] = make_float4(p4.w, p5.x, p5.y, p5.z);
    out[5] = make_float4(p5.w, wy2, __uint_as_float(gid), 0.f);
}

// Colour (x, y, z) of Gaussian `gid` in a view's slice of the colour array.
__device__ inline float4 bwd_colour(const float4* __restrict__ vcol, uint32_t gid) { return vcol[gid]; }

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kQueue = 112;            // queued emissions per wave
constexpr int kQueueGo = kQueue - 63;  // a round runs once this many are queued

template <int W>
__global__ void __launch_bounds__(kBwdThreads) k_render_bwd(const float* __restrict__ proj, uint32_t n_gauss,
                                                            const uint32_t* __restrict__ gids,
                                                            const uint32_t* __restrict__ ranges,
                                                            const uint32_t* __restrict__ items, BwdViews views,
                                                            Knobs kn, float* __restrict__ grad2d) {
    // Field-major: the lanes of a queue round read field k of different
    // entries, 16 bytes apart rather than an entry's 96 bytes apart, which
    // spreads them over the LDS banks.
    __shared__ float4 ring[6][kRing];
    // Value-major, so that the lanes of one atomic instruction (one value of
    // different entries) fall in different banks.
    __shared__ unsigned long long acc[kG][kRing];
    // Entry-major, so that a queue round reads an entry's twelve scales
    // with three 16-byte loads.
    static_assert(kG % 4 == 0, "scales are read four at a time");
    __shared__ __align__(16) int acc_scale[kRing][kG];
    __shared__ float4 queue[kBwdThreads / 64][kQueue];

    // The work item (the plan's, as rendered by the forward pass).
    const uint32_t item = items[blockIdx.x];
    const int v = item_view(item);
    const bool low = item_class(item) == VRS_CLASS_LOW;
    const int sub = item_sub(item);
    const uint32_t tile = item_tile(item);
    const BwdView& V = views.v[v];
    const int T = V.T;
    const int tx = int(tile % uint32_t(V.ntx)), ty = int(tile / uint32_t(V.ntx));
    const int ox = tx * T, oy = ty * T;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // Sample of a lane of this wave: as in the forward, wave wv owns the 8x8
    // quadrant (qx, qy) of the 16x16 samples -- pixels of a (sub)tile, lanes
    // 4q..4q+3 a 2x2 group, or the centres of a LOW tile's 2x2 groups.
    const int bx = (T == 32 && !low) ? (sub & 1) * 16 : 0, by = (T == 32 && !low) ? (sub >> 1) * 16 : 0;
    const int qx = wv & 1, qy = wv >> 1;
    auto sample_of = [&](int l, float& sx_, float& sy_, int& px_, int& py_) {
        if (low) {
            const int gx = 8 * qx + (l & 7), gy = 8 * qy + (l >> 3);
            px_ = ox + 2 * gx;
            py_ = oy + 2 * gy;
            sx_ = float(2 * gx + 1);
            sy_ = float(2 * gy + 1);
            return;
        }
        const int qd = l >> 2, kq = l & 3;
        const int lx = 8 * qx + 2 * (qd & 3) + (kq & 1), ly = 8 * qy + 2 * (qd >> 2) + (kq >> 1);
        px_ = ox + bx + lx;
        py_ = oy + by + ly;
        sx_ = float(bx + lx) + 0.5f;
        sy_ = float(by + ly) + 0.5f;
    };
    float sx, sy;
    int px, py;
    sample_of(lane, sx, sy, px, py);
    const bool inimg = px < V.W && py < V.H;

    // Forward final state and the incoming gradient of this sample.
    const size_t plane = size_t(V.W) * size_t(V.H);
    float gr[3] = {0.f, 0.f, 0.f}, ga = 0.f, gCf = 0.f, Tf = 1.f;
    if (inimg) {
        const size_t pix = size_t(py) * V.W + px;
        Tf = 1.f - V.rgba[3 * plane + pix];
#pragma unroll
        for (int c = 0; c < 3; ++c) gr[c] = V.grad[c * plane + pix];
#pragma unroll
        for (int c = 0; c < 3; ++c) gCf = fmaf(gr[c], V.rgba[c * plane + pix] - Tf * kn.bg[c], gCf);
        ga = V.grad[3 * plane + pix];
    }
    // The part of dL/dalpha_i (times 1 - alpha_i) that does not depend on i.
    const float gback = (ga - (gr[0] * kn.bg[0] + gr[1] * kn.bg[1] + gr[2] * kn.bg[2])) * Tf;

    float Tc = 1.f;
    float D = 0.f;  // g_rgb . (colour accumulated so far)
    bool alive = inimg;
    BWindow<W> win;
    win.init(kn.window);
    const float amax = kn.alpha_max, tmin = kn.t_min;

    const uint2 rg = reinterpret_cast<const uint2*>(ranges)[V.tile_off + tile];
    const uint32_t L = rg.y - rg.x;
    const float* vproj = proj + size_t(v) * size_t(n_gauss) * kRec;
    const float4* vcol = colour_array(proj, size_t(views.n) * size_t(n_gauss)) + size_t(v) * size_t(n_gauss);
    float* vgrad = grad2d + size_t(v) * size_t(n_gauss) * kG;
    // This wave's sample rectangle, for the per-wave box culling of the forward.
    const float rx0 = low ? float(ox + 16 * qx + 1) : float(ox + bx + 8 * qx) + 0.5f;
    const float rx1 = low ? float(ox + 16 * qx + 15) : float(ox + bx + 8 * qx) + 7.5f;
    const float ry0 = low ? float(oy + 16 * qy + 1) : float(oy + by + 8 * qy) + 0.5f;
    const float ry1 = low ? float(oy + 16 * qy + 15) : float(oy + by + 8 * qy) + 7.5f;
    uint32_t ring_lo = 0;  // smallest arrival index whose record is still in the ring

    // An emission (a blended (sample, entry) pair) is completed in three
    // steps.  At the push that emits it, the lane advances T and issues the
    // load of the entry's colour; the pair becomes the lane's pending one.
    // At the lane's next emission (or a drain) the colour has arrived: the
    // lane forms dL/dalpha from T, alpha and D = g_rgb . C (the colour in
    // front), adds the pair's colour to D, and queues the record (dL/dalpha,
    // weight T alpha, arrival index, lane).  Whenever enough records are
    // queued, every lane of the wave takes one -- whichever sample it came
    // from -- and accumulates its 12 gradient values, so the gradient work
    // and the atomics run on full waves instead of on the few lanes that emit
    // at a given push.
    bool pend = false;
    float p_T = 0.f, p_ea = 0.f;
    uint32_t p_ek = 0;
    float4 pc = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t qhead = 0, qcount = 0;  // wave-uniform: ring-buffer head and length

    // Fold every pending pair into a queue record.
    auto fold = [&]() {
        bool rec = pend;
        float rdA = 0.f, rw = 0.f;
        if (pend) {
            const float gc = fmaf(gr[0], pc.x, fmaf(gr[1], pc.y, gr[2] * pc.z));
            const float w = p_T * p_ea;
            const float inv1 = __builtin_amdgcn_rcpf(1.f - p_ea);  // 1 - alpha >= 0.01
            // dL/dalpha = g_rgb . (c T - S / (1 - alpha)) + g_a T_fin / (1 - alpha),
            // S = C_fin - C_<=i (+ background T_fin, folded into gback).
            rdA = fmaf(gback - (gCf - fmaf(w, gc, D)), inv1, p_T * gc);
            D = fmaf(w, gc, D);
            rw = w;
        }
        pend = false;
        const uint64_t rm = __ballot(rec);
        if (rm == 0ull) return;
        if (rec) {
            uint32_t pos = qhead + qcount + uint32_t(__popcll(rm & lt));
            pos = pos >= uint32_t(kQueue) ? pos - uint32_t(kQueue) : pos;
            pos = pos >= uint32_t(kQueue) ? pos - uint32_t(kQueue) : pos;
            queue[wv][pos] = make_float4(rdA, rw, __uint_as_float(p_ek), __int_as_float(lane));
        }
        qcount += uint32_t(__popcll(rm));
    };

    // One round: lane l takes the l-th queued record.
    auto round = [&]() {
        wave_sync_lds();
        const uint32_t nq = qcount < 64u ? qcount : 64u;
        const bool has = uint32_t(lane) < nq;
        float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
        if (has) {
            uint32_t pos = qhead + uint32_t(lane);
            pos = pos >= uint32_t(kQueue) ? pos - uint32_t(kQueue) : pos;
            r = queue[wv][pos];
        }
        const int pl = has ? __float_as_int(r.w) : 0;
        // g_rgb of the record's sample, from the lane that owns it.
        const float pg0 = __shfl(gr[0], pl), pg1 = __shfl(gr[1], pl), pg2 = __shfl(gr[2], pl);
        if (has) {
            const float dA = r.x, w = r.y;
            const uint32_t ek = __float_as_uint(r.z);
            float qsx, qsy;
            int qpx, qpy;
            sample_of(pl, qsx, qsy, qpx, qpy);
            const bool in_ring = ek >= ring_lo;
            const int sl = int(ek % uint32_t(kRing));
            float4 e[6];
            if (in_ring) {
#pragma unroll
                for (int k = 0; k < 6; ++k) e[k] = ring[k][sl];
            } else {
                const uint32_t gid = gids[rg.x + ek];
                stage_entry(reinterpret_cast<const float4*>(vproj + size_t(gid) * kRec), gid, ox, oy, e);
            }
            const uint32_t gid = __float_as_uint(e[5].z);
            float g[kG];
#pragma unroll
            for (int k = 0; k < kG; ++k) g[k] = 0.f;
            // dL/dcolour = g_rgb of the pair's sample times its weight.
            g[G_RGB] = pg0 * w;
            g[G_RGB + 1] = pg1 * w;
            g[G_RGB + 2] = pg2 * w;
            // alpha = opacity 2^(-E), E = q / h^2, q = |M delta|^2, delta =
            // sample - mean; a clamped alpha passes no gradient to the splat.
            const float dx = e[0].x + qsx, dy = e[0].y + qsy;
            const float M00 = e[0].z, M01 = e[0].w, M10 = e[1].x, M11 = e[1].y;
            const float a3x = e[1].z, a3y = e[1].w;
            const float z1 = fmaf(M00, dx, M01 * dy);
            const float z2 = fmaf(M10, dx, M11 * dy);
            const float h = fmaf(a3x, dx, fmaf(a3y, dy, 1.f));
            const float q = fmaf(z1, z1, z2 * z2);
            // Hardware reciprocal and exp2: h > 0 for a blended pair, and
            // both exponents below are at most log2(255) in magnitude (the
            // pair passed the alpha_min test), inside the normal range.
            const float ih = __builtin_amdgcn_rcpf(h);
            const float ih2 = ih * ih;
            const float E = q * ih2;
            const float a_un = __builtin_amdgcn_exp2f(e[2].x - E);  // unclamped alpha
            if (a_un < amax) {
                const float gE = dA * (-0.69314718055994531f) * a_un;  // dL/dE
                const float cz = 2.f * gE * ih2;
                const float ch = -2.f * gE * E * ih;
                g[G_M + 0] = cz * z1 * dx;
                g[G_M + 1] = cz * z1 * dy;
                g[G_M + 2] = cz * z2 * dx;
                g[G_M + 3] = cz * z2 * dy;
                g[G_A3 + 0] = ch * dx;
                g[G_A3 + 1] = ch * dy;
                g[G_XY + 0] = -(cz * fmaf(z1, M00, z2 * M10) + ch * a3x);
                g[G_XY + 1] = -(cz * fmaf(z1, M01, z2 * M11) + ch * a3y);
                g[G_SIG] = dA * __builtin_amdgcn_exp2f(-E);
            }
            float* dst = vgrad + size_t(gid) * kG;
            int sc[kG];
            if (in_ring) {
#pragma unroll
                for (int k4 = 0; k4 < kG / 4; ++k4) {
                    const int4 s4 = reinterpret_cast<const int4*>(acc_scale[sl])[k4];
                    sc[4 * k4] = s4.x; sc[4 * k4 + 1] = s4.y; sc[4 * k4 + 2] = s4.z; sc[4 * k4 + 3] = s4.w;
                }
            }
#pragma unroll
            for (int k = 0; k < kG; ++k) {
                if (g[k] == 0.f) continue;
                if (!in_ring || !fixed_add(&acc[k][sl], &acc_scale[sl][k], sc[k], g[k])) unsafeAtomicAdd(dst + k, g[k]);
            }
        }
        qhead += nq;
        qhead = qhead >= uint32_t(kQueue) ? qhead - uint32_t(kQueue) : qhead;
        qcount -= nq;
    };

    // Blend the entry leaving the window (alpha ea, arrival index ek).
    // Called at wave-uniform points.
    auto emit = [&](float ea, uint32_t ek) {
        bool valid = alive && ek != kNone;
        const float Tn = Tc * (1.f - ea);
        if (valid && Tn < tmin) {  // stops the sample; not blended
            alive = false;
            valid = false;
        }
        if (__ballot(valid) == 0ull) return;
        fold();
        if (valid) {
            const bool in_ring = ek >= ring_lo;
            const uint32_t gid =
                in_ring ? __float_as_uint(ring[5][ek % uint32_t(kRing)].z) : gids[rg.x + ek];
            pc = bwd_colour(vcol, gid);
            pend = true;
            p_T = Tc;
            p_ea = ea;
            p_ek = ek;
            Tc = Tn;
        }
        if (qcount >= uint32_t(kQueueGo)) round();
    };

    // Complete every pending pair and empty the queue.
    auto drain = [&]() {
        fold();
        while (qcount > 0u) round();
    };

    uint32_t last_b0 = 0, staged_end = 0;
    for (uint32_t b0 = 0; b0 < L; b0 += kBwdBatch) {
        // The forward stops a wave once all its samples have stopped; the
        // block stops when all four waves have.
        if (__syncthreads_or(alive ? 1 : 0) == 0) break;
        const int nb = int(min(uint32_t(kBwdBatch), L - b0));
        const int base = int(b0 % uint32_t(kRing));
        if (b0 >= uint32_t(kRing)) {
            // Flush the batch that leaves the ring.
            for (int w = t; w < kBwdBatch * kG; w += kBwdThreads) {
                const int s = base + w / kG, k = w % kG;
                const int sc = acc_scale[s][k];
                if (sc != kUnset && acc[k][s] != 0ull)
                    unsafeAtomicAdd(&vgrad[size_t(__float_as_uint(ring[5][s].z)) * kG + k],
                                    fixed_value(acc[k][s], sc));
            }
            __syncthreads();
            ring_lo = b0 + kBwdBatch - kRing;
        }
        if (t < nb) {
            const uint32_t gid = gids[rg.x + b0 + t];
            float4 e[6];
            stage_entry(reinterpret_cast<const float4*>(vproj + size_t(gid) * kRec), gid, ox, oy, e);
#pragma unroll
            for (int k = 0; k < 6; ++k) ring[k][base + t] = e[k];
        }
        for (int w = t; w < kBwdBatch * kG; w += kBwdThreads) {
            acc[w % kG][base + w / kG] = 0ull;
            acc_scale[base + w / kG][w % kG] = kUnset;
        }
        last_b0 = b0;
        staged_end = b0 + uint32_t(nb);
        // Each wave reads the boxes of the batch for its own culling.
        bool rel = false;
        if (lane < nb) {
            const uint32_t gid = gids[rg.x + b0 + lane];
            const float4 bb = reinterpret_cast<const float4*>(vproj + size_t(gid) * kRec)[7];
            rel = !(bb.z < rx0 || bb.x > rx1 || bb.w < ry0 || bb.y > ry1);
        }
        __syncthreads();
        uint64_t todo = __ballot(rel);
        if (__ballot(alive) == 0ull) todo = 0ull;
        while (todo) {
            const int j = __builtin_ctzll(todo);
            todo &= todo - 1;
            const float4 f0 = ring[0][base + j], f1 = ring[1][base + j], f2 = ring[2][base + j];
            const float dx = f0.x + sx, dy = f0.y + sy;
            const float z1 = fmaf(f0.z, dx, f0.w * dy);
            const float z2 = fmaf(f1.x, dx, f1.y * dy);
            const float h = fmaf(f1.z, dx, fmaf(f1.w, dy, 1.f));
            const float q = fmaf(z1, z1, z2 * z2);
            const float h2 = h * h;
            const bool pass = alive && (h > 0.f) && (q <= f2.y * h2);
            if (__ballot(pass) != 0ull) {  // wave-uniform
                const float4 f3 = ring[3][base + j], f4 = ring[4][base + j], f5 = ring[5][base + j];
                const float xa = pass ? splat_alpha(f2.x, q, h2, amax) : 0.f;
                const float num = fmaf(f2.w, dx, fmaf(f3.x, dy, f2.z));
                const float w0 = fmaf(f4.x, dx, fmaf(f4.w, dy, f3.y));
                const float w1 = fmaf(f4.y, dx, fmaf(f5.x, dy, f3.z));
                const float w2 = fmaf(f4.z, dx, fmaf(f5.y, dy, f3.w));
                const float den = fmaf(w0, w0, fmaf(w1, w1, w2 * w2));
                const float xt = pass ? num * __builtin_amdgcn_rcpf(den) : -INFINITY;
                float ea;
                uint32_t ek;
                win.push(xt, xa, pass ? b0 + uint32_t(j) : kNone, ea, ek);
                emit(ea, ek);
            }
            if (__ballot(alive) == 0ull) break;
        }
        // Every emission is accumulated before the next batch may leave
        // the ring.
        drain();
    }
    // Flush the window in ascending depth order.
#pragma unroll 1
    for (int i = 0; i < W; ++i) {
        const float ea = win.a[0];
        const uint32_t ek = win.k[0];
        win.shift();
        emit(ea, ek);
    }
    drain();
    __syncthreads();
    // Flush what is left in the ring: arrival indices [first, staged_end).
    const uint32_t span = uint32_t(kRing - kBwdBatch);
    const uint32_t first = last_b0 >= span ? last_b0 - span : 0u;
    for (int w = t; w < kRing * kG; w += kBwdThreads) {
        const int s = w / kG, k = w % kG;
        const uint32_t a = first + (uint32_t(s) + uint32_t(kRing) - first % uint32_t(kRing)) % uint32_t(kRing);
        if (a >= staged_end) continue;
        const int sc = acc_scale[s][k];
        if (sc != kUnset && acc[k][s] != 0ull)
            unsafeAtomicAdd(&vgrad[size_t(__float_as_uint(ring[5][s].z)) * kG + k], fixed_value(acc[k][s], sc));
    }
}

// ---------------------------------------------------------------------------
// K8b: FP64 forward-mode dual numbers.
// ---------------------------------------------------------------------------
struct Dual {
    double v, d;
};
__device__ inline Dual dconst(double x) { return Dual{x, 0.0}; }
__device__ inline Dual operator+(Dual a, Dual b) { return Dual{a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual{a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator-(Dual a) { return Dual{-a.v, -a.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual{a.v * b.v, a.v * b.d + a.d * b.v}; }
__device__ inline Dual operator*(double a, Dual b) { return Dual{a * b.v, a * b.d}; }
__device__ inline Dual operator+(double a, Dual b) { return Dual{a + b.v, b.d}; }
__device__ inline Dual operator-(double a, Dual b) { return Dual{a - b.v, -b.d}; }
__device__ inline Dual operator/(Dual a, Dual b) {
    const double iv = 1.0 / b.v;
    const double q = a.v * iv;
    return Dual{q, (a.d - q * b.d) * iv};
}
__device__ inline Dual dsqrt(Dual a) {
    const double s = sqrt(a.v);
    return Dual{s, a.d * (0.5 / s)};
}
__device__ inline Dual dexp(Dual a) {
    const double e = exp(a.v);
    return Dual{e, a.d * e};
}

// M (with the record's power-of-two scale), a3 and the mean's image point
// as functions of the mean, log-scales and quaternion: the formulas of
// load_gaussian and make_geo, in dual arithmetic.
__device__ inline void splat_params(const Dual mu[3], const Dual ls[3], const Dual q[4], const GeoView& V,
                                    double dil, Dual M[4], Dual a3[2], Dual xy[2]) {
    const Dual qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const Dual k2 = dconst(2.0) / qq;
    const Dual w = q[0], x = q[1], y = q[2], z = q[3];
    Dual R[9];
    R[0] = 1.0 - k2 * (y * y + z * z);
    R[1] = k2 * (x * y - w * z);
    R[2] = k2 * (x * z + w * y);
    R[3] = k2 * (x * y + w * z);
    R[4] = 1.0 - k2 * (x * x + z * z);
    R[5] = k2 * (y * z - w * x);
    R[6] = k2 * (x * z - w * y);
    R[7] = k2 * (y * z + w * x);
    R[8] = 1.0 - k2 * (x * x + y * y);
    Dual s[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = dexp(ls[c]);
    double Rv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rv[k] = double(V.R[k]);
    Dual muc[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
        muc[r] = Rv[3 * r] * mu[0] + Rv[3 * r + 1] * mu[1] + Rv[3 * r + 2] * mu[2] + dconst(double(V.t[r]));
    const Dual rr = dsqrt(muc[0] * muc[0] + muc[1] * muc[1] + muc[2] * muc[2]);
    const Dual ux = muc[0] / rr, uy = muc[1] / rr, uz = muc[2] / rr;
    const Dual kk = dconst(1.0) / (1.0 + uz);
    const Dual e1[3] = {1.0 - ux * ux * kk, -(ux * uy * kk), -ux};
    const Dual e2[3] = {-(ux * uy * kk), 1.0 - uy * uy * kk, -uy};
    // G2 = E^T R_c S with R_c = R_v R.
    Dual g0[3], g1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const Dual c0 = Rv[0] * R[c] + Rv[1] * R[3 + c] + Rv[2] * R[6 + c];
        const Dual c1 = Rv[3] * R[c] + Rv[4] * R[3 + c] + Rv[5] * R[6 + c];
        const Dual c2 = Rv[6] * R[c] + Rv[7] * R[3 + c] + Rv[8] * R[6 + c];
        g0[c] = (e1[0] * c0 + e1[1] * c1 + e1[2] * c2) * s[c];
        g1[c] = (e2[0] * c0 + e2[1] * c1 + e2[2] * c2) * s[c];
    }
    const Dual fr = dconst(V.f) / rr;
    const Dual sc = fr * fr;
    const Dual sa = sc * (g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2]) + dconst(dil);
    const Dual sb = sc * (g0[0] * g1[0] + g0[1] * g1[1] + g0[2] * g1[2]);
    const Dual scc = sc * (g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]) + dconst(dil);
    const Dual det = sa * scc - sb * sb;
    const Dual c00 = scc / det, c01 = -(sb / det), c11 = sa / det;
    const Dual l00 = dsqrt(c00);
    const Dual l01 = c01 / l00;
    const Dual l11 = dsqrt(c11 - l01 * l01);
    const double zs = double(float(sqrt(0.5 / M_LN2)));  // the record's scale, as rounded there
    M[0] = zs * (uz * (l00 * e1[0] + l01 * e2[0]));
    M[1] = zs * (uz * (l00 * e1[1] + l01 * e2[1]));
    M[2] = zs * (uz * (l11 * e2[0]));
    M[3] = zs * (uz * (l11 * e2[1]));
    a3[0] = V.inv_f * (uz * ux);
    a3[1] = V.inv_f * (uz * uy);
    xy[0] = double(V.cx) + V.f * (muc[0] / muc[2]);
    xy[1] = double(V.cy) + V.f * (muc[1] / muc[2]);
}

// Gradient of one Gaussian's render-record gradients of view v (12 floats).
__device__ inline void load_g12(const float* grad2d, int v, int n, int i, float gv[kG]) {
    const float4* gg = reinterpret_cast<const float4*>(grad2d + (size_t(v) * n + i) * kG);
    const float4 a = gg[0], b = gg[1], c = gg[2];
    gv[0] = a.x; gv[1] = a.y; gv[2] = a.z; gv[3] = a.w;
    gv[4] = b.x; gv[5] = b.y; gv[6] = b.z; gv[7] = b.w;
    gv[8] = c.x; gv[9] = c.y; gv[10] = c.z; gv[11] = c.w;
}

// Value and gradient (d/dx, d/dy, d/dz) of a polynomial in the direction.
struct Grad3 {
    float v, x, y, z;
};
__device__ inline Grad3 g3(float v, float x, float y, float z) { return Grad3{v, x, y, z}; }

// Real SH basis function k (the polynomials of sh_basis) and its gradient
// with respect to the (unnormalised) polynomial variables x, y, z.
__device__ inline Grad3 sh_basis_grad(int k, float x, float y, float z) {
    constexpr double pi = M_PI;
    switch (k) {
        case 0: return g3(float(0.5 / sqrt(pi)), 0.f, 0.f, 0.f);
        case 1: { const float c = float(sqrt(3.0 / (4.0 * pi))); return g3(-c * y, 0.f, -c, 0.f); }
        case 2: { const float c = float(sqrt(3.0 / (4.0 * pi))); return g3(c * z, 0.f, 0.f, c); }
        case 3: { const float c = float(sqrt(3.0 / (4.0 * pi))); return g3(-c * x, -c, 0.f, 0.f); }
        case 4: { const float c = float(sqrt(15.0 / (4.0 * pi))); return g3(c * x * y, c * y, c * x, 0.f); }
        case 5: { const float c = float(sqrt(15.0 / (4.0 * pi))); return g3(-c * y * z, 0.f, -c * z, -c * y); }
        case 6: {
            const float c = float(sqrt(5.0 / (16.0 * pi)));
            return g3(c * (3.f * z * z - 1.f), 0.f, 0.f, 6.f * c * z);
        }
        case 7: { const float c = float(sqrt(15.0 / (4.0 * pi))); return g3(-c * x * z, -c * z, 0.f, -c * x); }
        case 8: {
            const float c = float(sqrt(15.0 / (16.0 * pi)));
            return g3(c * (x * x - y * y), 2.f * c * x, -2.f * c * y, 0.f);
        }
        case 9: {
            const float c = float(sqrt(35.0 / (32.0 * pi)));
            return g3(-c * y * (3.f * x * x - y * y), -6.f * c * x * y, -c * (3.f * x * x - 3.f * y * y), 0.f);
        }
        case 10: {
            const float c = float(sqrt(105.0 / (4.0 * pi)));
            return g3(c * x * y * z, c * y * z, c * x * z, c * x * y);
        }
        case 11: {
            const float c = float(sqrt(21.0 / (32.0 * pi)));
            return g3(-c * y * (5.f * z * z - 1.f), 0.f, -c * (5.f * z * z - 1.f), -10.f * c * y * z);
        }
        case 12: {
            const float c = float(sqrt(7.0 / (16.0 * pi)));
            return g3(c * z * (5.f * z * z - 3.f), 0.f, 0.f, c * (15.f * z * z - 3.f));
        }
        case 13: {
            const float c = float(sqrt(21.0 / (32.0 * pi)));
            return g3(-c * x * (5.f * z * z - 1.f), -c * (5.f * z * z - 1.f), 0.f, -10.f * c * x * z);
        }
        case 14: {
            const float c = float(sqrt(105.0 / (16.0 * pi)));
            return g3(c * z * (x * x - y * y), 2.f * c * x * z, -2.f * c * y * z, c * (x * x - y * y));
        }
        default: {
            const float c = float(sqrt(35.0 / (32.0 * pi)));
            return g3(-c * x * (x * x - 3.f * y * y), -c * (3.f * x * x - 3.f * y * y), 6.f * c * x * y, 0.f);
        }
    }
}

// K8b, colour part: SH coefficients, and the mean through the view
// direction.  colour_c = max(0, sum_k sh_kc Y_k(u) + 0.5) with u = d / |d|,
// d = mean - eye centre: dL/dsh_kc = g_c Y_k(u) where the colour is not
// clamped, and dL/dmean = J_u^T sum_c g_c grad Y . sh_c with
// J_u = (I - u u^T) / |d|.  One thread per Gaussian; writes out.sh and
// out.means (the geometry part adds to the latter).  The SH degree is a
// template parameter: no per-coefficient branches, and the loads of a view
// can be issued together.
template <int kDeg>
__global__ void __launch_bounds__(256) k_color_bwd(GaussPtrs g, GeoViews views, const float* __restrict__ grad2d,
                                                   GradPtrs out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int n = g.n;
    constexpr int K = (kDeg + 1) * (kDeg + 1);
    const double mu[3] = {double(g.means[i]), double(g.means[n + i]), double(g.means[2 * n + i])};
    float gsh[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
    float gm[3] = {0.f, 0.f, 0.f};
    for (int v = 0; v < views.n; ++v) {
        const GeoView& V = views.v[v];
        const float4 gc = reinterpret_cast<const float4*>(grad2d + (size_t(v) * n + i) * kG)[2];
        const float grgb[3] = {gc.y, gc.z, gc.w};
        if (grgb[0] == 0.f && grgb[1] == 0.f && grgb[2] == 0.f) continue;
        double dir[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dir[c] = mu[c] + (double(V.R[c]) * V.t[0] + double(V.R[3 + c]) * V.t[1] + double(V.R[6 + c]) * V.t[2]);
        const double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        const float u[3] = {float(dir[0] / dn), float(dir[1] / dn), float(dir[2] / dn)};
        // Colour values and gradients with respect to u.
        Grad3 col[3] = {g3(0.5f, 0.f, 0.f, 0.f), g3(0.5f, 0.f, 0.f, 0.f), g3(0.5f, 0.f, 0.f, 0.f)};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const Grad3 y = sh_basis_grad(k, u[0], u[1], u[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float a = g.sh[(k * 3 + c) * n + i];
                col[c].v = fmaf(a, y.v, col[c].v);
                col[c].x = fmaf(a, y.x, col[c].x);
                col[c].y = fmaf(a, y.y, col[c].y);
                col[c].z = fmaf(a, y.z, col[c].z);
            }
        }
        float wc[3], gu[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            wc[c] = col[c].v > 0.f ? grgb[c] : 0.f;  // a clamped colour passes no gradient
            gu[0] = fmaf(wc[c], col[c].x, gu[0]);
            gu[1] = fmaf(wc[c], col[c].y, gu[1]);
            gu[2] = fmaf(wc[c], col[c].z, gu[2]);
        }
        // Through u = d / |d|: dL/dd = (gu - (gu . u) u) / |d|.
        const float gdotu = gu[0] * u[0] + gu[1] * u[1] + gu[2] * u[2];
        const float idn = float(1.0 / dn);
#pragma unroll
        for (int c = 0; c < 3; ++c) gm[c] = fmaf(gu[c] - gdotu * u[c], idn, gm[c]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float yv = sh_basis_grad(k, u[0], u[1], u[2]).v;
#pragma unroll
            for (int c = 0; c < 3; ++c) gsh[k][c] = fmaf(wc[c], yv, gsh[k][c]);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) out.means[c * n + i] = gm[c];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) out.sh[(k * 3 + c) * n + i] = gsh[k][c];
    }
}

// K8b, geometry part: means (added to the colour part), log-scales,
// quaternions and opacity logits.  The FP64 dual numbers take every register
// a wave can have; held to two waves per SIMD, the kernel spills a few
// values and runs faster than at one.
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) k_geom_bwd(GaussPtrs g, GeoViews views, Knobs kn,
                                                  const float* __restrict__ grad2d, GradPtrs out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int n = g.n;
    double p[10];
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = double(g.means[c * n + i]);
#pragma unroll
    for (int c = 0; c < 3; ++c) p[3 + c] = double(g.log_scales[c * n + i]);
#pragma unroll
    for (int c = 0; c < 4; ++c) p[6 + c] = double(g.quats[c * n + i]);
    const double sig = 1.0 / (1.0 + exp(-double(g.opac[i])));
    double gp[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) gp[k] = 0.0;
    double gop = 0.0;
    for (int v = 0; v < views.n; ++v) {
        const GeoView& V = views.v[v];
        float gv[kG];
        load_g12(grad2d, v, n, i, gv);
        bool any = false;
#pragma unroll
        for (int k = 0; k < G_RGB; ++k) any = any || gv[k] != 0.f;
        if (!any) continue;
        gop += double(gv[G_SIG]) * sig * (1.0 - sig);
        // One dual pass per mean, log-scale and quaternion entry.
#pragma unroll 1
        for (int pi = 0; pi < 10; ++pi) {
            Dual mu[3], ls[3], q[4];
            for (int c = 0; c < 3; ++c) {
                mu[c] = Dual{p[c], pi == c ? 1.0 : 0.0};
                ls[c] = Dual{p[3 + c], pi == 3 + c ? 1.0 : 0.0};
            }
            for (int c = 0; c < 4; ++c) q[c] = Dual{p[6 + c], pi == 6 + c ? 1.0 : 0.0};
            Dual M[4], a3[2], xy[2];
            splat_params(mu, ls, q, V, double(kn.dilation), M, a3, xy);
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) s += double(gv[G_M + k]) * M[k].d;
            s += double(gv[G_A3]) * a3[0].d + double(gv[G_A3 + 1]) * a3[1].d;
            s += double(gv[G_XY]) * xy[0].d + double(gv[G_XY + 1]) * xy[1].d;
            gp[pi] += s;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) out.means[c * n + i] = float(double(out.means[c * n + i]) + gp[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) out.log_scales[c * n + i] = float(gp[3 + c]);
#pragma unroll
    for (int c = 0; c < 4; ++c) out.quats[c * n + i] = float(gp[6 + c]);
    out.opac[i] = float(gop);
}

__global__ void __launch_bounds__(256) k_fill_f32(float* __restrict__ p, size_t n) {
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.f;
}

size_t backward_ws_bytes(size_t n, int n_views) { return n * size_t(n_views) * kG * sizeof(float); }

// ---------------------------------------------------------------------------
// Foveated views: dL/d(final image) back through the periphery blur and the
// nearest-neighbour upsampling, and through the HYBRID mix (Sec. 4.3), to
// the samples, deterministically (gathers, no atomics).
// ---------------------------------------------------------------------------
__device__ inline uint8_t fov_class(const FovGradView& V, int x, int y) {
    return V.cls[size_t(y >> 4) * V.ntx16 + (x >> 4)];
}

// dL/d(pre)[q] = dL/d(final)[q] if q is not LOW, plus, for every LOW pixel p
// whose edge-clamped 3x3 window reads q, K(delta) dL/d(final)[p] summed
// over the offsets delta that land on q.  One thread per pixel q.
__global__ void __launch_bounds__(256) k_fov_grad_pre(FovGradView V) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= V.W || y >= V.H) return;
    const size_t plane = size_t(V.W) * V.H, q = size_t(y) * V.W + x;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (fov_class(V, x, y) != VRS_CLASS_LOW)
        for (int c = 0; c < 4; ++c) acc[c] = V.gout[c * plane + q];
    for (int py = max(y - 1, 0); py <= min(y + 1, V.H - 1); ++py)
        for (int px = max(x - 1, 0); px <= min(x + 1, V.W - 1); ++px) {
            if (fov_class(V, px, py) != VRS_CLASS_LOW) continue;
            float w = 0.f;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int sx = min(max(px + dx, 0), V.W - 1), sy = min(max(py + dy, 0), V.H - 1);
                    if (sx == x && sy == y) w += float((2 - dx * dx) * (2 - dy * dy)) * (1.f / 16.f);
                }
            const size_t p = size_t(py) * V.W + px;
            for (int c = 0; c < 4; ++c) acc[c] = fmaf(w, V.gout[c * plane + p], acc[c]);
        }
    for (int c = 0; c < 4; ++c) V.gpre[c * plane + q] = acc[c];
}

// dL/d(sample): a HIGH pixel's is dL/d(pre); a HYBRID pixel q's is
// w_q dL/d(pre)[q] + sum over its 2x2 group's in-image pixels p of
// (1 - w_p) / n dL/d(pre)[p]; a LOW group's (at its top-left pixel) is the
// sum of dL/d(pre) over its in-image pixels.
__global__ void __launch_bounds__(256) k_fov_grad_samples(FovGradView V) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= V.W || y >= V.H) return;
    const size_t plane = size_t(V.W) * V.H, q = size_t(y) * V.W + x;
    const uint8_t k = fov_class(V, x, y);
    const int gx = x & ~1, gy = y & ~1;
    const int gx1 = min(gx + 1, V.W - 1), gy1 = min(gy + 1, V.H - 1);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (k == VRS_CLASS_LOW) {
        if (x != gx || y != gy) return;  // only the group's top-left pixel holds its sample
        for (int yy = gy; yy <= gy1; ++yy)
            for (int xx = gx; xx <= gx1; ++xx)
                for (int c = 0; c < 4; ++c) acc[c] += V.gpre[c * plane + size_t(yy) * V.W + xx];
    } else if (k == VRS_CLASS_HYBRID) {
        const float n = float((gx1 - gx + 1) * (gy1 - gy + 1));
        const float wq = fovea_weight(V.mask, x, y);
        for (int c = 0; c < 4; ++c) acc[c] = wq * V.gpre[c * plane + q];
        for (int yy = gy; yy <= gy1; ++yy)
            for (int xx = gx; xx <= gx1; ++xx) {
                const float f = (1.f - fovea_weight(V.mask, xx, yy)) / n;
                for (int c = 0; c < 4; ++c) acc[c] = fmaf(f, V.gpre[c * plane + size_t(yy) * V.W + xx], acc[c]);
            }
    } else {
        for (int c = 0; c < 4; ++c) acc[c] = V.gpre[c * plane + q];
    }
    for (int c = 0; c < 4; ++c) V.gsamp[c * plane + q] = acc[c];
}

int launch_fov_grads(const FovGradView& V, hipStream_t s) {
    const dim3 grid((V.W + 63) / 64, (V.H + 3) / 4);
    hipLaunchKernelGGL(k_fov_grad_pre, grid, dim3(256), 0, s, V);
    hipLaunchKernelGGL(k_fov_grad_samples, grid, dim3(256), 0, s, V);
    return launch_status(hipGetLastError());
}

template <int W>
static void launch_render_bwd(const float* proj, uint32_t n, const uint32_t* gids, const uint32_t* ranges,
                              const uint32_t* items, uint32_t n_items, const BwdViews& views, const Knobs& kn,
                              float* grad2d, hipStream_t s) {
    hipLaunchKernelGGL(k_render_bwd<W>, dim3(n_items), dim3(kBwdThreads), 0, s, proj, n, gids, ranges, items,
                       views, kn, grad2d);
}

int launch_backward(const GaussPtrs& g, const GeoViews& gv, const float* proj, const uint32_t* gids,
                    const uint32_t* ranges, const uint32_t* items, uint32_t n_items, const BwdViews& views,
                    const Knobs& kn, int window, float* grad2d, const GradPtrs& out, hipStream_t s) {
    const size_t ng = size_t(g.n) * size_t(views.n) * kG;
    if (ng > 0) {
        const size_t blocks = (ng + 255) / 256;
        hipLaunchKernelGGL(k_fill_f32, dim3(unsigned(blocks < 16384 ? blocks : 16384)), dim3(256), 0, s, grad2d,
                           ng);
    }
    if (n_items > 0 && g.n > 0) {
#define VRS_BWD_W(w)                                                                                      \
    case w:                                                                                               \
        launch_render_bwd<w>(proj, uint32_t(g.n), gids, ranges, items, n_items, views, kn, grad2d, s); \
        break;
        switch (window_network(window)) {
            VRS_BWD_W(1) VRS_BWD_W(2) VRS_BWD_W(3) VRS_BWD_W(4) VRS_BWD_W(6) VRS_BWD_W(8) VRS_BWD_W(12)
            VRS_BWD_W(16) VRS_BWD_W(24) VRS_BWD_W(32)
            default: return VRS_ERR_UNSUPPORTED;
        }
#undef VRS_BWD_W
    }
    if (g.n > 0) {
        const dim3 cg(unsigned((g.n + 255) / 256));
        switch (g.sh_degree) {
            case 0: hipLaunchKernelGGL(k_color_bwd<0>, cg, dim3(256), 0, s, g, gv, grad2d, out); break;
            case 1: hipLaunchKernelGGL(k_color_bwd<1>, cg, dim3(256), 0, s, g, gv, grad2d, out); break;
            case 2: hipLaunchKernelGGL(k_color_bwd<2>, cg, dim3(256), 0, s, g, gv, grad2d, out); break;
            default: hipLaunchKernelGGL(k_color_bwd<3>, cg, dim3(256), 0, s, g, gv, grad2d, out); break;
        }
        hipLaunchKernelGGL(k_geom_bwd, dim3(unsigned((g.n + 127) / 128)), dim3(128), 0, s, g, gv, kn, grad2d, out);
    }
    return launch_status(hipGetLastError());
}

}  // namespace vrs
