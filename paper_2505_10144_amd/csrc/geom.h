// FP64 per-Gaussian set-up geometry (preprocessing, K1) and the tangent-plane
// tile test with its per-tile depth (instantiation, K3).  The set-up runs
// once per Gaussian and view, the test once per candidate (Gaussian, tile);
// double precision costs little next to the memory traffic of those kernels
// and keeps the discrete decisions (near cull, tile test, key depth) within a
// few ulp of exact.
#pragma once

#include "vrs_internal.h"

namespace vrs {

struct GaussLocal {
    double mu[3];
    double R[9];   // rotation of the Gaussian (world), row-major
    double s[3];   // standard deviations
    double is[3];  // 1 / s
    double sigma;  // opacity
    bool ok;
    bool nonfinite;  // a raw parameter (mean, log-scale, quaternion, opacity logit) is NaN or infinite
};

__device__ inline GaussLocal load_gaussian(const GaussPtrs& g, int i) {
    GaussLocal L;
    const int n = g.n;
    double q[4];
    for (int c = 0; c < 3; ++c) {
        L.mu[c] = double(g.means[c * n + i]);
        L.s[c] = exp(double(g.log_scales[c * n + i]));
        L.is[c] = 1.0 / L.s[c];
    }
    for (int c = 0; c < 4; ++c) q[c] = double(g.quats[c * n + i]);
    L.sigma = 1.0 / (1.0 + exp(-double(g.opac[i])));
    bool fin = isfinite(g.opac[i]);
    for (int c = 0; c < 3; ++c) fin = fin && isfinite(g.means[c * n + i]) && isfinite(g.log_scales[c * n + i]);
    for (int c = 0; c < 4; ++c) fin = fin && isfinite(g.quats[c * n + i]);
    L.nonfinite = !fin;
    const double qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    bool ok = qq > 0.0 && isfinite(qq) && isfinite(L.sigma);
    for (int c = 0; c < 3; ++c) ok = ok && isfinite(L.mu[c]) && isfinite(L.s[c]) && L.s[c] > 0.0;
    L.ok = ok && fin;
    // Rotation matrix of the unit quaternion q/|q| (Hamilton convention),
    // written with 2/|q|^2 so that no square root is needed.
    const double k2 = 2.0 / qq;
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    L.R[0] = 1.0 - k2 * (y * y + z * z);
    L.R[1] = k2 * (x * y - w * z);
    L.R[2] = k2 * (x * z + w * y);
    L.R[3] = k2 * (x * y + w * z);
    L.R[4] = 1.0 - k2 * (x * x + z * z);
    L.R[5] = k2 * (y * z - w * x);
    L.R[6] = k2 * (x * z - w * y);
    L.R[7] = k2 * (y * z + w * x);
    L.R[8] = 1.0 - k2 * (x * x + y * y);
    return L;
}

// The FP64 tile-test set-up of one Gaussian in one view.  K1 derives it for
// the render record and the candidate rectangle; K3 derives it again from
// the Gaussian's parameters (the same code on the same inputs, so the same
// values) rather than reading 176 bytes per Gaussian-view back from memory.
struct TileGeo {
    double x0, y0;     // image point of the mean (pixels)
    double M[4];       // whitened tangent coords z = M delta / h, |z|^2 = D^2
    double a3x, a3y;   // h = 1 + a3 . delta  (> 0 iff the ray is in front)
    double kappa;      // keep iff D^2_min <= kappa = 2 ln(opacity / alpha_min)
    double r;          // |mu_c|: the depth when the mean lies in the tile (per-Gaussian
                       //   key depths: that key, after K1)
    double n0, nx, ny;         // depth numerator  n0 + nx dx + ny dy
    double w0[3], wx[3], wy[3];  // denominator |w0 + dx wx + dy wy|^2
};

// A Gaussian's candidate tiles in one view, stored by K1 for K3.
struct TileRect {
    int32_t tx0, ty0;    // candidate tile rectangle: origin,
    uint16_t ncx, ncy;   //   width and height (tiles),
    int32_t count;       //   and the number of its (visible) tiles
};
static_assert(sizeof(TileRect) == kTileRectBytes, "TileRect layout");

// Everything K1 derives for one Gaussian in one view.
struct Geo {
    TileGeo tg;
    double u[3];       // mean direction
    double muc[3];
    double lam_max;    // largest eigenvalue of Sigma_2D (px^2)
    double l2s;        // log2(opacity)
};

// Optimal Projection set-up (Sec. 3 end, Sec. 4.2).  Returns false when the
// Gaussian is culled from the view (camera z <= z_near, opacity below
// alpha_min, non-finite or degenerate input).
__device__ inline bool make_geo(const GaussLocal& G, const GeoView& V, const Knobs& kn, double ln_amin,
                                Geo& o) {
    if (!G.ok || !(G.sigma >= double(kn.alpha_min))) return false;
    double Rv[9];
    for (int k = 0; k < 9; ++k) Rv[k] = double(V.R[k]);
    for (int r = 0; r < 3; ++r)
        o.muc[r] = Rv[3 * r] * G.mu[0] + Rv[3 * r + 1] * G.mu[1] + Rv[3 * r + 2] * G.mu[2] + double(V.t[r]);
    if (!(o.muc[2] > double(kn.z_near))) return false;
    const double f = V.f, inv_f = V.inv_f;
    // Camera-frame rotation of the Gaussian, R_c = R_v R.
    double Rc[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            Rc[3 * r + c] = Rv[3 * r] * G.R[c] + Rv[3 * r + 1] * G.R[3 + c] + Rv[3 * r + 2] * G.R[6 + c];
    TileGeo& t = o.tg;
    t.r = sqrt(o.muc[0] * o.muc[0] + o.muc[1] * o.muc[1] + o.muc[2] * o.muc[2]);
    const double inv_r = 1.0 / t.r;
    for (int c = 0; c < 3; ++c) o.u[c] = o.muc[c] * inv_r;
    const double ux = o.u[0], uy = o.u[1], uz = o.u[2];
    // Tangent-plane basis: images of the camera x/y axes under the minimal
    // rotation taking +z to u (any orthonormal basis gives the same splat).
    const double k = 1.0 / (1.0 + uz);
    const double e1[3] = {1.0 - ux * ux * k, -ux * uy * k, -ux};
    const double e2[3] = {-ux * uy * k, 1.0 - uy * uy * k, -uy};
    // G2 = E^T R_c S; Sigma_2D = (f / r)^2 G2 G2^T + dilation I.
    double g0[3], g1[3];
    for (int c = 0; c < 3; ++c) {
        const double c0 = Rc[c], c1 = Rc[3 + c], c2 = Rc[6 + c];
        g0[c] = (e1[0] * c0 + e1[1] * c1 + e1[2] * c2) * G.s[c];
        g1[c] = (e2[0] * c0 + e2[1] * c1 + e2[2] * c2) * G.s[c];
    }
    const double sc = (f * inv_r) * (f * inv_r);
    const double dil = double(kn.dilation);
    const double sa = sc * (g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2]) + dil;
    const double sb = sc * (g0[0] * g1[0] + g0[1] * g1[1] + g0[2] * g1[2]);
    const double scc = sc * (g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]) + dil;
    const double det = sa * scc - sb * sb;
    if (!(det > 0.0)) return false;
    const double inv_det = 1.0 / det;
    // Conic C = Sigma_2D^-1 and its factor C = L^T L, L upper triangular.
    const double c00 = scc * inv_det, c01 = -sb * inv_det, c11 = sa * inv_det;
    const double l00 = sqrt(c00);
    const double l01 = c01 / l00;
    const double l11 = sqrt(fmax(c11 - l01 * l01, 0.0));
    // Tangent coordinate of the pixel offset delta from the mean's image
    // point: q = u_z A delta / (1 + a3 . delta), A the xy-block of E^T.
    const double A00 = e1[0], A01 = e1[1], A10 = e2[0], A11 = e2[1];
    t.M[0] = uz * (l00 * A00 + l01 * A10);
    t.M[1] = uz * (l00 * A01 + l01 * A11);
    t.M[2] = uz * (l11 * A10);
    t.M[3] = uz * (l11 * A11);
    t.a3x = uz * ux * inv_f;
    t.a3y = uz * uy * inv_f;
    const double inv_z = 1.0 / o.muc[2];
    t.x0 = double(V.cx) + f * o.muc[0] * inv_z;
    t.y0 = double(V.cy) + f * o.muc[1] * inv_z;
    const double ln_s = log(G.sigma);
    t.kappa = 2.0 * (ln_s - ln_amin);
    o.l2s = ln_s * M_LOG2E;
    const double tr = 0.5 * (sa + scc);
    o.lam_max = tr + sqrt(0.25 * (sa - scc) * (sa - scc) + sb * sb);
    // Depth along the pixel ray d(delta) = (x0 + dx - cx, y0 + dy - cy, f)/f:
    // t*(d) = d^T B mu_c / d^T B d with B = Sigma_c^-1 = W3^T W3, W3 =
    // S^-1 R_c^T, so with m = W3 mu_c and w(delta) = W3 d(delta):
    // w = m / z + dx W3[:,0] / f + dy W3[:,1] / f and numerator w . m.
    double m[3];
    for (int r = 0; r < 3; ++r) {
        // Row r of W3 is column r of R_c scaled by 1/s_r.
        const double w_0 = Rc[r] * G.is[r], w_1 = Rc[3 + r] * G.is[r], w_2 = Rc[6 + r] * G.is[r];
        m[r] = w_0 * o.muc[0] + w_1 * o.muc[1] + w_2 * o.muc[2];
        t.wx[r] = w_0 * inv_f;
        t.wy[r] = w_1 * inv_f;
        t.w0[r] = m[r] * inv_z;
    }
    t.n0 = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * inv_z;
    t.nx = t.wx[0] * m[0] + t.wx[1] * m[1] + t.wx[2] * m[2];
    t.ny = t.wy[0] * m[0] + t.wy[1] * m[1] + t.wy[2] * m[2];
    return true;
}

// Candidate tiles: the image of the cone of half-angle beta, tan(beta) =
// sqrt(kappa lam_max) / f, around u contains every ray where alpha reaches
// alpha_min (the footprint on the tangent plane lies in the disc of radius
// sqrt(kappa lam_max)).  Its image is bounded by the planes through the eye
// tangent to the cone; |n . u| = sin(beta) |n| with n = (1, 0, -x') gives
// the x' range, likewise for y.  The whole grid when the cone comes within
// 0.1 degree of the plane z = 0.  Only square roots: cos/sin of beta follow
// from tan(beta).
//
// The box is then intersected with the bounding box of the exact footprint:
// alpha >= alpha_min at pixel offset d from the mean's image point iff
// |M d|^2 <= kappa h^2 with h = 1 + a3 . d > 0, i.e. inside the conic
//   d^T (M^T M - kappa a3 a3^T) d - 2 kappa a3 . d - kappa <= 0.
// When its matrix A is positive definite the conic is an ellipse with
// centre kappa A^-1 a3 and "radius" r^2 = kappa^2 a3^T A^-1 a3 + kappa, whose
// half-extents along x and y are r sqrt((A^-1)_00) and r sqrt((A^-1)_11).
// Elongated splats get much tighter boxes than the cone's.
__device__ inline bool conic_box(const TileGeo& t, double& xlo, double& xhi, double& ylo, double& yhi) {
    const double k = fmax(t.kappa, 0.0);
    const double* M = t.M;
    const double A00 = M[0] * M[0] + M[2] * M[2] - k * t.a3x * t.a3x;
    const double A01 = M[0] * M[1] + M[2] * M[3] - k * t.a3x * t.a3y;
    const double A11 = M[1] * M[1] + M[3] * M[3] - k * t.a3y * t.a3y;
    const double det = A00 * A11 - A01 * A01;
    // Positive definite and not close to singular (the box's rounding error
    // grows with A's condition number; near-parabolic footprints keep the
    // cone's box).
    if (!(A00 > 0.0 && det > 1e-9 * A00 * A11)) return false;
    const double i00 = A11 / det, i01 = -A01 / det, i11 = A00 / det;
    const double ax = i00 * t.a3x + i01 * t.a3y, ay = i01 * t.a3x + i11 * t.a3y;  // A^-1 a3
    const double r2 = k * k * (t.a3x * ax + t.a3y * ay) + k;
    const double hx = sqrt(r2 * i00), hy = sqrt(r2 * i11);
    const double cx = t.x0 + k * ax, cy = t.y0 + k * ay;
    xlo = cx - hx; xhi = cx + hx; ylo = cy - hy; yhi = cy + hy;
    return isfinite(xlo) && isfinite(xhi) && isfinite(ylo) && isfinite(yhi);
}

__device__ inline void cone_tiles(const Geo& g, const GeoView& V, int& tx0, int& tx1, int& ty0, int& ty1,
                                  float bbox[4]) {
    const double rq = sqrt(fmax(g.tg.kappa, 0.0) * g.lam_max);
    const double hyp = sqrt(rq * rq + V.f * V.f);
    const double sb = rq / hyp, cb = V.f / hyp;
    const double uz = g.u[2];
    const double st = sqrt(fmax(1.0 - uz * uz, 0.0));
    const double m = 0.5;  // pixels of margin against rounding
    double pxlo = -INFINITY, pxhi = INFINITY, pylo = -INFINITY, pyhi = INFINITY;
    // cos(theta_u + beta) > cos(89.9 deg): the cone's image is bounded.
    if (uz * cb - st * sb > 1.7453283658983088e-3) {
        const double inv_a = 1.0 / (uz * uz - sb * sb);
        const double dx = sqrt(fmax(g.u[0] * g.u[0] + uz * uz - sb * sb, 0.0));
        const double dy = sqrt(fmax(g.u[1] * g.u[1] + uz * uz - sb * sb, 0.0));
        pxlo = double(V.cx) + V.f * (g.u[0] * uz - sb * dx) * inv_a - m;
        pxhi = double(V.cx) + V.f * (g.u[0] * uz + sb * dx) * inv_a + m;
        pylo = double(V.cy) + V.f * (g.u[1] * uz - sb * dy) * inv_a - m;
        pyhi = double(V.cy) + V.f * (g.u[1] * uz + sb * dy) * inv_a + m;
    }
    double exlo, exhi, eylo, eyhi;
    if (conic_box(g.tg, exlo, exhi, eylo, eyhi)) {
        pxlo = fmax(pxlo, exlo - m);
        pxhi = fmin(pxhi, exhi + m);
        pylo = fmax(pylo, eylo - m);
        pyhi = fmin(pyhi, eyhi + m);
    }
    if (!(isfinite(pxlo) && isfinite(pxhi) && isfinite(pylo) && isfinite(pyhi))) {
        tx0 = 0; ty0 = 0; tx1 = V.ntx - 1; ty1 = V.nty - 1;
        bbox[0] = -INFINITY; bbox[1] = -INFINITY; bbox[2] = INFINITY; bbox[3] = INFINITY;
        return;
    }
    // Pixel box, rounded outwards to whole pixels.
    bbox[0] = float(floor(pxlo));
    bbox[1] = float(floor(pylo));
    bbox[2] = float(ceil(pxhi));
    bbox[3] = float(ceil(pyhi));
    if (pxhi < 0.0 || pylo > double(V.H) || pyhi < 0.0 || pxlo > double(V.W)) {
        tx0 = 1; tx1 = 0; ty0 = 1; ty1 = 0;  // empty
        return;
    }
    const double iT = 1.0 / double(V.T);
    tx0 = int(fmax(floor(pxlo * iT), 0.0));
    ty0 = int(fmax(floor(pylo * iT), 0.0));
    tx1 = int(fmin(floor(pxhi * iT), double(V.ntx - 1)));
    ty1 = int(fmin(floor(pyhi * iT), double(V.nty - 1)));
}

// Tile test of Sec. 4.2 / Eq. 4 on the whitened tangent plane for the tile
// box [bx0, bx1] x [by0, by1] (continuous pixels).  Returns true when the
// maximum alpha over the tile reaches alpha_min (D^2_min <= kappa) and then
// writes the depth t* along the unit ray through the maximum point.
__device__ inline bool tile_test(const TileGeo& g, const GeoView& V, double bx0, double by0, double bx1,
                                 double by1, double* depth) {
    if (g.x0 >= bx0 && g.x0 <= bx1 && g.y0 >= by0 && g.y0 <= by1) {
        *depth = g.r;  // maximum at the mean: t*(u) = |mu_c|
        return true;
    }
    const double cxs[4] = {bx0, bx1, bx1, bx0};
    const double cys[4] = {by0, by0, by1, by1};
    double dx[4], dy[4], h[4], zx[4], zy[4];
    bool fr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dx[k] = cxs[k] - g.x0;
        dy[k] = cys[k] - g.y0;
        h[k] = 1.0 + g.a3x * dx[k] + g.a3y * dy[k];
        fr[k] = h[k] > 0.0;
        const double ih = fr[k] ? 1.0 / h[k] : 0.0;
        zx[k] = (g.M[0] * dx[k] + g.M[1] * dy[k]) * ih;
        zy[k] = (g.M[2] * dx[k] + g.M[3] * dy[k]) * ih;
    }
    double best = INFINITY, bx = 0.0, by = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int a = k, b = (k + 1) & 3;
        double px, py, ex, ey, t;
        if (fr[a] && fr[b]) {
            px = zx[a]; py = zy[a];
            ex = zx[b] - zx[a]; ey = zy[b] - zy[a];
            const double ee = ex * ex + ey * ey;
            t = ee > 0.0 ? -(px * ex + py * ey) / ee : 0.0;
            t = fmin(fmax(t, 0.0), 1.0);
        } else if (fr[a] != fr[b]) {
            // Half-line from the visible corner towards the horizon point
            // (where h = 0) of the edge.
            const int s = fr[a] ? a : b, oth = fr[a] ? b : a;
            const double s0 = h[s] / (h[s] - h[oth]);
            const double hx = dx[s] + s0 * (dx[oth] - dx[s]);
            const double hy = dy[s] + s0 * (dy[oth] - dy[s]);
            px = zx[s]; py = zy[s];
            ex = g.M[0] * hx + g.M[1] * hy;
            ey = g.M[2] * hx + g.M[3] * hy;
            const double ee = ex * ex + ey * ey;
            t = ee > 0.0 ? fmax(-(px * ex + py * ey) / ee, 0.0) : 0.0;
        } else {
            continue;
        }
        const double qx = px + t * ex, qy = py + t * ey;
        const double D2 = qx * qx + qy * qy;
        if (D2 < best) { best = D2; bx = qx; by = qy; }
    }
    if (!(best <= g.kappa)) return false;
    // Back to the image: delta = v / (1 - a3 . v), v = M^-1 z.
    const double inv_md = 1.0 / (g.M[0] * g.M[3] - g.M[1] * g.M[2]);
    const double vx = (g.M[3] * inv_md) * bx + (-g.M[1] * inv_md) * by;
    const double vy = (-g.M[2] * inv_md) * bx + (g.M[0] * inv_md) * by;
    const double s = 1.0 / (1.0 - (g.a3x * vx + g.a3y * vy));
    const double ddx = vx * s, ddy = vy * s;
    const double w0 = g.w0[0] + ddx * g.wx[0] + ddy * g.wy[0];
    const double w1 = g.w0[1] + ddx * g.wx[1] + ddy * g.wy[1];
    const double w2 = g.w0[2] + ddx * g.wx[2] + ddy * g.wy[2];
    const double num = g.n0 + ddx * g.nx + ddy * g.ny;
    const double d0 = (g.x0 + ddx - double(V.cx)) * V.inv_f;
    const double d1 = (g.y0 + ddy - double(V.cy)) * V.inv_f;
    *depth = num / (w0 * w0 + w1 * w1 + w2 * w2) * sqrt(d0 * d0 + d1 * d1 + 1.0);
    return true;
}

__device__ inline void tile_box(const GeoView& V, int tx, int ty, double& x0, double& y0, double& x1,
                                double& y1) {
    x0 = double(tx * V.T);
    y0 = double(ty * V.T);
    x1 = double(min((tx + 1) * V.T, V.W));
    y1 = double(min((ty + 1) * V.T, V.H));
}

__device__ inline uint32_t ord_f32(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b ^ 0x80000000u);
}

}  // namespace vrs
