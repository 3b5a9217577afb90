// FP64 per-Gaussian set-up geometry shared by the preprocessing (K1) and
// instantiation (K3) kernels.  Everything here runs once per Gaussian and
// view (or per Gaussian and candidate tile), so double precision costs little
// next to the memory traffic of those kernels and keeps the discrete
// decisions (near cull, tile test, key depth) within a few ulp of exact.
#pragma once

#include "vrs_internal.h"

namespace vrs {

struct Geo {
    double muc[3];   // camera-frame mean
    double r;        // |mu_c|
    double u[3];     // mu_c / r
    double M[4];     // whitened tangent coords: z = M delta / h, |z|^2 = D^2
    double Minv[4];
    double a3x, a3y; // h = 1 + a3 . delta
    double x0, y0;   // image point of the mean (pixels)
    double sigma;    // opacity
    double kappa;    // D^2 threshold: 2 ln(sigma / alpha_min)
    double lam_max;  // largest eigenvalue of Sigma_2D (px^2)
    double W3[9];    // S^-1 R_c^T (row-major): d^T Sigma_c^-1 d = |W3 d|^2
    double m[3];     // W3 mu_c
};

struct GaussLocal {
    double mu[3];
    double R[9];   // rotation of the Gaussian (world)
    double s[3];   // standard deviations
    double sigma;
    bool ok;
};

__device__ inline GaussLocal load_gaussian(const GaussPtrs& g, int i) {
    GaussLocal L;
    const int n = g.n;
    double q[4];
    for (int c = 0; c < 3; ++c) {
        L.mu[c] = double(g.means[c * n + i]);
        L.s[c] = exp(double(g.log_scales[c * n + i]));
    }
    for (int c = 0; c < 4; ++c) q[c] = double(g.quats[c * n + i]);
    const double o = double(g.opac[i]);
    L.sigma = 1.0 / (1.0 + exp(-o));
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    bool ok = qn > 0.0 && isfinite(qn) && isfinite(L.sigma);
    for (int c = 0; c < 3; ++c) ok = ok && isfinite(L.mu[c]) && isfinite(L.s[c]) && L.s[c] > 0.0;
    L.ok = ok;
    const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    // Rotation matrix of a unit quaternion (Hamilton convention).
    L.R[0] = 1.0 - 2.0 * (y * y + z * z);
    L.R[1] = 2.0 * (x * y - w * z);
    L.R[2] = 2.0 * (x * z + w * y);
    L.R[3] = 2.0 * (x * y + w * z);
    L.R[4] = 1.0 - 2.0 * (x * x + z * z);
    L.R[5] = 2.0 * (y * z - w * x);
    L.R[6] = 2.0 * (x * z - w * y);
    L.R[7] = 2.0 * (y * z + w * x);
    L.R[8] = 1.0 - 2.0 * (x * x + y * y);
    return L;
}

// Optimal Projection set-up of one Gaussian for one view.  Returns false when
// the Gaussian is culled from the view (camera z <= z_near, opacity below
// alpha_min, non-finite input).
__device__ inline bool make_geo(const GaussLocal& G, const GeoView& V, const Knobs& kn, Geo& o) {
    if (!G.ok || !(G.sigma >= double(kn.alpha_min))) return false;
    double Rv[9];
    for (int k = 0; k < 9; ++k) Rv[k] = double(V.R[k]);
    for (int r = 0; r < 3; ++r)
        o.muc[r] = Rv[3 * r] * G.mu[0] + Rv[3 * r + 1] * G.mu[1] + Rv[3 * r + 2] * G.mu[2] + double(V.t[r]);
    if (!(o.muc[2] > double(kn.z_near))) return false;
    const double f = V.f;
    // Camera-frame rotation of the Gaussian.
    double Rc[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            Rc[3 * r + c] = Rv[3 * r] * G.R[c] + Rv[3 * r + 1] * G.R[3 + c] + Rv[3 * r + 2] * G.R[6 + c];
    o.r = sqrt(o.muc[0] * o.muc[0] + o.muc[1] * o.muc[1] + o.muc[2] * o.muc[2]);
    for (int c = 0; c < 3; ++c) o.u[c] = o.muc[c] / o.r;
    const double ux = o.u[0], uy = o.u[1], uz = o.u[2];
    // Tangent-plane basis: images of the camera x/y axes under the minimal
    // rotation taking +z to u (any orthonormal basis gives the same splat).
    const double k = 1.0 / (1.0 + uz);
    const double e1[3] = {1.0 - ux * ux * k, -ux * uy * k, -ux};
    const double e2[3] = {-ux * uy * k, 1.0 - uy * uy * k, -uy};
    // G2 = E^T R_c S (2x3); Sigma_2D = (f/r)^2 G2 G2^T + dilation I.
    double g0[3], g1[3];
    for (int c = 0; c < 3; ++c) {
        const double col0 = Rc[c], col1 = Rc[3 + c], col2 = Rc[6 + c];
        g0[c] = (e1[0] * col0 + e1[1] * col1 + e1[2] * col2) * G.s[c];
        g1[c] = (e2[0] * col0 + e2[1] * col1 + e2[2] * col2) * G.s[c];
    }
    const double sc = (f / o.r) * (f / o.r);
    const double dil = double(kn.dilation);
    const double sa = sc * (g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2]) + dil;
    const double sb = sc * (g0[0] * g1[0] + g0[1] * g1[1] + g0[2] * g1[2]);
    const double scc = sc * (g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]) + dil;
    const double det = sa * scc - sb * sb;
    if (!(det > 0.0)) return false;
    // Conic C = Sigma_2D^-1 and its factor C = L^T L, L upper triangular.
    const double c00 = scc / det, c01 = -sb / det, c11 = sa / det;
    const double l00 = sqrt(c00);
    const double l01 = c01 / l00;
    const double l11 = sqrt(fmax(c11 - l01 * l01, 0.0));
    // Tangent coordinate of the pixel offset delta from the mean's image
    // point: q = u_z A delta / (1 + a3 . delta) with A the xy-block of E^T.
    const double A00 = e1[0], A01 = e1[1], A10 = e2[0], A11 = e2[1];
    o.M[0] = uz * (l00 * A00 + l01 * A10);
    o.M[1] = uz * (l00 * A01 + l01 * A11);
    o.M[2] = uz * (l11 * A10);
    o.M[3] = uz * (l11 * A11);
    const double md = o.M[0] * o.M[3] - o.M[1] * o.M[2];
    o.Minv[0] = o.M[3] / md;
    o.Minv[1] = -o.M[1] / md;
    o.Minv[2] = -o.M[2] / md;
    o.Minv[3] = o.M[0] / md;
    o.a3x = uz * ux / f;
    o.a3y = uz * uy / f;
    o.x0 = double(V.cx) + f * o.muc[0] / o.muc[2];
    o.y0 = double(V.cy) + f * o.muc[1] / o.muc[2];
    o.sigma = G.sigma;
    o.kappa = 2.0 * log(G.sigma / double(kn.alpha_min));
    const double tr = 0.5 * (sa + scc);
    o.lam_max = tr + sqrt(0.25 * (sa - scc) * (sa - scc) + sb * sb);
    // Depth along a ray: t*(d) = d^T B mu / d^T B d with B = Sigma_c^-1 =
    // W3^T W3, W3 = S^-1 R_c^T.
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) o.W3[3 * r + c] = Rc[3 * c + r] / G.s[r];
    for (int r = 0; r < 3; ++r)
        o.m[r] = o.W3[3 * r] * o.muc[0] + o.W3[3 * r + 1] * o.muc[1] + o.W3[3 * r + 2] * o.muc[2];
    return true;
}

// Inclusive tile-index ranges that can hold instances of the Gaussian: the
// image of the cone of half-angle beta = atan(sqrt(kappa lam_max) / f) around
// u, which contains every ray where alpha reaches alpha_min.  The whole grid
// when the cone reaches the plane z = 0.
__device__ inline void cone_tiles(const Geo& g, const GeoView& V, int& tx0, int& tx1, int& ty0,
                                  int& ty1) {
    const double beta = atan(sqrt(fmax(g.kappa, 0.0) * g.lam_max) / V.f);
    const double theta = acos(fmin(fmax(g.u[2], -1.0), 1.0));
    if (theta + beta >= 89.9 * (M_PI / 180.0)) {
        tx0 = 0; ty0 = 0; tx1 = V.ntx - 1; ty1 = V.nty - 1;
        return;
    }
    const double sb = sin(beta);
    const double uz = g.u[2];
    const double a = uz * uz - sb * sb;
    const double dx = sqrt(fmax(g.u[0] * g.u[0] + uz * uz - sb * sb, 0.0));
    const double dy = sqrt(fmax(g.u[1] * g.u[1] + uz * uz - sb * sb, 0.0));
    const double xlo = (g.u[0] * uz - sb * dx) / a, xhi = (g.u[0] * uz + sb * dx) / a;
    const double ylo = (g.u[1] * uz - sb * dy) / a, yhi = (g.u[1] * uz + sb * dy) / a;
    const double m = 0.5;  // pixels of margin against rounding
    const double pxlo = double(V.cx) + V.f * xlo - m, pxhi = double(V.cx) + V.f * xhi + m;
    const double pylo = double(V.cy) + V.f * ylo - m, pyhi = double(V.cy) + V.f * yhi + m;
    if (pxhi < 0.0 || pylo > double(V.H) || pyhi < 0.0 || pxlo > double(V.W)) {
        tx0 = 1; tx1 = 0; ty0 = 1; ty1 = 0;  // empty
        return;
    }
    const double T = double(V.T);
    tx0 = int(fmax(floor(pxlo / T), 0.0));
    ty0 = int(fmax(floor(pylo / T), 0.0));
    tx1 = int(fmin(floor(pxhi / T), double(V.ntx - 1)));
    ty1 = int(fmin(floor(pyhi / T), double(V.nty - 1)));
}

// Tile test of Sec. 4.2 / Eq. 4 on the whitened tangent plane for the tile
// box [bx0, bx1] x [by0, by1] (continuous pixels).  Returns true when the
// maximum alpha over the tile reaches alpha_min (D^2_min <= kappa) and then
// writes the depth t* along the unit ray through the maximum point.
__device__ inline bool tile_test(const Geo& g, const GeoView& V, double bx0, double by0, double bx1,
                                 double by1, double* depth) {
    if (g.x0 >= bx0 && g.x0 <= bx1 && g.y0 >= by0 && g.y0 <= by1) {
        if (depth) *depth = g.r;  // maximum at the mean: t*(u) = |mu_c|
        return true;
    }
    const double cxs[4] = {bx0, bx1, bx1, bx0};
    const double cys[4] = {by0, by0, by1, by1};
    double dx[4], dy[4], h[4], zx[4], zy[4];
    bool fr[4];
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
            const int s = fr[a] ? a : b, oth = fr[a] ? b : a;
            const double s0 = h[s] / (h[s] - h[oth]);
            const double hx = dx[s] + s0 * (dx[oth] - dx[s]);
            const double hy = dy[s] + s0 * (dy[oth] - dy[s]);
            px = zx[s]; py = zy[s];
            ex = g.M[0] * hx + g.M[1] * hy;  // direction towards the horizon
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
    if (depth) {
        // Back to the image: delta = v / (1 - a3 . v), v = M^-1 z.
        const double vx = g.Minv[0] * bx + g.Minv[1] * by;
        const double vy = g.Minv[2] * bx + g.Minv[3] * by;
        const double den = 1.0 - (g.a3x * vx + g.a3y * vy);
        const double ddx = vx / den, ddy = vy / den;
        const double d0 = (g.x0 + ddx - double(V.cx)) / V.f;
        const double d1 = (g.y0 + ddy - double(V.cy)) / V.f;
        const double w0 = g.W3[0] * d0 + g.W3[1] * d1 + g.W3[2];
        const double w1 = g.W3[3] * d0 + g.W3[4] * d1 + g.W3[5];
        const double w2 = g.W3[6] * d0 + g.W3[7] * d1 + g.W3[8];
        const double num = w0 * g.m[0] + w1 * g.m[1] + w2 * g.m[2];
        const double dd = w0 * w0 + w1 * w1 + w2 * w2;
        *depth = num / dd * sqrt(d0 * d0 + d1 * d1 + 1.0);
    }
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
