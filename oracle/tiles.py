"""Tile binning, tile culling on tangent-plane quadrilaterals, per-tile depth,
sort keys and tile ranges.  Test infrastructure only.

Sec. 3 (tile-based rasterisation): each Gaussian is instantiated for the tiles
its splat touches, the Gaussian/tile instances are sorted, and each tile reads
only its own list.

Sec. 4.2, Fig. 4 and Eq. 4: with Optimal Projection a screen tile maps to a
convex quadrilateral on the Gaussian's tangent plane.  If the projected mean
lies inside, the point of maximum density is the mean; otherwise it lies on an
edge, and along an edge p + t d the maximum is at
    t = d^T C (mu - p) / (d^T C d),  C = Sigma_2D^-1   (Eq. 4; here mu = 0).
The instance is culled when alpha at that point is below 1/255.  The point,
projected back to the image, is where the per-tile depth is taken.

Readings (paper silent):
* t is clamped to the segment [0, 1]; the minimum is taken over all four
  edges (equal to the minimum over the at most two reachable edges -- tested).
* Tile corners whose ray is not in front of the tangent plane (u . d <= 0):
  only the part of the tile with u . d > 0 can receive the splat (alpha is 0
  elsewhere).  An edge from a visible corner P to a hidden corner maps to the
  half-line from q(P) towards the horizon direction E^T d*, where d* is the
  edge point with u . d* = 0; t is then clamped to [0, inf).  Edges with both
  corners hidden are skipped.  The tile counts as containing the mean iff the
  mean's image point lies in the tile rectangle.
* Per-tile depth: t* (depth.py) on the unit ray through the back-projected
  maximum point; when the mean lies inside the tile this is |mu_c|.
* Key: (global tile id << 32) | ord(float32(depth)), ord flips all bits of a
  negative float and only the sign bit of a non-negative one, so that unsigned
  order equals float order.  Instances are sorted by (key, Gaussian id).
"""
import numpy as np

from . import camera as cam_mod
from . import depth as depth_mod


class TileGrid:
    """Tiles of size T over a W x H view: tile (tx, ty) covers the continuous
    pixel box [tx T, min((tx+1) T, W)] x [ty T, min((ty+1) T, H)]."""

    def __init__(self, width, height, T):
        self.W, self.H, self.T = int(width), int(height), int(T)
        self.ntx = -(-self.W // self.T)
        self.nty = -(-self.H // self.T)
        self.n = self.ntx * self.nty

    def box(self, tile):
        ty, tx = divmod(int(tile), self.ntx)
        x0, y0 = tx * self.T, ty * self.T
        return x0, y0, min(x0 + self.T, self.W), min(y0 + self.T, self.H)

    def boxes(self, tiles):
        tiles = np.asarray(tiles)
        ty, tx = np.divmod(tiles, self.ntx)
        x0 = tx * self.T
        y0 = ty * self.T
        return (x0.astype(np.float64), y0.astype(np.float64),
                np.minimum(x0 + self.T, self.W).astype(np.float64),
                np.minimum(y0 + self.T, self.H).astype(np.float64))


def cone_tile_bounds(u, lam_max, kappa, f, cam, grid, margin_px=0.5):
    """Accelerator only (the instance set is defined by ``quad_test`` over all
    tiles).  Every tile whose max alpha reaches alpha_min meets the cone of
    half-angle beta = atan(sqrt(kappa * lam_max) / f) around u: the footprint
    on the tangent plane {q^T C q <= kappa} lies in the disc of radius
    sqrt(kappa lam_max).  The image of that cone is bounded by the planes
    through the eye tangent to it; solving |n . u| = sin(beta) |n| for
    n = (1, 0, -x') gives the x' range, likewise for y.  If the cone reaches
    the plane z = 0 the whole view is returned.

    Returns integer tile-index ranges (tx0, tx1, ty0, ty1), inclusive, or a
    full-view range."""
    beta = np.arctan(np.sqrt(kappa * lam_max) / f)
    sb = np.sin(beta)
    theta_u = np.arccos(np.clip(u[:, 2], -1, 1))
    full = theta_u + beta >= np.deg2rad(89.9)

    def axis_range(ua):
        a = u[:, 2] ** 2 - sb ** 2
        disc = np.maximum(ua ** 2 + u[:, 2] ** 2 - sb ** 2, 0.0)
        a_safe = np.where(full, 1.0, a)
        lo = (ua * u[:, 2] - sb * np.sqrt(disc)) / a_safe
        hi = (ua * u[:, 2] + sb * np.sqrt(disc)) / a_safe
        return lo, hi

    xlo, xhi = axis_range(u[:, 0])
    ylo, yhi = axis_range(u[:, 1])
    pxlo = np.float64(cam.cx) + f * xlo - margin_px
    pxhi = np.float64(cam.cx) + f * xhi + margin_px
    pylo = np.float64(cam.cy) + f * ylo - margin_px
    pyhi = np.float64(cam.cy) + f * yhi + margin_px
    T = grid.T
    tx0 = np.clip(np.floor(pxlo / T), 0, grid.ntx - 1)
    tx1 = np.clip(np.floor(pxhi / T), -1, grid.ntx - 1)
    ty0 = np.clip(np.floor(pylo / T), 0, grid.nty - 1)
    ty1 = np.clip(np.floor(pyhi / T), -1, grid.nty - 1)
    # Boxes that end left of / above the view are empty (tx1 < tx0).
    tx1 = np.where(pxhi < 0, -1, tx1)
    ty1 = np.where(pyhi < 0, -1, ty1)
    tx0 = np.where(pxlo > grid.W, grid.ntx, tx0)
    ty0 = np.where(pylo > grid.H, grid.nty, ty0)
    tx0 = np.where(full, 0, tx0)
    ty0 = np.where(full, 0, ty0)
    tx1 = np.where(full, grid.ntx - 1, tx1)
    ty1 = np.where(full, grid.nty - 1, ty1)
    return tx0.astype(np.int64), tx1.astype(np.int64), ty0.astype(np.int64), ty1.astype(np.int64)


def quad_test(cam, f, u, E, C, x0, y0, bx0, by0, bx1, by1):
    """Eq. 4 on the tangent plane for K Gaussian/tile pairs (arrays of length K).

    u (K,3), E (K,3,2), C (K,2,2): per-pair Gaussian data; (x0, y0): image
    point of the mean; (bx0, by0, bx1, by1): tile box in continuous pixels.
    Returns dict(D2min (K,), qhat (K,2), inside (K,), Pq (K,4,2), front
    (K,4), edge_D2 (K,4)): qhat is the tangent-plane point of maximum density,
    Pq the corner images (NaN/inf where hidden), edge_D2 each edge's clamped
    minimum (inf for hidden edges).
    """
    K = u.shape[0]
    cx = [bx0, bx1, bx1, bx0]
    cy = [by0, by0, by1, by1]
    d = np.stack([cam_mod.ray_dirs(cam, cx[k], cy[k], normalize=False) for k in range(4)], axis=1)  # (K,4,3)
    h = np.einsum("kci,ki->kc", d, u)                                  # (K,4)
    front = h > 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        Pq = f * np.einsum("kci,kij->kcj", d, E) / h[..., None]        # (K,4,2)

    inside_img = (x0 >= bx0) & (x0 <= bx1) & (y0 >= by0) & (y0 <= by1)
    # Paper's formulation when the whole quad is on the plane: containment of
    # the projected mean (the origin) in the convex quadrilateral.
    all_front = front.all(axis=1)
    cross = np.empty((K, 4))
    for k in range(4):
        a = Pq[:, k]
        b = Pq[:, (k + 1) % 4]
        cross[:, k] = (b[:, 0] - a[:, 0]) * (-a[:, 1]) - (b[:, 1] - a[:, 1]) * (-a[:, 0])
    inside_quad = (cross >= 0).all(axis=1) | (cross <= 0).all(axis=1)
    inside = np.where(all_front, inside_quad, inside_img)

    best = np.full(K, np.inf)
    qbest = np.zeros((K, 2))
    edge_D2 = np.full((K, 4), np.inf)
    for k in range(4):
        ka, kb = k, (k + 1) % 4
        fa, fb = front[:, ka], front[:, kb]
        pa, pb = Pq[:, ka], Pq[:, kb]
        # Segment case.
        seg = fa & fb
        # Half-line case: start at the visible corner, head to the horizon.
        s0 = np.where(fa & ~fb, h[:, ka] / (h[:, ka] - h[:, kb]),
                      np.where(~fa & fb, h[:, kb] / (h[:, kb] - h[:, ka]), 0.0))
        start = np.where((fa & ~fb)[:, None], pa, pb)
        dstart = np.where((fa & ~fb)[:, None], d[:, ka], d[:, kb])
        dother = np.where((fa & ~fb)[:, None], d[:, kb], d[:, ka])
        dstar = dstart + s0[:, None] * (dother - dstart)
        vdir = np.einsum("ki,kij->kj", dstar, E)
        half = fa ^ fb
        e = np.where(seg[:, None], pb - pa, vdir)
        p = np.where(seg[:, None], pa, start)
        with np.errstate(divide="ignore", invalid="ignore"):
            Ce = np.einsum("kij,kj->ki", C, e)
            t = -np.einsum("ki,ki->k", Ce, p) / np.einsum("ki,ki->k", Ce, e)
        t_cl = np.where(seg, np.clip(t, 0.0, 1.0), np.maximum(t, 0.0))
        xq = p + t_cl[:, None] * e
        D2 = np.einsum("ki,kij,kj->k", xq, C, xq)
        valid = seg | half
        D2 = np.where(valid, D2, np.inf)
        edge_D2[:, k] = D2
        better = D2 < best
        best = np.where(better, D2, best)
        qbest = np.where(better[:, None], xq, qbest)
    best = np.where(inside, 0.0, best)
    qbest = np.where(inside[:, None], 0.0, qbest)
    return dict(D2min=best, qhat=qbest, inside=inside, Pq=Pq, front=front,
                edge_D2=edge_D2)


def tile_depth(u, E, f, qhat, mu_c, B):
    """Per-instance depth: t* on the unit ray through u + (q1 e1 + q2 e2)/f,
    the eye ray whose tangent-plane coordinate is qhat."""
    dd = u + np.einsum("kij,kj->ki", E, qhat) / f
    dd = dd / np.linalg.norm(dd, axis=1, keepdims=True)
    Bd = np.einsum("kij,kj->ki", B, dd)
    return np.einsum("ki,ki->k", Bd, mu_c) / np.einsum("ki,ki->k", Bd, dd)


def ord_f32(depth):
    """Order-preserving map of float32 bit patterns to uint32."""
    b = np.asarray(depth, np.float32).view(np.uint32).astype(np.uint64)
    neg = (b >> np.uint64(31)) & np.uint64(1)
    return np.where(neg == 1, (~b) & np.uint64(0xFFFFFFFF), b ^ np.uint64(0x80000000)).astype(np.uint64)


def make_keys(global_tile, depth):
    return (np.asarray(global_tile, np.uint64) << np.uint64(32)) | ord_f32(depth)


def sort_instances(keys, gids):
    """Ascending order of (key, gid)."""
    order = np.lexsort((np.asarray(gids), np.asarray(keys)))
    return np.asarray(keys)[order], np.asarray(gids)[order]


def tile_ranges(sorted_keys, n_tiles):
    """ranges[t] = [first, last+1) of tile t in the sorted keys; empty tiles
    are [0, 0)."""
    r = np.zeros((n_tiles, 2), dtype=np.uint32)
    if len(sorted_keys) == 0:
        return r
    tiles = (np.asarray(sorted_keys, np.uint64) >> np.uint64(32)).astype(np.int64)
    starts = np.flatnonzero(np.r_[True, tiles[1:] != tiles[:-1]])
    ends = np.r_[starts[1:], len(tiles)]
    r[tiles[starts], 0] = starts
    r[tiles[starts], 1] = ends
    return r
