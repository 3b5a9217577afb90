"""Single-pass foveated rendering layout and periphery reconstruction
(Sec. 4.3, Fig. 5a).  Test infrastructure only.

The image is cut into 32x32 tiles; tiles near the fovea are split into four
16x16 subtiles rendered at full resolution, the rest are rendered with one
sample per 2x2 pixel group (half resolution).  Transitional subtiles are
rendered at full resolution, and the mean of each 2x2 group is blended with the
per-pixel value by a continuous mask.  The periphery is reconstructed by
nearest-neighbour upsampling followed by a 3x3 Gaussian blur.

Readings (the paper gives a centre rectangle of half the image with a 10 %
linear band; the fovea here is circular in angle):
* eccentricity e(p) = angle between the pixel's ray and the fovea-centre ray;
  mask w(p) = clamp((rho (1 + b) - e) / (rho b), 0, 1) with radius rho and band
  fraction b (w = 1 inside rho, falls linearly to 0 at rho (1 + b)); rho = 0
  gives w = 0 everywhere.
* A 32x32 tile is LOW if w = 0 at all of its in-image pixel centres, otherwise
  SPLIT.  A subtile of a SPLIT tile is HIGH if w = 1 at all of its in-image
  pixel centres, otherwise HYBRID.  Subtiles entirely outside the image do not
  exist.
* LOW samples sit at the centre of each aligned 2x2 group (tile-local
  (2i+1, 2j+1)); the group value is written to its in-image pixels.
* HYBRID: out(p) = w(p) c(p) + (1 - w(p)) mean of c over p's aligned 2x2 group
  (in-image pixels only); applied to RGB and alpha alike.
* Blur: K = [1 2 1]^T [1 2 1] / 16 applied to LOW pixels only, reading the
  pre-blur image (any class) with coordinates clamped to the image; RGB and
  alpha alike.  HIGH/HYBRID pixels are not blurred.
"""
import numpy as np

from . import camera as cam_mod

LOW, HIGH, HYBRID = 0, 1, 2


def mask_weights(cam, fovea, px, py):
    """w(p) at continuous pixel positions."""
    if getattr(fovea, "shape", 0) == 1:
        return rect_weights(fovea, px, py)
    d = cam_mod.ray_dirs(cam, px, py)
    dc = cam_mod.ray_dirs(cam, np.float64(fovea.center_px[0]), np.float64(fovea.center_px[1]))
    cosang = np.clip(d @ dc, -1.0, 1.0)
    e = np.arccos(cosang)
    rho = np.deg2rad(np.float64(fovea.radius_deg))
    b = np.float64(fovea.band_frac)
    if rho <= 0:
        return np.zeros_like(e)
    if b <= 0:
        return (e <= rho).astype(np.float64)
    return np.clip((rho * (1.0 + b) - e) / (rho * b), 0.0, 1.0)


def rect_weights(fovea, px, py):
    """The paper's layout (Sec. 5): a centre rectangle with half-extents
    (hx, hy) around center_px and a band of band_frac of it in which the
    weights rise linearly.  Reading: per axis
    u = clamp((h (1 + b) - |p - c|) / (h b), 0, 1), and w = min(u_x, u_y)
    (w = 1 on the rectangle, 0 outside the padded one); without a band, w is
    1 on the closed rectangle and 0 elsewhere."""
    b = np.float64(fovea.band_frac)
    out = None
    for p, c, h in ((px, fovea.center_px[0], fovea.half_px[0]), (py, fovea.center_px[1], fovea.half_px[1])):
        dist = np.abs(np.asarray(p, np.float64) - np.float64(c))
        h = np.float64(h)
        if h <= 0:
            u = np.zeros_like(dist)
        elif b <= 0:
            u = (dist <= h).astype(np.float64)
        else:
            u = np.clip((h * (1.0 + b) - dist) / (h * b), 0.0, 1.0)
        out = u if out is None else np.minimum(out, u)
    return out


def classify(cam, fovea):
    """Classes of every 32x32 tile and 16x16 subtile of a view.

    Returns (tile_split (nty32, ntx32) bool, sub_class (nty16, ntx16) int8)
    where sub_class is LOW for subtiles of LOW tiles, HIGH or HYBRID for
    subtiles of SPLIT tiles, and -1 for subtiles entirely outside the image."""
    W, H = cam.width, cam.height
    nt32x, nt32y = -(-W // 32), -(-H // 32)
    nt16x, nt16y = 2 * nt32x, 2 * nt32y
    px, py = cam_mod.pixel_centers(0, 0, W, H)
    w = mask_weights(cam, fovea, px, py).reshape(H, W)
    split = np.zeros((nt32y, nt32x), dtype=bool)
    sub = np.full((nt16y, nt16x), -1, dtype=np.int8)
    for ty in range(nt32y):
        for tx in range(nt32x):
            blk = w[ty * 32:min(ty * 32 + 32, H), tx * 32:min(tx * 32 + 32, W)]
            split[ty, tx] = bool((blk > 0).any())
            for sy in range(2):
                for sx in range(2):
                    y0, x0 = ty * 32 + sy * 16, tx * 32 + sx * 16
                    if y0 >= H or x0 >= W:
                        continue
                    sb = w[y0:min(y0 + 16, H), x0:min(x0 + 16, W)]
                    if not split[ty, tx]:
                        sub[2 * ty + sy, 2 * tx + sx] = LOW
                    else:
                        sub[2 * ty + sy, 2 * tx + sx] = HIGH if bool((sb >= 1.0).all()) else HYBRID
    return split, sub, w


def hybrid_mix(vals, w, x0, y0, W, H):
    """HYBRID output for a 16x16 subtile at (x0, y0): vals (4, h, w) per-pixel
    values of its in-image pixels, w (h, w) mask.  Group means over aligned 2x2
    groups of in-image pixels."""
    h, wd = vals.shape[1:]
    out = np.empty_like(vals)
    for gy in range(0, h, 2):
        for gx in range(0, wd, 2):
            g = vals[:, gy:gy + 2, gx:gx + 2]
            mean = g.reshape(4, -1).mean(axis=1)
            ww = w[gy:gy + 2, gx:gx + 2]
            out[:, gy:gy + 2, gx:gx + 2] = ww[None] * g + (1.0 - ww[None]) * mean[:, None, None]
    return out


BLUR = np.outer([1.0, 2.0, 1.0], [1.0, 2.0, 1.0]) / 16.0


def blur_low(pre, low_mask, ys=None, xs=None):
    """Final image: LOW pixels take the 3x3 binomial blur of ``pre`` (clamped
    at the image edge), other pixels keep ``pre``.  ``ys, xs`` optionally
    restrict the output to a pixel box (slices)."""
    C, H, W = pre.shape
    out = pre.copy()
    yy, xx = np.nonzero(low_mask)
    if len(yy) == 0:
        return out
    acc = np.zeros((C, len(yy)))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ny = np.clip(yy + dy, 0, H - 1)
            nx = np.clip(xx + dx, 0, W - 1)
            acc += BLUR[dy + 1, dx + 1] * pre[:, ny, nx]
    out[:, yy, xx] = acc
    return out
