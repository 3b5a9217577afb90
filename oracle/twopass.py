"""Two-pass foveated rendering, the comparison baseline of App. A.  Test
infrastructure only.

App. A: a first pass renders the centre region at full resolution through a
tight projection frustum; a second pass renders the periphery at a lower
resolution; the low-resolution image is upsampled bilinearly, and the two are
blended by the continuous foveation mask in the transition band, which is
therefore rendered twice.  The centre and band are the ones of the
single-pass renderer (Sec. 4.3).

Readings (the appendix gives no formulas):
* Centre pass: a camera with the same pose and focal length whose image is
  the bounding box of the 32x32 tiles that hold a pixel centre with w > 0
  (the SPLIT tiles of the single-pass layout), principal point shifted by the
  box origin.  Plain 16x16 tiles.
* Periphery pass: the whole view at half resolution, ceil(W/2) x ceil(H/2),
  focal length f/2, principal point halved, dilation delta/4; low-resolution
  pixel (i, j) then evaluates the splats on exactly the ray of the
  single-pass LOW sample at full-resolution (2i+1, 2j+1).  Plain 16x16 tiles
  (the full-resolution 32x32 tiles).
* Upsampling: bilinear between low-resolution pixel centres, which sit at
  full-resolution coordinates 2i+1; a full-resolution pixel centre x + 1/2
  lies at low-resolution coordinate (x + 1/2)/2 - 1/2; indices clamped at the
  image edge.
* Blend: out = w c_centre + (1 - w) up(low), RGB and alpha alike, with w the
  mask of oracle.fovea (zero outside the centre box).
"""
import math

import numpy as np

from . import camera as cam_mod
from . import fovea as fov_mod


def centre_box(cam, fovea):
    """Pixel box (x0, y0, x1, y1) of the 32x32 tiles holding a pixel centre
    with w > 0; None if there is none."""
    split, _, _ = fov_mod.classify(cam, fovea)
    ty, tx = np.nonzero(split)
    if len(tx) == 0:
        return None
    return (int(tx.min()) * 32, int(ty.min()) * 32,
            min(int(tx.max() + 1) * 32, cam.width), min(int(ty.max() + 1) * 32, cam.height))


def _with(cam, fov_x_deg, cx, cy, width, height):
    return type(cam)(world_to_cam=cam.world_to_cam, fov_x_deg=fov_x_deg, cx=cx, cy=cy,
                     width=width, height=height)


def _f32(x):
    return float(np.float32(x))


def centre_camera(cam, box):
    """The tight-frustum camera of the centre pass: same pose and focal
    length, image = the box.  The horizontal FoV is re-derived from the box
    width (cameras are given by FoV and width) and rounded to float32."""
    x0, y0, x1, y1 = box
    f = cam_mod.focal(cam)
    fov = math.degrees(2.0 * math.atan((x1 - x0) / 2.0 / f))
    return _with(cam, _f32(fov), _f32(np.float64(cam.cx) - x0), _f32(np.float64(cam.cy) - y0), x1 - x0, y1 - y0)


def low_camera(cam):
    """The half-resolution camera of the periphery pass: focal length f/2."""
    wl, hl = (cam.width + 1) // 2, (cam.height + 1) // 2
    f = cam_mod.focal(cam) / 2.0
    fov = math.degrees(2.0 * math.atan(wl / 2.0 / f))
    return _with(cam, _f32(fov), _f32(np.float64(cam.cx) / 2.0), _f32(np.float64(cam.cy) / 2.0), wl, hl)


def bilinear_up(low, width, height):
    """Full-resolution image (C, height, width) from the half-resolution
    image low (C, hl, wl) by bilinear interpolation between low-resolution
    pixel centres (full-resolution coordinate 2i+1), clamped at the edge."""
    C, hl, wl = low.shape
    sx = (np.arange(width) + 0.5) / 2.0 - 0.5
    sy = (np.arange(height) + 0.5) / 2.0 - 0.5
    ix = np.floor(sx).astype(np.int64)
    iy = np.floor(sy).astype(np.int64)
    fx = sx - ix
    fy = sy - iy
    x0 = np.clip(ix, 0, wl - 1)
    x1 = np.clip(ix + 1, 0, wl - 1)
    y0 = np.clip(iy, 0, hl - 1)
    y1 = np.clip(iy + 1, 0, hl - 1)
    top = low[:, y0][:, :, x0] * (1.0 - fx)[None, None] + low[:, y0][:, :, x1] * fx[None, None]
    bot = low[:, y1][:, :, x0] * (1.0 - fx)[None, None] + low[:, y1][:, :, x1] * fx[None, None]
    return top * (1.0 - fy)[None, :, None] + bot * fy[None, :, None]


def compose(cam, fovea, centre_img, box, low_img):
    """Blend of the two passes (see the module readings)."""
    W, H = cam.width, cam.height
    out = bilinear_up(low_img, W, H)
    if box is not None:
        x0, y0, x1, y1 = box
        px, py = cam_mod.pixel_centers(x0, y0, x1, y1)
        w = fov_mod.mask_weights(cam, fovea, px, py).reshape(y1 - y0, x1 - x0)
        out[:, y0:y1, x0:x1] = w[None] * centre_img + (1.0 - w[None]) * out[:, y0:y1, x0:x1]
    return out


def render(scene, cams, foveas, params, opts=None):
    """Both passes with the oracle renderer, then the blend.  Returns the
    final images, the passes' own results and the centre boxes."""
    from .render import render as render_views
    from synth import fovea_off
    boxes = [centre_box(c, f) for c, f in zip(cams, foveas)]
    ccams = [centre_camera(c, b) for c, b in zip(cams, boxes) if b is not None]
    lcams = [low_camera(c) for c in cams]
    p1 = params.replace(tile=16)
    p2 = params.replace(tile=16, dilation=float(np.float32(params.dilation / 4.0)))
    centre = render_views(scene, ccams, [fovea_off()] * len(ccams), p1, opts) if ccams else None
    low = render_views(scene, lcams, [fovea_off()] * len(lcams), p2, opts)
    images = []
    k = 0
    for v, (cam, fov) in enumerate(zip(cams, foveas)):
        cimg = None
        if boxes[v] is not None:
            cimg = centre["images"][k]
            k += 1
        images.append(compose(cam, fov, cimg, boxes[v], low["images"][v]))
    return dict(images=images, boxes=boxes, centre=centre, low=low, centre_cams=ccams, low_cams=lcams)
