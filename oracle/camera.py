"""Pinhole cameras (Sec. 5 renders per-eye images at a fixed resolution; App. D
changes focal length and resolution together).  Test infrastructure only.

Readings (the paper does not state them): camera axes x right, y down,
z forward; ``world_to_cam`` = [R | t] with x_cam = R x + t; horizontal field of
view; square pixels, so f_x = f_y = (W/2) / tan(fov_x/2); pixel (i, j) is
sampled at its centre (i + 1/2, j + 1/2).
"""
import numpy as np


def rt(cam):
    m = np.asarray(cam.world_to_cam, np.float64)
    return m[:, :3], m[:, 3]


def focal(cam):
    """f = (W/2) / tan(fov_x / 2) in pixels."""
    return (cam.width / 2.0) / np.tan(np.deg2rad(np.float64(cam.fov_x_deg)) / 2.0)


def eye_center(cam):
    """o = -R^T t: the camera centre in world coordinates."""
    R, t = rt(cam)
    return -R.T @ t


def to_camera(cam, x_world):
    """x_cam = R x + t for points (N, 3)."""
    R, t = rt(cam)
    return np.asarray(x_world, np.float64) @ R.T + t


def ray_dirs(cam, px, py, normalize=True):
    """Camera-frame direction through continuous pixel position (px, py):
    ((px - cx)/f, (py - cy)/f, 1), optionally normalised."""
    f = focal(cam)
    px = np.asarray(px, np.float64)
    py = np.asarray(py, np.float64)
    d = np.stack([(px - np.float64(cam.cx)) / f, (py - np.float64(cam.cy)) / f,
                  np.ones(np.broadcast(px, py).shape)], axis=-1)
    if normalize:
        d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    return d


def pixel_centers(x0, y0, x1, y1):
    """Pixel-centre coordinates of the integer pixel box [x0,x1) x [y0,y1),
    row-major; returns (px, py) flattened."""
    ys, xs = np.mgrid[y0:y1, x0:x1]
    return xs.ravel() + 0.5, ys.ravel() + 0.5
