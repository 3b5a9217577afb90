"""Pins for the oracle's two-pass foveated baseline (App. A): the bilinear
upsampling against a library routine and against affine functions, the
limits of the centre region, and the periphery pass against the single-pass
renderer's LOW samples."""
import numpy as np
from scipy import ndimage

import oracle
import synth
from oracle import camera as ocam
from oracle import fovea as ofov
from oracle import twopass


def test_bilinear_up_equals_library_linear_interpolation():
    rng = np.random.default_rng(0)
    for W, H in [(64, 48), (33, 17), (2, 2), (1, 5)]:
        low = rng.uniform(0, 1, (4, (H + 1) // 2, (W + 1) // 2))
        up = twopass.bilinear_up(low, W, H)
        sy = (np.arange(H) + 0.5) / 2 - 0.5
        sx = (np.arange(W) + 0.5) / 2 - 0.5
        YY, XX = np.meshgrid(sy, sx, indexing="ij")
        for c in range(4):
            ref = ndimage.map_coordinates(low[c], [YY.ravel(), XX.ravel()], order=1, mode="nearest")
            np.testing.assert_allclose(up[c].ravel(), ref, atol=1e-12)


def test_bilinear_up_reproduces_affine_functions():
    """Low-resolution samples of a + b x + c y taken at full-resolution
    points (2i+1, 2j+1) upsample to the same function at every pixel centre
    between them."""
    W, H = 40, 30
    i = np.arange(W // 2)
    j = np.arange(H // 2)
    f = lambda x, y: 0.3 + 0.01 * x - 0.02 * y
    low = np.stack([f(2 * i[None, :] + 1.0, 2 * j[:, None] + 1.0)] * 4)
    up = twopass.bilinear_up(low, W, H)
    ys, xs = np.mgrid[1:H - 1, 1:W - 1]
    np.testing.assert_allclose(up[0, 1:H - 1, 1:W - 1], f(xs + 0.5, ys + 0.5), atol=1e-12)


def test_centre_box_holds_every_pixel_of_the_mask():
    cam = synth.camera_translate((0, 0, -3), 100.0, 203, 141)
    fov = synth.Fovea(True, (71.3, 88.9), 14.0, 0.25)
    box = twopass.centre_box(cam, fov)
    x0, y0, x1, y1 = box
    assert x0 % 32 == 0 and y0 % 32 == 0
    px, py = ocam.pixel_centers(0, 0, cam.width, cam.height)
    w = ofov.mask_weights(cam, fov, px, py).reshape(cam.height, cam.width)
    ys, xs = np.nonzero(w > 0)
    assert xs.min() >= x0 and xs.max() < x1 and ys.min() >= y0 and ys.max() < y1
    # The centre camera sees the box's pixels along the same rays.
    cc = twopass.centre_camera(cam, box)
    d_full = ocam.ray_dirs(cam, x0 + 3.5, y0 + 7.5)
    d_sub = ocam.ray_dirs(cc, 3.5, 7.5)
    np.testing.assert_allclose(d_full, d_sub, atol=1e-9)


def test_everything_central_equals_the_plain_render():
    """A fovea covering the whole image: the centre pass is the whole view
    (same camera) with w = 1 everywhere, so the result is the plain 16x16
    render."""
    scene = synth.cluster_scene(3, 3000, log_scale=(-4.0, 0.5))
    cam = synth.camera_translate((0, 0, -3), 90.0, 96, 64)
    fov = synth.Fovea(True, (48.0, 32.0), 80.0, 0.1)
    params = synth.default_params(tile=32, window=8)
    res = twopass.render(scene, [cam], [fov], params)
    assert res["boxes"][0] == (0, 0, 96, 64)
    plain = oracle.render(scene, [cam], synth.fovea_off(), params.replace(tile=16))
    np.testing.assert_allclose(res["images"][0], plain["images"][0], atol=1e-12)


def test_periphery_pass_equals_single_pass_low_samples():
    """The half-resolution periphery pass evaluates the same splats on the
    same rays as the single-pass renderer's LOW samples (fovea of radius 0:
    every tile LOW), tile for tile, so the two agree exactly."""
    scene = synth.cluster_scene(4, 3000, log_scale=(-4.0, 0.5))
    cam = synth.camera_translate((0, 0, -3), 90.0, 128, 96)
    params = synth.default_params(tile=32, window=8)
    fov0 = synth.Fovea(True, (64.0, 48.0), 0.0, 0.1)
    single = oracle.render(scene, [cam], [fov0], params)
    res = twopass.render(scene, [cam], [fov0], params)
    assert res["boxes"][0] is None
    low = res["low"]["images"][0]
    np.testing.assert_allclose(low, single["pre_images"][0][:, ::2, ::2], atol=1e-12)
    np.testing.assert_allclose(res["images"][0], twopass.bilinear_up(low, 128, 96), atol=1e-15)
