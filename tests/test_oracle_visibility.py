"""Pins for visibility culling (Sec. 4.3, Fig. 5b) and the paper's
rectangular foveation layout (Sec. 5): tile bitfield and summed-area counts
against brute force, the synthetic lens mask's tile split, masked renders
against unmasked ones, and the rectangle's blending weights."""
import numpy as np

import oracle
import synth
from oracle import camera as ocam
from oracle import fovea as ofov
from oracle import visibility as ovis


def test_tile_bits_and_summed_area_counts_equal_brute_force():
    rng = np.random.default_rng(0)
    for H, W, T in [(70, 100, 16), (64, 64, 32), (33, 17, 16)]:
        mask = (rng.random((H, W)) < 0.02).astype(np.uint8)
        bits = ovis.tile_bits(mask, T)
        nty, ntx = bits.shape
        for ty in range(nty):
            for tx in range(ntx):
                assert bits[ty, tx] == bool(mask[ty * T:(ty + 1) * T, tx * T:(tx + 1) * T].any())
        S = ovis.summed_area(bits)
        for _ in range(300):
            tx0, tx1 = sorted(rng.integers(0, ntx, 2))
            ty0, ty1 = sorted(rng.integers(0, nty, 2))
            assert ovis.rect_count(S, tx0, tx1, ty0, ty1) == bits[ty0:ty1 + 1, tx0:tx1 + 1].sum()
        assert ovis.rect_count(S, 3, 2, 0, 0) == 0  # empty rectangle


def test_lens_mask_tile_split_at_the_papers_resolution():
    """2064x2272 per eye in 32x32 tiles: 4615 tiles, of which the synthetic
    lens mask leaves 508 invisible (the paper's headset: 507, Sec. 5.4)."""
    bits = ovis.tile_bits(synth.lens_mask(2064, 2272), 32)
    assert bits.size == 4615
    assert int((~bits).sum()) == 508


def test_masked_plain_render_is_the_unmasked_render_with_invisible_tiles_at_background():
    scene = synth.cluster_scene(2, 4000, log_scale=(-4.0, 0.5))
    cam = synth.camera_translate((0, 0, -3), 90.0, 160, 128)
    params = synth.default_params(tile=16, window=8, background=(0.1, 0.2, 0.3))
    mask = synth.lens_mask(160, 128, (0.8, 0.8))
    full = oracle.render(scene, [cam], synth.fovea_off(), params)
    res = oracle.render(scene, [cam], synth.fovea_off(), params, masks=[mask])
    bits = ovis.tile_bits(mask, 16)
    assert (~bits).sum() > 10
    vis_px = np.repeat(np.repeat(bits, 16, 0), 16, 1)[:128, :160]
    np.testing.assert_allclose(res["images"][0][:, vis_px], full["images"][0][:, vis_px], atol=1e-12)
    bg = np.array([0.1, 0.2, 0.3, 0.0])
    assert np.all(res["images"][0][:, ~vis_px] == np.float32(bg)[:, None].astype(np.float64))
    # Fewer instances, none in an invisible tile.
    assert 0 < res["stats"]["n_inst"] < full["stats"]["n_inst"]
    tiles = (res["keys"] >> np.uint64(32)).astype(np.int64)
    assert bits.ravel()[tiles].all()


def test_masked_foveated_pre_image_keeps_visible_tiles():
    scene, cams, fovs, params = synth.config_stereo(4, n=4000, width=192, height=160, radius_deg=14.0)
    masks = [synth.lens_mask(192, 160, (0.85, 0.85))] * 2
    full = oracle.render(scene, cams, fovs, params)
    res = oracle.render(scene, cams, fovs, params, masks=masks)
    for v in range(2):
        bits = ovis.tile_bits(masks[v], 32)
        vis_px = np.repeat(np.repeat(bits, 32, 0), 32, 1)[:160, :192]
        np.testing.assert_allclose(res["pre_images"][v][:, vis_px], full["pre_images"][v][:, vis_px], atol=1e-12)
        assert np.all(res["pre_images"][v][:3, ~vis_px] == 0.0) and np.all(res["pre_images"][v][3, ~vis_px] == 0.0)


def test_rectangle_fovea_weights():
    """Centre rectangle of half the image (half-extents W/4, H/4) with a 10 %
    band: w = 1 on the rectangle, 0 beyond the padded one, linear across the
    band (0.5 halfway), and the weight of a point is set by its worse axis."""
    cam = synth.camera_translate((0, 0, -3), 90.0, 400, 300)
    fov = synth.fovea_rect(cam)
    hx, hy = 100.0, 75.0
    assert fov.half_px == (hx, hy)
    cx, cy = 200.0, 150.0
    w = lambda x, y: float(ofov.mask_weights(cam, fov, np.array([x]), np.array([y]))[0])
    b = np.float64(fov.band_frac)  # 0.1 rounded to float32
    assert w(cx + hx, cy) == 1.0 and w(cx, cy - hy) == 1.0
    assert w(cx + (1 + b) * hx, cy) == 0.0 and w(cx, cy + 1.2 * hy) == 0.0
    assert abs(w(cx + (1 + b / 2) * hx, cy) - 0.5) < 1e-12
    assert abs(w(cx + (1 + b / 4) * hx, cy + (1 + 3 * b / 4) * hy) - 0.25) < 1e-12
    split, sub, wm = ofov.classify(cam, fov)
    # Tiles: split exactly where the padded rectangle reaches a pixel centre.
    px, py = ocam.pixel_centers(0, 0, 400, 300)
    ref = ((np.abs(px - cx) < (1 + b) * hx) & (np.abs(py - cy) < (1 + b) * hy)).reshape(300, 400)
    pad = np.zeros((320, 416), bool)
    pad[:300, :400] = ref
    assert np.array_equal(split, pad.reshape(10, 32, 13, 32).any(axis=(1, 3)))
