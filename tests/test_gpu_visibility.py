"""Visibility culling (Sec. 4.3, Fig. 5b) and the paper's rectangular
foveation layout (Sec. 5) on the GPU through the C ABI: exact per-Gaussian
visible-tile counts from the plan's summed-area table, instance sets
restricted to visible tiles, and images against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import fovea as ofov
from oracle import visibility as ovis
from oracle.render import OracleOptions
from parity_check import check_render, workers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2505_10144_amd import render
    from paper_2505_10144_amd import _lib
    _lib.load()
    return render


def _tile_rects(r):
    """Candidate rectangle (tx0, ty0, ncx, ncy) and count per (view,
    Gaussian) from the rectangles the render's preprocess stored."""
    from paper_2505_10144_amd import _lib as L
    nslots = r.V * r.n
    off = nslots * L.VRS_RECORD_FLOATS * 4
    raw = r.proj[off:off + nslots * L.TILERECT_BYTES].cpu().numpy().reshape(nslots, L.TILERECT_BYTES)
    tx0 = raw[:, 0:4].view(np.int32)[:, 0]
    ty0 = raw[:, 4:8].view(np.int32)[:, 0]
    ncx = raw[:, 8:10].view(np.uint16)[:, 0].astype(np.int64)
    ncy = raw[:, 10:12].view(np.uint16)[:, 0].astype(np.int64)
    cnt = raw[:, 12:16].view(np.int32)[:, 0]
    return tx0, ty0, ncx, ncy, cnt


@pytest.mark.parametrize("case", ["stereo_lens", "plain_lens", "rect_fovea_lens"])
def test_visibility_culling_matches_oracle(R, case):
    if case == "stereo_lens":
        scene, cams, fovs, params = synth.config_stereo(3, n=8000, width=256, height=224)
        masks = [synth.lens_mask(256, 224, (0.9, 0.9))] * 2
    elif case == "plain_lens":
        scene = synth.cluster_scene(4, 6000, log_scale=(-4.3, 0.6))
        cams = [synth.camera_translate((0.0, 0.0, -3.0), 90.0, 200, 176)]
        fovs = [synth.fovea_off()]
        params = synth.default_params(tile=16, window=8)
        masks = [synth.lens_mask(200, 176, (0.8, 0.95))]
    else:
        scene, cams, fovs, params = synth.config_stereo(5, n=8000, width=256, height=224)
        fovs = [synth.fovea_rect(c) for c in cams]
        masks = [synth.lens_mask(256, 224, (0.9, 0.9)), None]
    print(f"[visibility] {case}", flush=True)
    r = R.Renderer(cams, fovs, params, scene.n, masks=masks)
    g = R.upload(scene)
    r.ensure_capacity(g)
    r.render(g)
    torch.cuda.synchronize()
    kept = r.check()
    ref = oracle.render(scene, cams, fovs, params,
                        OracleOptions(alternatives=True, workers=workers()), masks=masks)
    # Counts: exactly the visible tiles of each Gaussian's rectangle.
    tx0, ty0, ncx, ncy, cnt = _tile_rects(r)
    counts = r.counts[:r.V * r.n].cpu().numpy().astype(np.int64)
    for v in range(len(cams)):
        sl = slice(v * scene.n, (v + 1) * scene.n)
        valid = ref["pre"][v]["valid"]           # records exist for these only
        bits = ref["vis_bits"][v]
        if bits is None:
            assert np.array_equal(counts[sl][valid], (ncx * ncy)[sl][valid])
            continue
        S = ovis.summed_area(bits)
        a, b, w, h = tx0[sl][valid], ty0[sl][valid], ncx[sl][valid], ncy[sl][valid]
        want = ovis.rect_count(S, a, a + w - 1, b, b + h - 1)
        assert np.array_equal(counts[sl][valid], want)
        assert np.array_equal(cnt[sl][valid], want)
        assert np.all(counts[sl][~valid] == 0)
    # Instances: the oracle's set, all in visible tiles.
    keys = r.keys[:kept].cpu().numpy().view(np.uint64)
    gids = r.gids[:kept].cpu().numpy().view(np.uint32).astype(np.int64)
    s32 = np.uint64(32)
    assert int(ref["inst_border"].sum()) == 0
    got = set(zip((keys >> s32).tolist(), gids.tolist()))
    want_set = set(zip((ref["keys"] >> s32).tolist(), ref["gids"].tolist()))
    assert got == want_set
    check_render(r, ref, label=f"visibility {case}")
    if case == "rect_fovea_lens":
        # The rectangle's classes, decided in FP64, equal the oracle's.
        cls = r.plan_classes()
        off = 0
        for v, cam in enumerate(cams):
            _, sub, _ = ofov.classify(cam, fovs[v])
            m = cls[off:off + sub.size].reshape(sub.shape).astype(np.int16)
            m[m == 255] = -1
            assert np.array_equal(m, sub.astype(np.int16))
            off += sub.size


def test_stereo_full_size_with_lens_mask(R):
    """The 500k stereo workload at 2064x2208 per eye with the synthetic lens
    mask: fewer instances than without it, instance tiles all visible, and
    every SPLIT tile plus 32 LOW tiles per eye against the oracle."""
    scene, cams, fovs, params = synth.config_stereo(0)
    masks = [synth.lens_mask(2064, 2208)] * 2
    g = R.upload(scene)
    r0 = R.Renderer(cams, fovs, params, scene.n)
    r0.ensure_capacity(g)
    r0.render(g)
    torch.cuda.synchronize()
    n_full = r0.check()
    del r0
    r = R.Renderer(cams, fovs, params, scene.n, masks=masks)
    r.ensure_capacity(g)
    r.render(g)
    torch.cuda.synchronize()
    n_vis = r.check()
    bits = ovis.tile_bits(masks[0], 32)
    print(f"[visibility] instances {n_full} -> {n_vis} ({1 - n_vis / n_full:.1%} fewer); "
          f"invisible tiles {int((~bits).sum())} of {bits.size} per eye", flush=True)
    assert n_vis < n_full
    keys = r.keys[:n_vis].cpu().numpy().view(np.uint64)
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    allbits = np.concatenate([bits.ravel(), bits.ravel()])
    assert allbits[tiles].all()
    sel = {}
    rng = np.random.default_rng(17)
    for v in range(2):
        split, _, _ = ofov.classify(cams[v], fovs[v])
        flat = split.ravel()
        low = rng.choice(np.flatnonzero(~flat & bits.ravel()), 32, replace=False)
        sel[v] = sorted(np.flatnonzero(flat).tolist() + low.tolist())
    ref = oracle.render(scene, cams, fovs, params,
                        OracleOptions(alternatives=True, workers=workers(), tiles=sel), masks=masks)
    check_render(r, ref, label="stereo 500k with lens mask, split + 32 low tiles")
