"""GPU parity: every stage of the HIP path, called through the C ABI, against
the FP64 oracle on the same seeded inputs.

Bars: bit-exact for the foveation classes, the sort and the tile ranges;
instance sets equal except oracle-flagged borderline instances, key depths
within one float32 ulp; images within 2e-4 max-abs per channel on every
pixel, a borderline pixel against the outcomes the oracle admits for it
(see parity_check)."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import fovea as ofov
from oracle import tiles as otiles
from oracle.render import OracleOptions
from parity_check import check_render, ref_render, workers

pytestmark = pytest.mark.gpu

TOL = 2e-4


@pytest.fixture(scope="module")
def R():
    from paper_2505_10144_amd import render
    from paper_2505_10144_amd import _lib
    _lib.load()
    return render


def run_gpu(R, scene, cams, foveas, params):
    print(f"[gpu] n={scene.n} views={len(cams)} size={cams[0].width}x{cams[0].height} "
          f"tile={params.tile} W={params.window}", flush=True)
    r = R.Renderer(cams, foveas, params, scene.n)
    g = R.upload(scene)
    imgs = r.render(g)
    torch.cuda.synchronize()
    r.check()
    return r, g, [im.cpu().numpy().astype(np.float64) for im in imgs]


# ---------------------------------------------------------------------------
# Images
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_plain_full_image(R, seed):
    scene, cams, fov, params = synth.config_tiny(seed)
    r, _, _ = run_gpu(R, scene, cams, [fov], params)
    check_render(r, ref_render(scene, cams, fov, params), label=f"tiny seed {seed}")


@pytest.mark.parametrize("W", [1, 4, 5, 8, 12, 13, 20, 24, 32])
def test_window_lengths(R, W):
    scene, cams, fov, params = synth.config_tiny(2, n=4000, size=96, window=W)
    r, _, _ = run_gpu(R, scene, cams, [fov], params)
    check_render(r, ref_render(scene, cams, fov, params), label=f"tiny W={W}")


@pytest.mark.parametrize("size", [(250, 170), (33, 47), (1, 1), (17, 16)])
def test_ragged_image_sizes(R, size):
    w, h = size
    scene = synth.uniform_scene(3, 3000, log_scale=(-3.5, 0.5))
    cam = synth.camera_translate((0.05, -0.02, -3.0), 80.0, w, h)
    params = synth.default_params(tile=16, window=8)
    r, _, _ = run_gpu(R, scene, [cam], [synth.fovea_off()], params)
    check_render(r, ref_render(scene, [cam], synth.fovea_off(), params), label=f"ragged {w}x{h}")


def test_plain_view_with_32_tiles(R):
    scene = synth.uniform_scene(4, 3000, log_scale=(-3.5, 0.5))
    cam = synth.camera_translate((0.0, 0.0, -3.0), 90.0, 120, 88)
    params = synth.default_params(tile=32, window=12)
    r, _, _ = run_gpu(R, scene, [cam], [synth.fovea_off()], params)
    check_render(r, ref_render(scene, [cam], synth.fovea_off(), params), label="plain tile 32")


@pytest.mark.parametrize("seed,radius", [(0, 12.0), (1, 20.0)])
def test_foveated_stereo_small(R, seed, radius):
    scene, cams, fovs, params = synth.config_stereo(seed, n=6000, width=224, height=192, radius_deg=radius)
    r, _, _ = run_gpu(R, scene, cams, fovs, params)
    ref = ref_render(scene, cams, fovs, params)
    assert any((c[1] == ofov.HYBRID).any() for c in ref["classes"])
    assert any((c[1] == ofov.LOW).any() for c in ref["classes"])
    check_render(r, ref, label=f"foveated stereo seed {seed}")


def test_foveated_ragged_and_offcentre(R):
    scene = synth.cluster_scene(5, 8000, log_scale=(-4.5, 0.6))
    cam = synth.camera_translate((0.0, 0.0, -3.0), 100.0, 203, 141)
    fov = synth.Fovea(True, (71.3, 88.9), 14.0, 0.25)
    params = synth.default_params(tile=32, window=16)
    r, _, _ = run_gpu(R, scene, [cam], [fov], params)
    check_render(r, ref_render(scene, [cam], fov, params), label="foveated ragged off-centre")


def test_empty_and_all_culled(R):
    cam = synth.camera_translate((0, 0, -3), 90, 64, 48)
    params = synth.default_params(tile=16, window=4)
    # All Gaussians behind the camera: every count is zero.
    scene = synth.uniform_scene(6, 500)
    scene.means[2] = -10.0
    _, _, imgs = run_gpu(R, scene, [cam], [synth.fovea_off()], params)
    assert np.all(imgs[0][3] == 0.0) and np.all(imgs[0][:3] == 0.0)
    # Opacity below alpha_min everywhere.
    scene2 = synth.uniform_scene(7, 500)
    scene2.opacity_logits[:] = -20.0
    _, _, imgs = run_gpu(R, scene2, [cam], [synth.fovea_off()], params)
    assert np.all(imgs[0] == 0.0)


def test_background_colour(R):
    scene, cams, fov, params = synth.config_tiny(8, n=2000, size=64)
    params = params.replace(background=(0.25, 0.5, 1.0))
    r, _, _ = run_gpu(R, scene, cams, [fov], params)
    check_render(r, ref_render(scene, cams, fov, params), label="background")


def test_schedules_and_batches_are_bit_identical(R):
    """The blend schedule and the staging batch are performance knobs: every
    combination gives the same bits as one block per item with 64-entry
    batches, on mixed plain and foveated views."""
    scene = synth.cluster_scene(5, 20000, log_scale=(-4.5, 0.6))
    rng = np.random.default_rng(9)
    cams = synth.ring_cameras(rng, 3, 3.0, [(200, 150), (96, 130), (160, 160)])
    fovs = [synth.fovea_off(), synth.fovea_at_center(cams[1], 12.0), synth.fovea_off()]
    ref = None
    for schedule in (0, 1):
        for batch in (64, 32, 16):
            params = synth.default_params(tile=16, window=8, blend_batch=batch, schedule=schedule)
            _, _, imgs = run_gpu(R, scene, cams, fovs, params)
            if ref is None:
                ref = imgs
                continue
            for a, b in zip(imgs, ref):
                assert np.array_equal(a, b), (schedule, batch)


@pytest.mark.parametrize("window", [4, 16])
def test_inbox_blend_equals_immediate_insertion(R, window):
    """The blend batches window insertions through per-lane inboxes; the
    instrumented blend inserts immediately.  Both give the same bits."""
    scene = synth.cluster_scene(6, 30000, log_scale=(-4.5, 0.6))
    rng = np.random.default_rng(10)
    cams = synth.ring_cameras(rng, 2, 3.0, [(224, 176)])
    fovs = [synth.fovea_off(), synth.fovea_at_center(cams[1], 15.0)]
    params = synth.default_params(tile=16, window=window)
    r, g, imgs = run_gpu(R, scene, cams, fovs, params)
    work = r.blend_stats()
    r.compose()
    torch.cuda.synchronize()
    for a, b in zip(imgs, r.images):
        assert np.array_equal(a, b.cpu().numpy().astype(np.float64))
    assert work["push_steps"] > 0 and work["contrib"] > 0


def test_deterministic_repeat(R):
    scene, cams, fovs, params = synth.config_stereo(2, n=20000, width=320, height=288)
    r, g, a = run_gpu(R, scene, cams, fovs, params)
    b = [im.cpu().numpy() for im in r.render(g)]
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert np.array_equal(x.astype(np.float32), y)


# ---------------------------------------------------------------------------
# Stages
# ---------------------------------------------------------------------------

def test_fovea_plan_classes_bit_exact(R):
    scene, cams, fovs, params = synth.config_stereo(0, n=10, width=400, height=352, radius_deg=18.0)
    fovs[1] = synth.Fovea(True, (130.0, 201.0), 10.0, 0.3)
    r = R.Renderer(cams, fovs, params, scene.n)
    cls = r.plan_classes()
    items = r.plan_items()
    off = 0
    n_items = 0
    for v, cam in enumerate(cams):
        split, sub, _ = ofov.classify(cam, fovs[v])
        m = cls[off:off + sub.size].reshape(sub.shape).astype(np.int16)
        m[m == 255] = -1
        assert np.array_equal(m, sub.astype(np.int16)), f"view {v}"
        off += sub.size
        n_items += int((~split).sum()) + int(((sub >= 0) & np.repeat(np.repeat(split, 2, 0), 2, 1)).sum())
    assert r.n_items == n_items == len(items)
    # Items cover every in-image pixel exactly once.
    for v, cam in enumerate(cams):
        cover = np.zeros((cam.height, cam.width), np.int32)
        for it in items[(items >> 27) == v]:
            cl, s, t = (it >> 25) & 3, (it >> 23) & 3, it & 0x7FFFFF
            ntx = -(-cam.width // 32)
            tx, ty = t % ntx, t // ntx
            if cl == 0:
                cover[ty * 32:ty * 32 + 32, tx * 32:tx * 32 + 32] += 1
            else:
                x0, y0 = tx * 32 + (s & 1) * 16, ty * 32 + (s >> 1) * 16
                cover[y0:y0 + 16, x0:x0 + 16] += 1
        assert np.all(cover == 1)


def _stage_setup(R, scene, cams, fovs, params):
    r = R.Renderer(cams, fovs, params, scene.n)
    g = R.upload(scene)
    r.ensure_capacity(g)
    r.preprocess(g)
    r.duplicate(g)
    torch.cuda.synchronize()
    r.check()
    return r, g


def test_instances_and_keys_match_oracle(R):
    scene, cams, fovs, params = synth.config_stereo(3, n=8000, width=256, height=224)
    r, g = _stage_setup(R, scene, cams, fovs, params)
    n_cand, n_kept = (int(x) for x in r.n_inst.cpu().tolist())
    keys = r.keys[:n_cand].cpu().numpy().view(np.uint64)
    gids = r.gids[:n_cand].cpu().numpy().view(np.uint32).astype(np.int64)
    live = keys != np.uint64(0xFFFFFFFFFFFFFFFF)
    assert int(live.sum()) == n_kept
    keys, gids = keys[live], gids[live]
    ref = oracle.render(scene, cams, fovs, params, OracleOptions(shade=False))
    assert int(ref["inst_border"].sum()) == 0
    assert len(ref["gids"]) == n_kept
    s32 = np.uint64(32)
    gpu = {(int(k >> s32), int(gg)): int(k & np.uint64(0xFFFFFFFF)) for k, gg in zip(keys, gids)}
    ora = {(int(k >> s32), int(gg)): int(k & np.uint64(0xFFFFFFFF)) for k, gg in zip(ref["keys"], ref["gids"])}
    assert gpu.keys() == ora.keys()
    diffs = np.array([abs(gpu[k] - ora[k]) for k in ora])
    print(f"[keys] {len(diffs)} instances, {int((diffs > 0).sum())} differ by one ulp", flush=True)
    assert diffs.max() <= 1
    assert (diffs > 0).mean() < 1e-3
    # Instances are written in (view, Gaussian, tile) order.
    view = (keys >> s32).astype(np.int64) >= ref["view_offsets"][1]
    assert np.all(np.diff(view.astype(np.int64)) >= 0)
    for v in (False, True):
        gv = gids[view == v]
        assert np.all(np.diff(gv) >= 0)
    # Candidate counts bound the oracle's exact per-(view, Gaussian) counts.
    cnt = r.counts[: 2 * scene.n].cpu().numpy().reshape(2, scene.n)
    otile = (ref["keys"] >> s32).astype(np.int64)
    for v in range(2):
        inview = (otile >= ref["view_offsets"][v]) & (otile < ref["view_offsets"][v] + ref["grids"][v].n)
        oc = np.bincount(ref["gids"][inview].astype(np.int64), minlength=scene.n)
        assert np.all(cnt[v] >= oc)
        assert np.array_equal(cnt[v] > 0, ref["pre"][v]["valid"] & (cnt[v] > 0))


def test_instances_and_keys_full_stereo_frame(R):
    """Instantiation at full size (500k Gaussians, 2 x 2064x2208): the GPU's
    instance set equals the oracle's up to borderline tile tests (an
    instance only one side has must be within 1e-9 of the alpha_min cut in
    ln alpha by the oracle's own tile test), and the depth bits of shared
    instances differ by at most one float32 ulp."""
    scene, cams, fovs, params = synth.config_stereo(0)
    print(f"[keys] full stereo frame n={scene.n}", flush=True)
    r, g = _stage_setup(R, scene, cams, fovs, params)
    n_cand, n_kept = (int(x) for x in r.n_inst.cpu().tolist())
    keys = r.keys[:n_cand].cpu().numpy().view(np.uint64)
    gids = r.gids[:n_cand].cpu().numpy().view(np.uint32).astype(np.int64)
    live = keys != np.uint64(0xFFFFFFFFFFFFFFFF)
    assert int(live.sum()) == n_kept
    keys, gids = keys[live], gids[live]
    ref = oracle.render(scene, cams, fovs, params, OracleOptions(shade=False, workers=workers()))
    s32 = np.uint64(32)
    gtile = (keys >> s32).astype(np.int64)
    gcode = gtile * (1 << 20) + gids
    gbits = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    ocode = ref["inst_tile"] * (1 << 20) + ref["inst_gid"]
    obits = otiles.ord_f32(ref["inst_depth"]).astype(np.int64)
    _, gi, oi = np.intersect1d(gcode, ocode, assume_unique=True, return_indices=True)
    only_o = np.setdiff1d(np.arange(len(ocode)), oi)
    only_g = np.setdiff1d(np.arange(len(gcode)), gi)
    d = np.abs(gbits[gi] - obits[oi])
    print(f"[keys] {len(gi)} shared instances ({int((d > 0).sum())} one ulp apart), {len(only_o)} oracle-only, "
          f"{len(only_g)} GPU-only", flush=True)
    assert len(gi) > 2_000_000
    assert np.all(ref["inst_border"][only_o])
    ln_amin = math.log(np.float64(params.alpha_min))
    for k in only_g:
        t = int(gtile[k])
        v = 0 if t < ref["view_offsets"][1] else 1
        pre, grid, gg = ref["pre"][v], ref["grids"][v], int(gids[k])
        bx0, by0, bx1, by1 = grid.boxes(np.array([t - ref["view_offsets"][v]]))
        res = otiles.quad_test(cams[v], pre["f"], pre["u"][[gg]], pre["E"][[gg]], pre["C"][[gg]], pre["x0"][[gg]],
                               pre["y0"][[gg]], bx0, by0, bx1, by1)
        lnah = math.log(pre["sigma"][gg]) - 0.5 * float(res["D2min"][0])
        assert abs(lnah - ln_amin) < 1e-9, (t, gg, lnah - ln_amin)
    assert d.max() <= 1 and (d > 0).mean() < 1e-3


def test_sort_pairs_bit_exact_on_gpu_keys(R):
    from paper_2505_10144_amd import _lib as L
    import ctypes
    scene, cams, fovs, params = synth.config_stereo(4, n=20000, width=384, height=320)
    r, g = _stage_setup(R, scene, cams, fovs, params)
    n = int(r.n_inst[0].item())
    k0 = r.keys[:n].cpu().numpy().view(np.uint64).copy()
    v0 = r.gids[:n].cpu().numpy().view(np.uint32).copy()
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    L.call("vrs_sort_pairs", ctypes.c_void_p(r.keys.data_ptr()), ctypes.c_void_p(r.gids.data_ptr()),
           ctypes.c_void_p(r.n_inst.data_ptr()), ctypes.c_size_t(r.capacity), r.key_bits(),
           ctypes.c_void_p(r.sort_ws.data_ptr()), ctypes.c_size_t(r.sort_ws.numel()),
           ctypes.c_void_p(st.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ks = r.keys[:n].cpu().numpy().view(np.uint64)
    vs = r.gids[:n].cpu().numpy().view(np.uint32)
    order = np.argsort(k0, kind="stable")
    assert np.array_equal(ks, k0[order]) and np.array_equal(vs, v0[order])
    # The kept instances come out in (key, gid) order.
    n_kept = int(r.n_inst[1].item())
    live = k0 != np.uint64(0xFFFFFFFFFFFFFFFF)
    lo = np.lexsort((v0[live], k0[live]))
    assert np.array_equal(ks[:n_kept], k0[live][lo]) and np.array_equal(vs[:n_kept], v0[live][lo])
    # Ranges from the sorted keys equal the oracle's scan of the same keys.
    L.call("vrs_tile_ranges", ctypes.c_void_p(r.keys.data_ptr()), ctypes.c_void_p(r.n_inst.data_ptr() + 4),
           ctypes.c_size_t(r.capacity), ctypes.c_uint32(r.tiles_total), ctypes.c_void_p(r.ranges.data_ptr()),
           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    rg = r.ranges[: 2 * r.tiles_total].cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert np.array_equal(rg, otiles.tile_ranges(ks[:n_kept], r.tiles_total))


def _copies_scene(n_copies, n_random):
    """n_copies identical Gaussians (equal keys in every tile they reach) and
    n_random random ones."""
    a = synth.uniform_scene(11, 1, lo=-0.2, hi=0.2, log_scale=(-1.5, 0.0))
    a.opacity_logits[:] = 3.0
    b = synth.uniform_scene(12, n_random, lo=-1.0, hi=1.0)
    rep = lambda x, y: np.concatenate([np.repeat(x, n_copies, axis=-1), y], axis=-1)
    return synth.Scene(rep(a.means, b.means), rep(a.log_scales, b.log_scales), rep(a.quats, b.quats),
                       rep(a.opacity_logits, b.opacity_logits), rep(a.sh, b.sh), a.sh_degree)


@pytest.mark.parametrize("case", ["small", "copies", "stereo_full"])
def test_render_sort_is_stable_sort_of_candidates(R, case):
    """vrs_sort leaves the kept candidates exactly in stable (tile, depth)
    order -- ties in candidate order -- with matching ranges, also for tile
    lists longer than 2048 entries and runs of equal keys that long."""
    print(f"[render sort] {case}", flush=True)
    if case == "small":
        scene, cams, fovs, params = synth.config_stereo(3, n=8000, width=256, height=224)
    elif case == "copies":
        scene = _copies_scene(3000, 2000)
        cams = [synth.camera_translate((0.0, 0.0, -2.0), 90.0, 200, 160)]
        fovs = [synth.fovea_off()]
        params = synth.default_params(tile=16, window=8)
    else:
        scene, cams, fovs, params = synth.config_stereo(0)
    r = R.Renderer(cams, fovs, params, scene.n)
    g = R.upload(scene)
    r.ensure_capacity(g)
    r.preprocess(g)
    r.duplicate(g)
    torch.cuda.synchronize()
    r.check()
    n = int(r.n_inst[0].item())
    k0 = r.keys[:n].cpu().numpy().view(np.uint64).copy()
    v0 = r.gids[:n].cpu().numpy().view(np.uint32).copy()
    r.sort(g)
    torch.cuda.synchronize()
    r.check()
    n_kept = int(r.n_inst[1].item())
    live = k0 != np.uint64(0xFFFFFFFFFFFFFFFF)
    assert int(live.sum()) == n_kept
    order = np.argsort(k0[live], kind="stable")
    ks = r.keys[:n_kept].cpu().numpy().view(np.uint64)
    vs = r.gids[:n_kept].cpu().numpy().view(np.uint32)
    assert np.array_equal(ks, k0[live][order]) and np.array_equal(vs, v0[live][order])
    rg = r.ranges[: 2 * r.tiles_total].cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert np.array_equal(rg, otiles.tile_ranges(ks, r.tiles_total))
    lens = rg[:, 1].astype(np.int64) - rg[:, 0]
    print(f"[render sort] {n_kept} kept of {n}, longest list {int(lens.max())}", flush=True)
    if case != "small":
        assert lens.max() > 2048
    if case == "copies":
        # Some tile holds a run of equal keys longer than 2048.
        _, runs = np.unique(ks, return_counts=True)
        assert runs.max() > 2048


@pytest.mark.parametrize("n,bits,dups", [(0, 40, 1), (1, 40, 1), (4095, 64, 1), (4097, 33, 7),
                                         (100_003, 46, 50), (300_000, 64, 1000), (3_000_001, 64, 3),
                                         (2_500_000, 8, 1)])
def test_sort_pairs_random(R, n, bits, dups):
    from paper_2505_10144_amd import _lib as L
    import ctypes
    rng = np.random.default_rng(n + bits)
    print(f"[sort] n={n} bits={bits}", flush=True)
    hi = (1 << bits) - 1 if bits < 64 else (1 << 64) - 1
    base = rng.integers(0, hi, size=max(n // dups, 1), dtype=np.uint64, endpoint=True) if n else np.zeros(0, np.uint64)
    keys = base[rng.integers(0, len(base), size=n)] if n else np.zeros(0, np.uint64)
    vals = rng.permutation(n).astype(np.uint32)
    cap = n + 123
    kt = torch.zeros(cap, dtype=torch.int64, device="cuda")
    vt = torch.zeros(cap, dtype=torch.int32, device="cuda")
    if n:
        kt[:n] = torch.from_numpy(keys.view(np.int64)).cuda()
        vt[:n] = torch.from_numpy(vals.view(np.int32)).cuda()
    nt = torch.tensor([n], dtype=torch.int32, device="cuda")
    ws = torch.empty(int(L.load().vrs_sort_pairs_workspace_size(cap)), dtype=torch.uint8, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    L.call("vrs_sort_pairs", ctypes.c_void_p(kt.data_ptr()), ctypes.c_void_p(vt.data_ptr()),
           ctypes.c_void_p(nt.data_ptr()), ctypes.c_size_t(cap), bits, ctypes.c_void_p(ws.data_ptr()),
           ctypes.c_size_t(ws.numel()), ctypes.c_void_p(st.data_ptr()),
           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ks = kt[:n].cpu().numpy().view(np.uint64)
    vs = vt[:n].cpu().numpy().view(np.uint32)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(ks, keys[order]) and np.array_equal(vs, vals[order])
    assert np.all(kt[n:].cpu().numpy() == 0)


def test_capacity_overflow_is_reported_and_recoverable(R):
    from paper_2505_10144_amd import _lib as L
    scene, cams, fovs, params = synth.config_stereo(5, n=5000, width=192, height=160)
    r = R.Renderer(cams, fovs, params, scene.n, capacity=64)
    g = R.upload(scene)
    r.status.zero_()
    r.preprocess(g)
    r.sort(g)
    torch.cuda.synchronize()
    assert int(r.status.item()) == L.VRS_ERR_CAPACITY
    need = int(r.n_inst[0].item())
    assert need > 64 and r.keys.numel() == 64
    with pytest.raises(L.VrsError):
        r.check()
    r2 = R.Renderer(cams, fovs, params, scene.n, capacity=need)
    r2.render(g)
    torch.cuda.synchronize()
    assert 0 < r2.check() <= need


def test_record_colours_and_alpha(R):
    """K1 output: the colour array holds the oracle's SH colour, and the
    record's mean image point and opacity equal the oracle's."""
    scene, cams, fovs, params = synth.config_stereo(6, n=3000, width=256, height=224)
    r, g = _stage_setup(R, scene, cams, fovs, params)
    # Records of culled slots are never written: only valid rows are read.
    rec_all = r.records().cpu().numpy()
    cols = r.colours().cpu().numpy().astype(np.float64)
    from oracle.render import preprocess_view
    for v, cam in enumerate(cams):
        pre = preprocess_view(scene, cam, params)
        ok = pre["valid"]
        rec = np.zeros(rec_all.shape, np.float64)
        rec[v, ok] = rec_all[v, ok]
        np.testing.assert_allclose(cols[v, ok, :3], pre["color"][ok], atol=2e-6)
        assert np.all(cols[v, :, 3] == 0.0)
        x0 = rec[v, ok, 0] + rec[v, ok, 2]
        y0 = rec[v, ok, 1] + rec[v, ok, 3]
        np.testing.assert_allclose(x0, pre["x0"][ok], atol=1e-4, rtol=1e-6)
        np.testing.assert_allclose(y0, pre["y0"][ok], atol=1e-4, rtol=1e-6)
        np.testing.assert_allclose(np.exp2(rec[v, ok, 10]), pre["sigma"][ok], rtol=1e-6)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_colours_every_sh_degree(R, degree):
    """The colour array for SH degrees 0-3 equals the oracle's SH colour,
    through both the two-view kernel (one view) and the four-view kernel
    (three views, one padding slot), and a view's colour has the same bits
    in both."""
    from oracle.render import preprocess_view
    scene = synth.uniform_scene(11 + degree, 2000, sh_degree=degree, sh_std=0.5)
    cams = [synth.camera_translate((0.3 * k - 0.3, 0.1 * k, -3.0), 80.0 + 10 * k, 96, 64) for k in range(3)]
    params = synth.default_params(tile=16, window=8)
    print(f"[colours] degree={degree} n={scene.n}", flush=True)
    r3, _ = _stage_setup(R, scene, cams, [synth.fovea_off()] * 3, params)
    cols3 = r3.colours().cpu().numpy()
    r1, _ = _stage_setup(R, scene, cams[1:2], [synth.fovea_off()], params)
    cols1 = r1.colours().cpu().numpy()
    assert np.array_equal(cols1[0], cols3[1])
    for v, cam in enumerate(cams):
        pre = preprocess_view(scene, cam, params)
        ok = pre["valid"]
        assert ok.sum() > 100
        np.testing.assert_allclose(cols3[v, ok, :3].astype(np.float64), pre["color"][ok], atol=2e-6)


@pytest.mark.parametrize("scale", [(-3.5, 1.2), (-2.5, 0.5)])
def test_record_boxes_contain_the_footprint(R, scale):
    """K1's pixel box (cone bound intersected with the exact conic footprint
    box) contains every pixel centre where the oracle's alpha reaches
    alpha_min, for anisotropic splats near and far, including ones that
    cross the image border and ones close to the camera."""
    from oracle.render import preprocess_view, _alpha_fn
    from oracle import camera as ocam
    scene = synth.uniform_scene(7, 300, lo=-1.5, hi=1.5, log_scale=scale)
    cam = synth.camera_translate((0.0, 0.0, -2.2), 100.0, 96, 80)
    params = synth.default_params(tile=16, window=8)
    r, g = _stage_setup(R, scene, [cam], [synth.fovea_off()], params)
    rec = r.records().cpu().numpy().astype(np.float64)[0]
    pre = preprocess_view(scene, cam, params)
    px, py = ocam.pixel_centers(0, 0, cam.width, cam.height)
    rays = ocam.ray_dirs(cam, px, py)
    checked = 0
    for gi in np.nonzero(pre["valid"])[0]:
        a, lnag = _alpha_fn(pre, gi, cam, rays, params)
        hit = lnag >= np.log(np.float64(params.alpha_min)) + 1e-9
        if not hit.any():
            continue
        x0b, y0b, x1b, y1b = rec[gi, 28:32]
        inside = (px >= x0b) & (px <= x1b) & (py >= y0b) & (py <= y1b)
        assert np.all(inside[hit]), (int(gi), rec[gi, 28:32], px[hit & ~inside][:3], py[hit & ~inside][:3])
        checked += 1
    print(f"[boxes] {checked} splats checked", flush=True)
    assert checked > 50


def test_stereo_full_frame_every_pixel(R):
    """The full 500k-Gaussian stereo workload at 2064x2208 per eye, in the
    launch configuration of the benchmark: every pixel of both eyes against
    the oracle (borderline pixels against their admissible outcomes)."""
    scene, cams, fovs, params = synth.config_stereo(0)
    r, g, imgs = run_gpu(R, scene, cams, fovs, params)
    ref = ref_render(scene, cams, fovs, params)
    check_render(r, ref, label="stereo 500k 2x2064x2208 full frame")


def _split_and_low_tiles(cam, fov, n_low, seed):
    """Every SPLIT 32x32 tile of a foveated view plus n_low random LOW tiles."""
    split, _, _ = ofov.classify(cam, fov)
    flat = split.ravel()
    rng = np.random.default_rng(seed)
    low = rng.choice(np.flatnonzero(~flat), n_low, replace=False)
    return sorted(np.flatnonzero(flat).tolist() + low.tolist())


@pytest.mark.parametrize("frame", [0, 15, 29])
def test_unpruned_yaw_arc_split_and_low_tiles(R, frame):
    """The unpruned-density workload (3M smaller, fainter Gaussians, stereo
    foveated at 2064x2208) at both ends and the middle of its +-20 degree
    head-yaw arc: every SPLIT tile and 64 random LOW tiles per eye against
    the oracle."""
    scene, cams, fovs, params = synth.config_unpruned(0, frame=frame)
    r, g, imgs = run_gpu(R, scene, cams, fovs, params)
    sel = {v: _split_and_low_tiles(cams[v], fovs[v], 64, 100 + frame + v) for v in range(2)}
    ref = ref_render(scene, cams, fovs, params, tiles=sel)
    check_render(r, ref, label=f"unpruned 3M frame {frame} split+64 low tiles")


def test_unpruned_yaw_arc_all_frames_run(R):
    """Every frame of the 30-frame yaw arc renders through one renderer per
    frame with finite output, no capacity error and alpha in [0, 1]."""
    scene, cams, fovs, params = synth.config_unpruned(0, frame=0)
    g = R.upload(scene)
    for frame in range(0, 30, 3):
        _, cams, fovs, params = synth.config_unpruned(0, frame=frame, n=16)  # cameras only
        r = R.Renderer(cams, fovs, params, scene.n)
        r.ensure_capacity(g)
        imgs = r.render(g)
        torch.cuda.synchronize()
        kept = r.check()
        assert kept > 0
        for im in imgs:
            assert bool(torch.isfinite(im).all())
            a = im[3]
            assert float(a.min()) >= 0.0 and float(a.max()) <= 1.0
        print(f"[yaw] frame {frame} instances {kept}", flush=True)


# ---------------------------------------------------------------------------
# Failure reporting
# ---------------------------------------------------------------------------

def test_nonfinite_parameters_are_culled_and_reported(R):
    """Gaussians with a NaN or infinite mean, log-scale, quaternion or
    opacity logit are culled from every view and one with non-finite SH
    coefficients is coloured black; the status word says so, and the image
    equals (bit for bit) the render of the same scene with those Gaussians
    behind the camera and that colour clamped to black."""
    from paper_2505_10144_amd import _lib as L
    scene, cams, fovs, params = synth.config_stereo(7, n=4000, width=192, height=160)
    bad = synth.subset_scene(scene, np.arange(scene.n))
    bad.means[0, 5] = np.nan
    bad.log_scales[1, 7] = np.inf
    bad.quats[2, 9] = np.nan
    bad.opacity_logits[11] = -np.inf
    bad.sh[0, 1, 13] = np.nan
    good = synth.subset_scene(scene, np.arange(scene.n))
    for i in (5, 7, 9, 11):
        good.means[:, i] = (0.0, 0.0, -50.0)  # behind both eyes: culled by the near plane
    good.sh[0, :, 13] = -1e30                   # SH sum far below zero: colour clamped to 0
    print("[nonfinite] n=4000 stereo 192x160", flush=True)
    out = []
    for sc, want in ((bad, L.VRS_ERR_NONFINITE), (good, 0)):
        r = R.Renderer(cams, fovs, params, sc.n)
        g = R.upload(sc)
        r.ensure_capacity(g)
        r.status.zero_()
        imgs = [im.clone() for im in r.render(g)]
        torch.cuda.synchronize()
        assert int(r.status.item()) == want
        assert all(bool(torch.isfinite(im).all()) for im in imgs)
        out.append(imgs)
    for a, b in zip(*out):
        assert torch.equal(a, b)


def test_candidate_count_beyond_32_bits_is_reported(R):
    """More than 2^32 - 1 candidate (Gaussian, tile) pairs -- 20000 splats
    that each cover all 262144 tiles of an 8192x8192 view -- cannot be
    addressed by the 32-bit instance offsets: vrs_sort reports
    VRS_ERR_UNSUPPORTED, leaves zero instances and writes nothing."""
    from paper_2505_10144_amd import _lib as L
    scene = synth.uniform_scene(3, 20000, lo=-0.05, hi=0.05, log_scale=(0.5, 0.01))
    scene.opacity_logits[:] = 8.0
    cam = synth.camera_translate((0.0, 0.0, -3.0), 90.0, 8192, 8192)
    params = synth.default_params(tile=16, window=4)
    print("[overflow] 20000 splats x 262144 tiles", flush=True)
    r = R.Renderer([cam], [synth.fovea_off()], params, scene.n, capacity=4096)
    g = R.upload(scene)
    r.status.zero_()
    r.preprocess(g)
    torch.cuda.synchronize()
    counts = r.counts[:scene.n].cpu().numpy().astype(np.int64)
    assert counts.sum() >= 2 ** 32
    r.keys.fill_(7)
    r.sort(g)
    torch.cuda.synchronize()
    assert int(r.status.item()) == L.VRS_ERR_UNSUPPORTED
    assert r.n_inst.cpu().tolist() == [0, 0]
    assert bool((r.keys == 7).all())


@pytest.mark.parametrize("depth,W", [(1, 0), (2, 0), (1, 4), (2, 16), (0, 0)])
def test_global_sort_variants(R, depth, W):
    """Key depth per Gaussian (view z, distance) and/or no per-sample resort
    (W = 0): the global-sort orders of the comparison renderers."""
    scene, cams, fov, params = synth.config_tiny(6, n=4000, size=96, window=W)
    params = params.replace(depth=depth)
    r, _, _ = run_gpu(R, scene, cams, [fov], params)
    check_render(r, ref_render(scene, cams, fov, params), label=f"global sort depth={depth} W={W}")


def test_global_sort_foveated_stereo(R):
    scene, cams, fovs, params = synth.config_stereo(8, n=6000, width=224, height=192, radius_deg=12.0)
    params = params.replace(depth=2, window=0)
    r, _, _ = run_gpu(R, scene, cams, fovs, params)
    check_render(r, ref_render(scene, cams, fovs, params), label="global sort distance W=0 foveated stereo")
