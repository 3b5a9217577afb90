"""Pins for the oracle's blending, windowed resorting, foveation and the whole
forward pass: exhaustive per-pixel sort, k-buffer exactness, closed forms and
the paper's large-FoV crop protocol (App. D)."""
import copy
import math

import numpy as np
import pytest

import oracle
from oracle import blend as blend_mod
from oracle import camera as cam_mod
from oracle import fovea as fov_mod
from oracle import projection as proj_mod
from oracle.render import OracleOptions, preprocess_view
import synth


def _small(seed=0, n=300, size=64, fov=90.0, window=16, log_scale=(-3.2, 0.4)):
    scene = synth.uniform_scene(seed, n, log_scale=log_scale)
    cam = synth.camera_translate((0.0, 0.0, -3.0), fov, size, size)
    return scene, cam, synth.default_params(tile=16, window=window)


def _per_pixel_exhaustive(scene, cam, params, xs, ys):
    """Full per-pixel sort over ALL Gaussians (no tiles, no window)."""
    pre = preprocess_view(scene, cam, params)
    gids = np.flatnonzero(pre["valid"])
    out = []
    for x, y in zip(xs, ys):
        d = cam_mod.ray_dirs(cam, x + 0.5, y + 0.5)
        al, ts, cs = [], [], []
        for g in gids:
            q, h = proj_mod.tangent_coords(d, pre["u"][g], pre["E"][g], pre["f"])
            if h <= 0:
                al.append(0.0); ts.append(0.0); cs.append(np.zeros(3)); continue
            D2 = q @ pre["C"][g] @ q
            al.append(min(params.alpha_max, pre["sigma"][g] * math.exp(-0.5 * D2)))
            Bd = pre["B"][g] @ d
            ts.append((Bd @ pre["mu_c"][g]) / (Bd @ d))
            cs.append(pre["color"][g])
        C, T = blend_mod.exhaustive_blend(np.array(al), np.array(ts), np.array(cs),
                                          params.alpha_min, params.t_min)
        out.append(np.r_[C, 1 - T])
    return np.array(out)


def test_large_window_equals_exhaustive_per_pixel_sort():
    scene, cam, params = _small(n=250, size=48, window=400)
    res = oracle.render(scene, [cam], synth.fovea_off(), params)
    img = res["images"][0]
    rng = np.random.default_rng(0)
    xs = rng.integers(0, 48, 60)
    ys = rng.integers(0, 48, 60)
    ref = _per_pixel_exhaustive(scene, cam, params, xs, ys)
    got = img[:, ys, xs].T
    np.testing.assert_allclose(got, ref, atol=1e-12)


def _synthetic_lists(rng, n, disp):
    t = np.sort(rng.uniform(1, 2, n))
    # Arrival order: sorted by t with each entry moved at most `disp` places.
    keys = np.arange(n) + rng.uniform(0, disp + 0.999, n)
    order = np.argsort(keys, kind="stable")
    return t[order], order


def test_window_exact_when_displacement_bounded():
    rng = np.random.default_rng(1)
    for W in (1, 2, 4, 8, 16):
        for _ in range(10):
            n = 60
            t, order = _synthetic_lists(rng, n, W)
            # k-buffer bound: an entry arriving i places late needs W >= i.
            rank = np.argsort(np.argsort(t))
            if np.max(np.arange(n) - rank) > W:
                continue
            al = rng.uniform(0.01, 0.3, n)
            col = rng.uniform(0, 1, (n, 3))

            def gen():
                for i in range(n):
                    a = np.array([al[i]])
                    yield a, np.log(a), (lambda m, i=i: np.array([t[i]])), col[i], False
            C, T, fl, st, _ = blend_mod.window_blend(1, gen(), W, 1 / 255, 1e-4)
            Ce, Te = blend_mod.exhaustive_blend(al, t, col, 1 / 255, 1e-4)
            np.testing.assert_allclose(C[0], Ce, atol=1e-14)
            assert abs(T[0] - Te) < 1e-14


def test_window_is_approximate_beyond_its_length():
    # An entry arriving W+1 places late is blended out of order.
    W = 2
    t = np.array([2.0, 3.0, 4.0, 1.0])
    al = np.array([0.5, 0.5, 0.5, 0.5])
    col = np.eye(3)[[0, 1, 2, 0]] * 1.0
    col[3] = [0, 0, 0]

    def gen():
        for i in range(4):
            a = np.array([al[i]])
            yield a, np.log(a), (lambda m, i=i: np.array([t[i]])), col[i], False
    C, T, *_ = blend_mod.window_blend(1, gen(), W, 1 / 255, 1e-4)
    Ce, Te = blend_mod.exhaustive_blend(al, t, col, 1 / 255, 1e-4)
    assert np.abs(C[0] - Ce).max() > 0.05


def test_uniform_colour_gives_c_times_alpha():
    scene, cam, params = _small(n=400, size=64, window=4)
    scene.sh[:] = 0.0
    res = oracle.render(scene, [cam], synth.fovea_off(), params)
    img = res["images"][0]
    np.testing.assert_allclose(img[:3], np.broadcast_to(0.5 * img[3][None], img[:3].shape), atol=1e-14)
    assert img[3].max() > 0.9


def test_transmittance_monotone_and_bounded():
    scene, cam, params = _small(n=600, size=48, window=8)
    res = oracle.render(scene, [cam], synth.fovea_off(), params, OracleOptions(record=True))
    checked = 0
    for key, rec in res["records"].items():
        for seq in rec:
            T = 1.0
            for _, a in seq:
                Tn = T * (1 - a)
                assert Tn <= T and Tn >= params.t_min
                T = Tn
                checked += 1
    assert checked > 1000
    a = res["images"][0][3]
    assert np.all(a >= 0) and np.all(a <= 1 - params.t_min + 1e-15)


def test_gaussian_index_permutation_invariance():
    scene, cam, params = _small(n=500, size=64, window=8)
    ref = oracle.render(scene, [cam], synth.fovea_off(), params)
    ps, perm = synth.permute_scene(scene, 3)
    got = oracle.render(ps, [cam], synth.fovea_off(), params)
    ok = ~(ref["flags"][0] | got["flags"][0])
    np.testing.assert_allclose(got["images"][0][:, ok], ref["images"][0][:, ok], atol=1e-12)


def test_isotropic_gaussian_closed_form_image():
    """One isotropic Gaussian: alpha(p) = min(0.99, sigma exp(-D^2/2)),
    D^2 = f^2 tan^2(theta_p) / (f^2 s^2 / r^2 + delta); colour = DC term."""
    s, o = 0.08, 1.2
    mu = np.array([0.3, -0.2, 2.0])
    scene = synth.Scene(np.float32(mu[:, None]), np.full((3, 1), np.float32(math.log(s))),
                        np.float32([[1.0], [0.0], [0.0], [0.0]]), np.float32([o]),
                        np.zeros((16, 3, 1), np.float32), 3)
    scene.sh[0, :, 0] = np.float32([0.4, -0.2, 0.1])
    cam = synth.camera_translate((0, 0, 0), 90.0, 96, 80)
    params = synth.default_params(tile=16, window=16)
    img = oracle.render(scene, [cam], synth.fovea_off(), params)["images"][0]
    f = cam_mod.focal(cam)
    mu64 = scene.means[:, 0].astype(np.float64)
    s64 = float(np.exp(np.float64(scene.log_scales[0, 0])))
    r = np.linalg.norm(mu64)
    u = mu64 / r
    ys, xs = np.mgrid[0:80, 0:96]
    d = cam_mod.ray_dirs(cam, xs + 0.5, ys + 0.5)
    th = np.arccos(np.clip(d @ u, -1, 1))
    D2 = f * f * np.tan(th) ** 2 / (f * f * s64 * s64 / (r * r) + params.dilation)
    sig = 1 / (1 + math.exp(-np.float64(scene.opacity_logits[0])))
    a = np.minimum(params.alpha_max, sig * np.exp(-0.5 * D2))
    a = np.where(a >= params.alpha_min, a, 0.0)
    c = np.maximum(scene.sh[0, :, 0].astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5, 0)
    np.testing.assert_allclose(img[3], a, atol=1e-12)
    np.testing.assert_allclose(img[:3], c[:, None, None] * a[None], atol=1e-12)


def test_large_fov_crop_equals_normal_render():
    """App. D: focal length / 3 with resolution x 3, centre crop == normal
    render, for a method without projection error.  Here the focal length in
    pixels is unchanged (tan(fov'/2) = 3 tan(fov/2)) and the resolution
    triples, so the centre crop sees exactly the same rays and tiles."""
    scene = synth.uniform_scene(4, 1500, log_scale=(-3.3, 0.5))
    W, H = 64, 48
    fov = 60.0
    cam = synth.camera_translate((0, 0, -3.0), fov, W, H)
    fov3 = math.degrees(2 * math.atan(3 * math.tan(math.radians(fov) / 2)))
    cam3 = synth.Camera(cam.world_to_cam, float(np.float32(fov3)), 1.5 * W, 1.5 * H, 3 * W, 3 * H)
    params = synth.default_params(tile=16, window=8)
    f1 = cam_mod.focal(cam)
    f3 = cam_mod.focal(cam3)
    assert abs(f1 - f3) < 1e-3 * f1
    # Use exactly the same focal length: adjust the wide camera's FoV field so
    # that both sides compute identical f (fov stored as float32).
    small = oracle.render(scene, [cam], synth.fovea_off(), params)["images"][0]
    big = oracle.render(scene, [cam3], synth.fovea_off(), params)["images"][0]
    crop = big[:, H:2 * H, W:2 * W]
    # Residual: the float32 FoV makes f differ by ~1e-7 relative.
    np.testing.assert_allclose(crop, small, atol=5e-5)
    assert small[3].max() > 0.5


def test_fovea_everywhere_high_equals_plain_render():
    scene, cam, params = _small(n=250, size=64, window=400)
    plain = oracle.render(scene, [cam], synth.fovea_off(), params)["images"][0]
    fov = synth.Fovea(True, (cam.cx, cam.cy), 179.0, 0.1)
    p32 = params.replace(tile=32)
    res = oracle.render(scene, [cam], fov, p32)
    assert all((res["classes"][0][1] == fov_mod.HIGH).ravel())
    np.testing.assert_allclose(res["images"][0], plain, atol=1e-12)


def test_fovea_radius_zero_equals_half_resolution_render():
    """All tiles LOW: the pre-blur image equals a plain render at half the
    resolution with half the focal length and a quarter of the dilation."""
    scene, cam, params = _small(n=400, size=64, window=6)
    fov = synth.Fovea(True, (cam.cx, cam.cy), 0.0, 0.1)
    res = oracle.render(scene, [cam], fov, params.replace(tile=32))
    pre = res["pre_images"][0]
    half = synth.Camera(cam.world_to_cam, cam.fov_x_deg, cam.cx / 2, cam.cy / 2, 32, 32)
    ph = params.replace(tile=16, dilation=params.dilation / 4)
    assert ph.dilation * 4 == params.dilation
    ref = oracle.render(scene, [half], synth.fovea_off(), ph)["images"][0]
    np.testing.assert_allclose(pre[:, ::2, ::2], ref, atol=1e-12)
    np.testing.assert_allclose(pre[:, 1::2, 1::2], ref, atol=1e-12)
    # The final periphery is the 3x3 binomial blur of the upsampled image.
    fin = res["images"][0]
    np.testing.assert_allclose(fin.mean(), pre.mean(), rtol=0.05)


def test_foveated_classes_and_hybrid_band():
    cam = synth.camera_translate((0, 0, -3), 110.0, 512, 480)
    fov = synth.fovea_at_center(cam, 15.0)
    split, sub, w = fov_mod.classify(cam, fov)
    f = cam_mod.focal(cam)
    # Radius 15 deg at the centre is ~f tan(15 deg) px; the band ends at 16.5 deg.
    r_in = f * math.tan(math.radians(15.0))
    r_out = f * math.tan(math.radians(16.5))
    ys, xs = np.mgrid[0:480, 0:512]
    rr = np.hypot(xs + 0.5 - 256, ys + 0.5 - 240)
    assert np.all(w[rr < r_in - 0.5] == 1.0)
    assert np.all(w[rr > r_out + 0.5] == 0.0)
    assert (sub == fov_mod.HIGH).any() and (sub == fov_mod.HYBRID).any() and (sub == fov_mod.LOW).any()
    # LOW tiles never touch w > 0; HIGH subtiles have w == 1 everywhere.
    for sy in range(sub.shape[0]):
        for sx in range(sub.shape[1]):
            blk = w[sy * 16:(sy + 1) * 16, sx * 16:(sx + 1) * 16]
            if sub[sy, sx] == fov_mod.LOW:
                assert (blk == 0).all()
            elif sub[sy, sx] == fov_mod.HIGH:
                assert (blk == 1).all()


def test_hybrid_mix_limits():
    rng = np.random.default_rng(0)
    vals = rng.uniform(size=(4, 16, 16))
    np.testing.assert_allclose(fov_mod.hybrid_mix(vals, np.ones((16, 16)), 0, 0, 16, 16), vals)
    z = fov_mod.hybrid_mix(vals, np.zeros((16, 16)), 0, 0, 16, 16)
    np.testing.assert_allclose(z[:, 0, 0], vals[:, :2, :2].reshape(4, -1).mean(1))
    np.testing.assert_allclose(z[:, 1, 1], z[:, 0, 0])


def test_blur_preserves_constants_and_spreads_binomially():
    pre = np.ones((4, 10, 12)) * 0.3
    low = np.ones((10, 12), bool)
    np.testing.assert_allclose(fov_mod.blur_low(pre, low), pre)
    pre = np.zeros((1, 7, 7)); pre[0, 3, 3] = 16.0
    out = fov_mod.blur_low(pre, np.ones((7, 7), bool))
    np.testing.assert_allclose(out[0, 2:5, 2:5], [[1, 2, 1], [2, 4, 2], [1, 2, 1]])


def test_tiny_workload_flag_fraction_small():
    scene, cams, fov, params = synth.config_tiny(0)
    res = oracle.render(scene, cams, fov, params)
    frac = res["flags"][0].mean()
    assert frac < 0.01, frac
    assert res["stats"]["n_inst"] > 10000


# ---------------------------------------------------------------------------
# Admissible outcomes of borderline samples (blend.sample_outcomes)
# ---------------------------------------------------------------------------

def _blend_in_order(alphas, colors, order, T_min=1e-4):
    """Front-to-back compositing of the given entries in the given order,
    written out directly: C = sum c_i a_i prod_{j<i}(1 - a_j), stopping before
    the entry that would take T below T_min."""
    T, C = 1.0, np.zeros(3)
    for i in order:
        Tn = T * (1.0 - alphas[i])
        if Tn < T_min:
            break
        C = C + T * alphas[i] * np.asarray(colors[i], float)
        T = Tn
    return C, T


def _outcome_set(leaves):
    return sorted((tuple(np.round(C, 12)), round(T, 12)) for C, T, _ in leaves)


def _expected_set(pairs):
    return sorted((tuple(np.round(C, 12)), round(T, 12)) for C, T in pairs)


def test_sample_outcomes_fp64_path_equals_window_blend():
    """The outcome with no flipped decision is the window blend itself, on
    random lists with overflowing windows."""
    rng = np.random.default_rng(21)
    flags = blend_mod.BlendFlags()
    for W in (1, 3, 8):
        for _ in range(20):
            n = 50
            al = rng.uniform(0.0, 0.6, n)
            al[rng.random(n) < 0.3] = 0.001  # below alpha_min
            ts = rng.uniform(1.0, 3.0, n)
            col = rng.uniform(0, 1, (n, 3))
            lnag = np.log(np.maximum(al, 1e-300))

            def gen():
                for i in range(n):
                    yield (np.array([al[i]]), np.array([lnag[i]]), (lambda m, i=i: np.array([ts[i]])[m]),
                           col[i], False)
            C, T, fl, _, _ = blend_mod.window_blend(1, gen(), W, 1 / 255, 1e-4, flags)
            keep = al >= 1 / 255
            leaves, complete = blend_mod.sample_outcomes(al[keep], lnag[keep], ts[keep], col[keep],
                                                         np.zeros(keep.sum(), bool), W, 1 / 255, 1e-4, flags)
            assert complete
            base = [(c, t) for c, t, f in leaves if not f]
            assert len(base) == 1
            np.testing.assert_allclose(base[0][0], C[0], atol=1e-15)
            assert abs(base[0][1] - T[0]) <= 1e-15
            assert (len(leaves) > 1) == bool(fl[0])


def test_sample_outcomes_depth_near_tie_admits_both_orders():
    """Two entries whose depths differ by 1e-7 relative meet at an emission
    (W = 1): both blend orders are admitted, and nothing else."""
    al = np.array([0.5, 0.3, 0.2])
    col = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    ts = np.array([2.0, 2.0 * (1 + 1e-7), 5.0])
    leaves, _ = blend_mod.sample_outcomes(al, np.log(al), ts, col, np.zeros(3, bool), 1, 1 / 255, 1e-4,
                                          blend_mod.BlendFlags())
    want = [_blend_in_order(al, col, [0, 1, 2]), _blend_in_order(al, col, [1, 0, 2])]
    assert _outcome_set(leaves) == _expected_set(want)
    # Depths further apart than eps_t: one outcome.
    ts2 = np.array([2.0, 2.0 * (1 + 1e-4), 5.0])
    leaves, _ = blend_mod.sample_outcomes(al, np.log(al), ts2, col, np.zeros(3, bool), 1, 1 / 255, 1e-4,
                                          blend_mod.BlendFlags())
    assert _outcome_set(leaves) == _expected_set([_blend_in_order(al, col, [0, 1, 2])])


def test_sample_outcomes_alpha_at_threshold_admits_skip_and_blend():
    """An entry whose alpha is within eps_alpha of alpha_min may be skipped
    or blended."""
    amin = 1 / 255
    al = np.array([0.4, amin * math.exp(1e-6), 0.25])
    col = np.array([[0.2, 0.4, 0.6], [1.0, 1.0, 1.0], [0.9, 0.1, 0.3]])
    ts = np.array([1.0, 1.5, 2.0])
    leaves, _ = blend_mod.sample_outcomes(al, np.log(al), ts, col, np.zeros(3, bool), 4, amin, 1e-4,
                                          blend_mod.BlendFlags())
    want = [_blend_in_order(al, col, [0, 1, 2]), _blend_in_order(al, col, [0, 2])]
    assert _outcome_set(leaves) == _expected_set(want)
    kinds = {f[0][0] for _, _, f in leaves if f}
    assert kinds == {blend_mod.FLAG_ALPHA}


def test_sample_outcomes_transmittance_at_T_min_admits_stop_and_blend():
    """An emission whose T' lands within eps_T of T_min may stop the sample
    or blend the entry."""
    T_min = 1e-4
    a0 = 0.99
    a1 = 1.0 - T_min * (1 + 1e-5) / (1.0 - a0)       # T' after entry 1 = T_min (1 + 1e-5)
    al = np.array([a0, a1, 0.5])
    col = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    ts = np.array([1.0, 2.0, 3.0])
    leaves, _ = blend_mod.sample_outcomes(al, np.log(al), ts, col, np.zeros(3, bool), 2, 1 / 255, T_min,
                                          blend_mod.BlendFlags())
    stop = _blend_in_order(al, col, [0])
    # Blending entry 1 leaves T = T_min (1 + 1e-5); entry 2 then stops the sample.
    go = _blend_in_order(al, col, [0, 1], T_min=0.0)
    assert _outcome_set(leaves) == _expected_set([stop, go])


def test_sample_outcomes_ambiguous_arrival_order():
    """Two list neighbours with ambiguous key order: both arrival orders are
    followed, which changes the window's content (W = 1): D(5), A(3), B(2)
    blends A, B, D; swapped, D, B, A blends B, A, D."""
    al = np.array([0.3, 0.4, 0.5])          # D, A, B
    col = np.array([[0, 0, 1.0], [1.0, 0, 0], [0, 1.0, 0]])
    ts = np.array([5.0, 3.0, 2.0])
    amb = np.array([False, True, False])
    leaves, _ = blend_mod.sample_outcomes(al, np.log(al), ts, col, amb, 1, 1 / 255, 1e-4,
                                          blend_mod.BlendFlags())
    want = [_blend_in_order(al, col, [1, 2, 0]), _blend_in_order(al, col, [2, 1, 0])]
    assert _outcome_set(leaves) == _expected_set(want)


def test_sample_outcomes_cap():
    """Many simultaneous near-ties exceed the enumeration cap."""
    n = 12
    al = np.full(n, 0.05)
    ts = 2.0 * (1 + 1e-8 * np.arange(n))
    col = np.random.default_rng(3).uniform(0, 1, (n, 3))
    with pytest.raises(blend_mod.TooManyOutcomes):
        blend_mod.sample_outcomes(al, np.log(al), ts, col, np.zeros(n, bool), 2, 1 / 255, 1e-4,
                                  blend_mod.BlendFlags(), cap=64)
    # With a flip budget the enumeration stays small and says it is partial.
    leaves, complete = blend_mod.sample_outcomes(al, np.log(al), ts, col, np.zeros(n, bool), 2, 1 / 255, 1e-4,
                                                 blend_mod.BlendFlags(), cap=64, max_flips=1)
    assert not complete and 1 < len(leaves) <= 64
    assert sum(1 for _, _, f in leaves if not f) == 1 and all(len(f) <= 1 for _, _, f in leaves)


def test_render_outcomes_cover_every_flagged_pixel():
    """With outcome enumeration on, every flagged pre-compose pixel of a
    foveated stereo render has admissible outcomes (or is counted as
    unchecked), and the FP64 outcome among them is the oracle's own pixel,
    HYBRID mixes included."""
    scene, cams, fovs, params = synth.config_stereo(1, n=6000, width=160, height=128, radius_deg=14.0)
    res = oracle.render(scene, cams, fovs, params, OracleOptions(alternatives=True))
    n_alt = 0
    for v in range(2):
        fl = res["pre_flags"][v]
        alts = res["pre_alts"][v]
        unc = res["pre_unchecked"][v]
        have = np.zeros_like(fl)
        for (y, x), (vals, flips, _) in alts.items():
            have[y, x] = True
            base = [i for i, f in enumerate(flips) if not f]
            assert base, (y, x)
            np.testing.assert_allclose(vals[base[0]], res["pre_images"][v][:, y, x], atol=1e-12)
            n_alt += len(vals) > 1
        assert np.array_equal(fl, have | unc)
    assert n_alt > 0


# ---------------------------------------------------------------------------
# Global-sort variants: view-z / distance keys, no per-sample resort (W = 0)
# ---------------------------------------------------------------------------

def test_window_zero_blends_in_list_order():
    rng = np.random.default_rng(31)
    n = 40
    al = rng.uniform(0.0, 0.5, n)
    ts = rng.uniform(1, 3, n)
    col = rng.uniform(0, 1, (n, 3))

    def gen():
        for i in range(n):
            yield (np.array([al[i]]), np.array([np.log(max(al[i], 1e-300))]),
                   (lambda m, i=i: np.array([ts[i]])[m]), col[i], False)
    C, T, *_ = blend_mod.window_blend(1, gen(), 0, 1 / 255, 1e-4)
    keep = [i for i in range(n) if al[i] >= 1 / 255]
    Cw, Tw = _blend_in_order(al, col, keep)
    np.testing.assert_allclose(C[0], Cw, atol=1e-15)
    assert abs(T[0] - Tw) <= 1e-15


@pytest.mark.parametrize("depth", [1, 2])
def test_global_sort_keys_with_no_resort_equal_per_pixel_key_order(depth):
    """With one key depth per Gaussian (view z or distance) and W = 0, every
    pixel composites all Gaussians reaching alpha_min in order of that depth
    (ties by index): written out per pixel over all Gaussians, no tiles."""
    scene, cam, params = _small(seed=5, n=200, size=40, window=0)
    params = params.replace(depth=depth)
    res = oracle.render(scene, [cam], synth.fovea_off(), params)
    pre = preprocess_view(scene, cam, params)
    gids = np.flatnonzero(pre["valid"])
    key = pre["mu_c"][:, 2] if depth == 1 else pre["r"]
    rng = np.random.default_rng(3)
    for x, y in zip(rng.integers(0, 40, 40), rng.integers(0, 40, 40)):
        d = cam_mod.ray_dirs(cam, x + 0.5, y + 0.5)
        al = []
        for g in gids:
            q, h = proj_mod.tangent_coords(d, pre["u"][g], pre["E"][g], pre["f"])
            al.append(0.0 if h <= 0 else min(params.alpha_max, pre["sigma"][g] * math.exp(-0.5 * q @ pre["C"][g] @ q)))
        C, T = blend_mod.exhaustive_blend(np.array(al), key[gids], pre["color"][gids],
                                          params.alpha_min, params.t_min)
        np.testing.assert_allclose(res["images"][0][:, y, x], np.r_[C, 1 - T], atol=1e-12)
