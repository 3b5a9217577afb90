"""Pins for the oracle gradient (fine-tuning by backpropagation, Sec. 4.1):
the differentiable replay reproduces the NumPy forward pass, and its
gradient matches float64 central differences of the NumPy forward pass on
coordinates whose perturbation does not change any discrete decision."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import grad as ograd
from oracle import sh as osh


def test_sh_polynomial_form_matches_definition():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((200, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    a = osh.sh_basis(3, v)
    b = ograd.sh_basis_torch(3, torch.tensor(v)).numpy()
    np.testing.assert_allclose(b, a, atol=1e-13)


def fd_scene(seed=0, n=64, size=32):
    """64 Gaussians of a cluster scene around one cluster, seen by a 32x32
    camera aimed at their centroid from distance 3, FoV fitted to them."""
    base = synth.cluster_scene(seed, 20000, log_scale=(-5.0, 0.7))
    pts = base.means.T.astype(np.float64)
    c0 = pts[0]
    idx = np.argsort(np.linalg.norm(pts - c0, axis=1))[:n]
    sc = synth.subset_scene(base, idx)
    cen = sc.means.T.astype(np.float64).mean(0)
    rad = np.linalg.norm(sc.means.T - cen, axis=1).max()
    eye = cen + np.array([0.0, -0.3, -3.0])
    fov = 2 * math.degrees(math.atan(rad / 3.0)) * 1.1
    cam = synth.camera_lookat(eye, cen, fov, size, size)
    # Footprints of a few pixels: enlarge the scales (by e^2) so that the
    # gradients with respect to scale and rotation are well conditioned.
    f = (size / 2) / math.tan(math.radians(fov) / 2)
    if np.exp(np.median(sc.log_scales)) * f / 3.0 < 1.0:
        sc.log_scales += np.float32(2.0)
    s64 = synth.Scene(sc.means.astype(np.float64), sc.log_scales.astype(np.float64),
                      sc.quats.astype(np.float64), sc.opacity_logits.astype(np.float64),
                      sc.sh.astype(np.float64), sc.sh_degree)
    return s64, [cam]


def _targets(scene, cams, params, seed=1):
    rng = np.random.default_rng(seed)
    pert = synth.Scene(scene.means + rng.normal(0, 0.01, scene.means.shape),
                       scene.log_scales.copy(), scene.quats.copy(),
                       scene.opacity_logits + rng.normal(0, 0.2, scene.opacity_logits.shape),
                       scene.sh.copy(), scene.sh_degree)
    return oracle.render(pert, cams, [synth.fovea_off()] * len(cams), params)["images"]


def test_replay_reproduces_forward_image():
    scene, cams = fd_scene()
    params = synth.default_params(tile=16, window=8)
    tg = _targets(scene, cams, params)
    loss, grads, res, imgs = ograd.gradients(scene, cams, params, tg)
    np.testing.assert_allclose(imgs[0], res["images"][0], atol=1e-12)
    assert res["images"][0][3].max() > 0.5


def _state(res):
    return [tuple((a, ) for a, _ in seq) for rec in res["records"].values() for seq in rec]


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    scene, cams = fd_scene(seed)
    params = synth.default_params(tile=16, window=8)
    tg = _targets(scene, cams, params, seed + 7)
    loss, grads, res, _ = ograd.gradients(scene, cams, params, tg)
    base_state = _state(res)
    rng = np.random.default_rng(seed)
    fields = [("means", 3), ("log_scales", 3), ("quats", 4), ("opacity_logits", 1), ("sh", 48)]
    checked = {}
    for name, _ in fields:
        arr = getattr(scene, name)
        g = grads[name]
        flat = np.argsort(-np.abs(g).ravel())[:6]   # the most influential coordinates
        for k in flat:
            if abs(g.ravel()[k]) < 1e-9:
                continue
            h = 1e-7 * max(1.0, abs(arr.ravel()[k]))
            vals = []
            ok = True
            signs = []
            for sgn in (1, -1):
                a2 = arr.copy()
                a2.ravel()[k] += sgn * h
                sc2 = synth.Scene(**{**scene.__dict__, name: a2})
                l2, r2 = ograd.loss_numpy(sc2, cams, params, tg)
                ok = ok and _state(r2) == base_state
                signs.append(np.sign(r2["images"][0][:3] - tg[0][:3]))
                vals.append(l2)
            # The L1 term has a kink where a pixel equals its target.
            ok = ok and np.array_equal(signs[0], signs[1])
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            rel = abs(fd - g.ravel()[k]) / max(abs(fd), 1e-12)
            assert rel < 2e-5, (name, k, fd, g.ravel()[k])
            checked[name] = checked.get(name, 0) + 1
    assert all(checked.get(n, 0) >= 3 for n, _ in fields), checked


def test_vjp_matches_central_differences():
    """The vector-Jacobian product (all four channels, so the alpha path is
    covered too) against central differences of the NumPy forward pass."""
    scene, cams = fd_scene(2)
    params = synth.default_params(tile=16, window=8)
    rng = np.random.default_rng(5)
    Wt = [rng.standard_normal((4, c.height, c.width)) for c in cams]
    grads, res, _ = ograd.vjp(scene, cams, params, Wt)
    base_state = _state(res)

    def functional(sc):
        r = oracle.render(sc, cams, [synth.fovea_off()] * len(cams), params, oracle.OracleOptions(record=True))
        return sum(float((w * im).sum()) for w, im in zip(Wt, r["images"])), r

    checked = {}
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        arr = getattr(scene, name)
        g = grads[name]
        for k in np.argsort(-np.abs(g).ravel())[:4]:
            h = 1e-7 * max(1.0, abs(arr.ravel()[k]))
            vals, ok = [], True
            for sgn in (1, -1):
                a2 = arr.copy()
                a2.ravel()[k] += sgn * h
                val, r2 = functional(synth.Scene(**{**scene.__dict__, name: a2}))
                ok = ok and _state(r2) == base_state
                vals.append(val)
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g.ravel()[k]) <= 2e-5 * max(abs(fd), 1e-9), (name, k, fd, g.ravel()[k])
            checked[name] = checked.get(name, 0) + 1
    assert all(checked.get(n, 0) >= 2 for n in ("means", "log_scales", "quats", "opacity_logits", "sh")), checked


# ---------------------------------------------------------------------------
# Foveated views: the HYBRID mix and the periphery's upsampling and blur
# ---------------------------------------------------------------------------

def fov_fd_scene(seed=3):
    """The 64-Gaussian scene at 96x96 with a fovea of about 24 pixels around
    the corner point (16, 16) and a 30 % band: the four subtiles of the first
    tile are HIGH, the ring around them HYBRID, the far tiles LOW, so every
    class carries gradient."""
    scene, cams = fd_scene(seed, size=96)
    cam = cams[0]
    f = 48.0 / math.tan(math.radians(cam.fov_x_deg) / 2)
    fov = synth.Fovea(True, (16.0, 16.0), float(np.float32(math.degrees(math.atan(24.0 / f)))), 0.3)
    return scene, [cam], [fov]


def test_foveated_replay_reproduces_forward_image():
    scene, cams, fovs = fov_fd_scene()
    params = synth.default_params(tile=32, window=8)
    rng = np.random.default_rng(0)
    Wt = [rng.standard_normal((4, 96, 96))]
    grads, res, used, imgs = ograd.vjp_foveated(scene, cams, fovs, params, Wt)
    from oracle import fovea as ofov
    cls = res["classes"][0][1]
    assert (cls == ofov.LOW).any() and (cls == ofov.HYBRID).any() and (cls == ofov.HIGH).any()
    np.testing.assert_allclose(imgs[0], res["images"][0], atol=1e-12)


def test_foveated_vjp_matches_central_differences():
    scene, cams, fovs = fov_fd_scene()
    params = synth.default_params(tile=32, window=8)
    rng = np.random.default_rng(5)
    Wt = [rng.standard_normal((4, c.height, c.width)) for c in cams]
    grads, res, _, _ = ograd.vjp_foveated(scene, cams, fovs, params, Wt)
    base_state = _state(res)

    def functional(sc):
        r = oracle.render(sc, cams, fovs, params, oracle.OracleOptions(record=True))
        return sum(float((w * im).sum()) for w, im in zip(Wt, r["images"])), r

    checked = {}
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        arr = getattr(scene, name)
        g = grads[name]
        for k in np.argsort(-np.abs(g).ravel())[:4]:
            h = 1e-7 * max(1.0, abs(arr.ravel()[k]))
            vals, ok = [], True
            for sgn in (1, -1):
                a2 = arr.copy()
                a2.ravel()[k] += sgn * h
                val, r2 = functional(synth.Scene(**{**scene.__dict__, name: a2}))
                ok = ok and _state(r2) == base_state
                vals.append(val)
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g.ravel()[k]) <= 2e-5 * max(abs(fd), 1e-9), (name, k, fd, g.ravel()[k])
            checked[name] = checked.get(name, 0) + 1
    assert all(checked.get(n, 0) >= 2 for n in ("means", "log_scales", "quats", "opacity_logits", "sh")), checked
