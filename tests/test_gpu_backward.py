"""GPU backward pass (vrs_render_backward, through the C ABI) against the
oracle's vector-Jacobian product (oracle.grad.vjp: float64 autograd of the
recorded blends, itself pinned by central differences in
test_oracle_grad.py), on the same seeded inputs and the same upstream
gradient.  Pixels the oracle flags as borderline get a zero upstream
gradient on both sides (their blend order or stop may legitimately differ).

Tolerance: the GPU accumulates FP32 products of FP32 render records; per
Gaussian, each gradient value is a sum over its pixels of terms with
relative rounding error ~1e-6, and the "colour behind" term S_i is the
difference of two FP32 colours (absolute error ~1e-7 / (1 - alpha)), so
errors of a few 1e-6 of the group's largest gradient are expected (measured:
at most 2.2e-6).  The bar is |g_gpu - g_ref| <= RTOL |g_ref| + ATOL
max|g_ref| per parameter group."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import grad as ograd
from oracle import tiles as otiles

pytestmark = pytest.mark.gpu

RTOL = 1e-4
ATOL = 1e-5
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.fixture(scope="module")
def R():
    from paper_2505_10144_amd import render
    from paper_2505_10144_amd import _lib
    _lib.load()
    return render


def gpu_vjp(R, scene, cams, params, grad_images):
    print(f"[gpu-bwd] n={scene.n} views={len(cams)} size={cams[0].width}x{cams[0].height} "
          f"tile={params.tile} W={params.window}", flush=True)
    r = R.Renderer(cams, [synth.fovea_off()] * len(cams), params, scene.n)
    g = R.upload(scene)
    imgs = r.render(g)
    gi = [torch.from_numpy(np.ascontiguousarray(w, np.float32)).cuda() for w in grad_images]
    out = r.backward(g, gi)
    torch.cuda.synchronize()
    r.check()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}, [im.cpu().numpy() for im in imgs]


def compare_grads(got, ref, K, rtol=RTOL, atol=ATOL):
    report = {}
    for name in GROUPS:
        a, b = got[name], ref[name]
        if name == "sh":
            a, b = a[:K], b[:K]
        assert np.all(np.isfinite(a)), name
        scale = float(np.abs(b).max())
        err = np.abs(a - b)
        bound = rtol * np.abs(b) + atol * scale
        worst = float((err / np.maximum(bound, 1e-30)).max()) if err.size else 0.0
        report[name] = (scale, float(err.max()) if err.size else 0.0, worst)
        if worst > 1.0:
            k = int(np.argmax(err - bound))
            raise AssertionError(f"{name}: |err| {err.ravel()[k]:.3e} > bound {bound.ravel()[k]:.3e} "
                                 f"at {np.unravel_index(k, a.shape)}: got {a.ravel()[k]:.6e} "
                                 f"want {b.ravel()[k]:.6e} (group max {scale:.3e})")
    print("[grad] " + ", ".join(f"{n}: max {s:.2e} err {e:.2e} ({w:.2f} of bound)"
                                for n, (s, e, w) in report.items()), flush=True)
    return report


def cluster_views(seed, n, size, n_views=2, log_scale=(-4.5, 0.6)):
    scene = synth.cluster_scene(seed, n, log_scale=log_scale)
    rng = np.random.default_rng(seed + 100)
    cams = synth.ring_cameras(rng, n_views, 3.0, [size], fixed_fov=70.0)
    return scene, cams


def upstream(seed, cams):
    rng = np.random.default_rng(seed + 77)
    return [rng.standard_normal((4, c.height, c.width)) for c in cams]


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_oracle_vjp(R, seed):
    scene, cams = cluster_views(seed, 3000, (96, 80))
    params = synth.default_params(tile=16, window=16)
    Wt = upstream(seed, cams)
    ref, res, used = ograd.vjp(scene, cams, params, Wt, workers=8, mask_flagged=True)
    got, imgs = gpu_vjp(R, scene, cams, params, used)
    for v in range(len(cams)):
        ok = res["valid"][v] & ~res["flags"][v]
        assert np.abs(imgs[v][:, ok] - res["images"][v][:, ok]).max() <= 2e-4
    compare_grads(got, ref, 16)


@pytest.mark.parametrize("window,tile", [(4, 16), (1, 16), (8, 32), (32, 16), (5, 16), (24, 16), (20, 32), (0, 16)])
def test_backward_windows_and_tiles(R, window, tile):
    scene, cams = cluster_views(3, 2000, (72, 88), n_views=1)
    params = synth.default_params(tile=tile, window=window)
    Wt = upstream(3, cams)
    ref, res, used = ograd.vjp(scene, cams, params, Wt, workers=8, mask_flagged=True)
    got, _ = gpu_vjp(R, scene, cams, params, used)
    compare_grads(got, ref, 16)


def test_backward_low_sh_degree_and_background(R):
    scene, cams = cluster_views(4, 1500, (64, 64), n_views=1)
    scene = synth.Scene(scene.means, scene.log_scales, scene.quats, scene.opacity_logits,
                        np.ascontiguousarray(scene.sh[:4]), 1)
    params = synth.default_params(tile=16, window=16, background=(0.25, 0.5, 1.0))
    Wt = upstream(4, cams)
    ref, res, used = ograd.vjp(scene, cams, params, Wt, workers=8, mask_flagged=True)
    got, _ = gpu_vjp(R, scene, cams, params, used)
    compare_grads(got, ref, 4)


def test_backward_long_lists_leave_the_ring(R):
    """Dense overlapping splats: tile lists far longer than the four staged
    batches the kernel keeps in LDS, so window entries are emitted after
    their batch has left the ring (the global-memory path)."""
    scene, cams = cluster_views(5, 6000, (48, 48), n_views=1, log_scale=(-3.0, 0.3))
    scene.opacity_logits[:] = np.float32(-3.0)  # low alpha: long lists before T reaches t_min
    params = synth.default_params(tile=16, window=16)
    Wt = upstream(5, cams)
    ref, res, used = ograd.vjp(scene, cams, params, Wt, workers=8, mask_flagged=True)
    lens = np.diff(res["ranges"], axis=1).ravel()
    print(f"[lists] max {lens.max()} mean {lens.mean():.0f}", flush=True)
    assert lens.max() > 400
    got, _ = gpu_vjp(R, scene, cams, params, used)
    compare_grads(got, ref, 16)


def test_backward_upstream_spanning_many_octaves(R):
    """Upstream gradients log-uniform over 1e-4 .. 1e6 with random signs: an
    entry's contributions span far more than the fixed-point accumulators'
    headroom over their first contribution, so the overflow path (direct
    float atomics) is taken as well as the accumulators."""
    scene, cams = cluster_views(8, 3000, (80, 64), n_views=1)
    params = synth.default_params(tile=16, window=16)
    rng = np.random.default_rng(8)
    Wt = [np.exp(rng.uniform(np.log(1e-4), np.log(1e6), (4, c.height, c.width)))
          * rng.choice([-1.0, 1.0], (4, c.height, c.width)) for c in cams]
    ref, res, used = ograd.vjp(scene, cams, params, Wt, workers=8, mask_flagged=True)
    got, _ = gpu_vjp(R, scene, cams, params, used)
    compare_grads(got, ref, 16)


def test_backward_all_culled(R):
    scene, cams = cluster_views(6, 500, (64, 48), n_views=1)
    scene.opacity_logits[:] = np.float32(-10.0)  # opacity below alpha_min: all culled
    params = synth.default_params(tile=16, window=16)
    got, imgs = gpu_vjp(R, scene, cams, params, upstream(6, cams))
    assert np.allclose(imgs[0][3], 0.0)
    for name in GROUPS:
        assert np.all(got[name] == 0.0), name


@pytest.mark.parametrize("case", ["stereo", "mixed", "rect_lens"])
def test_foveated_backward_matches_oracle_vjp(R, case):
    """Gradients through the foveated forward -- the periphery's blur and
    nearest-neighbour upsampling, the HYBRID mix, LOW samples at group
    centres -- against the oracle's vector-Jacobian product of the foveated
    composition (oracle.grad.vjp_foveated, pinned by central differences),
    with a plain view in the same call for the mixed case."""
    masks = None
    if case == "stereo":
        scene, cams, fovs, params = synth.config_stereo(2, n=5000, width=160, height=128, radius_deg=14.0)
    elif case == "mixed":
        scene, cams = cluster_views(4, 3000, (128, 96), n_views=2)
        fovs = [synth.Fovea(True, (50.0, 40.0), 12.0, 0.3), synth.fovea_off()]
        params = synth.default_params(tile=16, window=8)
    else:
        scene, cams, fovs, params = synth.config_stereo(6, n=5000, width=160, height=128)
        fovs = [synth.fovea_rect(c) for c in cams]
        masks = [synth.lens_mask(160, 128, (0.9, 0.9))] * 2
    print(f"[gpu-bwd] foveated {case}", flush=True)
    Wt = upstream(7, cams)
    ref, res, used, _ = ograd.vjp_foveated(scene, cams, fovs, params, Wt, workers=8, mask_flagged=True,
                                           masks=masks)
    r = R.Renderer(cams, fovs, params, scene.n, masks=masks)
    g = R.upload(scene)
    r.render(g)
    gi = [torch.from_numpy(np.ascontiguousarray(w, np.float32)).cuda() for w in used]
    out = r.backward(g, gi)
    torch.cuda.synchronize()
    r.check()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    compare_grads(got, ref, 16)


def test_autograd_function(R):
    """rasterize() under torch.autograd: the loss L1 + 0.2 L2 of the paper's
    fine-tuning objective, gradients equal to a direct backward call with
    dL/dI, and a stale forward state is refused."""
    from paper_2505_10144_amd import rasterize
    scene, cams = cluster_views(7, 2000, (64, 64))
    params = synth.default_params(tile=16, window=16)
    r = R.Renderer(cams, [synth.fovea_off()] * len(cams), params, scene.n)
    g = R.upload(scene)
    leaves = [t.clone().requires_grad_(True) for t in (g.means, g.log_scales, g.quats, g.opacity_logits, g.sh)]
    tg = [torch.rand((4, c.height, c.width), device="cuda") for c in cams]
    imgs = rasterize(r, *leaves, sh_degree=3)
    n = sum(t[:3].numel() for t in tg)
    loss = sum((i[:3] - t[:3]).abs().sum() + 0.2 * ((i[:3] - t[:3]) ** 2).sum() for i, t in zip(imgs, tg)) / n
    loss.backward()
    dI = []
    for i, t in zip(imgs, tg):
        d = torch.zeros_like(i)
        diff = (i[:3] - t[:3]).detach()
        d[:3] = (torch.sign(diff) + 0.4 * diff) / n
        dI.append(d)
    direct = r.backward(g, dI, [i.detach() for i in imgs])
    torch.cuda.synchronize()
    for leaf, name in zip(leaves, GROUPS):
        assert leaf.grad is not None
        torch.testing.assert_close(leaf.grad, direct[name], rtol=1e-5, atol=1e-9)
    assert float(leaves[0].grad.abs().max()) > 0
    # A second forward pass invalidates the first one's backward.
    imgs1 = rasterize(r, *leaves, sh_degree=3)
    rasterize(r, *leaves, sh_degree=3)
    with pytest.raises(RuntimeError):
        sum(i.sum() for i in imgs1).backward()


def test_differentiation_config_sampled_tiles(R):
    """The 1M-Gaussian, 4 x 1024^2 fine-tuning workload in the launch
    configuration of the benchmark; the upstream gradient is random on
    sampled tiles and zero elsewhere, so the oracle replays only those."""
    scene, pert, cams, params = synth.config_diff(0)
    rng = np.random.default_rng(3)
    grid = otiles.TileGrid(cams[0].width, cams[0].height, params.tile)
    sel = {v: sorted(rng.choice(grid.n, 3, replace=False).tolist() + [grid.n // 2 + grid.ntx // 2])
           for v in range(len(cams))}
    Wt = upstream(11, cams)
    ref, res, used = ograd.vjp(scene, cams, params, Wt, tiles=sel, workers=8, mask_flagged=True)
    got, _ = gpu_vjp(R, scene, cams, params, used)
    nz = np.abs(ref["opacity_logits"]) > 0
    print(f"[diff] Gaussians with a gradient: {int(nz.sum())}", flush=True)
    assert nz.sum() > 100
    compare_grads(got, ref, 16)
