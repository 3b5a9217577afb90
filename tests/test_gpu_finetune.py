"""Fine-tuning on the GPU (Sec. 4.1, Sec. 5): the image loss kernel and the
Adam kernel against the oracle's definitions, and an end-to-end fine-tuning
loop (render, loss, backward, Adam) that lowers the loss of a perturbed
scene toward its targets."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import grad as ograd
from oracle import optim as ooptim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2505_10144_amd import render
    from paper_2505_10144_amd import _lib
    _lib.load()
    return render


def test_loss_kernel_matches_oracle(R):
    from paper_2505_10144_amd import finetune
    scene = synth.cluster_scene(2, 3000, log_scale=(-4.5, 0.6))
    cams = synth.ring_cameras(np.random.default_rng(3), 2, 3.0, [(96, 80), (64, 72)], fixed_fov=70.0)
    params = synth.default_params(tile=16, window=8)
    r = R.Renderer(cams, [synth.fovea_off()] * 2, params, scene.n)
    g = R.upload(scene)
    imgs = [im.clone() for im in r.render(g)]
    rng = np.random.default_rng(4)
    targets = [torch.from_numpy(rng.uniform(0, 1, (4, c.height, c.width)).astype(np.float32)).cuda() for c in cams]
    ft = finetune.FineTuner(r, g, targets)
    loss = float(ft.loss_and_grad(imgs).item())
    I = [im.cpu().numpy().astype(np.float64) for im in imgs]
    T = [t.cpu().numpy().astype(np.float64) for t in targets]
    want = float(ograd.loss_fn([torch.tensor(i) for i in I], [torch.tensor(t) for t in T]))
    # The kernel takes I - I* in FP32 (one rounding per term), sums in FP64.
    assert abs(loss - want) <= 1e-8 * max(1.0, abs(want))
    gw = ograd.loss_grad_images(I, T)
    for a, b in zip(ft.grad_img, gw):
        np.testing.assert_allclose(a.cpu().numpy().astype(np.float64), b, rtol=1e-6, atol=1e-12)


def test_adam_kernel_matches_oracle(R):
    from paper_2505_10144_amd import _lib as L
    import ctypes
    rng = np.random.default_rng(8)
    n = 100_003
    p0 = rng.standard_normal(n).astype(np.float32)
    p, m, v = (torch.from_numpy(x).cuda() for x in (p0.copy(), np.zeros(n, np.float32), np.zeros(n, np.float32)))
    pr, mr, vr = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 5):
        gr = rng.standard_normal(n).astype(np.float32)
        gt = torch.from_numpy(gr).cuda()
        L.call("vrs_adam_step", ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(gt.data_ptr()),
               ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), ctypes.c_size_t(n),
               ctypes.c_float(1e-2), ctypes.c_float(0.9), ctypes.c_float(0.999), ctypes.c_float(1e-15), step,
               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        pr, mr, vr = ooptim.adam_step(pr, gr.astype(np.float64), mr, vr, step, 1e-2, 0.9, 0.999, 1e-15)
    torch.cuda.synchronize()
    np.testing.assert_allclose(p.cpu().numpy().astype(np.float64), pr, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("foveated", [False, True])
def test_finetune_lowers_the_loss(R, foveated):
    """Targets rendered (by the oracle) from the scene with perturbed means
    and opacities; fine-tuning the unperturbed scene toward them for 40
    iterations lowers the loss by a quarter or more, and the first Adam step
    moves every parameter with a clear gradient by -lr sign(g) with the sign
    of the oracle's gradient."""
    from paper_2505_10144_amd import finetune
    scene = synth.cluster_scene(5, 2500, log_scale=(-4.3, 0.6))
    rng = np.random.default_rng(6)
    cams = synth.ring_cameras(rng, 2, 3.0, [(96, 96)], fixed_fov=70.0)
    fovs = ([synth.Fovea(True, (48.0, 48.0), 10.0, 0.3)] * 2) if foveated else [synth.fovea_off()] * 2
    params = synth.default_params(tile=32 if foveated else 16, window=8)
    pert = synth.Scene(np.float32(scene.means + rng.normal(0, 0.02, scene.means.shape)), scene.log_scales,
                       scene.quats, np.float32(scene.opacity_logits + rng.normal(0, 0.3, scene.n)), scene.sh,
                       scene.sh_degree)
    tgt_np = oracle.render(pert, cams, fovs, params)["images"]
    targets = [torch.from_numpy(np.float32(t)).cuda() for t in tgt_np]
    print(f"[finetune] foveated={foveated}", flush=True)
    r = R.Renderer(cams, fovs, params, scene.n)
    g = R.upload(scene)
    r.ensure_capacity(g, headroom=2.0)
    ft = finetune.FineTuner(r, g, targets)
    p0 = {k: getattr(g, k).clone() for k in finetune.GROUPS}
    losses = [float(ft.step().item())]
    # The first step against the oracle's gradient of the same loss.
    if not foveated:
        _, ref, _, _ = ograd.gradients(scene, cams, params, tgt_np)
        for k in finetune.GROUPS:
            d = (getattr(g, k) - p0[k]).cpu().numpy().astype(np.float64)
            gk = ref[k]
            clear = np.abs(gk) > 1e-2 * np.abs(gk).max()
            assert clear.sum() > 0
            np.testing.assert_allclose(d[clear], -ft.lr[k] * np.sign(gk[clear]), rtol=1e-3, atol=1e-6)
    for _ in range(39):
        losses.append(float(ft.step().item()))
    r.check()
    print(f"[finetune] loss {losses[0]:.5f} -> {losses[-1]:.5f}", flush=True)
    assert losses[-1] < 0.75 * losses[0]
