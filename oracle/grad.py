"""Gradients of the rendered images with respect to the Gaussian parameters
(the fine-tuning of Sec. 4.1 optimises position, rotation, scale, opacity and
SH coefficients by backpropagation through the renderer).  Test
infrastructure only.

Method: the NumPy forward pass (render.py) fixes every discrete decision --
instance sets, list order, which entries reach alpha_min, the window's
emission order and the stop index -- and records, per sample, the Gaussians
it blended in order.  This module replays exactly those blends in PyTorch
float64 on the CPU, as a differentiable function of the raw parameters
(means, log-scales, quaternions, opacity logits, SH), and lets autograd take
the derivative.  Decisions carry no gradient (they are piecewise constant);
the alpha clamp and the colour clamp pass zero gradient where active.

Loss (a reading of the L1 + L2 objective): L = mean|I - I*| + 0.2 mean((I - I*)^2)
over the RGB channels of all pixels of all views.

The replay reproduces the NumPy forward image to ~1e-13 (tested), and its
gradient is pinned by float64 central differences of the NumPy forward on
coordinates whose perturbation leaves the discrete state unchanged.
"""
import math

import numpy as np
import torch
from numpy.polynomial import polynomial as P

from . import camera as cam_mod
from .render import OracleOptions
from .render import render as render_full

DT = torch.float64


def _legendre_poly(l, m):
    """Coefficients of d^m/dx^m P_l(x) (Rodrigues' formula)."""
    base = P.polypow([-1.0, 0.0, 1.0], l)
    pl = P.polyder(base, l) / (2.0 ** l * math.factorial(l)) if l > 0 else np.array([1.0])
    return P.polyder(pl, m) if m > 0 else pl


def sh_basis_torch(degree, v):
    """Real SH (orthonormal, Condon-Shortley phase) at unit vectors v (..., 3)
    as a polynomial in (x, y, z): with x + iy = sin(theta) e^{i phi},
    sin^m(theta) cos(m phi) = Re (x + iy)^m and sin^m(theta) sin(m phi) =
    Im (x + iy)^m, so Y_lm = sqrt(2) K (-1)^m Q_lm(z) Re/Im (x + iy)^m with
    Q_lm = d^m/dz^m P_l.  Smooth everywhere (no atan2, no poles)."""
    x, y, z = v[..., 0], v[..., 1], v[..., 2]
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        r_prev, i_prev = re[-1], im[-1]
        re.append(r_prev * x - i_prev * y)
        im.append(r_prev * y + i_prev * x)
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            coeffs = _legendre_poly(l, am)
            q = torch.zeros_like(z)
            for c in reversed(coeffs):
                q = q * z + float(c)
            sgn = (-1.0) ** am
            if m == 0:
                out.append(K * q)
            elif m > 0:
                out.append(math.sqrt(2.0) * K * sgn * q * re[am])
            else:
                out.append(math.sqrt(2.0) * K * sgn * q * im[am])
    return torch.stack(out, dim=-1)


def quat_to_rotmat_torch(q):
    """q (4, N) -> (N, 3, 3) for q/|q| (Hamilton convention)."""
    q = q / torch.linalg.norm(q, dim=0, keepdim=True)
    w, x, y, z = q
    R = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], dim=1)
    return R.reshape(-1, 3, 3)


def emission_lists(res, cams):
    """Per view: (pixel index (P,), emitted Gaussian ids padded (P, K) with -1)
    from a recorded plain-mode forward pass."""
    out = []
    for v, cam in enumerate(cams):
        grid = res["grids"][v]
        off = res["view_offsets"][v]
        pix, seqs = [], []
        for (vv, kind, tile, sub), rec in res["records"].items():
            if vv != v:
                continue
            if kind != "plain":
                raise ValueError("gradients are defined for plain (non-foveated) views")
            s, e = res["ranges"][off + tile]
            lst = res["gids"][s:e]
            x0, y0, x1, y1 = grid.box(tile)
            ys, xs = np.mgrid[y0:y1, x0:x1]
            for k, seq in enumerate(rec):
                pix.append(int(ys.ravel()[k]) * cam.width + int(xs.ravel()[k]))
                seqs.append([int(lst[a]) for a, _ in seq])
        K = max([len(sq) for sq in seqs] + [1])
        E = np.full((len(seqs), K), -1, np.int64)
        for i, sq in enumerate(seqs):
            E[i, :len(sq)] = sq
        out.append((np.asarray(pix, np.int64), E))
    return out


def replay(tensors, sh_degree, cams, params, lists):
    """Differentiable images (list of (4, H, W) float64 tensors) from the raw
    parameters, blending each pixel's recorded Gaussians in recorded order."""
    means, log_scales, quats, logits, sh = tensors
    R = quat_to_rotmat_torch(quats)
    s = torch.exp(log_scales).T
    RS = R * s[:, None, :]
    Sigma = RS @ RS.transpose(1, 2)
    sigma = 1.0 / (1.0 + torch.exp(-logits))
    K = (sh_degree + 1) ** 2
    imgs = []
    for v, cam in enumerate(cams):
        pix, E = lists[v]
        Rv_np, tv_np = cam_mod.rt(cam)
        Rv = torch.tensor(Rv_np, dtype=DT)
        tv = torch.tensor(tv_np, dtype=DT)
        f = float(cam_mod.focal(cam))
        mu_c = means.T @ Rv.T + tv
        Sigma_c = Rv @ Sigma @ Rv.T
        r = torch.linalg.norm(mu_c, dim=1)
        u = mu_c / r[:, None]
        ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
        kk = 1.0 / (1.0 + uz)
        e1 = torch.stack([1 - ux * ux * kk, -ux * uy * kk, -ux], dim=1)
        e2 = torch.stack([-ux * uy * kk, 1 - uy * uy * kk, -uy], dim=1)
        Emat = torch.stack([e1, e2], dim=2)
        S2 = (f * f / (r * r))[:, None, None] * (Emat.transpose(1, 2) @ Sigma_c @ Emat)
        S2 = S2 + float(params.dilation) * torch.eye(2, dtype=DT)[None]
        C = torch.linalg.inv(S2)
        o = torch.tensor(cam_mod.eye_center(cam), dtype=DT)
        vd = means.T - o
        vd = vd / torch.linalg.norm(vd, dim=1, keepdim=True)
        Y = sh_basis_torch(sh_degree, vd)
        col = torch.clamp_min(torch.einsum("nk,kcn->nc", Y, sh[:K]) + 0.5, 0.0)
        H, W = cam.height, cam.width
        img = torch.zeros(4, H * W, dtype=DT)
        bg = torch.tensor(params.background, dtype=DT)
        if len(pix):
            px = torch.tensor(pix % W, dtype=DT) + 0.5
            py = torch.tensor(pix // W, dtype=DT) + 0.5
            d = torch.stack([(px - float(cam.cx)) / f, (py - float(cam.cy)) / f, torch.ones_like(px)], dim=1)
            d = d / torch.linalg.norm(d, dim=1, keepdim=True)
            Et = torch.tensor(E, dtype=torch.long)
            valid = Et >= 0
            g = Et.clamp_min(0)
            dd = d[:, None, :].expand(-1, g.shape[1], -1)
            h = (dd * u[g]).sum(-1)
            q = f * torch.einsum("pki,pkij->pkj", dd, Emat[g]) / h[..., None]
            D2 = torch.einsum("pki,pkij,pkj->pk", q, C[g], q)
            a = torch.minimum(torch.tensor(float(params.alpha_max), dtype=DT), sigma[g] * torch.exp(-0.5 * D2))
            a = torch.where(valid, a, torch.zeros_like(a))
            one_m = 1.0 - a
            T_excl = torch.cumprod(torch.cat([torch.ones(len(pix), 1, dtype=DT), one_m[:, :-1]], dim=1), dim=1)
            Tfin = torch.prod(one_m, dim=1)
            w = (a * T_excl)[..., None]
            rgb = (w * col[g]).sum(1) + Tfin[:, None] * bg[None]
            idx = torch.tensor(pix, dtype=torch.long)
            img = img.index_put((torch.arange(3)[:, None], idx[None, :]), rgb.T)
            img = img.index_put((torch.tensor([3])[:, None], idx[None, :]), (1.0 - Tfin)[None])
        imgs.append(img.reshape(4, H, W))
    return imgs


def loss_fn(imgs, targets):
    """mean |I - I*| + 0.2 mean (I - I*)^2 over RGB of all views."""
    l1 = sum(torch.abs(i[:3] - t[:3]).sum() for i, t in zip(imgs, targets))
    l2 = sum(((i[:3] - t[:3]) ** 2).sum() for i, t in zip(imgs, targets))
    n = sum(t[:3].numel() for t in targets)
    return l1 / n + 0.2 * l2 / n


def loss_grad_images(imgs, targets):
    """dL/dI for the loss above (images as NumPy arrays); zero on alpha."""
    n = sum(t[:3].size for t in targets)
    out = []
    for i, t in zip(imgs, targets):
        g = np.zeros_like(i)
        diff = i[:3] - t[:3]
        g[:3] = (np.sign(diff) + 0.4 * diff) / n
        out.append(g)
    return out


def gradients(scene, cams, params, targets, workers=1):
    """Loss and its gradients for a plain-mode render.  Returns
    (loss, dict(means, log_scales, quats, opacity_logits, sh) as NumPy arrays
    in the scene's layouts, forward result dict, replayed images)."""
    res = render_full(scene, cams, _plain(cams), params, OracleOptions(record=True, workers=workers))
    lists = emission_lists(res, cams)
    ts = [torch.tensor(np.asarray(a, np.float64), dtype=DT, requires_grad=True)
          for a in (scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh)]
    imgs = replay(ts, scene.sh_degree, cams, params, lists)
    tg = [torch.tensor(np.asarray(t, np.float64), dtype=DT) for t in targets]
    loss = loss_fn(imgs, tg)
    loss.backward()
    names = ("means", "log_scales", "quats", "opacity_logits", "sh")
    grads = {n: t.grad.numpy().copy() for n, t in zip(names, ts)}
    return float(loss.detach()), grads, res, [i.detach().numpy() for i in imgs]


def vjp(scene, cams, params, grad_images, tiles=None, workers=1, mask_flagged=False):
    """Vector-Jacobian product of the plain-mode renderer: the gradient of
    sum_v <grad_images[v], I_v> (all four channels) with respect to the raw
    parameters, for the discrete state of the NumPy forward pass.  With
    ``tiles`` ({view: [tile ids]}) only those tiles are shaded and replayed,
    and grad_images is taken as zero elsewhere.  With ``mask_flagged`` it is
    also taken as zero at pixels the forward pass flags as borderline (a
    near-tie that may order or cut differently in another precision).
    Returns (grads dict, forward result dict, the grad_images used)."""
    opts = OracleOptions(record=True, workers=workers, tiles=tiles)
    res = render_full(scene, cams, _plain(cams), params, opts)
    used = []
    for v, gi in enumerate(grad_images):
        gi = np.array(gi, np.float64, copy=True)
        keep = res["valid"][v].copy()
        if mask_flagged:
            keep &= ~res["flags"][v]
        gi[:, ~keep] = 0.0
        used.append(gi)
    grad_images = used
    lists = emission_lists(res, cams)
    ts = [torch.tensor(np.asarray(a, np.float64), dtype=DT, requires_grad=True)
          for a in (scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh)]
    imgs = replay(ts, scene.sh_degree, cams, params, lists)
    total = sum((torch.tensor(np.asarray(gi, np.float64), dtype=DT) * im).sum()
                for gi, im in zip(grad_images, imgs))
    total.backward()
    names = ("means", "log_scales", "quats", "opacity_logits", "sh")
    return {n: t.grad.numpy().copy() for n, t in zip(names, ts)}, res, used


def _plain(cams):
    from synth import fovea_off
    return [fovea_off() for _ in cams]


def loss_numpy(scene, cams, params, targets):
    """The loss from the NumPy forward pass (for central differences)."""
    res = render_full(scene, cams, _plain(cams), params, OracleOptions(record=True))
    imgs = res["images"]
    n = sum(t[:3].size for t in targets)
    l1 = sum(np.abs(i[:3] - t[:3]).sum() for i, t in zip(imgs, targets))
    l2 = sum(((i[:3] - t[:3]) ** 2).sum() for i, t in zip(imgs, targets))
    return l1 / n + 0.2 * l2 / n, res


# ---------------------------------------------------------------------------
# Foveated views: gradients through the HYBRID mix and the periphery's
# nearest-neighbour upsampling and blur (Sec. 4.3).
# ---------------------------------------------------------------------------

def _sample_positions(kind, box, cam):
    """Continuous image positions of a render job's samples, in the order the
    forward pass records them: pixel centres, or for a LOW tile the centres
    (2i + 1, 2j + 1) of its aligned 2x2 groups."""
    x0, y0, x1, y1 = box
    if kind == "low":
        GX, GY = np.meshgrid(np.arange(x0, x1, 2), np.arange(y0, y1, 2))
        return GX.ravel() + 1.0, GY.ravel() + 1.0
    return cam_mod.pixel_centers(x0, y0, x1, y1)


def fov_sample_lists(res, cams):
    """Per view: sample positions (px, py), the emitted Gaussian ids of every
    sample (S, K, -1 padded), and the two linear maps of the foveated
    composition as COO triplets: A (pre-compose pixel <- sample: identity for
    plain and HIGH pixels, w c_p + (1 - w)/n sum of the 2x2 group for HYBRID
    pixels, the group value for the pixels of a LOW group) and B (final pixel
    <- pre-compose pixel: the 3x3 binomial blur, edge-clamped, for LOW
    pixels, identity otherwise)."""
    from . import fovea as fov_mod
    out = []
    for v, cam in enumerate(cams):
        W, H = cam.width, cam.height
        grid = res["grids"][v]
        off = res["view_offsets"][v]
        cls = res["classes"][v]
        pxs, pys, seqs = [], [], []
        ar, ac, av = [], [], []
        for (vv, kind, tile, sub), rec in res["records"].items():
            if vv != v:
                continue
            s, e = res["ranges"][off + tile]
            lst = res["gids"][s:e]
            if kind == "sub":
                tx, ty = tile % grid.ntx, tile // grid.ntx
                bx0, by0 = tx * 32 + (sub % 2) * 16, ty * 32 + (sub // 2) * 16
                box = (bx0, by0, min(bx0 + 16, W), min(by0 + 16, H))
            else:
                box = grid.box(tile)
            px, py = _sample_positions(kind, box, cam)
            base = len(seqs)
            for k, seq in enumerate(rec):
                pxs.append(px[k]); pys.append(py[k])
                seqs.append([int(lst[a]) for a, _ in seq])
            x0, y0, x1, y1 = box
            if kind == "plain":
                for k in range(len(rec)):
                    ly, lx = divmod(k, x1 - x0)
                    ar.append((y0 + ly) * W + (x0 + lx)); ac.append(base + k); av.append(1.0)
                continue
            if kind == "low":
                gw = (x1 - x0 + 1) // 2
                for k in range(len(rec)):
                    gy, gx = divmod(k, gw)
                    for yy in range(y0 + 2 * gy, min(y0 + 2 * gy + 2, y1)):
                        for xx in range(x0 + 2 * gx, min(x0 + 2 * gx + 2, x1)):
                            ar.append(yy * W + xx); ac.append(base + k); av.append(1.0)
                continue
            wd = x1 - x0
            hybrid = kind == "sub" and cls[1][y0 // 16, x0 // 16] == fov_mod.HYBRID
            for k in range(len(rec)):
                ly, lx = divmod(k, wd)
                p = (y0 + ly) * W + (x0 + lx)
                if not hybrid:
                    ar.append(p); ac.append(base + k); av.append(1.0)
                    continue
                w = float(cls[2][y0 + ly, x0 + lx])
                gy0, gx0 = ly // 2 * 2, lx // 2 * 2
                members = [(yy, xx) for yy in range(gy0, min(gy0 + 2, y1 - y0))
                           for xx in range(gx0, min(gx0 + 2, wd))]
                ar.append(p); ac.append(base + k); av.append(w)
                for yy, xx in members:
                    ar.append(p); ac.append(base + yy * wd + xx); av.append((1.0 - w) / len(members))
        K = max([len(sq) for sq in seqs] + [1])
        E = np.full((len(seqs), K), -1, np.int64)
        for i, sq in enumerate(seqs):
            E[i, :len(sq)] = sq
        # B: blur of LOW pixels (none in a plain view).
        if cls is None:
            low = np.zeros((H, W), bool)
        else:
            low = np.repeat(np.repeat(cls[1] == fov_mod.LOW, 16, 0), 16, 1)[:H, :W]
        br, bc, bv = [], [], []
        ys, xs = np.nonzero(~low)
        br += list(ys * W + xs); bc += list(ys * W + xs); bv += [1.0] * len(ys)
        ys, xs = np.nonzero(low)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ny = np.clip(ys + dy, 0, H - 1)
                nx = np.clip(xs + dx, 0, W - 1)
                br += list(ys * W + xs); bc += list(ny * W + nx)
                bv += [float(fov_mod.BLUR[dy + 1, dx + 1])] * len(ys)
        out.append(dict(px=np.asarray(pxs), py=np.asarray(pys), E=E,
                        A=(np.asarray(ar, np.int64), np.asarray(ac, np.int64), np.asarray(av)),
                        B=(np.asarray(br, np.int64), np.asarray(bc, np.int64), np.asarray(bv))))
    return out


def _replay_samples(tensors, sh_degree, cam, params, px, py, E):
    """Differentiable RGBA (S, 4) of samples at continuous positions (px, py)
    blending their recorded Gaussians E (S, K) in order: the arithmetic of
    ``replay`` at arbitrary sample positions."""
    means, log_scales, quats, logits, sh = tensors
    R = quat_to_rotmat_torch(quats)
    s = torch.exp(log_scales).T
    RS = R * s[:, None, :]
    Sigma = RS @ RS.transpose(1, 2)
    sigma = 1.0 / (1.0 + torch.exp(-logits))
    K = (sh_degree + 1) ** 2
    Rv_np, tv_np = cam_mod.rt(cam)
    Rv = torch.tensor(Rv_np, dtype=DT)
    tv = torch.tensor(tv_np, dtype=DT)
    f = float(cam_mod.focal(cam))
    mu_c = means.T @ Rv.T + tv
    Sigma_c = Rv @ Sigma @ Rv.T
    r = torch.linalg.norm(mu_c, dim=1)
    u = mu_c / r[:, None]
    ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
    kk = 1.0 / (1.0 + uz)
    e1 = torch.stack([1 - ux * ux * kk, -ux * uy * kk, -ux], dim=1)
    e2 = torch.stack([-ux * uy * kk, 1 - uy * uy * kk, -uy], dim=1)
    Emat = torch.stack([e1, e2], dim=2)
    S2 = (f * f / (r * r))[:, None, None] * (Emat.transpose(1, 2) @ Sigma_c @ Emat)
    S2 = S2 + float(params.dilation) * torch.eye(2, dtype=DT)[None]
    C = torch.linalg.inv(S2)
    o = torch.tensor(cam_mod.eye_center(cam), dtype=DT)
    vd = means.T - o
    vd = vd / torch.linalg.norm(vd, dim=1, keepdim=True)
    Y = sh_basis_torch(sh_degree, vd)
    col = torch.clamp_min(torch.einsum("nk,kcn->nc", Y, sh[:K]) + 0.5, 0.0)
    bg = torch.tensor(params.background, dtype=DT)
    S = len(px)
    if S == 0:
        return torch.zeros(0, 4, dtype=DT)
    pxt = torch.tensor(px, dtype=DT)
    pyt = torch.tensor(py, dtype=DT)
    d = torch.stack([(pxt - float(cam.cx)) / f, (pyt - float(cam.cy)) / f, torch.ones_like(pxt)], dim=1)
    d = d / torch.linalg.norm(d, dim=1, keepdim=True)
    Et = torch.tensor(E, dtype=torch.long)
    valid = Et >= 0
    g = Et.clamp_min(0)
    dd = d[:, None, :].expand(-1, g.shape[1], -1)
    h = (dd * u[g]).sum(-1)
    q = f * torch.einsum("pki,pkij->pkj", dd, Emat[g]) / h[..., None]
    D2 = torch.einsum("pki,pkij,pkj->pk", q, C[g], q)
    a = torch.minimum(torch.tensor(float(params.alpha_max), dtype=DT), sigma[g] * torch.exp(-0.5 * D2))
    a = torch.where(valid, a, torch.zeros_like(a))
    one_m = 1.0 - a
    T_excl = torch.cumprod(torch.cat([torch.ones(S, 1, dtype=DT), one_m[:, :-1]], dim=1), dim=1)
    Tfin = torch.prod(one_m, dim=1)
    rgb = ((a * T_excl)[..., None] * col[g]).sum(1) + Tfin[:, None] * bg[None]
    return torch.cat([rgb, (1.0 - Tfin)[:, None]], dim=1)


def _apply(coo, x, n_out):
    """y = M x for M given as COO triplets (rows, cols, vals); x (n_in, C)."""
    rows, cols, vals = coo
    y = torch.zeros(n_out, x.shape[1], dtype=DT)
    return y.index_add(0, torch.tensor(rows), x[torch.tensor(cols)] * torch.tensor(vals, dtype=DT)[:, None])


def replay_foveated(tensors, sh_degree, cams, params, lists):
    """Differentiable final images (4, H, W) of foveated views from the raw
    parameters: recorded per-sample blends, then the HYBRID mix / LOW
    upsampling (A) and the periphery blur (B)."""
    imgs = []
    for cam, L in zip(cams, lists):
        s = _replay_samples(tensors, sh_degree, cam, params, L["px"], L["py"], L["E"])
        n = cam.width * cam.height
        pre = _apply(L["A"], s, n)
        fin = _apply(L["B"], pre, n)
        imgs.append(fin.T.reshape(4, cam.height, cam.width))
    return imgs


def vjp_foveated(scene, cams, foveas, params, grad_images, workers=1, mask_flagged=False, masks=None):
    """Vector-Jacobian product of the foveated renderer: the gradient of
    sum_v <grad_images[v], I_v> (final images, all four channels) with
    respect to the raw parameters, for the discrete state of the NumPy
    forward pass.  With ``mask_flagged`` grad_images is taken as zero at
    pixels the forward pass flags as borderline.  Returns (grads, forward
    result, the grad_images used)."""
    opts = OracleOptions(record=True, workers=workers)
    res = render_full(scene, cams, foveas, params, opts, masks=masks)
    used = []
    for v, gi in enumerate(grad_images):
        gi = np.array(gi, np.float64, copy=True)
        if mask_flagged:
            gi[:, res["flags"][v]] = 0.0
        used.append(gi)
    lists = fov_sample_lists(res, cams)
    ts = [torch.tensor(np.asarray(a, np.float64), dtype=DT, requires_grad=True)
          for a in (scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh)]
    imgs = replay_foveated(ts, scene.sh_degree, cams, params, lists)
    total = sum((torch.tensor(gi, dtype=DT) * im).sum() for gi, im in zip(used, imgs))
    total.backward()
    names = ("means", "log_scales", "quats", "opacity_logits", "sh")
    return {n: t.grad.numpy().copy() for n, t in zip(names, ts)}, res, used, [i.detach().numpy() for i in imgs]
