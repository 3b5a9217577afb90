"""The whole forward pass of the foveated tile rasterizer in FP64.  Test
infrastructure only.

Order of steps (Sec. 3 tile pipeline, Sec. 4.1-4.3):
1. per view, per Gaussian: camera transform, near cull, covariance (Eq. 1),
   Optimal Projection (2D conic on the tangent plane), view-dependent colour;
2. Gaussian/tile instances with the tangent-plane tile-culling test (Eq. 4),
   per-tile depth at the back-projected maximum point, keys;
3. sort by (key, Gaussian id) and tile ranges;
4. per tile (or 16x16 subtile, or LOW tile at half resolution): windowed
   per-sample resorting and front-to-back blending (Eq. 2);
5. foveated mode: hybrid blending, nearest-neighbour upsampling and 3x3 blur
   of the periphery (Sec. 4.3).

Readings shared with the other modules: the near cull drops a Gaussian from a
view when its camera-space z <= z_near; there is no other frustum test (tile
footprints decide everything), which keeps the App. D large-FoV crop exact.
A Gaussian whose opacity is below alpha_min is dropped too (it can never pass).

Borderline flags: a sample is flagged when a discrete decision touching it is
closer to its threshold than FP32 arithmetic can resolve (see ``BlendFlags``),
or when two adjacent list entries that both reach alpha_min at it carry float32
depths at most one ulp apart (their arrival order may differ in FP32).  The
flags propagate through the 2x2 group mean and the 3x3 blur.
"""
import dataclasses
import math
import multiprocessing as mp
import os
import time
from typing import Dict, List, Optional

import numpy as np

from . import blend as blend_mod
from . import camera as cam_mod
from . import fovea as fov_mod
from . import gaussian as g_mod
from . import projection as proj_mod
from . import sh as sh_mod
from . import tiles as tiles_mod


@dataclasses.dataclass
class OracleOptions:
    exhaustive_tiles: bool = False        # test every tile, no cone bound
    flags: Optional[blend_mod.BlendFlags] = dataclasses.field(default_factory=blend_mod.BlendFlags)
    tiles: Optional[Dict[int, List[int]]] = None  # view -> sort-grid tiles to shade (sampled mode)
    workers: int = 1
    record: bool = False
    eps_inst: float = 1e-9                # |ln alpha_hat - ln alpha_min| for instance flags
    shade: bool = True                    # False: stop after keys and ranges
    alternatives: bool = False            # enumerate admissible outcomes of flagged samples
    alt_cap: int = 256                    # most outcomes enumerated per sample or 2x2 group
    alt_flips: int = 3                    # most decisions against FP64 on an enumerated path


def preprocess_view(scene, cam, params):
    """Step 1 for one view.  Returns a dict of FP64 arrays over all N (rows of
    culled Gaussians are present but ``valid`` is False)."""
    N = scene.n
    mu = scene.means.astype(np.float64).T
    R_v, t_v = cam_mod.rt(cam)
    f = cam_mod.focal(cam)
    mu_c = mu @ R_v.T + t_v
    sigma = g_mod.opacity(scene.opacity_logits)
    valid = (mu_c[:, 2] > np.float64(params.z_near)) & (sigma >= np.float64(params.alpha_min))
    Sigma = g_mod.covariance(scene.quats, scene.log_scales)
    Sigma_c = R_v[None] @ Sigma @ R_v.T[None]
    # Guard culled rows against division by zero; they are never used.
    mu_safe = np.where(valid[:, None], mu_c, np.array([0.0, 0.0, 1.0]))
    op = proj_mod.optimal_projection(mu_safe, Sigma_c, f, np.float64(params.dilation))
    o = cam_mod.eye_center(cam)
    v = mu - o
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    color, color_raw = sh_mod.sh_color(scene.sh, scene.sh_degree, v)
    B = np.linalg.inv(Sigma_c)
    x0 = np.float64(cam.cx) + f * mu_safe[:, 0] / mu_safe[:, 2]
    y0 = np.float64(cam.cy) + f * mu_safe[:, 1] / mu_safe[:, 2]
    S2 = op["Sigma2D"]
    tr2 = 0.5 * (S2[:, 0, 0] + S2[:, 1, 1])
    lam_max = tr2 + np.sqrt(np.maximum(0.25 * (S2[:, 0, 0] - S2[:, 1, 1]) ** 2 + S2[:, 0, 1] ** 2, 0))
    with np.errstate(divide="ignore"):
        kappa = np.where(valid, 2.0 * np.log(np.maximum(sigma, 1e-300) / np.float64(params.alpha_min)), 0.0)
    return dict(valid=valid, mu_c=mu_safe, r=op["r"], u=op["u"], E=op["E"],
                Sigma_c=Sigma_c, B=B, Sigma2D=S2, C=op["conic"], sigma=sigma,
                color=color, color_raw=color_raw, x0=x0, y0=y0, kappa=kappa,
                lam_max=lam_max, f=f, near_gap=mu_c[:, 2] - np.float64(params.z_near))


def _candidates(pre, cam, grid, opts, tile_subset=None, visible=None):
    gid = np.flatnonzero(pre["valid"])
    if opts.exhaustive_tiles:
        tiles = np.arange(grid.n)
        if tile_subset is not None:
            tiles = np.intersect1d(tiles, tile_subset)
        G = np.repeat(gid, len(tiles))
        Tt = np.tile(tiles, len(gid))
        return G, Tt
    tx0, tx1, ty0, ty1 = tiles_mod.cone_tile_bounds(
        pre["u"][gid], pre["lam_max"][gid], pre["kappa"][gid], pre["f"], cam, grid)
    nx = np.maximum(tx1 - tx0 + 1, 0)
    ny = np.maximum(ty1 - ty0 + 1, 0)
    cnt = nx * ny
    G = np.repeat(gid, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    k = np.arange(len(G)) - start
    nxr = np.repeat(nx, cnt)
    Tt = (np.repeat(ty0, cnt) + k // np.maximum(nxr, 1)) * grid.ntx + np.repeat(tx0, cnt) + k % np.maximum(nxr, 1)
    if tile_subset is not None:
        keep = np.isin(Tt, tile_subset)
        G, Tt = G[keep], Tt[keep]
    if visible is not None:
        keep = visible[Tt]
        G, Tt = G[keep], Tt[keep]
    return G, Tt


def instances_view(pre, cam, grid, params, opts, tile_subset=None, chunk=400_000, visible=None):
    """Step 2 for one view: kept (tile, gid, depth) plus borderline flags.
    ``visible`` (bool per tile, or None) restricts instances to visible tiles
    (visibility culling, Sec. 4.3).  The key depth is the per-tile depth at
    the maximum point (params.depth 0, Sec. 4.2), or one depth per Gaussian:
    view-space z (1) or the distance from the eye (2), the orders of the
    Mini-Splatting (z) and (Dist) comparison renderers (Sec. 5)."""
    G, Tt = _candidates(pre, cam, grid, opts, tile_subset, visible)
    out_t, out_g, out_d, out_b, out_D2 = [], [], [], [], []
    f = pre["f"]
    ln_amin = math.log(np.float64(params.alpha_min))
    for s in range(0, len(G), chunk):
        g = G[s:s + chunk]
        t = Tt[s:s + chunk]
        bx0, by0, bx1, by1 = grid.boxes(t)
        res = tiles_mod.quad_test(cam, f, pre["u"][g], pre["E"][g], pre["C"][g],
                                  pre["x0"][g], pre["y0"][g], bx0, by0, bx1, by1)
        D2 = res["D2min"]
        lnah = np.log(pre["sigma"][g]) - 0.5 * D2
        keep = lnah >= ln_amin
        border = np.abs(lnah - ln_amin) < opts.eps_inst
        mode = int(getattr(params, "depth", 0))
        if mode == 0:
            dep = tiles_mod.tile_depth(pre["u"][g], pre["E"][g], f, res["qhat"], pre["mu_c"][g], pre["B"][g])
        elif mode == 1:
            dep = pre["mu_c"][g, 2]          # view-space z of the mean
        else:
            dep = pre["r"][g]                # distance from the eye to the mean
        out_t.append(t[keep]); out_g.append(g[keep]); out_d.append(dep[keep])
        out_b.append(border[keep]); out_D2.append(D2[keep])
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return dict(tile=cat(out_t, np.int64), gid=cat(out_g, np.int64), depth=cat(out_d, np.float64),
                border=cat(out_b, bool), D2=cat(out_D2, np.float64))


def _alpha_fn(pre, g, cam, rays, params):
    """alpha_raw and ln(sigma G) of Gaussian g at unit rays (S, 3)."""
    q, h = proj_mod.tangent_coords(rays, pre["u"][g], pre["E"][g], pre["f"])
    D2 = np.einsum("si,ij,sj->s", q, pre["C"][g], q)
    lnag = math.log(pre["sigma"][g]) - 0.5 * D2
    lnag = np.where(h > 0, lnag, -np.inf)
    a = np.minimum(np.float64(params.alpha_max), np.exp(lnag))
    return a, lnag


def shade_samples(pre, cam, params, rays, entries_g, amb, opts):
    """Step 4 for one list of Gaussian ids and a set of sample rays."""
    B = pre["B"]
    mu_c = pre["mu_c"]

    def gen():
        for i, g in enumerate(entries_g):
            a, lnag = _alpha_fn(pre, g, cam, rays, params)

            def tfn(m, g=g):
                d = rays[m]
                Bd = d @ B[g]
                return (Bd @ mu_c[g]) / np.einsum("si,si->s", Bd, d)
            yield a, lnag, tfn, pre["color"][g], bool(amb[i]) if len(amb) else False

    return blend_mod.window_blend(len(rays), gen(), int(params.window),
                                  np.float64(params.alpha_min), np.float64(params.t_min),
                                  opts.flags, opts.record)


def sample_alternatives(pre, cam, params, rays, entries_g, amb, samples, opts, chunk=16):
    """Admissible outcomes of the given (flagged) samples: for each, a pair
    (list of (rgba (4,), flips), complete) from ``blend.sample_outcomes`` over
    the entries of its list that might reach alpha_min, following paths with
    at most ``opts.alt_flips`` decisions against FP64 (fewer if that gives
    more than ``opts.alt_cap`` outcomes), or None if even one such decision
    gives too many."""
    out = {}
    g = np.asarray(entries_g, np.int64)
    if len(samples) == 0:
        return out
    ln_amin = math.log(np.float64(params.alpha_min))
    margin = opts.flags.eps_alpha * 1.5
    bg = np.asarray(params.background, np.float64)
    amb = np.asarray(amb, bool) if len(amb) else np.zeros(len(g), bool)
    u, E, Cc = pre["u"][g], pre["E"][g], pre["C"][g]
    lns = np.log(pre["sigma"][g])
    for s0 in range(0, len(samples), chunk):
        ss = np.asarray(samples[s0:s0 + chunk])
        d = rays[ss]                                             # (S, 3)
        h = d @ u.T                                              # (S, n)
        q = pre["f"] * np.einsum("si,nik->snk", d, E) / h[..., None]
        D2 = np.einsum("snk,nkl,snl->sn", q, Cc, q)
        lnag = np.where(h > 0, lns[None] - 0.5 * D2, -np.inf)
        for r, s in enumerate(ss):
            cand = np.flatnonzero(lnag[r] >= ln_amin - margin)
            gc = g[cand]
            la = lnag[r, cand]
            al = np.minimum(np.float64(params.alpha_max), np.exp(la))
            Bd = np.einsum("i,nij->nj", d[r], pre["B"][gc])
            ts = np.einsum("nj,nj->n", Bd, pre["mu_c"][gc]) / (Bd @ d[r])
            # amb between candidates k and k+1 only if they are neighbours in the list.
            ab = np.zeros(len(cand), bool)
            if len(cand) > 1:
                ab[:-1] = (cand[1:] == cand[:-1] + 1) & amb[cand[:-1]]
            res = None
            for mf in range(opts.alt_flips, 0, -1):
                try:
                    res = blend_mod.sample_outcomes(al, la, ts, pre["color"][gc], ab, int(params.window),
                                                    np.float64(params.alpha_min), np.float64(params.t_min),
                                                    opts.flags, opts.alt_cap, max_flips=mf)
                    break
                except blend_mod.TooManyOutcomes:
                    continue
            if res is None:
                out[int(s)] = None
                continue
            leaves, complete = res
            out[int(s)] = ([(np.r_[C + T * bg, 1.0 - T], flips) for C, T, flips in leaves], complete)
    return out


_WORK = {}


def _shade_job(job):
    v, kind, tile, sub = job
    st = _WORK
    cam = st["cams"][v]
    pre = st["pre"][v]
    params = st["params"]
    opts = st["opts"]
    grid = st["grids"][v]
    lst = st["lists"][v].get(tile, (np.zeros(0, np.int64), np.zeros(0, bool)))
    g_list, amb = lst
    W, H = cam.width, cam.height
    if kind == "plain":
        x0, y0, x1, y1 = grid.box(tile)
        px, py = cam_mod.pixel_centers(x0, y0, x1, y1)
    elif kind == "low":
        x0, y0, x1, y1 = grid.box(tile)
        gx = np.arange(x0, x1, 2)
        gy = np.arange(y0, y1, 2)
        GX, GY = np.meshgrid(gx, gy)
        px, py = GX.ravel() + 1.0, GY.ravel() + 1.0
    else:
        tx, ty = tile % grid.ntx, tile // grid.ntx
        x0 = tx * 32 + (sub % 2) * 16
        y0 = ty * 32 + (sub // 2) * 16
        x1, y1 = min(x0 + 16, W), min(y0 + 16, H)
        px, py = cam_mod.pixel_centers(x0, y0, x1, y1)
    rays = cam_mod.ray_dirs(cam, px, py)
    C, T, fl, stats, rec = shade_samples(pre, cam, params, rays, g_list, amb, opts)
    bg = np.asarray(params.background, np.float64)
    rgb = C + T[:, None] * bg[None]
    rgba = np.concatenate([rgb, (1.0 - T)[:, None]], axis=1)
    alts = None
    if opts.alternatives and opts.flags is not None:
        alts = sample_alternatives(pre, cam, params, rays, g_list, amb, np.flatnonzero(fl), opts)
    return (v, kind, tile, sub, (x0, y0, x1, y1), rgba, fl, stats, rec, alts)


def _place_alts(alts, unchecked, salts, pixels_of):
    """Record the admissible outcomes of flagged samples at the pre-image
    pixels each sample writes."""
    for s, res in salts.items():
        for yx in pixels_of(s):
            if res is None:
                unchecked[yx] = True
            else:
                leaves, complete = res
                alts[yx] = (np.array([r for r, _ in leaves]), [f for _, f in leaves], complete)


def _hybrid_alts(alts, unchecked, salts, base, wmask, x0, y0, x1, y1, cam, cap, max_flips):
    """Admissible HYBRID pre-image values: the combinations of the admissible
    outcomes of the samples of a 2x2 group (with at most ``max_flips``
    decisions against FP64 over the group), mixed as the HYBRID rule mixes
    them."""
    wd = x1 - x0
    groups = {}
    for s in salts:
        ly, lx = divmod(s, wd)
        groups.setdefault((ly // 2 * 2, lx // 2 * 2), []).append(s)
    for (gy, gx), _ in groups.items():
        ys = range(gy, min(gy + 2, y1 - y0))
        xs = range(gx, min(gx + 2, wd))
        members = [(ly, lx) for ly in ys for lx in xs]
        pix = [(y0 + ly, x0 + lx) for ly, lx in members]
        opts_per = []
        complete = True
        bad = False
        for ly, lx in members:
            s = ly * wd + lx
            if s in salts:
                if salts[s] is None:
                    bad = True
                    break
                leaves, comp = salts[s]
                opts_per.append(leaves)
                complete = complete and comp
            else:
                opts_per.append([(base[:, ly, lx], ())])
        if bad:
            for yx in pix:
                unchecked[yx] = True
            continue
        combos = []

        def walk(k, chosen, used):
            nonlocal complete
            if len(combos) > cap:
                return
            if k == len(opts_per):
                combos.append(list(chosen))
                return
            for r, fl in opts_per[k]:
                if used + len(fl) > max_flips:
                    complete = False
                    continue
                chosen.append((r, fl))
                walk(k + 1, chosen, used + len(fl))
                chosen.pop()

        walk(0, [], 0)
        if len(combos) > cap:
            for yx in pix:
                unchecked[yx] = True
            continue
        vals = {yx: [] for yx in pix}
        flips = {yx: [] for yx in pix}
        w = wmask[y0 + gy:y0 + gy + len(ys), x0 + gx:x0 + gx + len(xs)]
        for combo in combos:
            grp = np.empty((4, len(ys), len(xs)))
            for (ly, lx), (r, _) in zip(members, combo):
                grp[:, ly - gy, lx - gx] = r
            mixed = fov_mod.hybrid_mix(grp, w, x0 + gx, y0 + gy, cam.width, cam.height)
            fl = tuple(f for _, fs in combo for f in fs)
            for (ly, lx), yx in zip(members, pix):
                vals[yx].append(mixed[:, ly - gy, lx - gx])
                flips[yx].append(fl)
        for yx in pix:
            alts[yx] = (np.array(vals[yx]), flips[yx], complete)


def render(scene, cams, foveas, params, opts: Optional[OracleOptions] = None, masks=None):
    """Full forward pass.  ``foveas`` is one Fovea per view (or a single Fovea
    for all views); foveated views use 32x32 sort tiles, plain views use
    ``params.tile``.  ``masks`` optionally gives per view a visibility mask
    (uint8 [H][W], nonzero = visible, or None): instances in tiles without a
    visible pixel are culled (Sec. 4.3).  Returns a dict with per-view images
    (4, H, W) (NaN where not shaded in sampled mode), per-pixel flags,
    instance data, sorted keys/gids, ranges and counters."""
    from . import visibility as vis_mod
    opts = opts or OracleOptions()
    if not isinstance(foveas, (list, tuple)):
        foveas = [foveas] * len(cams)
    V = len(cams)
    masks = list(masks) if masks is not None else [None] * V
    vis_bits = []
    t_start = time.perf_counter()
    pres, grids, insts, offs = [], [], [], []
    off = 0
    for v, cam in enumerate(cams):
        pre = preprocess_view(scene, cam, params)
        T = 32 if foveas[v].enabled else int(params.tile)
        grid = tiles_mod.TileGrid(cam.width, cam.height, T)
        subset = None
        if opts.tiles is not None:
            want = np.asarray(opts.tiles.get(v, []), np.int64)
            if foveas[v].enabled and len(want):
                # LOW pixels blur across tile borders: shade the neighbours too.
                tx, ty = want % grid.ntx, want // grid.ntx
                nb = []
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        ok = (tx + dx >= 0) & (tx + dx < grid.ntx) & (ty + dy >= 0) & (ty + dy < grid.nty)
                        nb.append(((ty + dy) * grid.ntx + tx + dx)[ok])
                want = np.unique(np.concatenate(nb))
            subset = want
        vbits = vis_mod.tile_bits(masks[v], T) if masks[v] is not None else None
        vis_bits.append(vbits)
        inst = instances_view(pre, cam, grid, params, opts, subset,
                              visible=vbits.ravel() if vbits is not None else None)
        pres.append(pre); grids.append(grid); insts.append((inst, subset))
        offs.append(off)
        off += grid.n
    # Step 3: keys over all views, sort, ranges.
    all_tile = np.concatenate([insts[v][0]["tile"] + offs[v] for v in range(V)]) if V else np.zeros(0, np.int64)
    all_gid = np.concatenate([insts[v][0]["gid"] for v in range(V)]) if V else np.zeros(0, np.int64)
    all_dep = np.concatenate([insts[v][0]["depth"] for v in range(V)]) if V else np.zeros(0)
    all_border = np.concatenate([insts[v][0]["border"] for v in range(V)]) if V else np.zeros(0, bool)
    keys = tiles_mod.make_keys(all_tile, all_dep)
    order = np.lexsort((all_gid, keys))
    skeys, sgids = keys[order], all_gid[order]
    sdep = all_dep[order]
    ranges = tiles_mod.tile_ranges(skeys, off)
    # Adjacent entries whose float32 depths are within one ulp: ambiguous order.
    bits = tiles_mod.ord_f32(sdep).astype(np.int64)
    stile = (skeys >> np.uint64(32)).astype(np.int64)
    amb_next = np.zeros(len(skeys), bool)
    if len(skeys) > 1:
        amb_next[:-1] = (stile[1:] == stile[:-1]) & (np.abs(bits[1:] - bits[:-1]) <= 1) & (sgids[1:] != sgids[:-1])
    lists = []
    for v in range(V):
        d = {}
        lo, hi = offs[v], offs[v] + grids[v].n
        tiles_here = np.unique(stile[(stile >= lo) & (stile < hi)])
        for gt in tiles_here:
            s, e = ranges[gt]
            d[int(gt - lo)] = (sgids[s:e], amb_next[s:e])
        lists.append(d)

    t_keys = time.perf_counter() - t_start
    if not opts.shade:
        return dict(pre=pres, grids=grids, view_offsets=offs, n_tiles=off, inst_tile=all_tile, vis_bits=vis_bits,
                    inst_gid=all_gid, inst_depth=all_dep, inst_border=all_border, keys=skeys,
                    gids=sgids, depths=sdep, ranges=ranges,
                    stats=dict(n_inst=int(len(skeys)), t_keys=t_keys))
    # Step 4: shading jobs.
    jobs = []
    classes = []
    for v, cam in enumerate(cams):
        grid = grids[v]
        sel = insts[v][1]
        tiles_v = range(grid.n) if sel is None else sel.tolist()
        if foveas[v].enabled:
            split, sub, wmask = fov_mod.classify(cam, foveas[v])
            classes.append((split, sub, wmask))
            for t in tiles_v:
                tx, ty = t % grid.ntx, t // grid.ntx
                if not split[ty, tx]:
                    jobs.append((v, "low", t, -1))
                else:
                    for s in range(4):
                        sx, sy = 2 * tx + s % 2, 2 * ty + s // 2
                        if sub[sy, sx] >= 0:
                            jobs.append((v, "sub", t, s))
        else:
            classes.append(None)
            for t in tiles_v:
                jobs.append((v, "plain", t, -1))

    global _WORK
    t_shade0 = time.perf_counter()
    _WORK = dict(cams=cams, pre=pres, params=params, opts=opts, grids=grids, lists=lists)
    if opts.workers > 1 and len(jobs) > 1:
        ctx = mp.get_context("fork")
        with ctx.Pool(opts.workers) as pool:
            results = pool.map(_shade_job, jobs, chunksize=max(1, len(jobs) // (opts.workers * 8)))
    else:
        results = [_shade_job(j) for j in jobs]
    _WORK = {}
    t_shade = time.perf_counter() - t_shade0

    # Step 5: assemble and compose.
    images, flagged, shaded = [], [], []
    bits, alts, unchecked = [], [], []
    stats = dict(pairs=0, contrib=0, stopped=0, samples=0, jobs=len(jobs), t_keys=t_keys,
                 t_shade=t_shade)
    recs = {}
    for v, cam in enumerate(cams):
        images.append(np.full((4, cam.height, cam.width), np.nan))
        flagged.append(np.zeros((cam.height, cam.width), bool))
        shaded.append(np.zeros((cam.height, cam.width), bool))
        bits.append(np.zeros((cam.height, cam.width), np.uint8))
        alts.append({})
        unchecked.append(np.zeros((cam.height, cam.width), bool))
    for (v, kind, tile, sub, box, rgba, fl, st, rec, salts) in results:
        x0, y0, x1, y1 = box
        img, flg = images[v], flagged[v]
        for k in ("pairs", "contrib", "stopped"):
            stats[k] += st[k]
        stats["samples"] += len(fl)
        if rec is not None:
            recs[(v, kind, tile, sub)] = rec
        fb = fl.astype(np.uint8)
        fl = fl != 0
        if kind == "plain":
            img[:, y0:y1, x0:x1] = rgba.T.reshape(4, y1 - y0, x1 - x0)
            flg[y0:y1, x0:x1] = fl.reshape(y1 - y0, x1 - x0)
            bits[v][y0:y1, x0:x1] = fb.reshape(y1 - y0, x1 - x0)
            if salts is not None:
                _place_alts(alts[v], unchecked[v], salts, lambda s: [(y0 + s // (x1 - x0), x0 + s % (x1 - x0))])
        elif kind == "low":
            gw = (x1 - x0 + 1) // 2
            gh = (y1 - y0 + 1) // 2
            vals = rgba.T.reshape(4, gh, gw)
            fg = fl.reshape(gh, gw)
            up = np.repeat(np.repeat(vals, 2, axis=1), 2, axis=2)[:, :y1 - y0, :x1 - x0]
            fu = np.repeat(np.repeat(fg, 2, axis=0), 2, axis=1)[:y1 - y0, :x1 - x0]
            bu = np.repeat(np.repeat(fb.reshape(gh, gw), 2, axis=0), 2, axis=1)[:y1 - y0, :x1 - x0]
            img[:, y0:y1, x0:x1] = up
            flg[y0:y1, x0:x1] = fu
            bits[v][y0:y1, x0:x1] = bu
            if salts is not None:
                def pix(s, gw=gw, x0=x0, y0=y0, x1=x1, y1=y1):
                    gy, gx = divmod(s, gw)
                    return [(y, x) for y in range(y0 + 2 * gy, min(y0 + 2 * gy + 2, y1))
                            for x in range(x0 + 2 * gx, min(x0 + 2 * gx + 2, x1))]
                _place_alts(alts[v], unchecked[v], salts, pix)
        else:
            split, subc, wmask = classes[v]
            base = rgba.T.reshape(4, y1 - y0, x1 - x0)
            f2 = fl.reshape(y1 - y0, x1 - x0)
            b2 = fb.reshape(y1 - y0, x1 - x0)
            hybrid = subc[y0 // 16, x0 // 16] == fov_mod.HYBRID
            vals = base
            if hybrid:
                vals = fov_mod.hybrid_mix(base, wmask[y0:y1, x0:x1], x0, y0, cam.width, cam.height)
                # A flagged pixel taints its whole 2x2 group.
                g = np.zeros_like(f2)
                gb = np.zeros_like(b2)
                for gy in range(0, f2.shape[0], 2):
                    for gx in range(0, f2.shape[1], 2):
                        g[gy:gy + 2, gx:gx + 2] = f2[gy:gy + 2, gx:gx + 2].any()
                        gb[gy:gy + 2, gx:gx + 2] = np.bitwise_or.reduce(b2[gy:gy + 2, gx:gx + 2].ravel())
                f2, b2 = g, gb
            img[:, y0:y1, x0:x1] = vals
            flg[y0:y1, x0:x1] = f2
            bits[v][y0:y1, x0:x1] = b2
            if salts is not None:
                wd = x1 - x0
                if not hybrid:
                    _place_alts(alts[v], unchecked[v], salts, lambda s: [(y0 + s // wd, x0 + s % wd)])
                else:
                    _hybrid_alts(alts[v], unchecked[v], salts, base, wmask, x0, y0, x1, y1, cam, opts.alt_cap,
                                 opts.alt_flips)
        shaded[v][y0:y1, x0:x1] = True

    finals, fflags, valid_px = [], [], []
    for v, cam in enumerate(cams):
        if foveas[v].enabled:
            split, subc, wmask = classes[v]
            low = np.repeat(np.repeat(subc == fov_mod.LOW, 16, axis=0), 16, axis=1)[:cam.height, :cam.width]
            pre_img = images[v]
            low_ok = low & shaded[v]
            out = fov_mod.blur_low(np.nan_to_num(pre_img, nan=0.0), low_ok)
            # A blurred pixel is valid only if its whole 3x3 neighbourhood was shaded.
            H, W = cam.height, cam.width
            nbr_ok = np.ones((H, W), bool)
            nbr_fl = np.zeros((H, W), bool)
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    ys = np.clip(np.arange(H) + dy, 0, H - 1)
                    xs = np.clip(np.arange(W) + dx, 0, W - 1)
                    nbr_ok &= shaded[v][np.ix_(ys, xs)]
                    nbr_fl |= flagged[v][np.ix_(ys, xs)]
            valid = shaded[v] & (~low | nbr_ok)
            fl = np.where(low, nbr_fl, flagged[v])
            out[:, ~valid] = np.nan
            finals.append(out); fflags.append(fl & valid); valid_px.append(valid)
        else:
            finals.append(images[v]); fflags.append(flagged[v]); valid_px.append(shaded[v])
    if opts.tiles is not None:
        # Report only the requested tiles.
        for v, cam in enumerate(cams):
            want = opts.tiles.get(v, [])
            m = np.zeros((cam.height, cam.width), bool)
            for t in want:
                x0, y0, x1, y1 = grids[v].box(t)
                m[y0:y1, x0:x1] = True
            valid_px[v] = valid_px[v] & m
            finals[v][:, ~valid_px[v]] = np.nan
            fflags[v] = fflags[v] & valid_px[v]
    stats["n_inst"] = int(len(skeys))
    stats["n_inst_border"] = int(all_border.sum())
    return dict(images=finals, pre_images=images, flags=fflags, valid=valid_px,
                pre_flags=flagged, pre_flag_bits=bits, pre_alts=alts, pre_unchecked=unchecked, vis_bits=vis_bits,
                shaded=shaded,
                pre=pres, grids=grids, view_offsets=offs, n_tiles=off,
                inst_tile=all_tile, inst_gid=all_gid, inst_depth=all_dep,
                inst_border=all_border, keys=skeys, gids=sgids, depths=sdep,
                ranges=ranges, classes=classes, stats=stats, records=recs)
