"""Autotuner for multi-view rendering: picks the plain-view sort tile size,
the resort-window length W, the staging batch and the blend schedule for one
configuration (Gaussian count, cameras, foveae) by timing whole frames on
the GPU, and caches the choice in a JSON file.

Two kinds of knob:
  * output-invariant (blend_batch, schedule): only timed;
  * output-changing (tile, window): a candidate must also render images
    close to the reference setting's -- the window length trades residual
    ordering error for speed (Sec. 4.1), and the tile size changes the
    per-tile key depths that order the lists.  The bar is a fraction of
    pixels whose channels differ by more than 1/255 (8-bit display
    precision) from the reference render.

The search is a small grid: every (tile, window) candidate is timed with the
default invariant knobs and screened for quality; the fastest acceptable one
is then timed with every (blend_batch, schedule) pair.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence

import torch

from .render import Gaussians, Renderer

DEFAULT_SPACE = {
    "tile": (16, 32),
    "window": (8, 12, 16),
    "blend_batch": (64, 32),
    "schedule": (0, 1),
}


@dataclasses.dataclass
class TuneResult:
    params: object              # the chosen renderer params (same type as the input)
    ms_per_frame: float
    table: List[dict]           # every timed candidate
    cached: bool = False


def signature(n: int, cams: Sequence, foveas: Sequence, sh_degree: int, space: Dict, ref: Dict,
              max_bad_frac: float) -> str:
    """Cache key: the device, the Gaussian count (2 significant digits), the
    views (size, FoV, foveation) and the search space."""
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    nb = float(f"{n:.2g}")
    views = [(int(c.width), int(c.height), round(float(c.fov_x_deg), 1), bool(f.enabled),
              round(float(f.radius_deg), 1) if f.enabled else 0.0) for c, f in zip(cams, foveas)]
    blob = json.dumps(dict(dev=dev, n=nb, sh=sh_degree, views=views,
                           space={k: list(v) for k, v in sorted(space.items())},
                           ref=ref, bar=max_bad_frac), sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()[:24]


def _load_cache(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path: Optional[str], cache: dict):
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_frames(r: Renderer, g: Gaussians, steps: int, warmup: int = 2) -> float:
    """Mean ms of whole frames (preprocess, sort, blend, compose) on the
    renderer's stream, HIP events around `steps` frames."""
    for _ in range(warmup):
        r.render(g)
    s = r.stream if r.stream is not None else torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        r.render(g)
    e1.record(s)
    torch.cuda.synchronize()
    r.check()
    return e0.elapsed_time(e1) / steps


def bad_fraction(imgs: Sequence[torch.Tensor], ref: Sequence[torch.Tensor], thresh: float = 1.0 / 255.0) -> float:
    bad = total = 0
    for a, b in zip(imgs, ref):
        d = (a - b).abs().amax(dim=0) > thresh
        bad += int(d.sum())
        total += d.numel()
    return bad / max(total, 1)


def _renderer(cams, foveas, params, g: Gaussians, stream=None) -> Renderer:
    r = Renderer(cams, foveas, params, g.n, stream=stream)
    r.ensure_capacity(g)
    return r


def tune(g: Gaussians, cams: Sequence, foveas: Sequence, params, space: Optional[Dict] = None,
         cache_path: Optional[str] = None, steps: int = 5, ref: Optional[Dict] = None,
         max_bad_frac: float = 1e-3, log=None) -> TuneResult:
    """Choose renderer params for these Gaussians and views.  ``params`` gives
    the fixed knobs (thresholds, background); ``space`` the candidate values
    (DEFAULT_SPACE); ``ref`` the reference (tile, window) of the quality bar
    (default tile 16 and the largest window in the space)."""
    space = dict(DEFAULT_SPACE if space is None else space)
    ref = dict(ref or {"tile": 16, "window": max(space["window"])})
    key = signature(g.n, cams, foveas, g.sh_degree, space, ref, max_bad_frac)
    cache = _load_cache(cache_path)
    if key in cache:
        ent = cache[key]
        return TuneResult(params.replace(**ent["choice"]), ent["ms_per_frame"], ent["table"], cached=True)

    say = log or (lambda *a: None)
    base = dict(blend_batch=space["blend_batch"][0], schedule=space["schedule"][0])
    r_ref = _renderer(cams, foveas, params.replace(**ref, **base), g)
    ref_imgs = [im.clone() for im in r_ref.render(g)]
    torch.cuda.synchronize()
    r_ref.check()
    del r_ref
    table = []
    best = None
    for tile in space["tile"]:
        for window in space["window"]:
            p = params.replace(tile=tile, window=window, **base)
            r = _renderer(cams, foveas, p, g)
            imgs = r.render(g)
            torch.cuda.synchronize()
            r.check()
            bad = bad_fraction(imgs, ref_imgs)
            ms = time_frames(r, g, steps)
            ok = bad <= max_bad_frac
            row = dict(tile=tile, window=window, **base, ms=round(ms, 4), bad_frac=bad, accepted=ok)
            table.append(row)
            say(row)
            if ok and (best is None or ms < best[1]):
                best = (dict(tile=tile, window=window), ms)
            del r
            torch.cuda.empty_cache()
    if best is None:  # nothing but the reference passes: keep it
        best = (dict(ref), float("inf"))
    choice, best_ms = dict(best[0], **base), best[1]
    for bb in space["blend_batch"]:
        for sc in space["schedule"]:
            if dict(blend_batch=bb, schedule=sc) == base:
                continue
            p = params.replace(**best[0], blend_batch=bb, schedule=sc)
            r = _renderer(cams, foveas, p, g)
            ms = time_frames(r, g, steps)
            row = dict(**best[0], blend_batch=bb, schedule=sc, ms=round(ms, 4), bad_frac=None, accepted=True)
            table.append(row)
            say(row)
            if ms < best_ms:
                choice, best_ms = dict(best[0], blend_batch=bb, schedule=sc), ms
            del r
            torch.cuda.empty_cache()
    cache[key] = dict(choice=choice, ms_per_frame=best_ms, table=table, when=time.strftime("%Y-%m-%d %H:%M:%S"))
    _store_cache(cache_path, cache)
    return TuneResult(params.replace(**choice), best_ms, table)
