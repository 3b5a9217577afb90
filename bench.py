#!/usr/bin/env python
"""Benchmark of the foveated stereo Gaussian-splat renderer on one MI355X.

Workload: 500,000 synthetic Gaussians (64 anisotropic clusters + a ground
slab, log-scales N(-5, 0.7), SH degree 3) rendered to two eyes of
2064x2208 (110-degree FoV, 64 mm baseline), foveated with a 15-degree focus
radius and a half-resolution periphery in one launch, resort window 16.

A step is one whole stereo frame of the hot path -- preprocess, instance
keys, radix sort, tile ranges, single-launch blending and periphery compose
for both eyes -- starting from Gaussians resident in HBM and ending with both
RGBA images in HBM.  The foveation plan is built once per eye configuration
before timing (the paper precomputes it and reuses it across frames).

Prints one JSON line (value = stereo frames per second).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stereo frames/sec at 2064×2208/eye foveated (500k G); fwd+bwd ms/view"

# Algorithmic VALU lane-operations of the blending kernel:
# every evaluated (sample, entry) pair runs the alpha test; every pair whose
# alpha reaches alpha_min also evaluates alpha, the ray depth, the window
# insertion (11 per window slot + 5) and the blend.
OPS_PER_PAIR = 15
def ops_per_contrib(window):
    return 33 + 11 * window

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one FP32 VALU lane-op each.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--window", type=int, default=16)
    ap.add_argument("--schedule", type=int, default=0, help="blend schedule: 0 one block per item, 1 persistent")
    ap.add_argument("--blend-batch", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-diff", action="store_true", help="skip the fwd+bwd leg")
    ap.add_argument("--diff-steps", type=int, default=10)
    ap.add_argument("--diff-only", action="store_true", help="run only the fwd+bwd leg (for profiling)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched multi-view leg")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched multi-view leg")
    ap.add_argument("--batch-knobs", default=None,
                    help="tile,window,blend_batch,schedule for the batch leg instead of the autotuner's choice")
    ap.add_argument("--no-unpruned", action="store_true", help="skip the 3M-Gaussian yaw-arc leg")
    ap.add_argument("--unpruned-only", action="store_true", help="run only the 3M-Gaussian yaw-arc leg")
    ap.add_argument("--cpu-tiles", type=int, default=24, help="32x32 tiles per eye in the CPU sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def copy_probe():
    """A plain copy of exactly 1 GiB, three times: the reference that scales
    the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    x = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 4, "copies": 3}), flush=True)


def traffic_for(kernel_key):
    """HBM bytes per launch measured with rocprofv3 counters, if the kernel's
    source is unchanged since the measurement (else None)."""
    path = os.path.join(ROOT, "profiles", "blend_stereo_traffic.txt")
    src = os.path.join(ROOT, "paper_2505_10144_amd", "csrc", "render.hip")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if vals.get("render_hip_sha256") != sha or vals.get("kernel") != kernel_key:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(scene, cams, fovs, params, n_items, tiles_per_eye):
    """The FP64 oracle on this host: the full preprocess + instance + sort
    pass for both eyes, plus shading of a random sample of 32x32 tiles (and
    their blur neighbours), scaled to the whole frame by the number of render
    work items."""
    import numpy as np
    import oracle
    from oracle.render import OracleOptions
    cores = min(16, os.cpu_count() or 1)
    full = oracle.render(scene, cams, fovs, params, OracleOptions(shade=False))
    t_keys = full["stats"]["t_keys"]
    rng = np.random.default_rng(12345)
    ntiles = full["grids"][0].n
    sel = {v: sorted(rng.choice(ntiles, tiles_per_eye, replace=False).tolist()) for v in range(len(cams))}
    samp = oracle.render(scene, cams, fovs, params, OracleOptions(tiles=sel, workers=cores))
    jobs = samp["stats"]["jobs"]
    t_shade = samp["stats"]["t_shade"] * (n_items / max(jobs, 1))
    sec = t_keys + t_shade
    return {
        "value": 1.0 / sec, "unit": "stereo frames/s", "cores": cores, "kind": "oracle",
        "sample": (f"FP64 NumPy oracle: full preprocess+instances+sort of both eyes ({t_keys:.1f} s) plus "
                   f"shading of {jobs} of {n_items} work items ({2 * tiles_per_eye} random 32x32 tiles "
                   f"with blur neighbours, {samp['stats']['t_shade']:.1f} s on {cores} processes), "
                   f"scaled to the frame: {sec:.0f} s per stereo frame"),
    }


def diff_leg(steps, warmup):
    """fwd+bwd ms per view of the differentiable form: 1M cluster Gaussians,
    4 plain views at 1024^2, 90-degree FoV.  The upstream gradient is that
    of L1 + 0.2 L2 against targets rendered (by this renderer) from the
    scene with perturbed means and opacities; it is computed once before
    timing (the parameters do not change between timed steps).  A step is
    one forward render of the 4 views plus vrs_render_backward."""
    import torch
    import synth
    from paper_2505_10144_amd.render import Renderer, upload
    scene, pert, cams, params = synth.config_diff(0)
    fovs = [synth.fovea_off()] * len(cams)
    r = Renderer(cams, fovs, params, scene.n)
    gp = upload(pert)
    r.ensure_capacity(gp)
    targets = [im.clone() for im in r.render(gp)]
    g = upload(scene)
    r.ensure_capacity(g)
    imgs = r.render(g)
    n = sum(t[:3].numel() for t in targets)
    dI = []
    for i, t in zip(imgs, targets):
        d = torch.zeros_like(i)
        diff = i[:3] - t[:3]
        d[:3] = (torch.sign(diff) + 0.4 * diff) / n
        dI.append(d)
    for _ in range(warmup):
        r.render(g)
        r.backward(g, dI)
    torch.cuda.synchronize()
    r.check()
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        r.render(g)
        ev[k][1].record(stream)
        r.backward(g, dI)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r.check()
    V = len(cams)
    fwd = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    bwd = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    ms = (t1 - t0) * 1000.0 / steps
    return {"ms_per_view": round(ms / V, 4), "fwd_ms_per_view": round(fwd / V, 4),
            "bwd_ms_per_view": round(bwd / V, 4), "steps": steps, "warmup": warmup,
            "workload": "differentiation: 1M cluster Gaussians, 4 plain views 1024x1024, 90 deg FoV, "
                        "tile 16, W=16; dL/dI of L1 + 0.2 L2 against targets of the perturbed scene",
            "n_gaussians": scene.n, "views": V}


def unpruned_leg(reps=10, warmup=2, frames=30):
    """The unpruned-scale workload: 3M cluster Gaussians (smaller and fainter
    than the stereo workload's), stereo 2064x2208 foveated, W=16, along a
    30-frame +-20 degree head-yaw arc.  Per frame a renderer for that frame's
    cameras is set up (untimed), `warmup` frames run, then `reps` frames are
    timed one by one with HIP events; the frame's time is their median.
    Reports the mean, p50 and p99 over the frames."""
    import numpy as np
    import torch
    import synth
    from paper_2505_10144_amd.render import Renderer, upload
    scene, _, _, _ = synth.config_unpruned(0, frame=0)
    g = upload(scene)
    stream = torch.cuda.current_stream()
    per, inst = [], []
    for k in range(frames):
        _, cams, fovs, params = synth.config_unpruned(0, frame=k, n=16)  # this frame's cameras
        r = Renderer(cams, fovs, params, scene.n)
        r.ensure_capacity(g)
        for _ in range(warmup):
            r.render(g)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            r.render(g)
            b.record(stream)
        torch.cuda.synchronize()
        inst.append(r.check())
        per.append(float(np.median([a.elapsed_time(b) for a, b in ev])))
        del r
    torch.cuda.empty_cache()
    t = np.array(per)
    return {"ms_mean": round(float(t.mean()), 4), "ms_p50": round(float(np.percentile(t, 50)), 4),
            "ms_p99": round(float(np.percentile(t, 99)), 4), "fps_mean": round(1000.0 / float(t.mean()), 2),
            "frames": frames, "reps": reps, "instances_mean": int(np.mean(inst)),
            "workload": "unpruned: 3M cluster Gaussians (log-scale N(-5.5,0.8), opacity logit N(-1,1.5)), "
                        "2 eyes 2064x2208, 110 deg FoV, 15 deg fovea, W=16, head yaw -20..20 deg over 30 frames",
            "n_gaussians": scene.n}


def batch_leg(steps, log=None, knobs=None):
    """The batched multi-view form: 1M cluster Gaussians rendered to 16 views
    of mixed size (4 each of 512^2, 1024^2, 1920x1080, 2064x2208) and FoV, a
    random half foveated, in one call sequence (one preprocess, one sort, one
    blend launch over all views).  The renderer knobs come from the autotuner
    (cached per configuration in a JSON file); the same knobs are then timed
    as 16 separate single-view renders for comparison."""
    import tempfile
    import torch
    import synth
    from paper_2505_10144_amd.render import Renderer, upload
    from paper_2505_10144_amd.tune import time_frames, tune
    scene, cams, fovs, params = synth.config_batch(0)
    g = upload(scene)
    cache = os.environ.get("VRS_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "vrs_tune_cache.json"))
    t0 = time.perf_counter()
    if knobs:
        tile, window, bb, sc = (int(x) for x in knobs.split(","))
        p, cached = params.replace(tile=tile, window=window, blend_batch=bb, schedule=sc), None
    else:
        res = tune(g, cams, fovs, params, cache_path=cache, steps=3, log=log)
        p, cached = res.params, res.cached
    t_tune = time.perf_counter() - t0
    r = Renderer(cams, fovs, p, scene.n)
    r.ensure_capacity(g)
    batched = time_frames(r, g, steps)
    n_items = r.n_items
    del r
    torch.cuda.empty_cache()
    sep = 0.0
    for c, f in zip(cams, fovs):
        r1 = Renderer([c], [f], p, scene.n)
        r1.ensure_capacity(g)
        sep += time_frames(r1, g, steps)
        del r1
    torch.cuda.empty_cache()
    return {"batched_ms": round(batched, 4), "separate_ms": round(sep, 4),
            "speedup": round(sep / batched, 3), "views": len(cams), "items": n_items,
            "tuned": {k: getattr(p, k) for k in ("tile", "window", "blend_batch", "schedule")},
            "tune_s": round(t_tune, 1), "tune_cached": cached, "tune_cache": cache,
            "workload": "batch: 1M cluster Gaussians, 16 views (4 each 512^2, 1024^2, 1920x1080, 2064x2208), "
                        "FoV U[60,120] deg, 8 foveated (15 deg)"}


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU rendering is a design "
                                   "(views or screen tiles per GPU) and is not measured",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import synth
    from paper_2505_10144_amd.render import Renderer, upload

    torch.cuda.set_device(0)
    if args.diff_only:
        print(json.dumps({"fwd_bwd": diff_leg(args.diff_steps, 3)}), flush=True)
        return
    if args.unpruned_only:
        print(json.dumps({"unpruned": unpruned_leg()}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_leg(5, log=lambda row: print(row, file=sys.stderr, flush=True),
                                             knobs=args.batch_knobs)}), flush=True)
        return
    scene, cams, fovs, params = synth.config_stereo(0, n=args.n, window=args.window)
    params = params.replace(schedule=args.schedule, blend_batch=args.blend_batch)
    r = Renderer(cams, fovs, params, scene.n)
    g = upload(scene)
    n_cand = r.ensure_capacity(g)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        r.render(g)
    torch.cuda.synchronize()
    r.check()

    # Timed region: K whole stereo frames, events between the stages.
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        e = ev[k]
        e[0].record(stream)
        r.preprocess(g)
        e[1].record(stream)
        r.sort(g)
        e[2].record(stream)
        r.blend_only()
        e[3].record(stream)
        r.compose()
        e[4].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_kept = r.check()
    ms = (t1 - t0) * 1000.0 / K
    names = ["preprocess", "sort", "blend", "compose"]
    stages = {n: sum(ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)) / K for i, n in enumerate(names)}

    # Work units of the blend (instrumented launch, outside the timed region).
    work = r.blend_stats()
    torch.cuda.synchronize()
    ops = work["pairs"] * OPS_PER_PAIR + work["contrib"] * ops_per_contrib(args.window)
    blend_s = stages["blend"] / 1000.0
    achieved = ops / blend_s / 1e12
    kernel_key = f"k_render<{args.window},false> stereo 2064x2208 500k"
    traffic = traffic_for(kernel_key)

    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 3),
        "unit": "stereo frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "vr-stereo-foveated: 500k cluster+slab Gaussians, 2 eyes 2064x2208, "
                               "110 deg FoV, 64 mm baseline, 15 deg fovea, 10% band, W=16",
                   "n_gaussians": scene.n, "views": 2, "width": 2064, "height": 2208,
                   "fovea_deg": 15.0, "window": args.window, "sort_tile": 32,
                   "schedule": args.schedule, "blend_batch": args.blend_batch},
        "roofline": {"bound": "alu", "kernel": kernel_key, "achieved": round(achieved, 3),
                     "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tops/s (FP32 VALU lane-ops)",
                     "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": traffic},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "work": dict(work, candidates=n_cand, instances=n_kept, items=r.n_items),
    }
    n_items = r.n_items
    del r, g
    torch.cuda.empty_cache()
    if not args.no_diff:
        out["fwd_bwd"] = diff_leg(args.diff_steps, 3)
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batch"] = batch_leg(5, knobs=args.batch_knobs)
    if not args.no_unpruned:
        out["unpruned"] = unpruned_leg()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, cams, fovs, params, n_items, args.cpu_tiles)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
