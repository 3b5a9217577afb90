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

# Algorithmic VALU lane-operations of the blending kernel, per unit of work
# (what the method itself computes, independent of how the kernel is built):
# every evaluated (sample, entry) pair needs about 20 VALU operations and 2
# transcendentals (tangent-plane coordinates, the quadratic form, the
# exponential); every pair whose alpha reaches alpha_min adds about 12 for
# the ray depth t*, 3 per window slot for the insertion and 10 for blending.
OPS_PER_PAIR = 22
def ops_per_contrib(window):
    return 12 + 3 * window + 10

# The backward replays the blend (the work above) and adds, per contributing
# pair, about 150 VALU operations and 2 transcendentals of gradient work.
BWD_OPS_PER_CONTRIB = 152

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
    ap.add_argument("--no-two-pass", action="store_true", help="skip the two-pass foveated baseline leg")
    ap.add_argument("--no-visibility", action="store_true", help="skip the lens-mask (visibility culling) leg")
    ap.add_argument("--no-finetune", action="store_true", help="skip the fine-tuning leg")
    ap.add_argument("--stereo-only", action="store_true", help="only the stereo frame (for profiling)")
    ap.add_argument("--unpruned-only", action="store_true", help="run only the 3M-Gaussian yaw-arc leg")
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


def counters_for(kernel_key, name="blend_stereo_counters.txt", source="render.hip"):
    """Per-launch rocprofv3 counter figures of a kernel (HBM bytes, wave-level
    VALU instructions, launch time), if the kernel's source is unchanged
    since they were taken (else empty)."""
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2505_10144_amd", "csrc", source)
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if vals.get("source_sha256") != sha or vals.get("kernel") != kernel_key:
        return {}
    res = {}
    for k in ("hbm_bytes_per_launch", "valu_wave_insts_per_launch", "launch_us"):
        try:
            res[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return res


def host_cpu():
    """CPU model and logical CPU counts of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


def oracle_workers():
    """Worker processes for the oracle: every CPU this process may use, up to
    the 16 a one-GPU share of the host provides."""
    return max(1, min(16, host_cpu()[2]))


def cpu_baseline(scene, cams, fovs, params):
    """The FP64 oracle on this host, one whole stereo frame: preprocess,
    instances and sort of both eyes, then every work item shaded on a pool
    of worker processes, and the periphery compose."""
    import oracle
    from oracle.render import OracleOptions
    cores = oracle_workers()
    model, ncpu, avail = host_cpu()
    t0 = time.perf_counter()
    res = oracle.render(scene, cams, fovs, params, OracleOptions(workers=cores))
    sec = time.perf_counter() - t0
    st = res["stats"]
    return {
        "value": 1.0 / sec, "unit": "stereo frames/s", "cores": cores, "kind": "oracle",
        "cpu_model": model, "host_logical_cpus": ncpu, "cpus_available": avail,
        "sample": (f"the whole stereo frame, no sampling: FP64 NumPy oracle, preprocess+instances+sort "
                   f"of both eyes {st['t_keys']:.1f} s (one process), shading of all {st['jobs']} work items "
                   f"{st['t_shade']:.1f} s on {cores} processes; {sec:.1f} s per stereo frame"),
    }


def cpu_baseline_fwd_bwd(scene, cams, params, dI, tiles_per_view=16):
    """The FP64 oracle's forward + backward (vector-Jacobian product) for one
    view of the differentiation workload, on a sample of tiles stratified by
    candidate pairs (tile list length x pixels of the tile, one tile per
    1/16 quantile), scaled to the view by that pair count."""
    import numpy as np
    import oracle
    import synth
    from oracle import grad as ograd
    from oracle.render import OracleOptions
    cores = oracle_workers()
    model, ncpu, avail = host_cpu()
    cam = cams[:1]
    t0 = time.perf_counter()
    keys = oracle.render(scene, cam, [synth.fovea_off()], params, OracleOptions(shade=False))
    t_keys = time.perf_counter() - t0
    rg = keys["ranges"]
    grid = keys["grids"][0]
    lens = (rg[:, 1] - rg[:, 0]).astype(np.int64)
    boxes = [grid.box(t) for t in range(grid.n)]
    px = np.array([(x1 - x0) * (y1 - y0) for x0, y0, x1, y1 in boxes], np.int64)
    work = lens * px
    order = np.argsort(work, kind="stable")
    pick = sorted(set(order[np.linspace(0, len(order) - 1, tiles_per_view).astype(int)].tolist()))
    t1 = time.perf_counter()
    _, res, _ = ograd.vjp(scene, cam, params, [dI[0].cpu().numpy().astype(np.float64)], tiles={0: pick},
                          workers=cores)
    # The vjp repeats the view's preprocess+instances+sort (timed above); only
    # its shading, replay and backward are per-tile work.
    t_samp = time.perf_counter() - t1 - res["stats"]["t_keys"]
    scale = float(work.sum()) / max(float(work[pick].sum()), 1.0)
    sec = t_keys + t_samp * scale
    return {
        "value": sec * 1000.0, "unit": "ms/view (fwd+bwd)", "higher_is_better": False, "cores": cores,
        "kind": "oracle", "cpu_model": model, "host_logical_cpus": ncpu, "cpus_available": avail,
        "sample": (f"one 1024x1024 view of the 1M-Gaussian differentiation workload: FP64 NumPy "
                   f"preprocess+instances+sort {t_keys:.1f} s, then forward + PyTorch-FP64 vector-Jacobian "
                   f"product on {len(pick)} tiles stratified by candidate pairs ({t_samp:.1f} s on "
                   f"{cores} processes) scaled by candidate pairs x{scale:.0f}: {sec:.0f} s per view"),
    }


def diff_leg(steps, warmup, cpu=False):
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
    # Work units of the replayed blend (instrumented forward, untimed).
    work = r.blend_stats()
    W = params.window
    ops = work["pairs"] * OPS_PER_PAIR + work["contrib"] * (ops_per_contrib(W) + BWD_OPS_PER_CONTRIB)
    achieved = ops / (bwd / 1000.0) / 1e12
    roof = {"bound": "alu", "kernel": "vrs_render_backward (fill + k_render_bwd + k_color_bwd + k_geom_bwd)",
            "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "Tops/s (FP32 VALU lane-ops)", "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": None, "ops_per_launch": ops, "work": work}
    cpu_row = cpu_baseline_fwd_bwd(scene, cams, params, dI) if cpu else None
    return {"ms_per_view": round(ms / V, 4), "fwd_ms_per_view": round(fwd / V, 4),
            "bwd_ms_per_view": round(bwd / V, 4), "steps": steps, "warmup": warmup,
            "roofline": roof, "cpu_baseline": cpu_row,
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


def two_pass_leg(steps, warmup, single_ms):
    """The two-pass foveated baseline of App. A on the stereo workload: per
    stereo frame, a centre pass over both eyes' centre regions at full
    resolution (tight frustum), a periphery pass over both eyes at half
    resolution, and the bilinear-upsample blend.  Timed with HIP events over
    whole frames; compared with the single-pass frame time."""
    import torch
    import synth
    from paper_2505_10144_amd.render import TwoPassRenderer, upload
    scene, cams, fovs, params = synth.config_stereo(0)
    tp = TwoPassRenderer(cams, fovs, params, scene.n)
    g = upload(scene)
    tp.ensure_capacity(g)
    for _ in range(warmup):
        tp.render(g)
    torch.cuda.synchronize()
    tp.check()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        tp.render(g)
    e1.record(stream)
    torch.cuda.synchronize()
    tp.check()
    ms = e0.elapsed_time(e1) / steps
    boxes = [list(b) for b in tp.box_list]
    del tp, g
    torch.cuda.empty_cache()
    return {"ms_per_stereo_frame": round(ms, 4), "single_pass_ms": round(single_ms, 4),
            "single_over_two_pass": round(single_ms / ms, 4), "paper_ratio_tab2_deep_blending": round(8.14 / 10.35, 4),
            "centre_boxes": boxes, "steps": steps,
            "workload": "two-pass baseline of the stereo workload: centre pass (tight frustum over the 32x32 "
                        "tiles with mask > 0) at full resolution + periphery pass at half resolution for both "
                        "eyes, bilinear upsample and mask blend"}


def visibility_leg(steps, warmup, single_ms, single_instances):
    """The stereo workload with visibility culling (Sec. 4.3): a synthetic
    elliptical lens mask per eye (508 of the 4615 32x32 tiles of a
    2064x2272 eye invisible, like the paper's headset), whose tile bitfield's
    summed-area table gives the exact visible-tile count per splat."""
    import torch
    import synth
    from paper_2505_10144_amd.render import Renderer, upload
    scene, cams, fovs, params = synth.config_stereo(0)
    masks = [synth.lens_mask(c.width, c.height) for c in cams]
    r = Renderer(cams, fovs, params, scene.n, masks=masks)
    g = upload(scene)
    r.ensure_capacity(g)
    for _ in range(warmup):
        r.render(g)
    torch.cuda.synchronize()
    r.check()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        r.render(g)
    e1.record(stream)
    torch.cuda.synchronize()
    n_inst = r.check()
    ms = e0.elapsed_time(e1) / steps
    invisible = int(sum((m.reshape(-1) == 0).sum() for m in masks))
    del r, g
    torch.cuda.empty_cache()
    return {"ms_per_stereo_frame": round(ms, 4), "fps": round(1000.0 / ms, 2), "single_pass_ms": round(single_ms, 4),
            "instances": n_inst, "instances_without_mask": single_instances,
            "instance_reduction": round(1.0 - n_inst / max(single_instances, 1), 4),
            "masked_pixels": invisible, "steps": steps,
            "workload": "stereo workload with a synthetic elliptical lens mask per eye (visibility culling)"}


def finetune_leg(steps, warmup):
    """Fine-tuning iterations on the differentiation workload (1M Gaussians,
    4 plain views at 1024^2): render, L1 + L2 loss and its gradient,
    backward, one Adam step per parameter group -- all on the GPU."""
    import torch
    import synth
    from paper_2505_10144_amd import finetune
    from paper_2505_10144_amd.render import Renderer, upload
    scene, pert, cams, params = synth.config_diff(0)
    fovs = [synth.fovea_off()] * len(cams)
    r = Renderer(cams, fovs, params, scene.n)
    gp = upload(pert)
    r.ensure_capacity(gp)
    targets = [im.clone() for im in r.render(gp)]
    del gp
    g = upload(scene)
    r.ensure_capacity(g, headroom=1.5)
    ft = finetune.FineTuner(r, g, targets)
    first = float(ft.step().item())
    for _ in range(warmup):
        ft.step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        loss = ft.step()
    e1.record(stream)
    torch.cuda.synchronize()
    r.check()
    ms = e0.elapsed_time(e1) / steps
    last = float(loss.item())
    del ft, r, g
    torch.cuda.empty_cache()
    return {"ms_per_iteration": round(ms, 4), "ms_per_view": round(ms / len(cams), 4), "iterations": steps,
            "loss_first": round(first, 6), "loss_last": round(last, 6),
            "workload": "fine-tuning: 1M cluster Gaussians, 4 plain views 1024x1024; targets rendered from the "
                        "perturbed scene; Adam (3DGS learning rates, no schedule)"}


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
    if args.stereo_only:
        args.no_diff = args.no_batch = args.no_unpruned = args.no_cpu_baseline = True
        args.no_two_pass = args.no_visibility = args.no_finetune = True
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the renderer runs on one GPU only; multi-GPU rendering (views or screen "
                                   "tiles per GPU) is a design that is not implemented or measured",
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
    cnt = counters_for(kernel_key)
    executed = None
    if "valu_wave_insts_per_launch" in cnt and "launch_us" in cnt:
        # Lane slots the kernel executed (64 per wave-level VALU instruction)
        # per second of its profiled launch, against the same peak.
        executed = round(cnt["valu_wave_insts_per_launch"] * 64 / (cnt["launch_us"] * 1e-6) / 1e12
                         / VALU_PEAK_TOPS, 4)

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
                     "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": cnt.get("hbm_bytes_per_launch"),
                     "ops_per_launch": ops, "executed_frac": executed},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "work": dict(work, candidates=n_cand, instances=n_kept, items=r.n_items),
    }
    n_items = r.n_items
    del r, g
    torch.cuda.empty_cache()
    def progress(leg):
        print(f"[bench] {leg} done", file=sys.stderr, flush=True)

    progress("stereo")
    if not args.no_diff:
        out["fwd_bwd"] = diff_leg(args.diff_steps, 3, cpu=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
        progress("fwd_bwd")
    if not args.no_two_pass:
        out["two_pass"] = two_pass_leg(20, 3, ms)
        progress("two_pass")
    if not args.no_visibility:
        out["visibility"] = visibility_leg(20, 3, ms, n_kept)
        progress("visibility")
    if not args.no_finetune:
        out["finetune"] = finetune_leg(10, 3)
        progress("finetune")
    if not args.no_batch:
        out["batch"] = batch_leg(5, knobs=args.batch_knobs)
        progress("batch")
    if not args.no_unpruned:
        out["unpruned"] = unpruned_leg()
        torch.cuda.empty_cache()
        progress("unpruned")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, cams, fovs, params)
        progress("cpu_baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
