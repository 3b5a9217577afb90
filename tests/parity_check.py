"""Element-wise parity of GPU renders against the FP64 oracle, borderline
samples included.

A render is checked in two parts, so that every pixel is compared:

1. The blend output before the periphery compose (``Renderer.pre_images``:
   plain views, HIGH and HYBRID pixels, and the LOW group values written to
   their 2x2 pixels) against the oracle's pre-compose image.
   * A pixel whose samples take no borderline decision must be within ``tol``
     (2e-4 per channel) of the oracle.
   * A flagged pixel must be within ``tol`` of one of the outcomes the oracle
     enumerates for it (``oracle.blend.sample_outcomes``: both ways of every
     decision FP32 may take differently).  Which decisions the GPU took
     against FP64, and how close they were to their threshold, is reported:
     that is the measured resolution of the FP32 path the flag margins are
     calibrated against.
   * The oracle enumerates the outcomes with at most a few decisions taken
     against FP64 (every such decision is rare).  A flagged pixel that
     matches none of them is a failure if that enumeration was complete, and
     counted as unchecked if it was cut short (or if even one decision per
     path gives too many outcomes); the unchecked fraction is bounded.
2. The compose: the GPU's final image must equal the oracle's periphery
   reconstruction (``oracle.fovea.blur_low``) applied to the GPU's own
   pre-compose image, on every pixel, within FP32 rounding of a 9-tap sum.

Each check prints one line and, if ``VRS_PARITY_LOG`` names a file, appends a
JSON record to it.
"""
import json
import os

import numpy as np

import oracle
from oracle import blend as oblend
from oracle import fovea as ofov
from oracle.render import OracleOptions

TOL = 2e-4
COMPOSE_TOL = 2e-6


def workers():
    return max(1, min(16, os.cpu_count() or 1))


def ref_render(scene, cams, fovs, params, tiles=None, flags=None):
    """The oracle render with admissible outcomes of every flagged sample."""
    kw = dict(alternatives=True, workers=workers(), tiles=tiles)
    if flags is not None:
        kw["flags"] = flags
    return oracle.render(scene, cams, fovs, params, OracleOptions(**kw))


def low_mask(cam, classes):
    split, subc, _ = classes
    m = np.repeat(np.repeat(subc == ofov.LOW, 16, axis=0), 16, axis=1)
    return m[:cam.height, :cam.width]


def check_render(r, ref, tol=TOL, max_unchecked=1e-3, label="", views=None, ref_views=None):
    """Compare renderer ``r`` (after a render) with oracle result ``ref``.
    ``views`` are the renderer's view indices compared, ``ref_views`` the
    matching oracle view indices (default: the same)."""
    pres = r.pre_images()
    V = r.V
    views = list(range(V)) if views is None else list(views)
    ref_views = views if ref_views is None else list(ref_views)
    total = n_flagged = checked_alt = took_alt = unchecked = 0
    reasons = {name: 0 for name in oblend.FLAG_NAMES.values()}
    took = {name: [0, 0.0] for name in oblend.FLAG_NAMES.values()}
    dists = {name: [] for name in oblend.FLAG_NAMES.values()}
    worst = worst_alt = worst_compose = worst_final = 0.0
    failures = []
    for v, rv in zip(views, ref_views):
        cam = r.cams[v]
        got = pres[v].cpu().numpy().astype(np.float64)
        fin = r.images[v].cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(got)) and np.all(np.isfinite(fin)), "non-finite output"
        valid = ref["shaded"][rv]
        fl = ref["pre_flags"][rv]
        bits = ref["pre_flag_bits"][rv]
        total += int(valid.sum())
        n_flagged += int((valid & fl).sum())
        for b, name in oblend.FLAG_NAMES.items():
            reasons[name] += int((valid & ((bits & b) != 0)).sum())
        # 1a. pixels with no borderline decision
        ok = valid & ~fl
        err = np.abs(got - ref["pre_images"][rv]).max(axis=0)
        if ok.any():
            worst = max(worst, float(err[ok].max()))
            for y, x in np.argwhere(ok & (err > tol))[:5]:
                failures.append(f"view {v} px ({x},{y}) unflagged: got {got[:, y, x]} "
                                f"want {ref['pre_images'][rv][:, y, x]}")
        # 1b. flagged pixels against their admissible outcomes
        alts = ref["pre_alts"][rv]
        unc = ref["pre_unchecked"][rv] & valid
        unchecked += int(unc.sum())
        missing = valid & fl & ~unc
        for (y, x), (vals, flips, complete) in alts.items():
            if not valid[y, x]:
                continue
            missing[y, x] = False
            e = np.abs(vals - got[:, y, x][None]).max(axis=1)
            k = int(np.argmin(e))
            if e[k] > tol:
                if not complete:
                    # Only outcomes with few decisions against FP64 were
                    # enumerated, and none matches: not checked.
                    unchecked += 1
                    continue
                failures.append(f"view {v} px ({x},{y}) flagged, no admissible outcome within {tol}: "
                                f"got {got[:, y, x]}, closest {vals[k]} ({len(vals)} outcomes)")
                continue
            worst_alt = max(worst_alt, float(e[k]))
            checked_alt += 1
            base = [i for i, f in enumerate(flips) if not f]
            if base and e[base[0]] <= tol:
                continue
            took_alt += 1
            # The matching outcome with the fewest decisions against FP64.
            ok_k = [i for i in range(len(vals)) if e[i] <= tol]
            k = min(ok_k, key=lambda i: (len(flips[i]), e[i]))
            for bit, dist in flips[k]:
                t = took[oblend.FLAG_NAMES[bit]]
                t[0] += 1
                t[1] = max(t[1], float(dist))
                dists[oblend.FLAG_NAMES[bit]].append(float(dist))
        if missing.any():
            failures.append(f"view {v}: {int(missing.sum())} flagged pixels without outcomes")
        # 2. compose of the GPU's own pre-compose image
        if r.foveas[v].enabled:
            want = ofov.blur_low(got, low_mask(cam, ref["classes"][rv]))
        else:
            want = got
        ce = float(np.abs(fin - want).max()) if fin.size else 0.0
        worst_compose = max(worst_compose, ce)
        if ce > COMPOSE_TOL:
            failures.append(f"view {v}: compose differs from the periphery reconstruction of the "
                            f"GPU's pre-compose image by {ce:.3e}")
        # End to end on pixels the oracle's final image does not flag.
        okf = ref["valid"][rv] & ~ref["flags"][rv]
        if okf.any():
            fe = float(np.abs(fin - ref["images"][rv])[:, okf].max())
            worst_final = max(worst_final, fe)
            if fe > tol:
                failures.append(f"view {v}: final image differs by {fe:.3e} on unflagged pixels")
    rec = dict(label=label, pixels=total, flagged=n_flagged,
               flagged_frac=n_flagged / max(total, 1),
               reasons={k: c / max(total, 1) for k, c in reasons.items()},
               checked_against_outcomes=checked_alt, took_other_outcome=took_alt,
               took={k: dict(count=c, max_rel_dist=d) for k, (c, d) in took.items() if c},
               unchecked=unchecked, unchecked_frac=unchecked / max(total, 1),
               max_err_unflagged=worst, max_err_flagged=worst_alt,
               max_err_compose=worst_compose, max_err_final=worst_final)
    print("[parity] " + json.dumps(rec), flush=True)
    path = os.environ.get("VRS_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(rec) + "\n")
    assert not failures, "\n".join(failures[:10])
    assert total > 0
    assert unchecked <= max_unchecked * total, rec
    rec["took_dists"] = dists
    return rec
