"""Front-to-back alpha compositing with per-sample resorting.  Test
infrastructure only.

Eq. 2: C(p) = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j), with
alpha_i = sigma_i G_2D(p).  (The LaTeX source carries a revision macro whose
first argument -- the one that is printed -- is the product.)

Sec. 4.1: splats are re-sorted per pixel by depth along the view ray
(StopThePop's hierarchical per-pixel resorting).  Reading of that hierarchy
(the StopThePop paper is not available): level 1 is the per-tile list sorted
by the per-tile key; level 2 is a per-sample window of W entries.  For each
list entry in order (arrival index a) whose alpha at the sample reaches
alpha_min, (t*, a, alpha, colour) is inserted; whenever the window holds more
than W entries, the one with the smallest (t*, a) is blended.  At the end of
the list the rest is blended in ascending (t*, a) order.

Blending one entry (3DGS conventions, a reading): alpha is clamped to
alpha_max = 0.99; T' = T (1 - alpha); if T' < T_min = 1e-4 the sample stops and
this entry is not blended; otherwise C += T alpha c and T = T'.  The output is
rgb = C + T * background and alpha = 1 - T.

``exhaustive_blend`` is the full per-pixel sort (Sec. 3: the only ordering
free of popping), used to pin the window: they agree whenever no entry arrives
more than W places after an entry that is deeper than it.
"""
import numpy as np


class BlendFlags:
    """Relative distances to the discrete decisions below which a sample is
    flagged as borderline (FP32 vs FP64 may decide differently there)."""

    def __init__(self, eps_alpha=2e-5, eps_t=1e-5, eps_T=1e-3):
        self.eps_alpha = eps_alpha  # |ln(sigma G) - ln(alpha_min)|
        self.eps_t = eps_t          # |t1 - t2| / max(|t1|, |t2|) at an emission
        self.eps_T = eps_T          # |T' - T_min| / T_min at an emission


def _emit(state, idx, T_min, flags, fl, record):
    """Blend, for each sample index in idx, its window entry with the smallest
    (t*, a) and remove it from the window."""
    wt, wa, wal, wc, cnt, T, C, done = state
    rows_t = wt[idx]
    rows_a = wa[idx]
    tmin = rows_t.min(axis=1)
    cand = rows_t == tmin[:, None]
    amin = np.where(cand, rows_a, np.iinfo(np.int64).max).min(axis=1)
    j = np.argmax(cand & (rows_a == amin[:, None]), axis=1)
    # Borderline: another window entry with nearly the same depth.
    if flags is not None:
        tt = rows_t.copy()
        tt[np.arange(len(idx)), j] = np.inf
        t2 = tt.min(axis=1)
        scale = np.maximum(np.abs(tmin), np.abs(np.where(np.isfinite(t2), t2, 0)))
        close = np.isfinite(t2) & (np.abs(t2 - tmin) <= flags.eps_t * np.maximum(scale, 1e-30))
        fl[idx[close]] = True
    al = wal[idx, j]
    col = wc[idx, j]
    Tn = T[idx] * (1.0 - al)
    stop = Tn < T_min
    if flags is not None:
        fl[idx[np.abs(Tn - T_min) <= flags.eps_T * T_min]] = True
    go = ~stop
    gi = idx[go]
    C[gi] += (T[gi] * al[go])[:, None] * col[go]
    T[gi] = Tn[go]
    if record is not None:
        for s, g, a_ in zip(gi, wa[gi, j[go]], al[go]):
            record[int(s)].append((int(g), float(a_)))
    done[idx[stop]] = True
    # Remove slot j: move the last occupied slot into it.
    last = cnt[idx] - 1
    for arr in (wt, wa, wal):
        arr[idx, j] = arr[idx, last]
    wc[idx, j] = wc[idx, last]
    wt[idx, last] = np.inf
    wa[idx, last] = np.iinfo(np.int64).max
    cnt[idx] -= 1


def window_blend(n_samples, entries, W, alpha_min, T_min, flags=None,
                 record=False):
    """Per-sample windowed resorting and compositing.

    ``entries`` is an iterable over the tile's list in order, yielding
    (alpha_raw (S,), tstar_fn, color (3,), pair_ambiguous_with_next: bool)
    where alpha_raw = min(alpha_max, sigma G) already applied except for the
    threshold, and tstar_fn(mask) returns t* for the masked samples.

    Returns (C (S,3), T (S,), flagged (S,), stats dict, emitted list or None).
    """
    S = n_samples
    wt = np.full((S, W + 1), np.inf)
    wa = np.full((S, W + 1), np.iinfo(np.int64).max, dtype=np.int64)
    wal = np.zeros((S, W + 1))
    wc = np.zeros((S, W + 1, 3))
    cnt = np.zeros(S, dtype=np.int64)
    T = np.ones(S)
    C = np.zeros((S, 3))
    done = np.zeros(S, dtype=bool)
    fl = np.zeros(S, dtype=bool)
    rec = [[] for _ in range(S)] if record else None
    state = (wt, wa, wal, wc, cnt, T, C, done)
    pairs = 0
    contrib = 0
    prev_pass = np.zeros(S, dtype=bool)
    prev_amb = False
    ar = np.arange(S)
    for a, (alpha_raw, log_alpha_raw, tstar_fn, color, amb_next) in enumerate(entries):
        live = ~done
        pairs += int(live.sum())
        if flags is not None:
            with np.errstate(divide="ignore"):
                near = np.abs(log_alpha_raw - np.log(alpha_min)) <= flags.eps_alpha
            fl |= live & near
        m = live & (alpha_raw >= alpha_min)
        if flags is not None and prev_amb:
            fl |= m & prev_pass
        prev_pass = m
        prev_amb = amb_next
        if not m.any():
            continue
        contrib += int(m.sum())
        idx = ar[m]
        slot = cnt[idx]
        wt[idx, slot] = tstar_fn(m)
        wa[idx, slot] = a
        wal[idx, slot] = alpha_raw[m]
        wc[idx, slot] = color
        cnt[idx] += 1
        over = idx[cnt[idx] > W]
        if len(over):
            _emit(state, over, T_min, flags, fl, rec)
    while True:
        left = ar[(cnt > 0) & ~done]
        if len(left) == 0:
            break
        _emit(state, left, T_min, flags, fl, rec)
    return C, T, fl, dict(pairs=pairs, contrib=contrib, stopped=int(done.sum())), rec


def exhaustive_blend(alphas, tstars, colors, alpha_min, T_min):
    """Full per-pixel sort for one sample: alphas, tstars (n,), colors (n,3) in
    list order.  Entries below alpha_min are dropped, the rest are blended in
    ascending (t*, arrival) order with the same stop rule."""
    alphas = np.asarray(alphas, np.float64)
    keep = np.flatnonzero(alphas >= alpha_min)
    order = keep[np.lexsort((keep, np.asarray(tstars)[keep]))]
    T, C = 1.0, np.zeros(3)
    for i in order:
        Tn = T * (1.0 - alphas[i])
        if Tn < T_min:
            break
        C = C + T * alphas[i] * np.asarray(colors[i], np.float64)
        T = Tn
    return C, T
