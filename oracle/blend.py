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
the list the rest is blended in ascending (t*, a) order.  W = 0 blends every
entry on arrival, in list order: the renderers that only sort globally.

Blending one entry (3DGS conventions, a reading): alpha is clamped to
alpha_max = 0.99; T' = T (1 - alpha); if T' < T_min = 1e-4 the sample stops and
this entry is not blended; otherwise C += T alpha c and T = T'.  The output is
rgb = C + T * background and alpha = 1 - T.

``exhaustive_blend`` is the full per-pixel sort (Sec. 3: the only ordering
free of popping), used to pin the window: they agree whenever no entry arrives
more than W places after an entry that is deeper than it.
"""
import numpy as np


# Reasons a sample is flagged (bits of the flag mask).
FLAG_ALPHA = 1   # an entry's alpha is within eps_alpha of alpha_min
FLAG_TIE = 2     # an emission picks between window depths within eps_t
FLAG_STOP = 4    # an emission's T' is within eps_T of T_min
FLAG_ORDER = 8   # two adjacent list entries may arrive in either order
FLAG_NAMES = {FLAG_ALPHA: "alpha_min", FLAG_TIE: "depth tie", FLAG_STOP: "T_min",
              FLAG_ORDER: "arrival order"}


class BlendFlags:
    """Relative distances to the discrete decisions below which a sample is
    flagged as borderline (FP32 vs FP64 may decide differently there)."""

    def __init__(self, eps_alpha=1e-5, eps_t=2e-6, eps_T=1e-3):
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
        fl[idx[close]] |= FLAG_TIE
    al = wal[idx, j]
    col = wc[idx, j]
    Tn = T[idx] * (1.0 - al)
    stop = Tn < T_min
    if flags is not None:
        fl[idx[np.abs(Tn - T_min) <= flags.eps_T * T_min]] |= FLAG_STOP
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

    Returns (C (S,3), T (S,), flags (S,) uint8 mask of FLAG_* reasons, stats
    dict, emitted list or None).
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
    fl = np.zeros(S, dtype=np.uint8)
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
            fl[live & near] |= FLAG_ALPHA
        m = live & (alpha_raw >= alpha_min)
        if flags is not None and prev_amb:
            fl[m & prev_pass] |= FLAG_ORDER
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


class TooManyOutcomes(Exception):
    """More admissible outcomes than the enumeration cap."""


def sample_outcomes(alpha, lnag, tstar, color, amb, W, alpha_min, T_min, flags, cap=64, max_flips=None):
    """Every outcome of one sample's windowed blend that FP32 arithmetic could
    legitimately produce, given the FP64 values of its list entries.

    The entries are those of the sample's tile list that might reach
    alpha_min, in list order: alpha (clamped), lnag = ln(sigma G), tstar,
    color (n, 3), and amb[i] True when entry i and entry i+1 are neighbours in
    the list whose float32 key depths are at most one ulp apart (so the sort
    may deliver them in either order).

    The blend is the one of ``window_blend`` (insert entries reaching
    alpha_min; when the window exceeds W entries emit the smallest (t*,
    arrival); stop when T' < T_min, not blending that entry; flush in order).
    Wherever a decision is within the ``flags`` margins of its threshold --
    alpha vs alpha_min, two window depths at an emission, T' vs T_min, the
    order of an ambiguous pair -- both ways are followed.

    With ``max_flips`` only paths that take at most that many decisions
    against their FP64 outcome are followed (the likely ones: every decision
    FP32 may take differently is rare).

    Returns (outcomes, complete): outcomes is a list of (C (3,), T, flips),
    flips being the tuple of (FLAG_* bit, relative distance to the threshold)
    of every decision taken against the FP64 outcome on that path (the path
    with no flips is the FP64 blend); complete is False if ``max_flips`` cut
    off some path.  Raises TooManyOutcomes beyond ``cap`` outcomes."""
    n = len(alpha)
    ln_amin = np.log(alpha_min)
    eps_a, eps_t, eps_T = flags.eps_alpha, flags.eps_t, flags.eps_T
    color = np.asarray(color, np.float64)
    leaves = []
    calls = [0]
    complete = [True]
    budget = np.inf if max_flips is None else max_flips

    def can_flip(flips):
        if len(flips) < budget:
            return True
        complete[0] = False
        return False

    def leaf(C, T, flips):
        leaves.append((np.array(C, np.float64), float(T), flips))
        if len(leaves) > cap:
            raise TooManyOutcomes

    def emissions(win, T, C, flips):
        # win: list of (t*, position, alpha, entry index).  Candidates for the
        # emitted entry: the smallest (t*, position) and every entry whose t*
        # is within eps_t of it.
        k0 = min(range(len(win)), key=lambda k: (win[k][0], win[k][1]))
        t0 = win[k0][0]
        picks = [(k0, ())]
        for k, e in enumerate(win):
            if k != k0:
                rel = abs(e[0] - t0) / max(abs(e[0]), abs(t0), 1e-30)
                if rel <= eps_t and can_flip(flips):
                    picks.append((k, ((FLAG_TIE, rel),)))
        out = []
        for k, fl in picks:
            al = win[k][2]
            Tn = T * (1.0 - al)
            rest = win[:k] + win[k + 1:]
            blended = (rest, Tn, C + (T * al) * color[win[k][3]], False)
            halted = (rest, T, C, True)
            out.append(((halted if Tn < T_min else blended), fl))
            relT = abs(Tn - T_min) / T_min
            if relT <= eps_T and can_flip(flips + fl):
                out.append(((blended if Tn < T_min else halted), fl + ((FLAG_STOP, relT),)))
        return out

    def swappable(perm, p):
        i, j = perm[p], perm[p + 1]
        lo = min(i, j)
        return max(i, j) == lo + 1 and bool(amb[lo])

    def go(p, perm, win, T, C, flips, no_swap_at, forced):
        calls[0] += 1
        if calls[0] > 16 * cap:
            raise TooManyOutcomes
        while p < n:
            if no_swap_at != p and p + 1 < n and swappable(perm, p) and can_flip(flips):
                perm2 = list(perm)
                perm2[p], perm2[p + 1] = perm2[p + 1], perm2[p]
                go(p, perm2, list(win), T, C, flips + ((FLAG_ORDER, 0.0),), p, forced)
            i = perm[p]
            passes = bool(alpha[i] >= alpha_min) if forced is None else forced
            if forced is None:
                d = abs(lnag[i] - ln_amin)
                if d <= eps_a and can_flip(flips):
                    go(p, perm, list(win), T, C, flips + ((FLAG_ALPHA, d),), p, not passes)
            forced = None
            no_swap_at = None
            p += 1
            if not passes:
                continue
            win = win + [(tstar[i], p, alpha[i], i)]
            if len(win) > W:
                ch = emissions(win, T, C, flips)
                for (w2, T2, C2, stopped), fl in ch[1:]:
                    if stopped:
                        leaf(C2, T2, flips + fl)
                    else:
                        go(p, perm, w2, T2, C2, flips + fl, None, None)
                (win, T, C, stopped), fl = ch[0]
                flips = flips + fl
                if stopped:
                    leaf(C, T, flips)
                    return
        while win:
            ch = emissions(win, T, C, flips)
            for (w2, T2, C2, stopped), fl in ch[1:]:
                if stopped:
                    leaf(C2, T2, flips + fl)
                else:
                    go(n, perm, w2, T2, C2, flips + fl, None, None)
            (win, T, C, stopped), fl = ch[0]
            flips = flips + fl
            if stopped:
                break
        leaf(C, T, flips)

    go(0, list(range(n)), [], 1.0, np.zeros(3), (), None, None)
    return leaves, complete[0]
