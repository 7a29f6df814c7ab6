"""Two-detector coincidence, time slides, background counts and FAR (oracle).

Sec. I and Sec. II: background is built by shifting one detector's triggers by
multiples of a fixed step and recomputing coincidences; Eq. (6) gives
FAR = (1 + n_b(Lambda_b >= Lambda*_f)) / T_b.  Readings taken where the paper
is silent:

* Coincidence (Sec. I asks for agreement in time and in template parameters):
  same template id, and circular |delta| <= window with
  delta = ((t_H - t_L - k step + T/2) mod T) - T/2 on the integer tick grid,
  T = wrap (the analysed time on the concatenated timeline).  Slide k = 0 is the
  foreground; k = 1..K shift detector L by k * step.
* Statistic: the ranking statistic Lambda of Eq. (5) needs PyCBC's signal and
  noise models, which the paper does not give; Appendix A uses the network
  SNR rho_c = sqrt(rho_H^2 + rho_L^2) as the coincident statistic, and so
  does this reading.  Decisions are taken on stat = rho_c^2 in the precision
  of the GPU path: float32(float64(rho_H)^2 + float64(rho_L)^2) for float32
  triggers (float64 products of float32 values are exact), float64 otherwise.
* Clustering per slide: coincidence c survives iff no other coincidence c' of
  the same slide with circular |tick_H(c') - tick_H(c)| <= W_c has a larger
  stat, or an equal stat and a lexicographically smaller (tmpl, tick_H, tick_L).
* Background counts: n_b(x) = number of surviving coincidences with k >= 1 and
  rho_c >= x (inclusive), evaluated as float64(stat) >= float64(x)^2;
  T_b = K * T.
* Statistic floor (optional): coincidences with float64(stat) < float64(floor)^2
  are discarded before the clustering.  A coincidence is only ever removed by a
  better one, so the survivors at or above the floor and the counts at edges at
  or above it are unchanged (pinned against the plain definition in the tests).
"""
import math

import numpy as np


def coinc_stat(snr_h, snr_l):
    """rho_c^2 in the decision precision (see module docstring)."""
    snr_h = np.asarray(snr_h)
    snr_l = np.asarray(snr_l)
    s = snr_h.astype(np.float64) ** 2 + snr_l.astype(np.float64) ** 2
    if snr_h.dtype == np.float32 and snr_l.dtype == np.float32:
        return s.astype(np.float32)
    return s


def _circ(x, T):
    return (x + T // 2) % T - T // 2


def _pairs(h_tmpl, h_tick, l_tmpl, l_tick, n_slides, step, window, wrap, keep_pair=None):
    """All (i_H, j_L, k) with equal template and |circ(t_H - t_L - k step)| <= window.
    keep_pair(I, J) -> bool mask restricts the pairs first (the statistic floor)."""
    out_i, out_j, out_k = [], [], []
    l_order = np.argsort(l_tmpl, kind="stable")
    l_sorted = l_tmpl[l_order]
    j_max = (n_slides * step + window) // wrap + 1
    for t in np.unique(h_tmpl):
        ih_all = np.nonzero(h_tmpl == t)[0]
        a = np.searchsorted(l_sorted, t, "left")
        b = np.searchsorted(l_sorted, t, "right")
        jl = l_order[a:b]
        if len(jl) == 0:
            continue
        # H triggers of the template in chunks, so nH x nL never materialises at once
        chunk = max(1, (1 << 22) // len(jl))
        for c0 in range(0, len(ih_all), chunk):
            ih = ih_all[c0:c0 + chunk]
            I = np.repeat(ih, len(jl))
            J = np.tile(jl, len(ih))
            if keep_pair is not None:
                m = keep_pair(I, J)
                I, J = I[m], J[m]
            d = (h_tick[I] - l_tick[J]) % wrap                        # in [0, T)
            for j in range(-1, j_max + 1):
                # k step must lie in [d - window + j T, d + window + j T]
                k_lo = -((-(d - window + j * wrap)) // step)           # ceil
                k_hi = (d + window + j * wrap) // step                 # floor
                k_lo = np.maximum(k_lo, 0)
                k_hi = np.minimum(k_hi, n_slides)
                width = int(np.max(k_hi - k_lo + 1)) if len(d) else 0
                for o in range(max(width, 0)):
                    k = k_lo + o
                    ok = k <= k_hi
                    out_i.append(I[ok])
                    out_j.append(J[ok])
                    out_k.append(k[ok])
    if not out_i:
        z = np.zeros(0, np.int64)
        return z, z, z
    i = np.concatenate(out_i)
    j = np.concatenate(out_j)
    k = np.concatenate(out_k)
    # definition check: every emitted pair is coincident at its slide
    assert np.all(np.abs(_circ(h_tick[i] - l_tick[j] - k * step, wrap)) <= window)
    return i, j, k


def _cluster_slide(tick_h, stat, tmpl, tick_l, cluster_w, wrap):
    """Indices surviving the per-slide clustering rule (module docstring)."""
    n = len(tick_h)
    order = np.lexsort((tick_l, tmpl, tick_h))
    th = tick_h[order]
    keep = []
    all_nb = 2 * cluster_w + 1 >= wrap
    for p in range(n):
        t = th[p]
        if all_nb:
            nb = np.arange(n)
        else:
            lo, hi = t - cluster_w, t + cluster_w
            if lo < 0:
                rng = [(0, hi), (lo + wrap, wrap - 1)]
            elif hi >= wrap:
                rng = [(lo, wrap - 1), (0, hi - wrap)]
            else:
                rng = [(lo, hi)]
            nb = np.concatenate([np.arange(np.searchsorted(th, a, "left"),
                                           np.searchsorted(th, b, "right")) for a, b in rng])
        c = order[p]
        o = order[nb]
        o = o[o != c]
        better = (stat[o] > stat[c]) | (
            (stat[o] == stat[c]) & (
                (tmpl[o] < tmpl[c]) | ((tmpl[o] == tmpl[c]) & (
                    (tick_h[o] < tick_h[c]) | ((tick_h[o] == tick_h[c]) & (tick_l[o] < tick_l[c]))))))
        if not np.any(better):
            keep.append(c)
    return np.asarray(keep, np.int64)


def timeslide_coinc(h, l, n_slides: int, step: int, window: int, wrap: int, cluster_w: int,
                    edges, ticks_per_second: int, min_snr_c: float = 0.0):
    """Coincidences over slides 0..n_slides, clustered per slide, plus background counts.

    ``h`` and ``l`` are dicts with arrays tmpl (int), tick (int64 in [0, wrap)), snr.
    Returns dict(coincs=dict of columns sorted by (slide, tick_h, tmpl, tick_l),
    bg_counts=int64 [len(edges)], t_b=seconds).
    """
    if 2 * window >= wrap:
        raise ValueError("coincidence window must be below half the wrap period")
    h_tmpl = np.asarray(h["tmpl"], np.int64)
    h_tick = np.asarray(h["tick"], np.int64)
    l_tmpl = np.asarray(l["tmpl"], np.int64)
    l_tick = np.asarray(l["tick"], np.int64)
    if np.any((h_tick < 0) | (h_tick >= wrap)) or np.any((l_tick < 0) | (l_tick >= wrap)):
        raise ValueError("trigger ticks must lie in [0, wrap)")
    hs_, ls_ = np.asarray(h["snr"]), np.asarray(l["snr"])
    keep = None
    if min_snr_c > 0:
        # the floor is a property of the pair alone, so it may be applied before the slides
        keep = lambda I, J: np.asarray(coinc_stat(hs_[I], ls_[J]), np.float64) >= np.float64(min_snr_c) ** 2
    i, j, k = _pairs(h_tmpl, h_tick, l_tmpl, l_tick, n_slides, step, window, wrap, keep)
    snr_h = hs_[i]
    snr_l = ls_[j]
    stat = coinc_stat(snr_h, snr_l)
    tmpl = h_tmpl[i]
    th = h_tick[i]
    tl = l_tick[j]
    kept = []
    for s in np.unique(k):
        sel = np.nonzero(k == s)[0]
        kk = _cluster_slide(th[sel], stat[sel], tmpl[sel], tl[sel], cluster_w, wrap)
        kept.append(sel[kk])
    kept = np.concatenate(kept) if kept else np.zeros(0, np.int64)
    order = np.lexsort((tl[kept], tmpl[kept], th[kept], k[kept]))
    kept = kept[order]
    coincs = dict(slide=k[kept], tmpl=tmpl[kept], tick_h=th[kept], tick_l=tl[kept],
                  snr_h=snr_h[kept], snr_l=snr_l[kept], stat=stat[kept],
                  snr_c=np.sqrt(np.asarray(stat[kept], np.float64)))
    edges = np.asarray(edges)
    bg = coincs["stat"][coincs["slide"] >= 1].astype(np.float64)
    e2 = edges.astype(np.float64) ** 2
    counts = np.array([np.count_nonzero(bg >= x) for x in e2], dtype=np.int64)
    t_b = n_slides * wrap / ticks_per_second
    return dict(coincs=coincs, bg_counts=counts, t_b=t_b)


def false_alarm_rate(bg_count_above, t_b: float):
    """Eq. (6): FAR = (1 + n_b(>= statistic of the foreground event)) / T_b (per second)."""
    return (1.0 + np.asarray(bg_count_above, np.float64)) / t_b
