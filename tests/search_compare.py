"""Comparison of a whole GPU search with the oracle's, under the tolerance rule.

Floating point on the two sides differs by the FP32 error of the GPU path (rho within 1e-4
relative, re-weighted rho within ~2e-4), so near a decision boundary either outcome is correct.
A difference between the two results is accepted only where such a boundary explains it:

* triggers (per detector, the filter's own rho before re-weighting): an oracle trigger missing
  on the GPU, or a GPU trigger absent from the oracle's list, must lie in the threshold band
  thr (1 +- delta) or have a competing sample within the clustering window whose oracle rho is
  within 2 delta of its own (the oracle's SNR series is recomputed for those templates);
  common triggers agree within delta;
* coincidences above a statistic ``hi``: a coincidence present on one side only must have its
  network SNR within dstat of ``hi``, or share its slide and clustering window (circular
  |tick_H' - tick_H| <= W_c) with a pre-clustering coincidence of either side that holds a
  "fragile" trigger (one of the differing triggers, a trigger of a template only one side
  filtered, or a trigger whose rho sits within delta of the chi-square cut, where re-weighting
  switches on), or with another coincidence whose statistic is within dstat of its own;
* background counts: |n_gpu(x) - n_oracle(x)| is at most the number of differing background
  coincidences at or above x (1 - dstat) plus those within dstat of x.

Every such exemption is counted and returned, so the callers can also bound how many there are.
"""
import numpy as np

import oracle
from oracle import coinc as _oc


def _seg_sample(tick, seg_ticks, tps, m_off=0):
    """Segment and sample of a tick: segment s covers [s seg_ticks, (s + 1) seg_ticks) of the
    timeline, starting at its sample m_off (the start of its valid region)."""
    s = int(tick) // seg_ticks
    return s, (int(tick) - s * seg_ticks) // tps + m_off


def compare_triggers(g, o_tick, o_tmpl, o_snr_raw, thr, delta, series, window, seg_ticks, tps, only_tmpls=None,
                     m_off=0):
    """g: GPU trigger records (filter's own rho); o_*: the oracle's triggers (raw rho).
    series(seg, tmpl) -> the oracle's complex SNR series of that template on that segment.
    only_tmpls(seg) -> set of templates filtered on both sides (None: all).
    Returns (set of differing (tmpl, tick) keys, number of common triggers)."""
    G = {(int(t), int(k)): float(r) for t, k, r in zip(g["tmpl"], g["tick"], g["snr"])}
    O = {(int(t), int(k)): float(r) for t, k, r in zip(o_tmpl, o_tick, o_snr_raw)}
    assert len(G) == len(g) and len(O) == len(o_tick), "duplicate triggers"
    diff = set()
    cache = {}

    def rho_o(s, t):
        if (s, t) not in cache:
            cache[(s, t)] = np.abs(series(s, t))
        return cache[(s, t)]

    lo_band, hi_band = thr * (1 - delta), thr * (1 + delta)
    for key in set(O) ^ set(G):
        t, tick = key
        s, m = _seg_sample(tick, seg_ticks, tps, m_off)
        if only_tmpls is not None and t not in only_tmpls(s):
            diff.add(key)
            continue
        r = rho_o(s, t)
        n = len(r)
        here = r[m]
        assert here >= lo_band, ("trigger below the threshold band", key, here)
        if here < hi_band:
            diff.add(key)
            continue
        lo, hi = max(0, m - window), min(n - 1, m + window)
        nb = np.r_[r[lo:m], r[m + 1:hi + 1]]
        if key in O:
            # the oracle's peak: the GPU must have seen a competitor within 2 delta of it
            ok = nb.size and nb.max() >= here * (1 - 2 * delta)
        else:
            # the GPU's peak: the oracle's own peak in the window may not exceed it by more than 2 delta
            ok = (not nb.size) or nb.max() <= here * (1 + 2 * delta)
        assert ok, ("trigger differs without a near-tie", key, here, nb.max() if nb.size else None)
        diff.add(key)
    common = set(O) & set(G)
    for key in common:
        assert abs(G[key] / O[key] - 1.0) <= delta, ("rho differs", key, G[key], O[key])
    return diff, len(common)


def _pairs_index(trig_h, trig_l, n_slides, step, window, wrap, fragile_h, fragile_l):
    """Every coincident (slide, pair) of one side before clustering: slide, tick_h, stat and
    whether a fragile trigger takes part; sorted by (slide, tick_h)."""
    th, tl = np.asarray(trig_h["tick"], np.int64), np.asarray(trig_l["tick"], np.int64)
    mh, ml = np.asarray(trig_h["tmpl"], np.int64), np.asarray(trig_l["tmpl"], np.int64)
    i, j, k = _oc._pairs(mh, th, ml, tl, n_slides, step, window, wrap)
    stat = _oc.coinc_stat(np.asarray(trig_h["snr"])[i], np.asarray(trig_l["snr"])[j]).astype(np.float64)
    fh = np.array([(int(a), int(b)) in fragile_h for a, b in zip(mh[i], th[i])], bool)
    fl = np.array([(int(a), int(b)) in fragile_l for a, b in zip(ml[j], tl[j])], bool)
    order = np.lexsort((th[i], k))
    return dict(slide=k[order], tick=th[i][order], stat=stat[order], fragile=(fh | fl)[order],
                key=list(zip(k[order].tolist(), mh[i][order].tolist(), th[i][order].tolist(), tl[j][order].tolist())))


def _near(ix, slide, tick, cw, wrap):
    """Indices of ix's pairs in `slide` with circular |tick_h - tick| <= cw."""
    a = np.searchsorted(ix["slide"], slide, "left")
    b = np.searchsorted(ix["slide"], slide, "right")
    t = ix["tick"][a:b]
    d = np.abs((t - tick + wrap // 2) % wrap - wrap // 2)
    return a + np.nonzero(d <= cw)[0]


def compare_coincs(gc, oc, g_trig, o_trig, fragile, n_slides, step, window, wrap, cw, hi, dstat, edges=None,
                   g_bg=None, o_bg=None):
    """gc: GPU coincidence records; oc: the oracle's coincidence columns; g_trig / o_trig: (H, L)
    triggers with re-weighted snr as each side fed them to the coincidence; fragile: (set H, set L)
    of (tmpl, tick) keys.  Returns the number of exempt differences."""
    key = lambda c, sel: set(zip(np.asarray(c["slide"])[sel].tolist(), np.asarray(c["tmpl"])[sel].tolist(),
                                 np.asarray(c["tick_h"])[sel].tolist(), np.asarray(c["tick_l"])[sel].tolist()))
    snr_of = {}
    for c in (gc, oc):
        for k_, s_ in zip(zip(np.asarray(c["slide"]).tolist(), np.asarray(c["tmpl"]).tolist(),
                              np.asarray(c["tick_h"]).tolist(), np.asarray(c["tick_l"]).tolist()),
                          np.asarray(c["snr_c"], np.float64)):
            snr_of.setdefault(k_, float(s_))
    ix = [_pairs_index(t[0], t[1], n_slides, step, window, wrap, fragile[0], fragile[1]) for t in (g_trig, o_trig)]

    def exempt(c):
        sl, _, th, _ = c
        s = snr_of[c]
        if abs(s / hi - 1.0) <= dstat:
            return True
        for side in ix:
            near = _near(side, sl, th, cw, wrap)
            if side["fragile"][near].any():
                return True
            others = [q for q in near if side["key"][q] != c]
            if others and np.any(np.abs(side["stat"][others] / (s * s) - 1.0) <= 2 * dstat):
                return True
        return False

    sg = key(gc, np.asarray(gc["snr_c"]) >= hi)
    so = key(oc, np.asarray(oc["snr_c"]) >= hi)
    n_exempt = 0
    for c in sg ^ so:
        assert exempt(c), ("coincidence differs without a boundary or fragile trigger near it", c, snr_of[c])
        n_exempt += 1
    if edges is not None:
        allg = key(gc, np.asarray(gc["slide"]) >= 1)
        allo = key(oc, np.asarray(oc["slide"]) >= 1)
        d = allg ^ allo
        both = allg | allo
        for e, (a, b) in enumerate(zip(g_bg, o_bg)):
            x = float(edges[e])
            slack = sum(1 for c in d if snr_of[c] >= x * (1 - dstat))
            slack += sum(1 for c in both if abs(snr_of[c] / x - 1.0) <= dstat)
            assert abs(int(a) - int(b)) <= slack, ("background count", x, int(a), int(b), slack)
    return n_exempt


def check_followed(fg, fo, gc1, oc1, thresholds, dstat, coarse_mc, fine_mc, frac=0.05, fragile_rows=None):
    """Followed fine templates of one segment (sets fg GPU, fo oracle): a template followed on one
    side only must lie in the neighbourhood of a stage-1 coincidence present on one side only, at
    one of the follow-up thresholds (within dstat), or marked in fragile_rows (oracle rows whose
    proposer cell selection rounding can change).  Returns the number of such templates."""
    if fg == fo:
        return 0
    key = lambda c, i: (int(c["slide"][i]), int(c["tmpl"][i]), int(c["tick_h"][i]), int(c["tick_l"][i]))
    gk = {key(gc1, i) for i in range(len(gc1["tmpl"]))}
    ok_ = {key(oc1, i) for i in range(len(oc1["tmpl"]))}
    ok_tmpl = {int(gc1["tmpl"][i]) for i in range(len(gc1["tmpl"])) if key(gc1, i) not in ok_}
    for i in range(len(oc1["tmpl"])):
        s = float(oc1["snr_c"][i])
        if (key(oc1, i) not in gk or any(abs(s / x - 1) <= dstat for x in thresholds)
                or (fragile_rows is not None and len(fragile_rows) and fragile_rows[i])):
            ok_tmpl.add(int(oc1["tmpl"][i]))
    for f in fg ^ fo:
        assert any(abs(fine_mc[f] - coarse_mc[c]) <= frac * coarse_mc[c] for c in ok_tmpl), ("followed set differs", f)
    return len(fg ^ fo)


def oracle_series(st_segments, psds, n, fs, f_low, bank):
    """series(seg, tmpl) for compare_triggers: the oracle's SNR series of a template on a segment
    (st_segments: full-rate data transforms; the leading n/2 + 1 bins are used at length n)."""
    def f(s, t):
        a, b = oracle.band_edges(n, fs, f_low, bank.kstart[t], bank.k1[t])
        return oracle.snr_series(st_segments[s][: n // 2 + 1], bank.spectrum(t), psds[s][: n // 2 + 1], n, fs, a, b)
    return f


def cols(rec):
    """Trigger records as the oracle's coincidence input columns."""
    return dict(tmpl=np.asarray(rec["tmpl"], np.int64), tick=np.asarray(rec["tick"], np.int64), snr=rec["snr"])


def check_stage(hs, g_raw, g_rw, o_trig, series, thr, delta, dstat, window, seg_ticks, tps, rho_min, only=None,
                say=print, m_off=0):
    """Triggers of both detectors under the tolerance rule, and the re-weighted rho of the common
    ones within dstat / 2.  g_raw / g_rw: (H, L) GPU trigger tensors before / after re-weighting;
    o_trig: the oracle's (H, L) trigger columns (with snr_raw); series: (H, L) series functions.
    Returns the fragile trigger keys (H, L) and the GPU's re-weighted triggers as columns."""
    fragile, g_cols = [], []
    for det in (0, 1):
        g = hs.as_records(g_raw[det], hs.TRIGGER)
        gr = hs.as_records(g_rw[det], hs.TRIGGER)
        o = o_trig[det]
        diff, common = compare_triggers(g, o["tick"], o["tmpl"], o["snr_raw"], thr, delta, series[det], window,
                                        seg_ticks, tps, only, m_off)
        assert np.array_equal(g["tick"], gr["tick"]) and np.array_equal(g["tmpl"], gr["tmpl"])
        near_cut = {(int(a), int(b)) for a, b, r in zip(g["tmpl"], g["tick"], g["snr"])
                    if abs(r / rho_min - 1.0) <= delta}
        near_cut |= {(int(a), int(b)) for a, b, r in zip(o["tmpl"], o["tick"], o["snr_raw"])
                     if abs(r / rho_min - 1.0) <= delta}
        okey = {(int(a), int(b)): r for a, b, r in zip(o["tmpl"], o["tick"], o["snr"])}
        worst = 0.0
        for a, b, r in zip(gr["tmpl"], gr["tick"], gr["snr"]):
            k = (int(a), int(b))
            if k in okey and k not in near_cut:
                worst = max(worst, abs(float(r) / okey[k] - 1.0))
        assert worst <= dstat / 2, worst
        say(f"  detector {det}: {len(g)} GPU / {len(o['tick'])} oracle triggers, {common} common, "
            f"{len(diff)} differing (all exempt), re-weighted rho error {worst:.1e}")
        assert len(diff) <= 0.01 * common + 3
        fragile.append(diff | near_cut)
        g_cols.append(cols(gr))
    return fragile, g_cols


def exact_coinc(hs, coincs, bg_counts, g_cols, n_slides, step, window, wrap, cw, edges, ticks_per_second):
    """The oracle's coincidence step on the GPU's own triggers: identical records (slide, template,
    ticks, statistic) and background counts.  Returns the number of records."""
    ref = oracle.timeslide_coinc(g_cols[0], g_cols[1], n_slides, step, window, wrap, cw,
                                 np.asarray(edges, np.float32), ticks_per_second)
    c = hs.as_records(coincs, hs.COINC)
    r = ref["coincs"]
    for f in ("slide", "tmpl", "tick_h", "tick_l"):
        assert np.array_equal(c[f].astype(np.int64), np.asarray(r[f], np.int64)), f
    assert np.array_equal(c["stat"], np.asarray(r["stat"], np.float32))
    if bg_counts is not None:
        assert np.array_equal(np.asarray(bg_counts, np.int64), ref["bg_counts"])
    return len(c)
