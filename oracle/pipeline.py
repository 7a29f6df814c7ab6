"""Flat and two-stage hierarchical searches composed from the oracle steps.

Sec. II (flat): every template of the full bank filters every segment at the
full sample rate, threshold 4, coincidence and time slides.  Sec. III
(hierarchical): stage 1 filters with the coarse bank at a reduced rate
(threshold 3.5), coincides over zero lag plus a small set of long slides,
selects coincidences with Lambda_1 >= 7, and stage 2 re-filters each selected
segment at the full rate with the union of the fine-bank neighbourhoods
(threshold 4), followed by coincidence and time slides.

Stage-1 data: the paper re-samples to 512 Hz without saying how; reading:
ideal decimation, i.e. the stage-1 transform is the leading N/8 bins of the
full-rate transform of the same segment (same df), and the stage-1 PSD the
leading bins of the full-rate PSD.

A run is ``n_seg`` segments of ``n`` samples laid back to back: sample m of
segment s has tick s * seg_ticks + m * ticks_per_sample.  With pads (``segments``:
overlapping segments of a block, each keeping only its valid region), segments start
every stride = n - pad_lo - pad_hi samples, only samples pad_lo <= m < n - pad_hi are
candidates, sample m of segment s has tick (s * stride + m - pad_lo) * ticks_per_sample and
the timeline (the slide ring and the follow-up's segment of a tick) has stride-long segments.
"""
import numpy as np

from .spectral import strain_fft
from .filter import filter_bank, triggers_from_candidates
from .coinc import timeslide_coinc
from .followup import followup_templates
from .filter import band_edges, template_sigma
from .chisq import chisq_bin_edges, bin_snrs, chisq_terms, reweighted_snr
from .segments import valid_mask
from . import proposer as _proposer


def _concat(parts):
    keys = parts[0].keys()
    return {k: np.concatenate([p[k] for p in parts]) for k in keys}


def reweight_triggers(tr, st, psd, n, fs, f_low, bank, chisq_bins: int, rho_min: float, tps: int, seg_t0: int):
    """Eq. (4) on one segment's triggers: snr -> rho~ for triggers with snr >= rho_min
    (chi-square per ``chisq``); adds columns snr_raw and chisq."""
    snr = np.asarray(tr["snr"], np.float64)
    chi = np.zeros(len(snr))
    bins = np.zeros((len(snr), chisq_bins))
    for i in np.nonzero(snr >= rho_min)[0]:
        t = int(tr["tmpl"][i])
        h = bank.spectrum(t)
        k_lo, k_hi = band_edges(n, fs, f_low, bank.kstart[t], bank.k1[t])
        sig = template_sigma(h, psd, n, fs, k_lo, k_hi)
        e = chisq_bin_edges(h, psd, k_lo, k_hi, chisq_bins)
        m = (int(tr["tick"][i]) - seg_t0) // tps
        zl = bin_snrs(st, h, psd, n, fs, sig, m, e)
        bins[i] = chisq_terms(zl)
        chi[i] = bins[i].sum() / (2 * chisq_bins - 2)
    out = dict(tr)
    out["snr_raw"] = snr
    out["chisq"] = chi
    out["bins"] = bins
    out["snr"] = reweighted_snr(snr, chi)
    return out


def detector_triggers(segments, psds, fs: float, f_low: float, bank, tmpl_ids_per_seg, thr: float,
                      window_sec: float, ticks_per_second: int, decim: int = 1, chisq_bins: int = 8,
                      chisq_rho_min: float = None, pad_lo: int = 0, pad_hi: int = 0):
    """Triggers of one detector over all segments.  ``decim`` > 1 filters at fs/decim.
    With ``chisq_rho_min`` set, snr is the re-weighted SNR of Eq. (4).  pad_lo / pad_hi (full-rate
    samples, multiples of decim) restrict candidates to the valid region (``segments`` module)."""
    out = []
    for s, seg in enumerate(segments):
        n_full = len(seg)
        n = n_full // decim
        f = fs / decim
        st = strain_fft(seg, fs)[: n // 2 + 1]
        psd = psds[s][: n // 2 + 1]
        ids = np.asarray(tmpl_ids_per_seg[s], np.int64)
        c = filter_bank(st, psd, n, f, f_low, bank, ids, thr)
        keep = valid_mask(c["m"], n, pad_lo // decim, pad_hi // decim)
        c = {k: (v[keep] if k != "sigma" else v) for k, v in c.items()}
        tps = int(round(ticks_per_second / f))
        stride = n_full - pad_lo - pad_hi
        seg_t0 = (s * stride - pad_lo) * int(round(ticks_per_second / fs))
        tr = triggers_from_candidates(c["tpos"], c["m"], c["rho2"], c["phase"], ids,
                                      int(round(window_sec * f)), s, seg_t0, tps)
        if chisq_rho_min is not None:
            tr = reweight_triggers(tr, st, psd, n, f, f_low, bank, chisq_bins, chisq_rho_min, tps, seg_t0)
        out.append(tr)
    return _concat(out)


def flat_search(h_segments, l_segments, h_psds, l_psds, fs, f_low, bank, thr=4.0, window_sec=1.0,
                ticks_per_second=51200, n_slides=2000, step_sec=0.1, coinc_window_sec=0.015,
                cluster_sec=1.0, edges=(8.0,), chisq_bins=8, chisq_rho_min=None, pad_lo=0, pad_hi=0):
    ids = [np.arange(bank.n_tmpl)] * len(h_segments)
    kw = dict(chisq_bins=chisq_bins, chisq_rho_min=chisq_rho_min, pad_lo=pad_lo, pad_hi=pad_hi)
    th = detector_triggers(h_segments, h_psds, fs, f_low, bank, ids, thr, window_sec, ticks_per_second, **kw)
    tl = detector_triggers(l_segments, l_psds, fs, f_low, bank, ids, thr, window_sec, ticks_per_second, **kw)
    wrap = len(h_segments) * (len(h_segments[0]) - pad_lo - pad_hi) * int(round(ticks_per_second / fs))
    co = timeslide_coinc(th, tl, n_slides, int(round(step_sec * ticks_per_second)),
                         int(round(coinc_window_sec * ticks_per_second)), wrap,
                         int(round(cluster_sec * ticks_per_second)), np.asarray(edges, np.float32),
                         ticks_per_second)
    return dict(trig_h=th, trig_l=tl, coinc=co)


def hierarchical_search(h_segments, l_segments, h_psds, l_psds, fs, f_low, coarse, fine,
                        decim=4, thr1=3.5, thr2=4.0, window_sec=1.0, ticks_per_second=51200,
                        n_sh1=16, t_sh1_sec=15.0, rho1=7.0, mc_frac=0.05,
                        n_slides=2000, step_sec=0.1, coinc_window_sec=0.015, cluster_sec=1.0,
                        edges=(8.0,), chisq_bins=8, chisq_rho_min=None, proposer=None, pad_lo=0, pad_hi=0):
    """``proposer`` = (model, q_edges, p_cum[, rho_low, p_cum_low]) switches the follow-up to the
    learned cell rule (``proposer`` module): coincidences with rho_c >= rho1 keep the cells of
    cumulative probability p_cum, those with rho_low <= rho_c < rho1 the cells of p_cum_low; the
    bank objects then need ``q`` (mass ratio m1/m2 >= 1) as well."""
    n_seg = len(h_segments)
    n_full = len(h_segments[0])
    tpt = int(round(ticks_per_second / fs))
    seg_ticks = (n_full - pad_lo - pad_hi) * tpt          # one segment's share of the timeline
    wrap = n_seg * seg_ticks
    win = int(round(coinc_window_sec * ticks_per_second))
    cw = int(round(cluster_sec * ticks_per_second))
    e = np.asarray(edges, np.float32)
    ids1 = [np.arange(coarse.n_tmpl)] * n_seg
    kw = dict(chisq_bins=chisq_bins, chisq_rho_min=chisq_rho_min, pad_lo=pad_lo, pad_hi=pad_hi)
    t1h = detector_triggers(h_segments, h_psds, fs, f_low, coarse, ids1, thr1, window_sec,
                            ticks_per_second, decim, **kw)
    t1l = detector_triggers(l_segments, l_psds, fs, f_low, coarse, ids1, thr1, window_sec,
                            ticks_per_second, decim, **kw)
    c1 = timeslide_coinc(t1h, t1l, n_sh1, int(round(t_sh1_sec * ticks_per_second)), win, wrap, cw,
                         e, ticks_per_second)
    if proposer is None:
        fine_ids = followup_templates(c1["coincs"], rho1, coarse.mchirp, fine.mchirp, mc_frac,
                                      seg_ticks, n_seg)
    else:
        # learned proposer: cells of each followed neighbourhood ranked by the MLP
        model, q_edges, p_cum = proposer[:3]
        rho_low, p_low = proposer[3:5] if len(proposer) >= 5 else (rho1, p_cum)
        cc = c1["coincs"]
        feats = _proposer.features(cc, t1h, t1l, coarse.mchirp, coarse.q, int(round(t_sh1_sec * ticks_per_second)),
                                   wrap, ticks_per_second, chisq_bins)
        if len(feats):
            masks = _proposer.select_cells(_proposer.forward(model, feats)[0], p_cum,
                                           feats[:, 2].astype(np.float32), rho1, p_low)
        else:
            masks = np.zeros(0, np.uint64)
        fine_ids = _proposer.followup_cells(cc, rho_low, coarse.mchirp, fine.mchirp, fine.q, q_edges, mc_frac,
                                            seg_ticks, n_seg, masks)
    t2h = detector_triggers(h_segments, h_psds, fs, f_low, fine, fine_ids, thr2, window_sec,
                            ticks_per_second, **kw)
    t2l = detector_triggers(l_segments, l_psds, fs, f_low, fine, fine_ids, thr2, window_sec,
                            ticks_per_second, **kw)
    c2 = timeslide_coinc(t2h, t2l, n_slides, int(round(step_sec * ticks_per_second)), win, wrap, cw,
                         e, ticks_per_second)
    return dict(stage1_h=t1h, stage1_l=t1l, coinc1=c1, fine_ids=fine_ids, trig_h=t2h, trig_l=t2l,
                coinc=c2)
