"""Flat and two-stage hierarchical searches composed from the libhs entry points.

Control flow only: every numerical step is one of the C-ABI calls in ``hs``.

Flat (Sec. II): each segment of each detector is whitened, filtered with the full fine bank
at the full rate (threshold 4), clustered into triggers; two-detector coincidence over K
slides gives the foreground and the background counts of Eq. (6).

Hierarchical (Sec. III): stage 1 filters the leading quarter of the same whitened spectrum
(ideal decimation to fs/4, same df) with the coarse bank at threshold 3.5, coincides over
zero lag plus N_sh1 long slides, follows every coincidence with network SNR >= rho1 into the
union of fine-bank chirp-mass neighbourhoods of its segments, filters those templates at the
full rate (threshold 4) and coincides over the K background slides.  With the learned
proposer, each followed neighbourhood is cut down to the cells an MLP selects from features of
the stage-1 coincidence.

Time is int64 ticks of 1/ticks_per_second s; sample m of segment s has tick
s * seg_ticks + m * ticks_per_sample.  With overlapping segments of a block (pad_lo_sec /
pad_hi_sec, Sec. V) only each segment's valid region pad_lo <= m < n - pad_hi gives triggers,
seg_ticks is the stride n - pad_lo - pad_hi and sample m lies at s * seg_ticks + (m - pad_lo) *
ticks_per_sample: the valid regions laid end to end are the timeline (slide ring, follow-up).
"""
from dataclasses import dataclass, field

import numpy as np
import torch

from . import hs


@dataclass
class SearchConfig:
    fs: float = 2048.0
    f_low: float = 20.0
    decim: int = 4                # stage-1 rate = fs / decim
    thr1: float = 3.5
    thr2: float = 4.0
    window_sec: float = 1.0       # trigger clustering window
    ticks_per_second: int = 51200
    n_sh1: int = 16               # stage-1 slides (reading of Sec. III, scaled to the data length)
    t_sh1_sec: float = 15.0
    rho1: float = 7.0             # stage-1 follow-up threshold on the network SNR
    mc_frac: float = 0.05         # neighbourhood: |Mc_f - Mc_c| <= frac Mc_c
    n_slides: int = 2000          # stage-2 / flat background slides
    step_sec: float = 0.1
    coinc_window_sec: float = 0.015
    cluster_sec: float = 1.0      # per-slide coincidence clustering window
    coinc_min_snr: float = 0.0    # background / stage-2 coincidences below this network SNR are not formed
    stage1_min_snr: float = 0.0   # stage-1 coincidences below this are not formed (at most the follow-up bar)
    # overlapping segments of a block (Sec. V): each segment keeps the samples pad_lo <= t < T_seg - pad_hi
    # (its valid region); segments start every T_seg - pad_lo - pad_hi and their valid regions, laid end
    # to end, are the timeline.  0 / 0: segments are circular and laid back to back.
    pad_lo_sec: float = 0.0
    pad_hi_sec: float = 0.0
    edges: tuple = tuple(round(6.0 + 0.1 * i, 1) for i in range(81))   # background count grid, 6.0 .. 14.0
    chisq_rho_min: float = 5.5    # triggers at or above this SNR get the chi-square re-weighting (None: off)
    far_x_min: float = 7.0        # Eq. (7) fit over the edges >= far_x_min with non-zero counts
    far_x_fit: float = 8.0        # the fitted tail replaces the counted background at and above this


@dataclass
class SearchResult:
    trig_h: torch.Tensor
    trig_l: torch.Tensor
    coincs: torch.Tensor
    bg_counts: np.ndarray
    t_b: float
    templates_filtered: int              # (template, segment, detector) applications at full rate
    template_seconds: float              # full-rate template-seconds filtered
    stage1_template_seconds: float = 0.0
    stage1_coincs: torch.Tensor = None
    stage1_trig: tuple = None                       # (H, L) stage-1 triggers, re-weighted
    followed: list = field(default_factory=list)
    mf_ms: float = 0.0                   # device time inside matched-filter calls (events)
    mf_calls: int = 0
    mf_units: list = field(default_factory=list)   # (n, ids, bank, device ms) per matched-filter call
    far: dict = None                                # background_far() output, when computed
    fine_ids: list = None                           # per segment: followed fine template ids (device)
    raw: dict = None                                # the filter's own triggers before re-weighting:
                                                    # keys "h", "l" (full rate), "h1", "l1" (stage 1)


class _MFTimer:
    """Accumulates device time of matched-filter calls with events on the library's stream."""

    def __init__(self, ctx, enabled):
        self.ctx, self.enabled, self.ms, self.calls, self.units = ctx, enabled, 0.0, 0, []

    def run(self, fn, n, ids, bank):
        if not self.enabled:
            return fn()
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record(self.ctx.stream)
        out = fn()
        e.record(self.ctx.stream)
        e.synchronize()
        ms = s.elapsed_time(e)
        self.ms += ms
        self.calls += 1
        self.units.append((n, ids, bank, ms))
        return out


def whiten_all(ctx, strains, psds, cfg: SearchConfig):
    """Whitened spectra [n_seg, n/2] for one detector (strains [n_seg, n] float32 device)."""
    n_seg, n = strains.shape
    out = torch.empty((n_seg, n // 2), dtype=torch.complex64, device=strains.device)
    for s in range(n_seg):
        hs.hs_whiten(ctx, strains[s], cfg.fs, cfg.f_low, psds[s], out=out[s])
    return out


def timeline(cfg: SearchConfig, n_full: int):
    """(ticks per full-rate sample, pad_lo and pad_hi in full-rate samples, ticks of one segment's
    share of the timeline): sample m (full rate) of segment s lies at tick
    s * share + (m - pad_lo) * ticks_per_sample."""
    tpt = int(round(cfg.ticks_per_second / cfg.fs))
    plo = int(round(cfg.pad_lo_sec * cfg.fs))
    phi = int(round(cfg.pad_hi_sec * cfg.fs))
    if plo < 0 or phi < 0 or plo + phi >= n_full or plo % cfg.decim or phi % cfg.decim:
        raise ValueError("segment pads must be non-negative multiples of the stage-1 decimation within a segment")
    return tpt, plo, phi, (n_full - plo - phi) * tpt


def detector_triggers(ctx, specs, n, fs, bank, ids_per_seg, thr, cfg: SearchConfig, timer=None, with_chisq=False,
                      raw_sink=None):
    """Filter + cluster every segment of one detector; returns concatenated trigger records, and
    with ``with_chisq`` also the chi2_r values and per-bin chi-square terms of those triggers.
    The chi-square writes the re-weighted triggers to a new buffer: the filter's own triggers
    (rho and arg z at the peak, what hs_chisq_at_peaks needs) stay intact and, with a list as
    ``raw_sink``, are appended to it (concatenated over segments)."""
    tps = int(round(cfg.ticks_per_second / fs))
    n_full = specs.shape[1] * 2
    tpt, plo, phi, share = timeline(cfg, n_full)
    decim = n_full // n
    valid = (plo // decim, (n_full - phi) // decim)
    window = int(round(cfg.window_sec * fs))
    parts, chis, bins, raws = [], [], [], []
    p = max(1, bank.chisq_bins)
    use_chisq = cfg.chisq_rho_min is not None and bank.chisq_bins
    for s in range(specs.shape[0]):
        ids = ids_per_seg[s]
        if ids.numel() == 0:
            continue
        f = lambda: hs.hs_matched_filter(ctx, specs[s], n, fs, bank, ids, thr)
        cand = timer.run(f, n, ids, bank) if timer else f()
        seg_t0 = s * share - plo * tpt
        trig = hs.hs_cluster_triggers(ctx, cand, n, ids, window, seg=s, seg_t0=seg_t0, ticks_per_sample=tps,
                                      valid=valid)
        if use_chisq:
            # Eq. (4): the coincidence statistic combines re-weighted SNRs
            # the triggers carry the filter's own rho and arg z: the widest bin is formed from them
            r = hs.hs_chisq(ctx, specs[s], n, fs, bank, trig, seg_t0=seg_t0, ticks_per_sample=tps,
                            rho_min=cfg.chisq_rho_min, bins=with_chisq, at_peaks=True)
            raws.append(trig)
            trig = r[1]
            if with_chisq:
                chis.append(r[0])
                bins.append(r[2])
        else:
            raws.append(trig)
            if with_chisq:
                chis.append(torch.zeros(trig.shape[0], dtype=torch.float32, device=specs.device))
                bins.append(torch.zeros((trig.shape[0], p), dtype=torch.float32, device=specs.device))
        parts.append(trig)
    cat = lambda xs, shape: torch.cat(xs) if xs else torch.zeros(shape, dtype=torch.float32, device=specs.device)
    trig = torch.cat(parts) if parts else torch.zeros((0, 6), dtype=torch.int32, device=specs.device)
    if raw_sink is not None:
        raw_sink.append(torch.cat(raws) if raws else torch.zeros((0, 6), dtype=torch.int32, device=specs.device))
    if not with_chisq:
        return trig
    return trig, cat(chis, (0,)), cat(bins, (0, p))


YEAR = 365.25 * 86400.0


def speedup_eq8(n_seg: int, n_flat: int, n_stage1: int, n_stage2: int, f_flat: float, f_coarse: float,
                t_seg: float, gamma: float = 1.0) -> float:
    """Sec. V, Eq. (8): matched-filter speed-up of the two-stage search over the flat one when one
    template on one segment costs kappa N log N (N = f t_seg samples; kappa and the logarithm's
    base cancel); n_stage2 counts (template, segment) applications, gamma the per-segment overhead."""
    def cost(f):
        m = f * t_seg
        return m * np.log(m)
    return float(n_seg * n_flat * cost(f_flat) / (n_seg * n_stage1 * cost(f_coarse) + n_stage2 * gamma * cost(f_flat)))


def background_far(ctx, res: "SearchResult", cfg: SearchConfig):
    """Sec. IV: Eq. (7) fit of the background counts, hybrid FAR of every zero-lag coincidence
    (device float64 per record, -1 for background records, per second) and the statistic
    thresholds for inverse FARs of 1 and 10 years; None when the tail has fewer than two points."""
    e = np.asarray(cfg.edges, np.float32)
    try:
        a, b, m = hs.hs_far_fit(e, res.bg_counts, cfg.far_x_min)
    except hs.HsError:
        return None
    far = hs.hs_far(ctx, res.coincs, res.t_b, a, b, cfg.far_x_fit)
    return dict(alpha=a, beta=b, n_fit=m, far=far, t_b=res.t_b,
                ifar_1yr=hs.hs_far_threshold(a, b, res.t_b, YEAR),
                ifar_10yr=hs.hs_far_threshold(a, b, res.t_b, 10 * YEAR))


def _coinc(ctx, th, tl, n_tmpl, n_slides, step_sec, cfg, wrap, edges, min_snr_c=0.0):
    tk = cfg.ticks_per_second
    return hs.hs_timeslide_coinc(ctx, th, tl, n_tmpl, n_slides, int(round(step_sec * tk)),
                                 int(round(cfg.coinc_window_sec * tk)), wrap, int(round(cfg.cluster_sec * tk)),
                                 edges, min_snr_c=min_snr_c)


def flat_search(ctx, spec_h, spec_l, fine_h, fine_l, cfg: SearchConfig, time_mf=False) -> SearchResult:
    """Flat search; fine_h / fine_l are the fine bank prepared with each detector's PSD."""
    n = spec_h.shape[1] * 2
    n_seg = spec_h.shape[0]
    fine = fine_h
    all_ids = torch.arange(fine.n_tmpl, dtype=torch.int32, device=spec_h.device)
    timer = _MFTimer(ctx, time_mf)
    rh, rl = [], []
    th = detector_triggers(ctx, spec_h, n, cfg.fs, fine_h, [all_ids] * n_seg, cfg.thr2, cfg, timer, raw_sink=rh)
    tl = detector_triggers(ctx, spec_l, n, cfg.fs, fine_l, [all_ids] * n_seg, cfg.thr2, cfg, timer, raw_sink=rl)
    wrap = n_seg * timeline(cfg, n)[3]
    co, bg = _coinc(ctx, th, tl, fine.n_tmpl, cfg.n_slides, cfg.step_sec, cfg, wrap, np.asarray(cfg.edges, np.float32),
                    cfg.coinc_min_snr)
    T = n / cfg.fs
    apps = 2 * n_seg * fine.n_tmpl
    return SearchResult(th, tl, co, bg, cfg.n_slides * wrap / cfg.ticks_per_second, apps, apps * T,
                        mf_ms=timer.ms, mf_calls=timer.calls, mf_units=timer.units, raw=dict(h=rh[0], l=rl[0]))


def stage1(ctx, spec_h, spec_l, coarse_h, coarse_l, cfg: SearchConfig, timer=None, with_chisq=False, raw=None):
    """Stage 1 of Sec. III: the coarse bank on the leading quarter of each whitened spectrum
    (ideal decimation to fs / decim, same df), threshold thr1, coincidence over zero lag and
    n_sh1 slides of t_sh1.  Returns (trig_h, trig_l, coincs) where with ``with_chisq`` each
    trigger entry is (records, chi2_r, per-bin terms)."""
    n = spec_h.shape[1] * 2
    n1, fs1 = n // cfg.decim, cfg.fs / cfg.decim
    n_seg = spec_h.shape[0]
    c_ids = torch.arange(coarse_h.n_tmpl, dtype=torch.int32, device=spec_h.device)
    rh, rl = [], []
    th = detector_triggers(ctx, spec_h, n1, fs1, coarse_h, [c_ids] * n_seg, cfg.thr1, cfg, timer, with_chisq, rh)
    tl = detector_triggers(ctx, spec_l, n1, fs1, coarse_l, [c_ids] * n_seg, cfg.thr1, cfg, timer, with_chisq, rl)
    if raw is not None:
        raw.update(h1=rh[0], l1=rl[0])
    wrap = n_seg * timeline(cfg, n)[3]
    c1, _ = _coinc(ctx, th[0] if with_chisq else th, tl[0] if with_chisq else tl, coarse_h.n_tmpl, cfg.n_sh1,
                   cfg.t_sh1_sec, cfg, wrap, np.zeros(0, np.float32), cfg.stage1_min_snr)
    return th, tl, c1


def stage1_features(ctx, th, tl, c1, coarse, n_seg: int, n: int, cfg: SearchConfig):
    """Proposer features of the stage-1 coincidences (th / tl as returned by stage1 with chisq)."""
    seg_ticks = timeline(cfg, n)[3]
    return hs.hs_proposer_features(ctx, c1, th[0], th[1], th[2], tl[0], tl[1], tl[2], seg_ticks, coarse.mchirp,
                                   coarse.q, int(round(cfg.t_sh1_sec * cfg.ticks_per_second)), n_seg * seg_ticks,
                                   cfg.ticks_per_second)


def hierarchical_search(ctx, spec_h, spec_l, coarse_h, coarse_l, fine_h, fine_l, cfg: SearchConfig,
                        time_mf=False, proposer=None) -> SearchResult:
    """Two-stage search; each bank is given per detector (prepared with that detector's PSD).
    With a ``proposer`` (paper_2309_00019_amd.proposer.Proposer) the follow-up keeps only the
    neighbourhood cells the learned proposer selects; the banks then need ``q`` (m1 / m2)."""
    coarse, fine = coarse_h, fine_h
    n = spec_h.shape[1] * 2
    n_seg = spec_h.shape[0]
    timer = _MFTimer(ctx, time_mf)
    seg_ticks = timeline(cfg, n)[3]          # one segment's share of the timeline
    wrap = n_seg * seg_ticks
    use_p = proposer is not None
    raw = {}
    t1h, t1l, c1 = stage1(ctx, spec_h, spec_l, coarse_h, coarse_l, cfg, timer, with_chisq=use_p, raw=raw)
    if use_p:
        # two tiers: rho_c >= rho1 keeps the cells of probability p_cum, rho_low <= rho_c < rho1
        # (marginal stage-1 coincidences, followed only through the proposer) those of p_cum_low
        feats = stage1_features(ctx, t1h, t1l, c1, coarse, n_seg, n, cfg)
        masks = hs.hs_mlp_propose(ctx, proposer.model, feats, proposer.p_cum, cfg.rho1, proposer.p_cum_low)
        ids2, counts = hs.hs_followup_cells(ctx, c1, min(proposer.rho_low, cfg.rho1), coarse.mchirp, fine.mchirp,
                                            fine.q, cfg.mc_frac, proposer.q_edges, masks, seg_ticks, n_seg)
    else:
        ids2, counts = hs.hs_followup(ctx, c1, cfg.rho1, coarse.mchirp, fine.mchirp, cfg.mc_frac, seg_ticks, n_seg)
    per_seg = [ids2[s, :counts[s]] for s in range(n_seg)]
    rh, rl = [], []
    th = detector_triggers(ctx, spec_h, n, cfg.fs, fine_h, per_seg, cfg.thr2, cfg, timer, raw_sink=rh)
    tl = detector_triggers(ctx, spec_l, n, cfg.fs, fine_l, per_seg, cfg.thr2, cfg, timer, raw_sink=rl)
    raw.update(h=rh[0], l=rl[0])
    co, bg = _coinc(ctx, th, tl, fine.n_tmpl, cfg.n_slides, cfg.step_sec, cfg, wrap, np.asarray(cfg.edges, np.float32),
                    cfg.coinc_min_snr)
    T = n / cfg.fs
    apps = 2 * int(sum(counts))
    return SearchResult(th, tl, co, bg, cfg.n_slides * wrap / cfg.ticks_per_second, apps, apps * T,
                        stage1_template_seconds=2 * n_seg * coarse.n_tmpl * T, stage1_coincs=c1, followed=counts,
                        stage1_trig=(t1h[0] if use_p else t1h, t1l[0] if use_p else t1l),
                        mf_ms=timer.ms, mf_calls=timer.calls, mf_units=timer.units, fine_ids=per_seg, raw=raw)
