"""Synthetic candidate, trigger and coincidence lists for unit tests of the post-filter steps.

The record layouts mirror the C ABI structs so the same arrays can be handed to
the GPU library and (as plain columns) to the oracle:
  candidate  {int32 tpos; int32 m; float rho2; float phase}                 16 B
  trigger    {int32 seg; int32 tmpl; int64 tick; float snr; float phase}     24 B
  coinc      {int32 slide; int32 tmpl; int64 tick_h; int64 tick_l;
              float snr_h; float snr_l; float stat; float snr_c}             40 B
"""
import numpy as np

CANDIDATE_DTYPE = np.dtype([("tpos", "<i4"), ("m", "<i4"), ("rho2", "<f4"), ("phase", "<f4")])
TRIGGER_DTYPE = np.dtype([("seg", "<i4"), ("tmpl", "<i4"), ("tick", "<i8"), ("snr", "<f4"),
                          ("phase", "<f4")])
COINC_DTYPE = np.dtype([("slide", "<i4"), ("tmpl", "<i4"), ("tick_h", "<i8"), ("tick_l", "<i8"),
                        ("snr_h", "<f4"), ("snr_l", "<f4"), ("stat", "<f4"), ("snr_c", "<f4")])
assert CANDIDATE_DTYPE.itemsize == 16 and TRIGGER_DTYPE.itemsize == 24 and COINC_DTYPE.itemsize == 40


def synthetic_candidates(gen: np.random.Generator, n_tpos: int, n: int, per_tmpl: int,
                         thr: float, clumps: int = 0, clump_len: int = 0, ties: int = 0):
    """Random above-threshold samples of an SNR series for ``n_tpos`` templates.

    Background candidates are uniform in time with rho^2 = thr^2 + Exp(2); ``clumps``
    dense runs of ``clump_len`` consecutive samples per template imitate glitch
    responses; ``ties`` pairs of candidates share an rho2 value exactly.
    Returns an unsorted CANDIDATE_DTYPE array with unique (tpos, m).
    """
    recs = []
    for t in range(n_tpos):
        ms = gen.choice(n, size=min(per_tmpl, n), replace=False)
        for _ in range(clumps):
            c0 = int(gen.integers(0, max(1, n - clump_len)))
            ms = np.concatenate([ms, np.arange(c0, min(n, c0 + clump_len))])
        ms = np.unique(ms)
        r2 = (thr * thr + gen.exponential(2.0, len(ms))).astype(np.float32)
        if clumps and clump_len:
            # smooth bumps inside the dense runs
            r2 = np.maximum(r2, (thr * thr + 30.0 * np.abs(np.sin(ms / 97.0))).astype(np.float32))
        for _ in range(ties):
            if len(ms) >= 2:
                a, b = gen.choice(len(ms), 2, replace=False)
                r2[b] = r2[a]
        rec = np.zeros(len(ms), CANDIDATE_DTYPE)
        rec["tpos"] = t
        rec["m"] = ms
        rec["rho2"] = r2
        rec["phase"] = gen.uniform(-np.pi, np.pi, len(ms)).astype(np.float32)
        recs.append(rec)
    out = np.concatenate(recs) if recs else np.zeros(0, CANDIDATE_DTYPE)
    return out[gen.permutation(len(out))]


def synthetic_triggers(gen: np.random.Generator, n_tmpl: int, wrap_ticks: int, per_tmpl: float,
                       tick_step: int, seg_ticks: int, snr=(4.0, 12.0), tmpl_ids=None):
    """Random triggers on a tick grid, sorted by (tmpl, tick); Poisson count per template."""
    tmpl_ids = np.arange(n_tmpl) if tmpl_ids is None else np.asarray(tmpl_ids)
    recs = []
    n_steps = wrap_ticks // tick_step
    for t in tmpl_ids:
        c = gen.poisson(per_tmpl)
        ticks = np.unique(gen.integers(0, n_steps, c)) * tick_step
        rec = np.zeros(len(ticks), TRIGGER_DTYPE)
        rec["seg"] = ticks // seg_ticks
        rec["tmpl"] = t
        rec["tick"] = ticks
        rec["snr"] = gen.uniform(snr[0], snr[1], len(ticks)).astype(np.float32)
        rec["phase"] = gen.uniform(-np.pi, np.pi, len(ticks)).astype(np.float32)
        recs.append(rec)
    return np.concatenate(recs) if recs else np.zeros(0, TRIGGER_DTYPE)


def synthetic_coincs(gen: np.random.Generator, count: int, n_tmpl: int, wrap_ticks: int,
                     seg_ticks: int, n_slides: int, stat=(20.0, 120.0)):
    """Random coincidence records (for follow-up tests)."""
    rec = np.zeros(count, COINC_DTYPE)
    rec["slide"] = gen.integers(0, n_slides + 1, count)
    rec["tmpl"] = gen.integers(0, n_tmpl, count)
    rec["tick_h"] = gen.integers(0, wrap_ticks, count)
    rec["tick_l"] = gen.integers(0, wrap_ticks, count)
    s = gen.uniform(stat[0], stat[1], count).astype(np.float32)
    rec["stat"] = s
    rec["snr_c"] = np.sqrt(s).astype(np.float32)
    rec["snr_h"] = np.sqrt(s / 2).astype(np.float32)
    rec["snr_l"] = np.sqrt(s / 2).astype(np.float32)
    return rec


def synthetic_coinc_set(gen: np.random.Generator, n_tmpl: int, n_seg: int, seg_ticks: int, n_trig: int,
                        n_coinc: int, n_slides: int, p: int = 8):
    """Random H and L trigger lists (sorted by (seg, tmpl, tick)) with per-trigger chi-square
    values and p bin terms, and coincidence records that each reference one H and one L trigger
    of the same template (for feature tests).  Returns (trig_h, chisq_h, bins_h, trig_l, chisq_l,
    bins_l, coincs); the numbers are arbitrary draws, not outputs of any search step."""
    def trig_list(count):
        seg = gen.integers(0, n_seg, count)
        rec = np.zeros(count, TRIGGER_DTYPE)
        rec["seg"] = seg
        rec["tmpl"] = gen.integers(0, n_tmpl, count)
        rec["tick"] = seg * seg_ticks + gen.integers(0, seg_ticks, count)
        rec = np.unique(rec)          # sorted by (seg, tmpl, tick); duplicates dropped
        rec["snr"] = gen.uniform(3.5, 15.0, len(rec)).astype(np.float32)
        rec["phase"] = gen.uniform(-np.pi, np.pi, len(rec)).astype(np.float32)
        chi = np.where(gen.random(len(rec)) < 0.3, 0.0, gen.gamma(2.0, 0.8, len(rec))).astype(np.float32)
        bins = (gen.gamma(1.5, 1.2, (len(rec), p)) * (chi[:, None] > 0)).astype(np.float32)
        return rec, chi, bins

    th, ch, bh = trig_list(n_trig)
    tl, cl, bl = trig_list(n_trig)
    co = np.zeros(n_coinc, COINC_DTYPE)
    k = 0
    while k < n_coinc:
        i = int(gen.integers(0, len(th)))
        js = np.nonzero(tl["tmpl"] == th["tmpl"][i])[0]
        if len(js) == 0:
            continue
        j = int(js[gen.integers(0, len(js))])
        co[k]["slide"] = gen.integers(0, n_slides + 1)
        co[k]["tmpl"] = th["tmpl"][i]
        co[k]["tick_h"] = th["tick"][i]
        co[k]["tick_l"] = tl["tick"][j]
        co[k]["snr_h"] = th["snr"][i]
        co[k]["snr_l"] = tl["snr"][j]
        co[k]["stat"] = np.float32(gen.uniform(20.0, 200.0))
        co[k]["snr_c"] = np.float32(gen.uniform(4.5, 14.0))
        k += 1
    return th, ch, bh, tl, cl, bl, co
