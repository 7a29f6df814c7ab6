"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types an oracle formula: each compares the oracle with an
independent route (time-domain sums, Parseval, the Rayleigh law of Appendix A,
brute-force enumeration of a set definition, a library routine for a special
case, or a number the paper prints).
"""
import json
import os

import numpy as np
import pytest
import scipy.signal

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _analytic_psd(n, fs):
    k = np.arange(n // 2 + 1)
    p = np.empty(n // 2 + 1)
    p[1:] = synth.aligo_psd_fit(k[1:] * fs / n)
    p[0] = p[1]
    return p


# --------------------------------------------------------------------------------------
# Inner product and FFT conventions: brute-force time-domain circular correlation
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,k_lo,k_hi", [(64, 3, 31), (256, 5, 100), (1024, 40, 511)])
def test_snr_series_equals_time_domain_correlation(n, k_lo, k_hi):
    fs = float(n) / 4.0
    df, dt = fs / n, 1.0 / fs
    g = np.random.default_rng(n)
    s = g.standard_normal(n) * 3.0
    h = np.zeros(n // 2 + 1, complex)
    h[k_lo:k_hi + 1] = g.standard_normal(k_hi - k_lo + 1) + 1j * g.standard_normal(k_hi - k_lo + 1)
    psd = 0.5 + g.random(n // 2 + 1)
    z = oracle.snr_series(oracle.strain_fft(s, fs), h, psd, n, fs, k_lo, k_hi, sigma=1.0)
    # filter g[j] = 4 df dt sum_k h[k]/S[k] e^{2 pi i k j / N} by a direct sum over the band
    j = np.arange(n)
    filt = np.zeros(n, complex)
    for k in range(k_lo, k_hi + 1):
        filt += h[k] / psd[k] * np.exp(2j * np.pi * k * j / n)
    filt *= 4.0 * df * dt
    # z_m = sum_n s[n] conj(g[(n - m) mod N])
    brute = np.array([np.sum(s * np.conj(filt[(j - m) % n])) for m in range(n)])
    assert np.max(np.abs(z - brute)) <= 1e-12 * np.max(np.abs(brute))


def test_strain_fft_parseval():
    n, fs = 4096, 512.0
    s = np.random.default_rng(1).standard_normal(n)
    st = oracle.strain_fft(s, fs)
    df = fs / n
    two_sided = np.abs(st[0]) ** 2 + 2 * np.sum(np.abs(st[1:n // 2]) ** 2) + np.abs(st[n // 2]) ** 2
    assert np.isclose(np.sum(s * s) / fs, two_sided * df, rtol=1e-12)


def test_strain_fft_is_the_dt_weighted_dft():
    n, fs = 128, 64.0
    s = np.random.default_rng(2).standard_normal(n)
    st = oracle.strain_fft(s, fs)
    j = np.arange(n)
    for k in (0, 1, 17, 64):
        direct = np.sum(s * np.exp(-2j * np.pi * k * j / n)) / fs
        assert abs(st[k] - direct) < 1e-12 * max(1.0, abs(direct))


# --------------------------------------------------------------------------------------
# Normalisation, lag and phase: a noiseless injection is recovered at SNR sqrt((h,h))
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("mass,m0,phi0,amp", [(9.0, 1234, 0.7, 1.0), (14.0, 7001, -2.1, 3.5)])
def test_noiseless_injection_recovers_optimal_snr_lag_and_phase(mass, m0, phi0, amp):
    n, fs, f_low = 8192, 512.0, 30.0
    bank = synth.taylorf2_bank([mass], [mass], n, fs, f_low)
    h = bank.spectrum(0)
    psd = _analytic_psd(n, fs)
    # time series of the template with phase phi0, rolled to coalesce at sample m0
    x = np.fft.irfft(np.exp(1j * phi0) * h, n=n) * fs
    data = amp * np.roll(x, m0)
    k_lo, k_hi = oracle.band_edges(n, fs, f_low, bank.kstart[0], bank.k1[0])
    # (h, h) from the time-domain energy of the whitened template (Parseval, real signal):
    # 4 df sum_band |w~|^2 = 2 dt sum_n w[n]^2 with w~ = h~/sqrt(S) on the band.
    wt = np.zeros(n // 2 + 1, complex)
    wt[k_lo:k_hi + 1] = h[k_lo:k_hi + 1] / np.sqrt(psd[k_lo:k_hi + 1])
    w = np.fft.irfft(wt, n=n) * fs
    hh = 2.0 * np.sum(w * w) / fs
    z = oracle.snr_series(oracle.strain_fft(data, fs), h, psd, n, fs, k_lo, k_hi)
    m = int(np.argmax(np.abs(z)))
    assert m == m0
    assert np.isclose(np.abs(z[m]), amp * np.sqrt(hh), rtol=1e-10)
    assert abs(np.angle(z[m] * np.exp(-1j * phi0))) < 1e-9
    # and sigma itself equals sqrt((h,h))
    assert np.isclose(oracle.template_sigma(h, psd, n, fs, k_lo, k_hi), np.sqrt(hh), rtol=1e-10)


# --------------------------------------------------------------------------------------
# Gaussian noise: rho follows the Rayleigh law of Appendix A (rho^2 ~ chi^2_2)
# --------------------------------------------------------------------------------------
def test_snr_in_gaussian_noise_is_rayleigh():
    n, fs, f_low = 8192, 512.0, 30.0
    psd = _analytic_psd(n, fs)
    m1, m2 = synth.equal_mass_bank([8.0, 11.0, 15.0])
    bank = synth.taylorf2_bank(m1, m2, n, fs, f_low)
    r2 = []
    for seed in range(24):
        s, _ = synth.make_strain(900, 0, seed, n, fs, f_low)
        c = oracle.filter_bank(oracle.strain_fft(s, fs), psd, n, fs, f_low, bank, [0, 1, 2], 0.0,
                               keep_series=True)
        for z in c["series"]:
            r2.append(np.abs(z) ** 2)
    r2 = np.concatenate(r2)
    # E[rho^2] = 2 (each quadrature has unit variance)
    assert abs(np.mean(r2) - 2.0) < 0.06
    for x in (2.0, 3.0, 3.5):
        p = np.mean(r2 >= x * x)
        assert abs(p / np.exp(-x * x / 2.0) - 1.0) < 0.2, (x, p)


# --------------------------------------------------------------------------------------
# Peak clustering: brute force of the set definition
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_cluster_matches_bruteforce_definition(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(10, 200))
    m = g.choice(5000, n, replace=False)
    r2 = np.round(g.uniform(16, 30, n), 1)  # coarse values force exact ties
    W = int(g.integers(1, 400))
    kept = set(oracle.cluster_peaks(m, r2, W).tolist())
    brute = set()
    for i in range(n):
        ok = True
        for j in range(n):
            if i != j and abs(m[j] - m[i]) <= W:
                if r2[j] > r2[i] or (r2[j] == r2[i] and m[j] < m[i]):
                    ok = False
        if ok:
            brute.add(i)
    assert kept == brute


def test_threshold_is_inclusive():
    z = np.array([4.0 + 0j, np.nextafter(4.0, 0) + 0j, 0 + 4j, 5.0 + 0j])
    m, r2, _ = oracle.threshold_candidates(z, 4.0)
    assert m.tolist() == [0, 2, 3]


# --------------------------------------------------------------------------------------
# Coincidence and time slides: brute-force triple loop over (slide, i, j)
# --------------------------------------------------------------------------------------
def _brute_coinc(h, l, K, step, window, wrap, cw):
    pairs = []
    for k in range(K + 1):
        for i in range(len(h["tick"])):
            for j in range(len(l["tick"])):
                if h["tmpl"][i] != l["tmpl"][j]:
                    continue
                d = (int(h["tick"][i]) - int(l["tick"][j]) - k * step + wrap // 2) % wrap - wrap // 2
                if abs(d) <= window:
                    pairs.append((k, i, j))
    stat = {p: np.float32(np.float64(h["snr"][p[1]]) ** 2 + np.float64(l["snr"][p[2]]) ** 2)
            for p in pairs}

    def key(p):  # larger is better
        return (stat[p], -h["tmpl"][p[1]], -h["tick"][p[1]], -l["tick"][p[2]])

    kept = []
    for p in pairs:
        ok = True
        for q in pairs:
            if q == p or q[0] != p[0]:
                continue
            d = (int(h["tick"][q[1]]) - int(h["tick"][p[1]]) + wrap // 2) % wrap - wrap // 2
            if abs(d) <= cw and key(q) > key(p):
                ok = False
                break
        if ok:
            kept.append(p)
    return pairs, kept, stat


@pytest.mark.parametrize("seed", range(5))
def test_timeslide_coinc_matches_bruteforce(seed):
    g = np.random.default_rng(100 + seed)
    wrap = int(g.choice([20000, 20001, 30000]))
    step, window, cw, K = 1000, 150, int(g.integers(100, 3000)), 12
    th = synth.synthetic_triggers(g, 4, wrap, 9, 25, wrap)
    tl = synth.synthetic_triggers(g, 4, wrap, 9, 25, wrap)
    # plant exact ties and wrap-around coincidences
    tl["snr"][: len(tl) // 3] = th["snr"][0]
    h = dict(tmpl=th["tmpl"], tick=th["tick"], snr=th["snr"])
    l = dict(tmpl=tl["tmpl"], tick=tl["tick"], snr=tl["snr"])
    edges = np.array([4.0, 6.0, 8.0, 10.0, 14.0], np.float32)
    out = oracle.timeslide_coinc(h, l, K, step, window, wrap, cw, edges, 100)
    pairs, kept, stat = _brute_coinc(h, l, K, step, window, wrap, cw)
    c = out["coincs"]
    got = sorted(zip(c["slide"].tolist(), c["tmpl"].tolist(), c["tick_h"].tolist(), c["tick_l"].tolist()))
    exp = sorted((k, int(h["tmpl"][i]), int(h["tick"][i]), int(l["tick"][j])) for k, i, j in kept)
    assert got == exp
    assert len(pairs) >= len(kept) > 0
    bg = [stat[p] for p in kept if p[0] >= 1]
    for e, cnt in zip(edges, out["bg_counts"]):
        assert cnt == sum(1 for s in bg if np.float64(s) >= np.float64(e) ** 2)
    assert out["t_b"] == K * wrap / 100


def test_far_is_eq6():
    # Eq. (6): one more than the louder background count, over the background time
    assert oracle.false_alarm_rate(0, 10.0) == 0.1
    assert np.allclose(oracle.false_alarm_rate([3, 9], 20.0), [0.2, 0.5])


# --------------------------------------------------------------------------------------
# Follow-up: set algebra
# --------------------------------------------------------------------------------------
def test_followup_matches_set_algebra():
    g = np.random.default_rng(7)
    coarse_mc = np.sort(g.uniform(1.4, 10, 40))
    fine_mc = np.sort(g.uniform(1.4, 10, 500))
    seg_ticks, n_seg = 1000, 3
    co = synth.synthetic_coincs(g, 60, 40, seg_ticks * n_seg, seg_ticks, 4)
    out = oracle.followup_templates(co, 7.0, coarse_mc, fine_mc, 0.05, seg_ticks, n_seg)
    for s in range(n_seg):
        exp = set()
        for c in co:
            if float(c["stat"]) >= 49.0 and s in (c["tick_h"] // seg_ticks, c["tick_l"] // seg_ticks):
                mc = coarse_mc[c["tmpl"]]
                exp |= {f for f in range(len(fine_mc)) if abs(fine_mc[f] - mc) <= 0.05 * mc}
        assert out[s].tolist() == sorted(exp)


# --------------------------------------------------------------------------------------
# Welch PSD: special case of a library routine, and consistency with the true PSD
# --------------------------------------------------------------------------------------
def test_welch_matches_scipy():
    fs, L = 512.0, 1024
    s = np.random.default_rng(3).standard_normal(16384) * 5.0
    mine = oracle.welch_psd(s, fs, L)
    _, ref = scipy.signal.welch(s, fs=fs, window="hann", nperseg=L, noverlap=L // 2,
                                detrend=False, scaling="density", average="mean")
    assert np.allclose(mine, ref, rtol=1e-12, atol=0)


def test_welch_estimates_the_synthetic_psd():
    n, fs, f_low = 2 ** 16, 512.0, 30.0
    s, _ = synth.make_strain(901, 0, 0, n, fs, f_low)
    L = 4 * int(fs)
    p = oracle.psd_on_grid(oracle.welch_psd(s, fs, L), fs, L, n)
    f = np.arange(n // 2 + 1) * fs / n
    band = (f > 40) & (f < 200)
    ratio = p[band] / synth.aligo_psd_fit(f[band])
    assert abs(np.mean(ratio) - 1.0) < 0.05


# --------------------------------------------------------------------------------------
# Cost model: the paper's printed Hanford speed-ups
# --------------------------------------------------------------------------------------
def test_eq8_reproduces_printed_hanford_speedup():
    g = json.load(open(os.path.join(GOLDEN, "eq8_costmodel.json")))
    a = g["inputs"]
    s1 = oracle.speedup_eq8(a["n_seg"], a["n_flat"], a["n_stage1"], a["n_stage2"], a["f_flat"],
                            a["f_coarse"], a["t_seg"], 1.0)
    assert abs(s1 - g["printed"]["speedup_gamma1"]) < 0.005
    s3 = oracle.speedup_eq8(a["n_seg"], a["n_flat"], a["n_stage1"], a["n_stage2"], a["f_flat"],
                            a["f_coarse"], a["t_seg"], 3.0)
    assert abs(s3 - g["printed"]["speedup_gamma3"]) / g["printed"]["speedup_gamma3"] < 0.01


# --------------------------------------------------------------------------------------
# Band edge, whitened data and PSD interpolation: hand cases and direct sums
# --------------------------------------------------------------------------------------
def test_lowest_bin_hand_cases():
    # df = 512 / 4096 = 0.125 Hz: 30.1 Hz sits between bins 240 (30.0 Hz) and 241 (30.125 Hz);
    # the band starts at the first bin at or above f_low (a floor would give 240)
    assert oracle.lowest_bin(4096, 512.0, 30.1) == 241
    # f_low exactly on a bin: that bin is in the band
    assert oracle.lowest_bin(4096, 512.0, 30.0) == 240
    # just above a bin by one part in 1e12 of df still moves to the next bin
    assert oracle.lowest_bin(4096, 512.0, 30.0 + 0.125e-9) == 241
    # DC never enters the band
    assert oracle.lowest_bin(4096, 512.0, 0.0) == 1
    assert oracle.lowest_bin(4096, 512.0, 0.01) == 1
    # a non-power-of-two length: df = 100 / 1000 = 0.1 Hz, 20.05 Hz -> bin 201
    assert oracle.lowest_bin(1000, 100.0, 20.05) == 201


@pytest.mark.parametrize("n,fs,f_low", [(256, 64.0, 7.3), (512, 100.0, 11.11), (1024, 512.0, 30.2)])
def test_whitened_spectrum_is_direct_dft_over_sqrt_psd(n, fs, f_low):
    # f_low * n / fs is not an integer in any case, so a floor for the ceiling shows
    assert abs(f_low * n / fs - round(f_low * n / fs)) > 0.05
    g = np.random.default_rng(int(n + fs))
    s = g.standard_normal(n) * 2.0
    psd = 0.3 + g.random(n // 2 + 1)
    d = oracle.whitened_spectrum(s, fs, f_low, psd)
    assert d.shape == (n // 2,)                      # bins 0 .. n/2 - 1: Nyquist is not stored
    first = int(np.floor(f_low * n / fs)) + 1        # first bin with k df >= f_low
    j = np.arange(n)
    for k in range(n // 2):
        if k < first:
            assert d[k] == 0, k                      # DC and bins below f_low
        else:
            direct = np.sum(s * np.exp(-2j * np.pi * k * j / n)) / fs / np.sqrt(psd[k])
            assert abs(d[k] - direct) <= 1e-12 * max(1.0, abs(direct)), k
    assert d[first] != 0 and d[n // 2 - 1] != 0      # the band's first bin and the last stored bin


def test_psd_on_grid_interpolates_linearly():
    fs, L, n = 64.0, 16, 64
    # a PSD linear in f is reproduced exactly on the finer grid
    fw = np.arange(L // 2 + 1) * fs / L
    lin = 2.0 + 0.25 * fw
    out = oracle.psd_on_grid(lin, fs, L, n)
    fk = np.arange(n // 2 + 1) * fs / n
    assert out.shape == (n // 2 + 1,)
    assert np.allclose(out, 2.0 + 0.25 * fk, rtol=0, atol=1e-13)
    # hand case: the Welch grid has 4 Hz spacing, the segment grid 1 Hz; at 1/4, 1/2, 3/4 of
    # the way between two Welch bins the value moves that fraction of the way
    p = np.array([1.0, 5.0, 3.0, 3.0, 7.0, 1.0, 2.0, 2.0, 9.0])
    out = oracle.psd_on_grid(p, fs, L, n)
    assert out[0] == 1.0 and out[4] == 5.0 and out[8] == 3.0 and out[32] == 9.0
    assert np.allclose(out[1:4], [2.0, 3.0, 4.0], rtol=0, atol=1e-15)
    assert np.allclose(out[5:8], [4.5, 4.0, 3.5], rtol=0, atol=1e-15)
    assert np.allclose(out[17:20], [5.5, 4.0, 2.5], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_timeslide_coinc_matches_bruteforce_over_many_wraps(seed):
    # the slides go round the ring several times (K step = 1.5 .. 8 wraps), windows reach from a
    # few ticks to beyond one step, so a pair is coincident at several slides of one wrap or of
    # several wraps
    g = np.random.default_rng(300 + seed)
    wrap = int(g.choice([3000, 3001, 2999]))
    step = int(g.integers(70, 401))
    K = int(g.integers(20, 61))
    window = int(g.choice([int(g.integers(3, 40)), int(g.integers(40, step // 2 + 1)),
                           int(g.integers(step, min(1400, wrap // 2 - 1)))]))
    cw = int(g.integers(20, 1000))
    th = synth.synthetic_triggers(g, 3, wrap, 6, 7, wrap)
    tl = synth.synthetic_triggers(g, 3, wrap, 6, 7, wrap)
    tl["snr"][: len(tl) // 3] = th["snr"][0]
    h = dict(tmpl=th["tmpl"], tick=th["tick"], snr=th["snr"])
    l = dict(tmpl=tl["tmpl"], tick=tl["tick"], snr=tl["snr"])
    assert K * step >= 1.5 * wrap
    edges = np.array([4.0, 6.0, 8.0, 11.0, 14.0], np.float32)
    out = oracle.timeslide_coinc(h, l, K, step, window, wrap, cw, edges, 100)
    pairs, kept, stat = _brute_coinc(h, l, K, step, window, wrap, cw)
    c = out["coincs"]
    got = sorted(zip(c["slide"].tolist(), c["tmpl"].tolist(), c["tick_h"].tolist(), c["tick_l"].tolist()))
    exp = sorted((k, int(h["tmpl"][i]), int(h["tick"][i]), int(l["tick"][j])) for k, i, j in kept)
    assert got == exp and len(exp) > 0
    # a pair really coincides on more than one wrap of the ring in these cases
    ks = {}
    for k, i, j in pairs:
        ks.setdefault((i, j), []).append(k * step // wrap)
    assert any(len(set(v)) > 1 for v in ks.values())
    bg = [stat[p] for p in kept if p[0] >= 1]
    for e, cnt in zip(edges, out["bg_counts"]):
        assert cnt == sum(1 for s in bg if np.float64(s) >= np.float64(e) ** 2)


@pytest.mark.parametrize("seed", range(4))
def test_timeslide_coinc_floor_keeps_everything_at_or_above_it(seed):
    # the floor only drops coincidences below it: survivors at or above it and counts at edges at
    # or above it equal those of the plain definition (itself pinned by the brute force above)
    g = np.random.default_rng(400 + seed)
    wrap, step, window, cw, K = 40000, 700, 120, int(g.integers(300, 3000)), 50
    th = synth.synthetic_triggers(g, 5, wrap, 12, 5, wrap, snr=(3.5, 7.5))
    tl = synth.synthetic_triggers(g, 5, wrap, 12, 5, wrap, snr=(3.5, 7.5))
    h = dict(tmpl=th["tmpl"], tick=th["tick"], snr=th["snr"])
    l = dict(tmpl=tl["tmpl"], tick=tl["tick"], snr=tl["snr"])
    floor = float(g.choice([6.0, 7.0, 8.0]))
    edges = np.array([floor, floor + 0.5, floor + 1.5, 12.0], np.float32)
    full = oracle.timeslide_coinc(h, l, K, step, window, wrap, cw, edges, 100)
    cut = oracle.timeslide_coinc(h, l, K, step, window, wrap, cw, edges, 100, min_snr_c=floor)
    f, c = full["coincs"], cut["coincs"]
    keep = np.asarray(f["stat"], np.float64) >= floor ** 2
    assert 0 < len(c["slide"]) < len(f["slide"]) and np.any(~keep)
    for k in ("slide", "tmpl", "tick_h", "tick_l", "stat"):
        assert np.array_equal(np.asarray(f[k])[keep], np.asarray(c[k])), k
    assert np.array_equal(full["bg_counts"], cut["bg_counts"])
    # and the brute force with the floor applied to its pairs agrees too
    small = np.nonzero(th["tmpl"] < 2)[0], np.nonzero(tl["tmpl"] < 2)[0]
    hs_ = {k: v[small[0]] for k, v in h.items()}
    ls_ = {k: v[small[1]] for k, v in l.items()}
    cut2 = oracle.timeslide_coinc(hs_, ls_, 12, step, window, wrap, cw, edges, 100, min_snr_c=floor)
    pairs, _, stat = _brute_coinc(hs_, ls_, 12, step, window, wrap, cw)
    pairs = [p for p in pairs if np.float64(stat[p]) >= floor ** 2]

    def key(p):
        return (stat[p], -hs_["tmpl"][p[1]], -hs_["tick"][p[1]], -ls_["tick"][p[2]])
    kept = [p for p in pairs if not any(q != p and q[0] == p[0] and key(q) > key(p) and
            abs((int(hs_["tick"][q[1]]) - int(hs_["tick"][p[1]]) + wrap // 2) % wrap - wrap // 2) <= cw
            for q in pairs)]
    got = sorted(zip(cut2["coincs"]["slide"].tolist(), cut2["coincs"]["tick_h"].tolist(),
                     cut2["coincs"]["tick_l"].tolist()))
    assert got == sorted((k, int(hs_["tick"][i]), int(ls_["tick"][j])) for k, i, j in kept)
