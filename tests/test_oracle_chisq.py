"""Pins of the oracle's power-consistency chi-square and the re-weighted SNR of Eq. (4)."""
import numpy as np

import oracle
import synth


def _psd(n, fs):
    k = np.arange(n // 2 + 1)
    p = np.empty(n // 2 + 1)
    p[1:] = synth.aligo_psd_fit(k[1:] * fs / n)
    p[0] = p[1]
    return p


def _setup(mass=10.0, n=8192, fs=512.0, f_low=30.0):
    b = synth.taylorf2_bank([mass], [mass], n, fs, f_low)
    h = b.spectrum(0)
    psd = _psd(n, fs)
    k_lo, k_hi = oracle.band_edges(n, fs, f_low, b.kstart[0], b.k1[0])
    sig = oracle.template_sigma(h, psd, n, fs, k_lo, k_hi)
    return b, h, psd, k_lo, k_hi, sig


def test_bins_split_power_equally_up_to_one_bin():
    b, h, psd, k_lo, k_hi, sig = _setup()
    p = 8
    e = oracle.chisq_bin_edges(h, psd, k_lo, k_hi, p)
    assert e[0] == k_lo and e[-1] == k_hi + 1 and np.all(np.diff(e) > 0)
    pw = np.abs(h[k_lo:k_hi + 1]) ** 2 / psd[k_lo:k_hi + 1]
    parts = np.array([pw[e[l] - k_lo:e[l + 1] - k_lo].sum() for l in range(p)])
    assert np.all(np.abs(parts - pw.sum() / p) <= pw.max() + 1e-12 * pw.sum())


def test_chisq_reduced_has_unit_mean_in_gaussian_noise():
    n, fs, f_low = 8192, 512.0, 30.0
    b, h, psd, k_lo, k_hi, sig = _setup(12.0, n, fs, f_low)
    e = oracle.chisq_bin_edges(h, psd, k_lo, k_hi, 8)
    vals = []
    for seed in range(12):
        s, _ = synth.make_strain(910, 0, seed, n, fs, f_low)
        st = oracle.strain_fft(s, fs)
        for m in range(0, n, 257):
            vals.append(oracle.chisq_at(st, h, psd, n, fs, sig, m, e)[0])
    vals = np.asarray(vals)
    # chi2 has 2p - 2 = 14 degrees of freedom: mean 1, variance 2/14 per independent draw
    assert abs(vals.mean() - 1.0) < 0.06
    assert abs(vals.var() - 2.0 / 14.0) < 0.05


def test_chisq_vanishes_for_the_matching_signal_and_z_is_the_snr():
    n, fs = 8192, 512.0
    b, h, psd, k_lo, k_hi, sig = _setup(10.0, n, fs)
    m0, amp = 3001, 2.0
    x = np.fft.irfft(np.exp(0.3j) * h, n=n) * fs
    st = oracle.strain_fft(amp * np.roll(x, m0), fs)
    e = oracle.chisq_bin_edges(h, psd, k_lo, k_hi, 8)
    chi2_r, z = oracle.chisq_at(st, h, psd, n, fs, sig, m0, e)
    zs = oracle.snr_series(st, h, psd, n, fs, k_lo, k_hi, sig)
    assert abs(z - zs[m0]) < 1e-9 * abs(z)
    assert chi2_r < 1e-3 * abs(z) ** 2 / 8


def test_bin_snrs_sum_to_the_fft_snr_at_every_sample_in_noise():
    # the p bins tile the filter's band, so the per-bin sums add up to z[m] of the inverse FFT at
    # any sample, signal or not (the identity that lets the widest bin be formed from z)
    n, fs, f_low = 8192, 512.0, 30.0
    b, h, psd, k_lo, k_hi, sig = _setup(14.0, n, fs, f_low)
    s, _ = synth.make_strain(911, 0, 3, n, fs, f_low)
    st = oracle.strain_fft(s, fs)
    zs = oracle.snr_series(st, h, psd, n, fs, k_lo, k_hi, sig)
    for p in (2, 5, 8, 16):
        e = oracle.chisq_bin_edges(h, psd, k_lo, k_hi, p)
        for m in (0, 1, 777, n // 2, n - 1):
            zl = oracle.bin_snrs(st, h, psd, n, fs, sig, m, e)
            assert abs(zl.sum() - zs[m]) < 1e-9 * max(1.0, abs(zs[m]))
            assert abs(oracle.chisq_at(st, h, psd, n, fs, sig, m, e)[1] - zs[m]) < 1e-9 * max(1.0, abs(zs[m]))


def test_chisq_flags_a_loud_sine_gaussian():
    n, fs, f_low = 8192, 512.0, 30.0
    b, h, psd, k_lo, k_hi, sig = _setup(9.0, n, fs, f_low)
    t = np.arange(n) / fs
    tau = 9.0 / (np.sqrt(2) * np.pi * 120.0)
    g = 4000.0 * np.exp(-((t - 8.0) / tau) ** 2) * np.sin(2 * np.pi * 120.0 * (t - 8.0))
    s, _ = synth.make_strain(911, 0, 0, n, fs, f_low)
    st = oracle.strain_fft(s + g, fs)
    zs = oracle.snr_series(st, h, psd, n, fs, k_lo, k_hi, sig)
    m = int(np.argmax(np.abs(zs)))
    e = oracle.chisq_bin_edges(h, psd, k_lo, k_hi, 8)
    chi2_r, _ = oracle.chisq_at(st, h, psd, n, fs, sig, m, e)
    rho = abs(zs[m])
    assert rho > 8 and chi2_r > 5
    assert oracle.reweighted_snr([rho], [chi2_r])[0] < 0.75 * rho


def test_reweighted_snr_properties_of_eq4():
    rho = np.full(5, 10.0)
    c = np.array([0.0, 0.5, 1.0, 2.0, 8.0])
    r = oracle.reweighted_snr(rho, c)
    assert np.all(r[:3] == 10.0)                      # identity up to chi2_r = 1 (continuous there)
    assert np.all(np.diff(r[2:]) < 0)                 # decreasing above
    big = oracle.reweighted_snr([10.0], [1e4])[0]
    assert abs(big / (10.0 * 2 ** (1 / 6) * 1e4 ** -0.5) - 1) < 1e-6   # tends to rho (2/chi2_r^3)^(1/6)
