"""Sine-Gaussian glitches: g(t) = A exp(-(t-t0)^2/tau^2) sin(2 pi f0 (t-t0) + phi), tau = Q/(sqrt(2) pi f0).

Times follow a Poisson process of the given rate on the circular segment; f0 is
uniform in [f_lo, f_hi]; the loudness is log-uniform in [snr_lo, snr_hi] and is
converted to an amplitude with the narrow-band approximation
  snr^2 ~= 2 h_rss^2 / S(f0),   h_rss^2 = int g^2 dt ~= A^2 tau sqrt(pi/2) / 2,
which is a property of the synthetic noise, not of the search.
"""
import numpy as np

from .psd import aligo_psd_fit


def sine_gaussian_glitches(n: int, fs: float, gen: np.random.Generator, rate: float,
                           q: float = 9.0, f_lo: float = 40.0, f_hi: float = 300.0,
                           snr_lo: float = 6.0, snr_hi: float = 50.0, psd_fn=aligo_psd_fit):
    """Return (float64 series of length n, list of glitch parameter dicts)."""
    T = n / fs
    out = np.zeros(n, dtype=np.float64)
    count = gen.poisson(rate * T)
    t0s = np.sort(gen.uniform(0.0, T, count))
    params = []
    for t0 in t0s:
        f0 = gen.uniform(f_lo, f_hi)
        snr = np.exp(gen.uniform(np.log(snr_lo), np.log(snr_hi)))
        phi = gen.uniform(0.0, 2.0 * np.pi)
        tau = q / (np.sqrt(2.0) * np.pi * f0)
        hrss_per_amp2 = tau * np.sqrt(np.pi / 2.0) / 2.0
        amp = snr * np.sqrt(psd_fn(f0) / 2.0) / np.sqrt(hrss_per_amp2)
        half = int(np.ceil(6.0 * tau * fs))
        j0 = int(np.round(t0 * fs))
        idx = np.arange(j0 - half, j0 + half + 1)
        d = idx / fs - t0
        out[idx % n] += amp * np.exp(-(d / tau) ** 2) * np.sin(2.0 * np.pi * f0 * d + phi)
        params.append(dict(t0=t0, f0=f0, snr=snr, phi=phi, amp=amp, tau=tau))
    return out, params
