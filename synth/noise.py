"""Stationary coloured Gaussian noise with a prescribed one-sided PSD.

Frequency-domain synthesis on the circular grid f_k = k / T:
  n~_k = sqrt(S(f_k) / (4 df)) (x + i y),  x, y ~ N(0, 1),  0 < k < N/2,
with DC and Nyquist zero and an ideal high-pass below ``f_min`` (bins with
f_k < f_min are zero so the FP32 strain is not dominated by sub-band power).
The time series is n[j] = df * sum_k n~_k e^{2 pi i k j / N} (the inverse of
n~_k = dt sum_j n[j] e^{-2 pi i k j / N}), which for this draw has
E|n~_k|^2 = S_k / (2 df), i.e. one-sided PSD S.
"""
import numpy as np

from .psd import aligo_psd_fit


def coloured_noise(n: int, fs: float, gen: np.random.Generator, f_min: float,
                   psd_fn=aligo_psd_fit) -> np.ndarray:
    """Return float64 noise of length ``n`` sampled at ``fs`` Hz."""
    # numpy's irfft carries a 1/N; multiplying by N*df = fs undoes it and applies df.
    return np.fft.irfft(coloured_noise_spectrum(n, fs, gen, f_min, psd_fn), n=n) * fs


def coloured_noise_spectrum(n: int, fs: float, gen: np.random.Generator, f_min: float,
                            psd_fn=aligo_psd_fit) -> np.ndarray:
    """The one-sided spectrum n~_k (k = 0..n/2, complex128) of ``coloured_noise``."""
    df = fs / n
    k = np.arange(n // 2 + 1)
    f = k * df
    spec = np.zeros(n // 2 + 1, dtype=np.complex128)
    sel = (k > 0) & (k < n // 2) & (f >= f_min)
    amp = np.sqrt(psd_fn(f[sel]) / (4.0 * df))
    x = gen.standard_normal(sel.sum())
    y = gen.standard_normal(sel.sum())
    spec[sel] = amp * (x + 1j * y)
    return spec
