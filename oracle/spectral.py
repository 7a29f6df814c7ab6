"""Data Fourier transform, PSD estimate and whitened data (oracle, float64).

Conventions (Sec. II, Eq. (2) uses Fourier transforms x~(f) and a one-sided PSD
S_n(f) without fixing a discretisation; the reading taken here):
  x~[k] = dt * sum_j x[j] exp(-2 pi i k j / N),  f_k = k df,  df = 1/(N dt).
The paper does not say how S_n is estimated.  Reading: Welch's method with a
periodic Hann window, 50 % overlap, mean average, no detrending, one-sided
density scaling, linearly interpolated onto the segment's grid f_k.
"""
import math

import numpy as np


def strain_fft(s, fs: float) -> np.ndarray:
    """x~[k] for k = 0..N/2 (complex128)."""
    s = np.asarray(s, dtype=np.float64)
    return np.fft.rfft(s) / fs


def lowest_bin(n: int, fs: float, f_low: float) -> int:
    """First bin of the integration band, ceil(f_low / df) with df = fs / n (Eq. (2) lower limit)."""
    return max(1, int(math.ceil(f_low * n / fs)))


def welch_psd(s, fs: float, seg_len: int) -> np.ndarray:
    """One-sided Welch PSD on the grid j * fs / seg_len, j = 0..seg_len/2.

    Segments of ``seg_len`` samples start every seg_len/2 samples; each is
    multiplied by w[i] = 1/2 - 1/2 cos(2 pi i / seg_len); its periodogram
    |DFT|^2 is scaled by 1 / (fs sum w^2) and doubled for 0 < j < seg_len/2;
    the periodograms are averaged.
    """
    s = np.asarray(s, dtype=np.float64)
    L = int(seg_len)
    if L % 2 or L > len(s):
        raise ValueError("seg_len must be even and not longer than the data")
    step = L // 2
    n_seg = (len(s) - L) // step + 1
    i = np.arange(L)
    w = 0.5 - 0.5 * np.cos(2.0 * np.pi * i / L)
    acc = np.zeros(L // 2 + 1)
    for j in range(n_seg):
        x = s[j * step: j * step + L] * w
        X = np.fft.rfft(x)
        acc += np.abs(X) ** 2
    p = acc / n_seg / (fs * np.sum(w * w))
    p[1:L // 2] *= 2.0
    return p


def psd_on_grid(psd_w: np.ndarray, fs: float, seg_len: int, n: int) -> np.ndarray:
    """Linear interpolation of a Welch PSD onto f_k = k fs / n, k = 0..n/2."""
    fw = np.arange(len(psd_w)) * (fs / seg_len)
    fk = np.arange(n // 2 + 1) * (fs / n)
    return np.interp(fk, fw, psd_w)


def whitened_spectrum(s, fs: float, f_low: float, psd: np.ndarray) -> np.ndarray:
    """d~[k] = x~[k] / sqrt(S[k]) for lowest_bin <= k <= N/2 - 1, zero elsewhere; k = 0..N/2-1.

    The product d~ conj(w~) with w~ = h~/sqrt(S) is the integrand of Eq. (2);
    DC and Nyquist are excluded from the band.
    """
    n = len(s)
    st = strain_fft(s, fs)
    out = np.zeros(n // 2, dtype=np.complex128)
    k_lo = lowest_bin(n, fs, f_low)
    out[k_lo:n // 2] = st[k_lo:n // 2] / np.sqrt(psd[k_lo:n // 2])
    return out
