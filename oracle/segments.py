"""Blocks of data cut into overlapping segments, with a valid region per segment (oracle, float64)
-- TEST INFRASTRUCTURE (see the package docstring).

Sec. V: the data come in blocks, each divided into overlapping segments of 512 s, which are
filtered one by one.  The paper gives neither the overlap nor the part of a segment's output
that is kept, nor how often the PSD is estimated.  Readings taken here:

* A segment of n samples starts every ``stride`` samples of its block; its transform is
  circular, so an output sample m is exact (equal to the linear correlation of the block's data
  with the template) only when the template's support before coalescence (its duration) fits
  in the pad_lo samples before m and the support after coalescence in the pad_hi samples after.
  The valid region is pad_lo <= m < n - pad_hi and stride = n - pad_lo - pad_hi, so the valid
  regions of consecutive segments tile the block's data from pad_lo on, each sample once.
  Defaults for 512 s segments at 2048 Hz: pad_lo = 144 s (longer than the longest 20 Hz template
  of the banks, ~125 s), pad_hi = 16 s, stride = 352 s.
* Candidates are the samples of the valid region with rho >= thr; peak clustering runs among
  them only (an invalid sample cannot suppress a valid one).
* The PSD of Eq. (2) is estimated once per block: the Welch estimate of ``spectral`` over the
  whole block, linearly interpolated onto each segment's frequency grid.
* Time: the analysed timeline is the concatenation of the valid regions; sample m of segment s
  lies at tick (s * stride + m - pad_lo) * ticks_per_sample, so the valid regions of a block map
  onto [0, n_seg * stride) without gaps or overlaps.
"""
import numpy as np

from .spectral import welch_psd, psd_on_grid


def segment_starts(block_len: int, n: int, pad_lo: int, pad_hi: int) -> np.ndarray:
    """Starts of the segments of a block: every stride = n - pad_lo - pad_hi samples, as many as
    fit entirely in the block."""
    stride = n - pad_lo - pad_hi
    if stride <= 0 or n > block_len:
        raise ValueError("segment geometry does not fit")
    return np.arange(0, block_len - n + 1, stride, dtype=np.int64)


def block_psd(block, fs: float, welch_len: int, n: int) -> np.ndarray:
    """The block's Welch PSD on a segment's grid k fs / n, k = 0..n/2."""
    return psd_on_grid(welch_psd(np.asarray(block, np.float64), fs, welch_len), fs, welch_len, n)


def valid_mask(m, n: int, pad_lo: int, pad_hi: int) -> np.ndarray:
    """True for output samples inside the valid region pad_lo <= m < n - pad_hi."""
    m = np.asarray(m, np.int64)
    return (m >= pad_lo) & (m < n - pad_hi)


def linear_correlation(block, g, t: int) -> complex:
    """sum_j block[t + j] conj(g[j]) over the template's support j in [-len_pre, len_post):
    ``g`` is a dict with arrays ``j`` (integer lags, may be negative) and ``v`` (values);
    the plain non-circular correlation of the block with the filter, used to pin the valid
    region."""
    j = np.asarray(g["j"], np.int64)
    idx = t + j
    if idx.min() < 0 or idx.max() >= len(block):
        raise ValueError("lag outside the block")
    return complex(np.sum(np.asarray(block)[idx] * np.conj(np.asarray(g["v"]))))
