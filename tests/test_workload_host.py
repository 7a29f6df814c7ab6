"""Input preparation of the benchmark workload, on the host (CPU).

The injection amplitude factors that the benchmark's campaign, the proposer's training data and
the day run use (``workload.injection_amplitudes``: snr / sigma in the analytic PSD of the
synthetic noise) against the oracle's template sigma (Sec. II, Eq. (2) with x = y = h) over the
oracle's band of each waveform.  The two are written independently and must agree to rounding,
for light systems whose band runs to Nyquist and heavy ones cut at ISCO.  And the timeline of
overlapping segments (Sec. V): where each segment's valid samples lie in ticks.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import analytic_psd


@pytest.mark.parametrize("n,fs", [(2 ** 17, 2048.0), (2 ** 15, 512.0)])
def test_injection_amplitudes_equal_snr_over_oracle_sigma(n, fs):
    from paper_2309_00019_amd import workload
    f_low = 20.0
    m1 = np.array([1.4, 2.0, 5.0, 12.0, 30.0])
    m2 = np.array([1.4, 1.5, 3.0, 8.0, 25.0])
    snr = np.array([6.0, 9.5, 12.0, 20.0, 7.25])
    amp = workload.injection_amplitudes(m1, m2, snr, n, fs, f_low, chunk=2)   # chunks of 2, 2, 1
    psd = analytic_psd(n, fs)
    b = synth.taylorf2_bank(m1, m2, n, fs, f_low)
    assert b.k1.max() == n // 2 - 1 and b.k1.min() < n // 2 - 1             # Nyquist and ISCO ends
    for t in range(len(m1)):
        a, c = oracle.band_edges(n, fs, f_low, b.kstart[t], b.k1[t])
        sigma = oracle.template_sigma(b.spectrum(t), psd, n, fs, a, c)
        assert amp[t] * sigma == pytest.approx(snr[t], rel=1e-12)


def test_timeline_of_overlapping_segments():
    """Sample m of segment s lies at tick s * share + (m - pad_lo) * ticks_per_sample: 512 s
    segments at 2048 Hz with 144 s / 16 s pads share 352 s of the timeline each; pads that are
    negative, fill the segment or are not multiples of the stage-1 decimation are refused."""
    from paper_2309_00019_amd import search
    n = 2 ** 20
    cfg = search.SearchConfig(pad_lo_sec=144.0, pad_hi_sec=16.0)
    tpt, plo, phi, share = search.timeline(cfg, n)
    assert (tpt, plo, phi) == (25, 144 * 2048, 16 * 2048)
    assert share == 352 * 51200
    assert search.timeline(search.SearchConfig(), n) == (25, 0, 0, n * 25)
    for lo, hi in ((-1.0, 0.0), (256.0, 256.0), (144.0 + 1.0 / 2048, 16.0)):
        with pytest.raises(ValueError):
            search.timeline(search.SearchConfig(pad_lo_sec=lo, pad_hi_sec=hi), n)
