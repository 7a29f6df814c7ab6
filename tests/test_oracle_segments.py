"""Pins of the oracle's blocks of overlapping segments (valid regions, per-block PSD, timeline)
against brute force and library routines."""
import numpy as np
import pytest
import scipy.signal

import oracle
import synth
from helpers import loud
from oracle import segments as S


def _compact_filter(g, P_lo, P_hi):
    """A real filter on lags -P_lo..P_hi with zero sum and zero alternating sum (so dropping DC and
    Nyquist from a one-sided spectrum leaves it unchanged)."""
    j = np.arange(-P_lo, P_hi + 1)
    v = g.standard_normal(len(j))
    a = (-1.0) ** (j % 2)
    M = np.stack([np.ones_like(v), a])
    v -= M.T @ np.linalg.lstsq(M.T, v, rcond=None)[0]     # project out both constraints
    return dict(j=j, v=v)


@pytest.mark.parametrize("n,pad_lo,pad_hi,P_lo,P_hi", [(256, 40, 12, 37, 11), (1024, 300, 50, 300, 49),
                                                        (512, 64, 64, 10, 3)])
def test_valid_region_equals_linear_correlation(n, pad_lo, pad_hi, P_lo, P_hi):
    """Inside the valid region a segment's circular filter output equals the plain linear
    correlation of the block's data (exactly, for a filter whose support fits the pads); just
    before it the circular wrap makes them differ."""
    g = np.random.default_rng(n + pad_lo)
    fs = 64.0
    block = g.standard_normal(5 * n)
    filt = _compact_filter(g, P_lo, P_hi)
    # one-sided spectrum of the filter on the segment grid, dt-weighted like the data transform
    full = np.zeros(n)
    full[filt["j"] % n] = filt["v"]
    h = np.fft.rfft(full) / fs
    psd = np.ones(n // 2 + 1)
    starts = S.segment_starts(len(block), n, pad_lo, pad_hi)
    assert len(starts) >= 3
    for st in starts:
        seg = block[st:st + n]
        z = oracle.snr_series(oracle.strain_fft(seg, fs), h, psd, n, fs, 1, n // 2 - 1, sigma=1.0)
        for m in range(n):
            t = st + m
            if not (0 <= t - P_lo and t + P_hi < len(block)):
                continue
            lin = 2.0 / fs * S.linear_correlation(block, filt, t).real
            if S.valid_mask(m, n, pad_lo, pad_hi):
                assert abs(z[m].real - lin) <= 1e-12 * max(1.0, abs(lin)), (st, m)
        # the sample just before the valid region sees the wrap whenever the filter reaches it
        if P_lo >= pad_lo - 1 and st > 0:
            m = pad_lo - P_lo // 2 - 1
            lin = 2.0 / fs * S.linear_correlation(block, filt, st + m).real
            assert abs(z[m].real - lin) > 1e-6


def test_valid_regions_tile_the_block():
    for n, pad_lo, pad_hi, L in ((1024, 288, 32, 8192), (2 ** 20, 144 * 2048, 16 * 2048, 2 ** 23)):
        starts = S.segment_starts(L, n, pad_lo, pad_hi)
        stride = n - pad_lo - pad_hi
        covered = np.zeros(L, np.int64)
        for st in starts:
            m = np.arange(n)
            covered[st + m[S.valid_mask(m, n, pad_lo, pad_hi)]] += 1
        lo, hi = pad_lo, pad_lo + len(starts) * stride
        assert np.all(covered[lo:hi] == 1) and covered[:lo].sum() == 0 and covered[hi:].sum() == 0
        assert starts[-1] + n <= L < starts[-1] + stride + n
    # the paper-shaped block: 2^23 samples hold 11 segments of 512 s at a 352 s stride
    assert len(S.segment_starts(2 ** 23, 2 ** 20, 144 * 2048, 16 * 2048)) == 11


def test_block_psd_is_welch_of_the_block_on_the_segment_grid():
    fs, L, n = 512.0, 2048, 2 ** 14
    block = synth.make_strain(902, 0, 0, 2 ** 17, fs, 30.0)[0].astype(np.float64)
    p = S.block_psd(block, fs, L, n)
    f_w, ref_w = scipy.signal.welch(block, fs=fs, window="hann", nperseg=L, noverlap=L // 2, detrend=False,
                                    scaling="density", average="mean")
    fk = np.arange(n // 2 + 1) * fs / n
    assert np.allclose(p, np.interp(fk, f_w, ref_w), rtol=1e-9, atol=1e-12 * ref_w.max())
    # the block-length grid and the segment grid share every 8th bin exactly
    p_block = S.block_psd(block, fs, L, 2 ** 17)
    assert np.array_equal(p_block[::8], p)


def test_block_search_finds_an_injection_once_on_the_valid_timeline():
    """Oracle flat search over the overlapping segments of one block: an injection whose
    coalescence lies in the part two segments overlap is reported once, by the segment whose
    valid region holds it, at its time on the valid timeline."""
    fs, f_low = 512.0, 30.0
    n, pad_lo, pad_hi = 8192, 2048, 512            # 16 s segments, 4 s / 1 s pads, 10 s stride
    L = 4 * n
    m1, m2 = synth.equal_mass_bank([9.0, 12.0, 15.0])
    t_inj = 25.3                                    # block time (s): inside segments 1 and 2
    inj = [dict(m1=12.0, m2=12.0, t_c=t_inj, phi_c=0.3, snr=14.0)]
    bh = synth.make_strain(903, 0, 0, L, fs, f_low, injections=loud(inj, L, fs, f_low))[0]
    bl = synth.make_strain(903, 1, 0, L, fs, f_low,
                           injections=loud([dict(inj[0], t_c=t_inj + 0.004, phi_c=1.2)], L, fs, f_low))[0]
    starts = S.segment_starts(L, n, pad_lo, pad_hi)
    covering = [st for st in starts if st <= t_inj * fs < st + n]
    assert len(covering) == 2
    bank = synth.taylorf2_bank(m1, m2, n, fs, f_low)
    psd = [S.block_psd(bh, fs, 1024, n)] * len(starts)
    psl = [S.block_psd(bl, fs, 1024, n)] * len(starts)
    ref = oracle.flat_search([bh[st:st + n] for st in starts], [bl[st:st + n] for st in starts], psd, psl, fs,
                             f_low, bank, n_slides=3, step_sec=1.0, edges=(8.0,), pad_lo=pad_lo, pad_hi=pad_hi)
    c = ref["coinc"]["coincs"]
    z = np.nonzero((np.asarray(c["slide"]) == 0) & (np.asarray(c["snr_c"]) >= 10.0))[0]
    assert len(z) == 1
    tick = int(c["tick_h"][z[0]])
    assert abs(tick - (t_inj * fs - pad_lo) * 100) <= 100
    assert int(c["tmpl"][z[0]]) == 1
    # every trigger sits on the valid timeline [0, n_seg * stride) in ticks
    stride = n - pad_lo - pad_hi
    for tr in (ref["trig_h"], ref["trig_l"]):
        assert np.all((tr["tick"] >= 0) & (tr["tick"] < len(starts) * stride * 100))
