"""The benchmark's host-side statistics of the injection campaign (CPU).

``found_injections`` (a zero-lag coincidence within the tolerance of an injection's H arrival at
or above the network-SNR bar) on hand-built records, and ``paired_miss_interval`` (the paired
extra-missed fraction, its Wald interval and the exact upper bound of the lost fraction) against
values worked by hand and against the binomial distribution that the exact bound inverts.
"""
import numpy as np
import pytest

import bench

COINC = np.dtype([("slide", np.int32), ("tick_h", np.int64), ("snr_c", np.float32)])


def test_found_injections_by_hand():
    rec = np.array([(0, 1000, 9.0),      # found: zero lag, at the tick, above the bar
                    (3, 5000, 20.0),     # a slid coincidence never finds an injection
                    (0, 9050, 8.0),      # at the bar (inclusive), 50 ticks late: within 50
                    (0, 12051, 30.0),    # 51 ticks late: outside
                    (0, 20000, 7.999)],  # below the bar
                   dtype=COINC)
    got = bench.found_injections(rec, [1000, 5000, 9000, 12000, 20000], 50, snr_c_min=8.0)
    assert got.tolist() == [True, False, True, False, False]


def test_paired_miss_interval_by_hand():
    ref = np.zeros(100, bool)
    new = np.zeros(100, bool)
    ref[:60] = True
    new[:55] = True                      # 5 found by the reference only
    new[60] = True                       # 1 found by the new pipeline only
    r = bench.paired_miss_interval(ref, new)
    d = (5 - 1) / 100
    half = 1.96 * np.sqrt(((5 + 1) / 100 - d * d) / 100)
    assert (r["lost"], r["gained"]) == (5, 1)
    assert r["extra_missed"] == pytest.approx(0.04, abs=1e-12)
    assert r["ci95"] == pytest.approx([round(d - half, 5), round(d + half, 5)], abs=1e-12)
    assert r["ci95"] == pytest.approx([-0.00737, 0.08737], abs=1e-5)


@pytest.mark.parametrize("n,lost", [(2040, 13), (288, 2), (500, 0)])
def test_exact_bound_inverts_the_binomial(n, lost):
    """The upper bound u of the lost fraction is the p at which losing at most `lost` of n
    injections has probability 2.5 %: binom.cdf(lost, n, u) = 0.025 (u = 1 - 0.025^(1/n) when
    nothing is lost)."""
    from scipy.stats import binom
    ref = np.ones(n, bool)
    new = np.ones(n, bool)
    new[:lost] = False
    r = bench.paired_miss_interval(ref, new)
    u = r["lost_fraction_upper95"]
    assert binom.cdf(lost, n, u) == pytest.approx(0.025, abs=2e-4)
    if lost == 0:
        assert u == pytest.approx(1.0 - 0.025 ** (1.0 / n), abs=1e-5)
    assert r["extra_missed"] == pytest.approx(lost / n, abs=1e-5)


def test_no_difference_gives_a_zero_interval():
    found = np.array([True, False, True, True, False] * 40)
    r = bench.paired_miss_interval(found, found.copy())
    assert r["extra_missed"] == 0.0 and r["ci95"] == [0.0, 0.0] and r["lost"] == 0 and r["gained"] == 0
