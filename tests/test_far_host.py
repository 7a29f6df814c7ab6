"""The library's host-side tail fit (hs_far_fit, hs_far_threshold) against the oracle: pure host
code, so it runs without a GPU."""
import numpy as np

from oracle import farfit as F


def test_far_fit_matches_oracle():
    from paper_2309_00019_amd import hs
    g = np.random.default_rng(3)
    for trial in range(5):
        edges = np.arange(6.0, 12.0, 0.1, dtype=np.float32)
        counts = np.sort(g.integers(0, 10 ** 7, len(edges)))[::-1].copy()
        counts[g.integers(0, len(edges), 5)] = 0
        x_min = float(g.uniform(6.0, 9.0))
        a, b, m = hs.hs_far_fit(edges, counts, x_min)
        ra, rb, rm = F.tail_fit(edges, counts, x_min)
        assert m == rm
        assert abs(a - ra) <= 1e-12 * abs(ra) and abs(b - rb) <= 1e-12 * abs(rb)


def test_far_fit_rejects_fewer_than_two_points():
    import pytest
    from paper_2309_00019_amd import hs
    with pytest.raises(hs.HsError):
        hs.hs_far_fit(np.float32([8.0, 9.0, 10.0]), np.int64([5, 0, 0]), 7.0)


def test_far_threshold_matches_oracle():
    from paper_2309_00019_amd import hs
    yr = 365.25 * 86400.0
    for ifar in (yr, 10 * yr):
        assert abs(hs.hs_far_threshold(14.2, -1.7, 5.12e5, ifar) - F.ifar_threshold(14.2, -1.7, 5.12e5, ifar)) < 1e-12


def test_package_eq8_matches_the_oracle_cost_model():
    """The package's own Eq. (8) (used by the benchmark) against the oracle's pinned one."""
    import oracle
    from paper_2309_00019_amd import search
    for args in ((1493, 428725, 85080, 6274846, 2048.0, 512.0, 512.0), (1, 30000, 1500, 10666, 2048.0, 512.0, 256.0)):
        for gamma in (1.0, 3.0):
            a = search.speedup_eq8(*args, gamma=gamma)
            b = oracle.speedup_eq8(*args, gamma=gamma)
            assert abs(a - b) <= 1e-12 * b
