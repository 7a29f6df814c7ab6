"""Pins of the oracle's background tail fit and extrapolated FAR (Sec. IV, Eqs. (6)-(7))."""
import math

import numpy as np

from oracle import farfit as F


def test_fit_recovers_an_exact_exponential_tail():
    edges = np.arange(8.0, 12.01, 0.25, dtype=np.float32)
    a, b = 30.0, -1.5
    counts = np.round(np.exp(a + b * edges.astype(np.float64))).astype(np.int64)
    alpha, beta, used = F.tail_fit(edges, counts, 8.0)
    assert used == len(edges)
    assert abs(beta - b) < 1e-5 and abs(alpha - a) < 1e-4


def test_fit_is_the_least_squares_line_of_numpy_polyfit():
    g = np.random.default_rng(1)
    edges = np.arange(6.0, 11.0, 0.1, dtype=np.float32)
    counts = g.integers(1, 10 ** 6, len(edges))
    counts[[3, 17]] = 0                            # zero counts are left out of the fit
    alpha, beta, used = F.tail_fit(edges, counts, 7.0)
    x = edges.astype(np.float64)
    sel = (x >= np.float32(7.0)) & (counts > 0)
    pb, pa = np.polyfit(x[sel], np.log(counts[sel]), 1)
    assert used == sel.sum()
    assert abs(beta - pb) < 1e-10 * abs(pb) and abs(alpha - pa) < 1e-10 * abs(pa)


def test_gaussian_network_snr_tail_slope():
    # two detectors, Gaussian noise: rho_c^2 is chi-square with 4 degrees of freedom (Appendix A),
    # P(rho_c >= x) = (1 + x^2 / 2) exp(-x^2 / 2); its log-slope at x is -x + x / (1 + x^2 / 2)
    N = 1e22                      # counts 4e9 .. 1e8: rounding is negligible
    edges = np.arange(8.0, 8.5, 0.05, dtype=np.float32)
    x = edges.astype(np.float64)
    counts = np.round(N * (1 + x ** 2 / 2) * np.exp(-x ** 2 / 2)).astype(np.int64)
    _, beta, _ = F.tail_fit(edges, counts, 8.0)
    xm = x.mean()
    assert abs(beta - (-xm + xm / (1 + xm ** 2 / 2))) < 0.02


def test_counts_are_inclusive_at_the_edge():
    bg = np.float32([49.0, 48.999996, 64.0, 81.0])
    assert list(F.cumulative_counts(bg, [7.0, 8.0, 9.0, 9.5])) == [3, 2, 1, 0]


def test_hybrid_far_by_hand():
    bg = np.float32([50.0, 60.0, 70.0, 90.0])
    t_b = 1000.0
    alpha, beta = 12.0, -1.5
    got = F.far(np.float32([55.0, 60.0, 100.0]), bg, t_b, alpha, beta, 9.0)
    assert got[0] == (1 + 3) / t_b                # 60, 70, 90 >= 55
    assert got[1] == (1 + 3) / t_b                # inclusive
    assert abs(got[2] - math.exp(alpha + beta * 10.0) / t_b) < 1e-18


def test_ifar_threshold_inverts_the_fitted_far():
    alpha, beta, t_b = 14.2, -1.7, 5.12e5
    yr = 365.25 * 86400.0
    for ifar in (yr, 10 * yr):
        x = F.ifar_threshold(alpha, beta, t_b, ifar)
        assert abs(math.exp(alpha + beta * x) / t_b - 1.0 / ifar) < 1e-9 / ifar
    assert F.ifar_threshold(alpha, beta, t_b, 10 * yr) > F.ifar_threshold(alpha, beta, t_b, yr)
