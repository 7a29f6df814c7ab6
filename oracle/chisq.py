"""Power-consistency chi-square and re-weighted SNR (oracle, float64).

Sec. II down-weights triggers with the chi-square test it cites (Allen's p-bin
power-consistency test) through the re-weighted SNR of Eq. (4):

  rho~ = rho / [(1 + (chi2_r)^3) / 2]^(1/6)   if chi2_r >= 1,   rho otherwise.

The test itself is not written out in the paper; the reading taken (Allen's
construction): split the template's band into p contiguous frequency bins of
equal template power |h~|^2/S, evaluate the complex SNR restricted to each bin
at the trigger sample,

  z_l = (4 df / sigma) sum_{k in bin l} s~[k] conj(h~[k]) / S[k] exp(+2 pi i k m / N),

so that z = sum_l z_l, and form chi2 = p sum_l |z_l - z/p|^2 with 2p - 2 degrees
of freedom, chi2_r = chi2 / (2p - 2).  Bin edge l (l = 1..p-1) is the first bin
whose cumulative power from k_lo reaches l/p of the total.  The test is
evaluated for triggers with rho >= rho_min (a parameter); weaker triggers keep
chi2_r = 0 and rho~ = rho.
"""
import numpy as np


def chisq_bin_edges(htilde, psd, k_lo: int, k_hi: int, p: int) -> np.ndarray:
    """Edges e_0 = k_lo < e_1 <= ... <= e_{p-1} < e_p = k_hi + 1 of p equal-power bins."""
    h = np.asarray(htilde[k_lo:k_hi + 1], np.complex128)
    pw = (h.real ** 2 + h.imag ** 2) / psd[k_lo:k_hi + 1]
    c = np.cumsum(pw)
    total = c[-1]
    edges = [k_lo]
    for l in range(1, p):
        edges.append(k_lo + int(np.searchsorted(c, l * total / p, side="left")))
    edges.append(k_hi + 1)
    return np.asarray(edges, np.int64)


def bin_snrs(stilde, htilde, psd, n: int, fs: float, sigma: float, m: int, edges) -> np.ndarray:
    """The p band-limited complex SNRs z_l of one template at sample m."""
    df = fs / n
    p = len(edges) - 1
    zl = np.zeros(p, np.complex128)
    for l in range(p):
        k = np.arange(edges[l], edges[l + 1])
        q = np.asarray(stilde[k], np.complex128) * np.conj(np.asarray(htilde[k], np.complex128)) / psd[k]
        zl[l] = np.sum(q * np.exp(2j * np.pi * (k * m % n) / n)) * (4.0 * df / sigma)
    return zl


def chisq_terms(zl) -> np.ndarray:
    """Per-bin terms X_l = p |z_l - z/p|^2 (their sum is chi2)."""
    zl = np.asarray(zl, np.complex128)
    p = len(zl)
    return p * np.abs(zl - zl.sum() / p) ** 2


def chisq_at(stilde, htilde, psd, n: int, fs: float, sigma: float, m: int, edges) -> tuple:
    """(chi2_r, z) of one template at sample m for the given bin edges."""
    zl = bin_snrs(stilde, htilde, psd, n, fs, sigma, m, edges)
    p = len(zl)
    chi2 = p * np.sum(np.abs(zl - zl.sum() / p) ** 2)
    return chi2 / (2 * p - 2), zl.sum()


def reweighted_snr(rho, chi2_r):
    """Eq. (4)."""
    rho = np.asarray(rho, np.float64)
    chi2_r = np.asarray(chi2_r, np.float64)
    out = rho.copy()
    sel = chi2_r >= 1.0
    out[sel] = rho[sel] / ((1.0 + chi2_r[sel] ** 3) / 2.0) ** (1.0 / 6.0)
    return out
