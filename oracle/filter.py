"""Matched filter, threshold and peak clustering (oracle, float64).

Sec. II, Eqs. (1)-(2): the SNR is the noise-weighted inner product of the data
with the template, maximised over coalescence time and phase.  Eq. (1) as
printed takes |(s, (1+i) h)|, which read literally is |Re z + Im z|; the reading
taken here is the quadrature form of Appendix A, rho = sqrt(c_0^2 + c_{pi/2}^2)
for an orthonormal pair of template phases, i.e.

  z[m] = (4 df / sigma) sum_{k in band} s~[k] conj(h~[k]) / S[k] exp(+2 pi i k m / N)
  rho[m] = |z[m]|,   phase[m] = arg z[m],   sigma^2 = (h, h) = 4 df sum |h~|^2 / S

with the band k_lo = max(ceil(f_low/df), first template bin) .. k_hi =
min(last template bin, N/2 - 1) (f_high = the template's ISCO cut or Nyquist;
DC and Nyquist excluded).  The time index m is the coalescence sample on the
circular segment (t_c = m / fs).

Threshold (Sec. II: inclusive): rho >= thr, compared as rho^2 >= thr^2.
Peak clustering (Sec. II keeps the maximum of the SNR series as the trigger; the
rule is not given): a candidate m is a trigger iff every other candidate m'
with |m' - m| <= W has rho^2[m'] < rho^2[m], or rho^2[m'] == rho^2[m] and
m' > m (ties go to the earlier sample); distance is linear within a segment.
"""
import numpy as np

from .spectral import lowest_bin


def band_edges(n: int, fs: float, f_low: float, kstart: int, k1: int):
    """Inclusive integration band (k_lo, k_hi) for one template."""
    k_lo = max(lowest_bin(n, fs, f_low), int(kstart))
    k_hi = min(int(k1), n // 2 - 1)
    return k_lo, k_hi


def template_sigma(htilde: np.ndarray, psd: np.ndarray, n: int, fs: float, k_lo: int, k_hi: int) -> float:
    """sigma = sqrt((h, h)) over the band (Eq. (2) with x = y = h)."""
    df = fs / n
    h = np.asarray(htilde[k_lo:k_hi + 1], dtype=np.complex128)
    return float(np.sqrt(4.0 * df * np.sum((h.real ** 2 + h.imag ** 2) / psd[k_lo:k_hi + 1])))


def snr_series(stilde: np.ndarray, htilde: np.ndarray, psd: np.ndarray, n: int, fs: float,
               k_lo: int, k_hi: int, sigma: float = None) -> np.ndarray:
    """Complex SNR series z[m], m = 0..N-1 (see module docstring)."""
    df = fs / n
    if sigma is None:
        sigma = template_sigma(htilde, psd, n, fs, k_lo, k_hi)
    q = np.zeros(n, dtype=np.complex128)
    sl = slice(k_lo, k_hi + 1)
    q[sl] = np.asarray(stilde[sl], np.complex128) * np.conj(np.asarray(htilde[sl], np.complex128)) / psd[sl]
    # numpy's ifft carries 1/N: multiply by N to obtain the plain sum over k.
    return np.fft.ifft(q) * (n * 4.0 * df / sigma)


def threshold_candidates(z: np.ndarray, thr: float):
    """Samples with |z|^2 >= thr^2: returns (m int64, rho2 float64, phase float64)."""
    r2 = z.real ** 2 + z.imag ** 2
    m = np.nonzero(r2 >= thr * thr)[0]
    return m, r2[m], np.angle(z[m])


def cluster_peaks(m: np.ndarray, rho2: np.ndarray, window: int) -> np.ndarray:
    """Indices (into the inputs) of the candidates that are peaks within +-window samples.

    Candidate i survives iff for every other candidate j with |m_j - m_i| <= window:
    rho2_j < rho2_i, or rho2_j == rho2_i and m_j > m_i.  Returned in increasing m.
    """
    m = np.asarray(m, dtype=np.int64)
    rho2 = np.asarray(rho2)
    order = np.argsort(m, kind="stable")
    ms = m[order]
    rs = rho2[order]
    lo = np.searchsorted(ms, ms - window, side="left")
    hi = np.searchsorted(ms, ms + window, side="right")
    keep = []
    for i in range(len(ms)):
        nb_r = rs[lo[i]:hi[i]]
        nb_m = ms[lo[i]:hi[i]]
        beats = (nb_r > rs[i]) | ((nb_r == rs[i]) & (nb_m < ms[i]))
        if not np.any(beats):
            keep.append(order[i])
    return np.asarray(keep, dtype=np.int64)


def filter_bank(stilde: np.ndarray, psd: np.ndarray, n: int, fs: float, f_low: float, bank,
                tmpl_ids, thr: float, keep_series: bool = False):
    """Matched-filter every template in ``tmpl_ids`` and threshold.

    ``stilde`` holds x~[k] for k = 0..N/2 at least up to the largest band bin
    (a stage at a lower sample rate passes the leading bins of the full-rate
    transform; ideal decimation keeps x~[k] for |f_k| < fs/2 unchanged).
    Returns dict(tpos, m, rho2, phase, sigma[, series]).
    """
    tp, ms, r2s, phs, sig, series = [], [], [], [], [], []
    for p, t in enumerate(tmpl_ids):
        h = bank.spectrum(int(t))
        k_lo, k_hi = band_edges(n, fs, f_low, bank.kstart[t], bank.k1[t])
        s = template_sigma(h, psd, n, fs, k_lo, k_hi)
        z = snr_series(stilde, h, psd, n, fs, k_lo, k_hi, s)
        m, r2, ph = threshold_candidates(z, thr)
        tp.append(np.full(len(m), p, np.int64))
        ms.append(m)
        r2s.append(r2)
        phs.append(ph)
        sig.append(s)
        if keep_series:
            series.append(z)
    out = dict(tpos=np.concatenate(tp) if tp else np.zeros(0, np.int64),
               m=np.concatenate(ms) if ms else np.zeros(0, np.int64),
               rho2=np.concatenate(r2s) if r2s else np.zeros(0),
               phase=np.concatenate(phs) if phs else np.zeros(0),
               sigma=np.asarray(sig))
    if keep_series:
        out["series"] = series
    return out


def triggers_from_candidates(tpos, m, rho2, phase, tmpl_ids, window: int, seg: int,
                             seg_t0_ticks: int, ticks_per_sample: int):
    """Cluster each template's candidates and emit triggers sorted by (tpos, m).

    tick = seg_t0 + m * ticks_per_sample (no sub-sample interpolation);
    snr = sqrt(rho2).  Returns dict of column arrays (seg, tmpl, tick, snr, phase, rho2, tpos).
    """
    tpos = np.asarray(tpos, np.int64)
    m = np.asarray(m, np.int64)
    cols = dict(seg=[], tmpl=[], tick=[], snr=[], phase=[], rho2=[], tpos=[])
    for p in np.unique(tpos):
        sel = np.nonzero(tpos == p)[0]
        k = sel[cluster_peaks(m[sel], rho2[sel], window)]
        cols["seg"].append(np.full(len(k), seg, np.int64))
        cols["tmpl"].append(np.full(len(k), int(tmpl_ids[p]), np.int64))
        cols["tick"].append(seg_t0_ticks + m[k] * ticks_per_sample)
        cols["snr"].append(np.sqrt(np.asarray(rho2[k], np.float64)))
        cols["phase"].append(np.asarray(phase[k], np.float64))
        cols["rho2"].append(rho2[k])
        cols["tpos"].append(np.full(len(k), p, np.int64))
    return {c: (np.concatenate(v) if v else np.zeros(0)) for c, v in cols.items()}
