"""Compact-binary injections (TaylorF2, same signal model as the banks).

Loudness is specified as the optimal SNR of the injected waveform in the
ANALYTIC PSD of the synthetic noise (the standard way to label an injection);
the search never sees this number - it normalises with its own PSD estimate.
"""
import numpy as np

from .bank import taylorf2_bank, tau0, masses_from_mchirp_q, MSUN_SEC
from .psd import aligo_psd_fit


def injection_strain(n: int, fs: float, f_start: float, m1: float, m2: float, t_c: float,
                     phi_c: float, snr: float, psd_fn=aligo_psd_fit) -> np.ndarray:
    """Time series (float64, length n, circular) of one injection with optimal SNR ``snr``."""
    b = taylorf2_bank([m1], [m2], n, fs, f_start, tc=[t_c], phic=[phi_c])
    h = b.spectrum(0)
    df = fs / n
    k = np.arange(n // 2 + 1)
    band = (k >= b.kstart[0]) & (k <= b.k1[0])
    opt2 = 4.0 * df * np.sum(np.abs(h[band]) ** 2 / psd_fn(k[band] * df))
    h *= snr / np.sqrt(opt2)
    return np.fft.irfft(h, n=n) * fs


def injection_params(count: int, gen: np.random.Generator, mc_min: float, mc_max: float,
                     q_min: float, q_max: float, T: float, net_snr=(6.0, 20.0),
                     dt_max: float = 0.010, margin: float = 2.0, f_ref: float = 20.0):
    """Draw injection parameters: uniform in tau0 and q, network SNR uniform, split equally
    between two detectors, L arrival offset uniform in +-dt_max, independent phases."""
    t_hi = tau0(mc_min, f_ref)
    t_lo = tau0(mc_max, f_ref)
    t = gen.uniform(t_lo, t_hi, count)
    q = gen.uniform(q_min, q_max, count)
    mc = (t / (5.0 / 256.0 * (np.pi * f_ref) ** (-8.0 / 3.0))) ** (-3.0 / 5.0) / MSUN_SEC
    m1, m2 = masses_from_mchirp_q(mc, q)
    rho = gen.uniform(net_snr[0], net_snr[1], count)
    tc_h = gen.uniform(margin, T - margin, count)
    dt = gen.uniform(-dt_max, dt_max, count)
    ph_h = gen.uniform(0.0, 2.0 * np.pi, count)
    ph_l = gen.uniform(0.0, 2.0 * np.pi, count)
    return dict(m1=m1, m2=m2, mchirp=mc, q=q, net_snr=rho, snr_h=rho / np.sqrt(2.0),
                snr_l=rho / np.sqrt(2.0), tc_h=tc_h, tc_l=tc_h + dt, phi_h=ph_h, phi_l=ph_l)
