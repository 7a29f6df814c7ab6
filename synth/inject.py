"""Compact-binary injections (TaylorF2, same signal model as the banks).

An injection is the TaylorF2 spectrum of ``synth.bank`` scaled by a plain amplitude factor
``amp``.  The generator draws target SNRs (``injection_params``) but sets no loudness itself:
turning a target SNR into ``amp`` needs an inner product against the PSD, which belongs to the
callers (the oracle's in the tests, the workload's own in the benchmark and training scripts).
"""
import numpy as np

from .bank import taylorf2_bank, tau0, masses_from_mchirp_q, MSUN_SEC


def injection_strain(n: int, fs: float, f_start: float, m1: float, m2: float, t_c: float,
                     phi_c: float, amp: float) -> np.ndarray:
    """Time series (float64, length n, circular) of one injection of amplitude factor ``amp``."""
    return np.fft.irfft(injection_spectrum(n, fs, f_start, m1, m2, t_c, phi_c, amp), n=n) * fs


def injection_spectrum(n: int, fs: float, f_start: float, m1: float, m2: float, t_c: float,
                       phi_c: float, amp: float) -> np.ndarray:
    """One-sided spectrum (k = 0..n/2, complex128) of ``injection_strain``: ``amp`` times the
    TaylorF2 spectrum of the pair (coalescence at t_c, phase phi_c)."""
    b = taylorf2_bank([m1], [m2], n, fs, f_start, tc=[t_c], phic=[phi_c])
    return b.spectrum(0) * amp


def injection_params(count: int, gen: np.random.Generator, mc_min: float, mc_max: float,
                     q_min: float, q_max: float, T: float, net_snr=(6.0, 20.0),
                     dt_max: float = 0.010, margin: float = 2.0, f_ref: float = 20.0, slots: bool = False):
    """Draw injection parameters: uniform in tau0 and q, network SNR uniform, split equally
    between two detectors, L arrival offset uniform in +-dt_max, independent phases.
    With ``slots`` the H arrival of injection k is drawn in the middle 80 % of the k-th of
    ``count`` equal slots of [margin, T - margin] (several injections per segment, apart)."""
    t_hi = tau0(mc_min, f_ref)
    t_lo = tau0(mc_max, f_ref)
    t = gen.uniform(t_lo, t_hi, count)
    q = gen.uniform(q_min, q_max, count)
    mc = (t / (5.0 / 256.0 * (np.pi * f_ref) ** (-8.0 / 3.0))) ** (-3.0 / 5.0) / MSUN_SEC
    m1, m2 = masses_from_mchirp_q(mc, q)
    rho = gen.uniform(net_snr[0], net_snr[1], count)
    if slots:
        w = (T - 2.0 * margin) / count
        tc_h = margin + (np.arange(count) + 0.1 + 0.8 * gen.random(count)) * w
    else:
        tc_h = gen.uniform(margin, T - margin, count)
    dt = gen.uniform(-dt_max, dt_max, count)
    ph_h = gen.uniform(0.0, 2.0 * np.pi, count)
    ph_l = gen.uniform(0.0, 2.0 * np.pi, count)
    return dict(m1=m1, m2=m2, mchirp=mc, q=q, net_snr=rho, snr_h=rho / np.sqrt(2.0),
                snr_l=rho / np.sqrt(2.0), tc_h=tc_h, tc_l=tc_h + dt, phi_h=ph_h, phi_l=ph_l)


def realisation_params(cfg: int, r: int, T: float, per_seg: int, mc_range, q_range, margin: float = 8.0):
    """Injection parameters of two-detector realisation r of seed family cfg (``injection_params``
    drawn from the stream rng(cfg, 0, r, INJECT); several per segment are spread over slots)."""
    from .seeds import rng, INJECT
    return injection_params(per_seg, rng(cfg, 0, r, INJECT), mc_range[0], mc_range[1], q_range[0], q_range[1], T,
                            margin=margin, slots=per_seg > 1)


def realisation(cfg: int, r: int, n: int, fs: float, f_low: float, ip, amp_h, amp_l, glitch_rate: float):
    """Two-detector realisation r of seed family cfg: independent noise and glitches with the
    injections of ``ip`` (``realisation_params``) at amplitude factors amp_h / amp_l.  Returns
    (strain_h, strain_l, ip)."""
    from .strain import make_strain
    out = []
    for det, key, amp in ((0, "h", amp_h), (1, "l", amp_l)):
        injs = [dict(m1=ip["m1"][k], m2=ip["m2"][k], t_c=ip["tc_" + key][k], phi_c=ip["phi_" + key][k],
                     amp=amp[k]) for k in range(len(amp))]
        out.append(make_strain(cfg, det, r, n, fs, f_low, glitch_rate=glitch_rate, injections=injs)[0])
    return out[0], out[1], ip


def realisation_job(args):
    """Process-pool entry: (r, cfg, n, fs, f_low, ip, amp_h, amp_l, glitch_rate) -> (r, realisation(...)).
    Lives here so spawned workers import only numpy and synth."""
    r, cfg, n, fs, f_low, ip, amp_h, amp_l, glitch = args
    return r, realisation(cfg, r, n, fs, f_low, ip, amp_h, amp_l, glitch)


def single_threaded():
    """Process-pool initialiser: one OpenMP thread for the TaylorF2 generator."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(1)
    except OSError:
        pass
