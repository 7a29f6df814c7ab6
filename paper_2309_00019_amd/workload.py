"""The two-detector search workload shared by the benchmark and the proposer training: synthetic
stand-ins for the paper's O3 segments (coloured Gaussian noise from the analytic aLIGO-like PSD
fit, sine-Gaussian glitches at 0.05/s, TaylorF2 injections) and TaylorF2 banks placed uniformly
in tau0 and q.  Banks are generated on the host in chunks (``synth``) and prepared on the device
through hs_prepare_bank; everything else here is seeding and marshalling.
"""
import numpy as np
import torch

import synth

from . import hs

CFG = 2                      # seed family of this workload
FS, F_LOW = 2048.0, 20.0
MC_RANGE = (1.4, 10.0)
Q_RANGE = (1.0, 4.0)
GLITCH_RATE = 0.05


def bank_masses(n_tmpl: int, which: int):
    """(m1, m2) of the fine (which = 0) or coarse (which = 1) bank, sorted by chirp mass."""
    return synth.bank_by_tau0(n_tmpl, MC_RANGE[0], MC_RANGE[1], Q_RANGE[0], Q_RANGE[1],
                              synth.rng(CFG, which, 0, synth.BANK))


def make_banks(ctx, n, fs, f_low, m1, m2, psds, dtype="f32", chunk=2048, chisq_bins=8):
    """One prepared bank per PSD (device), with ``mchirp`` and ``q`` (m1 / m2) attached."""
    from synth.bank import bank_layout
    k0, kstart, k1, offset, total = bank_layout(m1, m2, n, fs, f_low)
    banks = [hs.PreparedBank.allocate(n, fs, dtype, offset, k0, total, ctx.device, chisq_bins=chisq_bins)
             for _ in psds]
    T = len(m1)
    for t0 in range(0, T, chunk):
        t1 = min(T, t0 + chunk)
        b = synth.taylorf2_bank(m1[t0:t1], m2[t0:t1], n, fs, f_low)
        raw = torch.as_tensor(b.data).to(ctx.device)
        off = torch.as_tensor(b.offset, device=ctx.device)
        kk0 = torch.as_tensor(b.k0, device=ctx.device)
        kks = torch.as_tensor(b.kstart, device=ctx.device)
        kk1 = torch.as_tensor(b.k1, device=ctx.device)
        for bank, psd in zip(banks, psds):
            hs.hs_prepare_bank(ctx, n, fs, f_low, psd, raw, off, kk0, kks, kk1, dtype, bank=bank, t0=t0,
                               elem0=int(offset[t0]))
        del raw
    mc = torch.as_tensor(synth.mchirp_eta(m1, m2)[0], device=ctx.device)
    q = torch.as_tensor(np.asarray(m1, np.float64) / np.asarray(m2, np.float64), device=ctx.device)
    for bank in banks:
        bank.mchirp = mc
        bank.q = q
    return banks


def background_strains(n: int):
    """The background segment pair (noise + glitches, no signal): float32 [n] per detector."""
    return [synth.make_strain(CFG, det, 0, n, FS, F_LOW, glitch_rate=GLITCH_RATE)[0] for det in (0, 1)]


def injection_amplitudes(m1, m2, snr, n: int, fs: float = FS, f_low: float = F_LOW, chunk: int = 256):
    """Loudness of the synthetic injections: the factor on synth's TaylorF2 spectrum of each pair
    (m1, m2) that makes its optimal SNR ``snr`` in the analytic PSD of the synthetic noise,
    snr / sigma with sigma^2 = 4 df sum |h~_k|^2 / S(f_k) over the waveform's bins kstart..k1
    (float64, on the host: part of preparing the inputs, not of the search)."""
    m1, m2, snr = (np.atleast_1d(np.asarray(x, np.float64)) for x in (m1, m2, snr))
    df = fs / n
    sig = np.empty(len(m1))
    for c0 in range(0, len(m1), chunk):
        b = synth.taylorf2_bank(m1[c0:c0 + chunk], m2[c0:c0 + chunk], n, fs, f_low)
        for t in range(b.n_tmpl):
            lo, hi = int(b.kstart[t]), int(b.k1[t])
            h = b.spectrum(t)[lo:hi + 1]
            psd = synth.aligo_psd_fit(np.arange(lo, hi + 1) * df)
            sig[c0 + t] = np.sqrt(4.0 * df * np.sum(np.abs(h) ** 2 / psd))
    return snr / sig


def realisation_jobs(seeds, per_seg: int, n: int, cfg: int = CFG, mc_range=MC_RANGE, q_range=Q_RANGE,
                     glitch_rate: float = GLITCH_RATE, margin: float = 8.0):
    """Process-pool jobs (synth.realisation_job) of the two-detector realisations ``seeds``: each
    with ``per_seg`` injections (network SNR 6-20 split equally between the detectors, L arrival
    within +-10 ms) and their amplitude factors.  A generator: the amplitudes of a realisation are
    computed when the pool asks for its job."""
    for r in seeds:
        ip = synth.realisation_params(cfg, r, n / FS, per_seg, mc_range, q_range, margin)
        amp_h = injection_amplitudes(ip["m1"], ip["m2"], ip["snr_h"], n) if per_seg else np.empty(0)
        amp_l = amp_h * (ip["snr_l"] / ip["snr_h"]) if per_seg else np.empty(0)
        yield (r, cfg, n, FS, F_LOW, ip, amp_h, amp_l, glitch_rate)


def injection_realisation(r: int, n: int, per_seg: int = 1, margin: float = 8.0):
    """Realisation r: independent noise + glitches in both detectors with ``per_seg`` injections.
    Returns (strain_h, strain_l, params) with the parameter arrays of synth.injection_params."""
    return synth.realisation_job(next(realisation_jobs([r], per_seg, n, margin=margin)))[1]
