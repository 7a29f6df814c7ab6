"""Shared test helpers: inputs from ``synth``, device upload, and the tolerance rule.

Tolerance rule for floating-point parity (FP32 path against the FP64 oracle):
  rho agrees within DELTA relative; every oracle candidate with rho >= thr (1 + DELTA) must be
  found at the same sample, and every GPU candidate must have oracle rho >= thr (1 - DELTA).
Candidates in the band thr (1 +- DELTA) may go either way.
"""
import numpy as np

import synth

DELTA = {"f32": 1e-4, "bf16": 4e-3, "f16": 1e-3}


def analytic_psd(n, fs):
    k = np.arange(n // 2 + 1)
    p = np.empty(n // 2 + 1)
    p[1:] = synth.aligo_psd_fit(k[1:] * fs / n)
    p[0] = p[1]
    return p


def loud(injections, n, fs, f_low):
    """Injection dicts with a target SNR (keys m1, m2, t_c, phi_c, snr) as synth wants them (amp in
    place of snr): the amplitude factor is snr / sigma, sigma the oracle's template sigma of the
    injected waveform in the analytic PSD over its band."""
    import oracle
    psd = analytic_psd(n, fs)
    out = []
    for inj in injections:
        b = synth.taylorf2_bank([inj["m1"]], [inj["m2"]], n, fs, f_low)
        a, c = oracle.band_edges(n, fs, f_low, b.kstart[0], b.k1[0])
        sigma = oracle.template_sigma(b.spectrum(0), psd, n, fs, a, c)
        d = {k: v for k, v in inj.items() if k != "snr"}
        d["amp"] = inj["snr"] / sigma
        out.append(d)
    return out


def device_bank(ctx, bank, psd_dev, f_low, dtype="f32"):
    """Prepare a synth.Bank on the device through hs_prepare_bank."""
    import torch
    from paper_2309_00019_amd import hs
    dev = ctx.device
    raw = torch.as_tensor(bank.data, device=dev)
    off = torch.as_tensor(bank.offset, device=dev)
    k0 = torch.as_tensor(bank.k0, device=dev)
    ks = torch.as_tensor(bank.kstart, device=dev)
    k1 = torch.as_tensor(bank.k1, device=dev)
    pb = hs.hs_prepare_bank(ctx, bank.n, bank.fs, f_low, psd_dev, raw, off, k0, ks, k1, dtype)
    pb.mchirp = torch.as_tensor(bank.mchirp, device=dev)
    return pb


def check_candidates(gpu_m, gpu_r2, z_oracle, thr, delta):
    """Apply the tolerance rule to one template, given the oracle's full complex SNR series.

    Returns the largest relative rho error over the GPU candidates."""
    gpu_m = np.asarray(gpu_m, np.int64)
    gpu_r2 = np.asarray(gpu_r2, np.float64)
    r2o = np.abs(z_oracle) ** 2
    hi = (thr * (1 + delta)) ** 2
    lo = (thr * (1 - delta)) ** 2
    must = np.nonzero(r2o >= hi)[0]
    missing = np.setdiff1d(must, gpu_m)
    assert len(missing) == 0, f"{len(missing)} oracle candidates missing on GPU, e.g. m={missing[:5]}"
    assert len(np.unique(gpu_m)) == len(gpu_m), "duplicate GPU candidates"
    assert np.all(r2o[gpu_m] >= lo), "GPU candidate below the tolerance band of the oracle"
    if len(gpu_m) == 0:
        return 0.0
    err = np.abs(np.sqrt(gpu_r2) / np.sqrt(r2o[gpu_m]) - 1.0)
    return float(err.max())
