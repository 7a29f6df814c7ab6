"""One detector segment of synthetic strain: noise + glitches + injections, cast to float32."""
import numpy as np

from .seeds import rng, NOISE, GLITCH
from .noise import coloured_noise_spectrum
from .glitch import sine_gaussian_glitches
from .inject import injection_spectrum
from .psd import aligo_psd_fit


def make_strain(cfg: int, det: int, seg: int, n: int, fs: float, f_low: float,
                glitch_rate: float = 0.0, injections=(), psd_fn=aligo_psd_fit,
                noise: bool = True):
    """Return (float32 strain [n], info dict).

    ``injections`` is a sequence of dicts with keys m1, m2, t_c, phi_c, amp (the factor on the
    TaylorF2 spectrum, see ``inject``).
    Noise is high-passed at 0.75 f_low.  Noise and injections are summed in the frequency
    domain and transformed once; glitches are added in the time domain.
    """
    spec = np.zeros(n // 2 + 1, dtype=np.complex128)
    if noise:
        spec += coloured_noise_spectrum(n, fs, rng(cfg, det, seg, NOISE), 0.75 * f_low, psd_fn)
    for inj in injections:
        spec += injection_spectrum(n, fs, f_low, inj["m1"], inj["m2"], inj["t_c"], inj["phi_c"], inj["amp"])
    s = np.fft.irfft(spec, n=n) * fs
    glitches = []
    if glitch_rate > 0:
        g, glitches = sine_gaussian_glitches(n, fs, rng(cfg, det, seg, GLITCH), glitch_rate,
                                             psd_fn=psd_fn)
        s += g
    return s.astype(np.float32), dict(glitches=glitches)
