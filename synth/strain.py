"""One detector segment of synthetic strain: noise + glitches + injections, cast to float32."""
import numpy as np

from .seeds import rng, NOISE, GLITCH
from .noise import coloured_noise
from .glitch import sine_gaussian_glitches
from .inject import injection_strain
from .psd import aligo_psd_fit


def make_strain(cfg: int, det: int, seg: int, n: int, fs: float, f_low: float,
                glitch_rate: float = 0.0, injections=(), psd_fn=aligo_psd_fit,
                noise: bool = True):
    """Return (float32 strain [n], info dict).

    ``injections`` is a sequence of dicts with keys m1, m2, t_c, phi_c, snr.
    Noise is high-passed at 0.75 f_low.
    """
    s = np.zeros(n, dtype=np.float64)
    if noise:
        s += coloured_noise(n, fs, rng(cfg, det, seg, NOISE), 0.75 * f_low, psd_fn)
    glitches = []
    if glitch_rate > 0:
        g, glitches = sine_gaussian_glitches(n, fs, rng(cfg, det, seg, GLITCH), glitch_rate,
                                             psd_fn=psd_fn)
        s += g
    for inj in injections:
        s += injection_strain(n, fs, f_low, inj["m1"], inj["m2"], inj["t_c"], inj["phi_c"],
                              inj["snr"], psd_fn)
    return s.astype(np.float32), dict(glitches=glitches)
