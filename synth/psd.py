"""Analytic aLIGO-like one-sided noise PSD fit used to colour the synthetic strain.

S(f) = S0 [ x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2) / (1 + x^2/2) ],  x = f / 215 Hz.

S0 is arbitrary for the search (the SNR does not depend on it); S0 = 1 keeps
strain values O(1..1e3) so FP32 data stays well inside its range.
"""
import numpy as np


def aligo_psd_fit(f, s0: float = 1.0):
    """Evaluate the fit at frequencies ``f`` (Hz, > 0).  Returns float64."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    return s0 * (x ** -4.14 - 5.0 * x ** -2 + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))
