"""Seeded synthetic inputs for the hierarchical matched-filter search.

This package produces INPUTS only: coloured Gaussian strain drawn from the
analytic aLIGO-like PSD fit, sine-Gaussian glitches, TaylorF2 template banks,
compact-binary injections and synthetic trigger lists.  It holds none of the
search's arithmetic (no whitening, no PSD weighting, no template
normalisation, no filtering, thresholding, clustering or coincidence), so the
FP64 oracle and the GPU library can both consume its outputs without sharing
any method code.

Every random draw comes from ``numpy.random.Generator(PCG64)`` seeded by
``numpy.random.SeedSequence([cfg, det, seg, stream])`` with stream
0 = noise, 1 = glitches, 2 = injections, 3 = bank, 4 = triggers.
"""
from .seeds import rng, NOISE, GLITCH, INJECT, BANK, TRIG
from .psd import aligo_psd_fit
from .noise import coloured_noise
from .bank import Bank, taylorf2_bank, mchirp_eta, bank_by_tau0, equal_mass_bank
from .glitch import sine_gaussian_glitches
from .inject import (injection_strain, injection_params, realisation_params, realisation, realisation_job,
                     single_threaded)
from .strain import make_strain
from .triggers import (TRIGGER_DTYPE, CANDIDATE_DTYPE, COINC_DTYPE,
                       synthetic_triggers, synthetic_candidates, synthetic_coincs,
                       synthetic_coinc_set)

__all__ = [
    "rng", "NOISE", "GLITCH", "INJECT", "BANK", "TRIG",
    "aligo_psd_fit", "coloured_noise", "Bank", "taylorf2_bank", "mchirp_eta",
    "bank_by_tau0", "equal_mass_bank", "sine_gaussian_glitches",
    "injection_strain", "injection_params", "realisation_params", "realisation", "realisation_job",
    "single_threaded",
    "make_strain",
    "TRIGGER_DTYPE", "CANDIDATE_DTYPE", "COINC_DTYPE",
    "synthetic_triggers", "synthetic_candidates", "synthetic_coincs", "synthetic_coinc_set",
]
