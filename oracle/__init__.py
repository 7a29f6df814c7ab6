"""FP64 CPU oracle for the hierarchical matched-filter search -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything in this package.  The product
path (the HIP library and its Python binding) never touches it, and this
package never imports the product path: the two share no code.  The only
module both consume is ``synth`` (seeded inputs, none of the method's
arithmetic).

Each function is the plain definition of one step of the method, in float64
NumPy/SciPy, citing the passage of the paper it follows:

* ``spectral``  -- data Fourier transform, Welch PSD, whitened data (Sec. II, Eq. (2))
* ``filter``    -- band, template sigma, complex SNR series, threshold, peak
                   clustering (Sec. II, Eqs. (1)-(2); Appendix A quadrature form)
* ``coinc``     -- two-detector coincidence, time slides, background counts,
                   false-alarm rate (Sec. I, Sec. II, Eq. (6); Appendix A network SNR)
* ``followup``  -- stage-1 selection and neighbourhood union (Sec. III)
* ``pipeline``  -- flat and two-stage hierarchical searches (Secs. II-III)
* ``costmodel`` -- matched-filter speed-up model (Sec. V, Eq. (8))
* ``chisq``     -- power-consistency chi-square, its per-bin terms, re-weighted SNR (Eq. (4))
* ``proposer``  -- learned follow-up proposer: coincidence features, MLP forward/backward,
                   Adam, cell selection and the cell-restricted neighbourhood rule
* ``farfit``    -- background tail fit and extrapolated FAR (Sec. IV, Eqs. (6)-(7))
* ``segments``  -- blocks cut into overlapping segments: valid regions, per-block PSD (Sec. V)

Where the paper is silent or garbled the reading taken is stated in the
docstring of the function that takes it.
"""
from .spectral import strain_fft, welch_psd, psd_on_grid, whitened_spectrum, lowest_bin
from .filter import (band_edges, template_sigma, snr_series, threshold_candidates,
                     cluster_peaks, filter_bank, triggers_from_candidates)
from .coinc import timeslide_coinc, false_alarm_rate, coinc_stat
from .followup import followup_templates
from .pipeline import flat_search, hierarchical_search
from .costmodel import speedup_eq8

__all__ = [
    "strain_fft", "welch_psd", "psd_on_grid", "whitened_spectrum", "lowest_bin",
    "band_edges", "template_sigma", "snr_series", "threshold_candidates", "cluster_peaks",
    "filter_bank", "triggers_from_candidates",
    "timeslide_coinc", "false_alarm_rate", "coinc_stat", "followup_templates",
    "flat_search", "hierarchical_search", "speedup_eq8",
]
from .chisq import chisq_bin_edges, chisq_at, bin_snrs, chisq_terms, reweighted_snr  # noqa: E402
from . import proposer  # noqa: E402
from . import farfit  # noqa: E402
from . import segments  # noqa: E402

__all__ += ["chisq_bin_edges", "chisq_at", "bin_snrs", "chisq_terms", "reweighted_snr", "proposer", "farfit",
            "segments"]
