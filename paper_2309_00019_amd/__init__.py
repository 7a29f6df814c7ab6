"""MI355X (gfx950) hierarchical matched-filter search: HIP kernels behind a C ABI (libhs).

Importing the package loads ``libhs.so``; a missing library raises ImportError (there
is no CPU fallback).  ``hs`` is the thin binding with the C entry-point names;
``search`` composes them into the flat and two-stage hierarchical searches.
"""
from . import hs
from .hs import (Context, PreparedBank, HsError, hs_abi_version, hs_welch_psd, hs_whiten, hs_prepare_bank,
                 hs_matched_filter, hs_snr_series, hs_cluster_triggers, hs_chisq, hs_timeslide_coinc, hs_followup,
                 as_records, to_device_records, CANDIDATE, TRIGGER, COINC)

hs.load_library()

__all__ = ["hs", "Context", "PreparedBank", "HsError", "hs_abi_version", "hs_welch_psd", "hs_whiten",
           "hs_prepare_bank", "hs_matched_filter", "hs_snr_series", "hs_cluster_triggers", "hs_chisq",
           "hs_timeslide_coinc", "hs_followup", "as_records", "to_device_records", "CANDIDATE",
           "TRIGGER", "COINC"]
