"""Stage-1 follow-up selection and neighbourhood union (oracle, float64).

Sec. III: segments holding stage-1 coincidences with Lambda_1 >= 7 are
re-filtered at 2048 Hz with the templates in the neighbourhoods (nbhds) of the
followed coarse templates; the nbhds of one segment are merged into a union.
Readings: Lambda_1 is the network SNR (see ``coinc``) and the selection is
float64(stat) >= rho_min^2; the nbhd of coarse template c is every fine
template f with |Mc_f - Mc_c| <= frac * Mc_c in float64 (inclusive; chirp-mass
neighbourhood); a coincidence contributes to the segment of its H trigger and
to the segment of its (unshifted) L trigger, and a segment's union is applied
to both detectors.
"""
import numpy as np


def followup_templates(coincs, rho_min: float, coarse_mchirp, fine_mchirp, frac: float,
                       seg_ticks: int, n_seg: int):
    """Per-segment sorted unique fine-template ids (list of int64 arrays, one per segment)."""
    stat = np.asarray(coincs["stat"]).astype(np.float64)
    sel = np.nonzero(stat >= float(rho_min) ** 2)[0]
    coarse_mchirp = np.asarray(coarse_mchirp, np.float64)
    fine_mchirp = np.asarray(fine_mchirp, np.float64)
    per_seg = [set() for _ in range(n_seg)]
    for c in sel:
        mc = coarse_mchirp[int(coincs["tmpl"][c])]
        nb = np.nonzero(np.abs(fine_mchirp - mc) <= frac * mc)[0]
        segs = {int(coincs["tick_h"][c]) // seg_ticks, int(coincs["tick_l"][c]) // seg_ticks}
        for s in segs:
            if 0 <= s < n_seg:
                per_seg[s].update(int(x) for x in nb)
    return [np.asarray(sorted(s), dtype=np.int64) for s in per_seg]
