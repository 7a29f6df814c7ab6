"""Independent re-count of a day's background on identical triggers (test infrastructure).

Reads the file ``python -m paper_2309_00019_amd.day --save-subset PATH`` writes (the stage-2
triggers of every 100th template of a day-long search and the GPU coincidence step's records and
background counts over exactly those triggers), runs the oracle's coincidence step (Secs. I-II,
Eq. (6)) with the same slides, window, clustering and statistic floor, and compares: records and
counts must be identical.  Then both sets of counts go through the oracle's Eq. (7) tail fit and
the network SNRs at inverse FARs of 1 and 10 years are printed side by side as one JSON line.

    python tests/day_oracle_check.py PATH
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from oracle import farfit  # noqa: E402

YEAR = 365.25 * 86400.0


def main(path):
    z = np.load(path)
    th, tl, gc = z["trig_h"], z["trig_l"], z["coincs"]
    edges = z["edges"]
    K, step, window, wrap, cw = (int(z[k]) for k in ("n_slides", "step", "window", "wrap", "cluster_w"))
    floor = float(z["min_snr_c"])
    tk = int(z["ticks_per_second"])
    t0 = time.perf_counter()
    ref = oracle.timeslide_coinc(dict(tmpl=th["tmpl"].astype(np.int64), tick=th["tick"], snr=th["snr"]),
                                 dict(tmpl=tl["tmpl"].astype(np.int64), tick=tl["tick"], snr=tl["snr"]),
                                 K, step, window, wrap, cw, edges, tk, min_snr_c=floor)
    secs = time.perf_counter() - t0
    c = ref["coincs"]
    same = len(gc) == len(c["slide"])
    for f in ("slide", "tmpl", "tick_h", "tick_l"):
        same = same and np.array_equal(gc[f].astype(np.int64), np.asarray(c[f], np.int64))
    same = same and np.array_equal(gc["stat"], np.asarray(c["stat"], np.float32))
    counts_same = bool(np.array_equal(z["bg_counts"], ref["bg_counts"]))
    t_b = K * wrap / tk
    out = {"templates": int(len(np.unique(th["tmpl"]))), "triggers": [int(len(th)), int(len(tl))],
           "coincidences": [int(len(gc)), int(len(c["slide"]))], "records_identical": bool(same),
           "bg_counts_identical": counts_same, "oracle_seconds": round(secs, 1),
           "background_years": round(t_b / YEAR, 1)}
    for name, counts in (("gpu", z["bg_counts"]), ("oracle", ref["bg_counts"])):
        a, b, m = farfit.tail_fit(edges, counts, 7.0)
        out[name] = {"alpha": a, "beta": b, "fit_points": m,
                     "rho_c_ifar_1yr": farfit.ifar_threshold(a, b, t_b, YEAR),
                     "rho_c_ifar_10yr": farfit.ifar_threshold(a, b, t_b, 10 * YEAR),
                     "counts_7_8_9_10": [int(counts[list(np.round(edges, 1)).index(x)]) for x in (7.0, 8.0, 9.0, 10.0)]}
    print(json.dumps(out), flush=True)
    return 0 if same and counts_same else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))
