"""A day of two-detector data through the whole search: the full background estimation.

24 h of strain per detector at 2048 Hz in 338 segments of 256 s (coloured noise with
sine-Gaussian glitches at 0.05/s), searched hierarchically with the learned proposer and BF16
template storage.  The stage-2 triggers of the whole day coincide over 100,000 time slides of
0.1 s (the ring is the day, Sec. II), which counts the background; Eq. (7) extrapolates its tail
and gives the network SNR at inverse false-alarm rates of 1 and 10 years (Sec. IV).  The flat
search over the same day is the comparator.  A second day of the same noise and glitches with
one injection per segment (network SNR 6-20) is searched at zero lag by both pipelines; the
injections found above each pipeline's own IFAR thresholds compare their sensitivity.

Coincidences below network SNR 7 are not formed (hs_timeslide_coinc's statistic floor: exact for
every count at or above it, and the background grid and the fit start there), so the work is
bounded by the pairs above the floor.  With ``--save-subset`` the stage-2 triggers of every
``--subset-every``-th template and the GPU's coincidence counts over them are written out, for an
independent re-count.

    python -m paper_2309_00019_amd.day [--segments 338] [--slides 100000] [--dtype bf16]
"""
import argparse
import json
import multiprocessing as mp
import sys
import time

import numpy as np

YEAR = 365.25 * 86400.0
CFG = 5                       # seed family of this workload
EDGES = tuple(round(7.0 + 0.1 * i, 1) for i in range(71))   # 7.0 .. 14.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _segment_job(args):
    """Process-pool entry: one detector segment (noise + glitches [+ one injection])."""
    import synth
    det, seg, n, fs, f_low, glitch, inj = args
    return det, seg, synth.make_strain(CFG, det, seg, n, fs, f_low, glitch_rate=glitch,
                                       injections=[inj] if inj else [])[0]


def injections_of_day(n_seg, n, fs, mc_range, q_range, margin=8.0):
    """One injection per segment (parameters from the segment's own injection stream), with the
    amplitude factors of its H and L SNRs."""
    import synth
    from . import workload
    out = []
    for s in range(n_seg):
        ip = synth.injection_params(1, synth.rng(CFG, 0, s, synth.INJECT), mc_range[0], mc_range[1], q_range[0],
                                    q_range[1], n / fs, margin=margin)
        out.append({k: float(v[0]) for k, v in ip.items()})
    amp_h = workload.injection_amplitudes([p["m1"] for p in out], [p["m2"] for p in out],
                                          [p["snr_h"] for p in out], n, fs)
    for p, a in zip(out, amp_h):
        p["amp_h"] = float(a)
        p["amp_l"] = float(a * p["snr_l"] / p["snr_h"])
    return out


def whitened_day(ctx, pool, n_seg, n, fs, f_low, glitch, psds, injections=None):
    """Whitened spectra [n_seg, n/2] of both detectors; strain made on the host pool, whitened on
    the device with the run-level PSD of each detector."""
    import torch
    from . import hs
    specs = [torch.empty((n_seg, n // 2), dtype=torch.complex64, device=ctx.device) for _ in (0, 1)]
    jobs = []
    for s in range(n_seg):
        for det, key in ((0, "h"), (1, "l")):
            inj = None
            if injections is not None:
                p = injections[s]
                inj = dict(m1=p["m1"], m2=p["m2"], t_c=p["tc_" + key], phi_c=p["phi_" + key], amp=p["amp_" + key])
            jobs.append((det, s, n, fs, f_low, glitch, inj))
    done = 0
    for det, s, x in pool.imap_unordered(_segment_job, jobs, chunksize=4):
        hs.hs_whiten(ctx, torch.as_tensor(x, device=ctx.device), fs, f_low, psds[det], out=specs[det][s])
        done += 1
        if done % 128 == 0:
            log(f"[day] {done}/{len(jobs)} segments generated and whitened")
    return specs


def found_above(res, inj, thr, n, cfg, tol_sec=0.1):
    """Injections with a zero-lag coincidence within tol of their H arrival at or above network
    SNR thr; returns a boolean per injection."""
    from . import hs
    rec = hs.as_records(res.coincs, hs.COINC)
    ok = (rec["slide"] == 0) & (rec["snr_c"].astype(np.float64) >= thr)
    t = np.sort(rec["tick_h"][ok])
    tk = cfg.ticks_per_second
    seg_ticks = n * int(round(tk / cfg.fs))
    out = np.zeros(len(inj), bool)
    for s, p in enumerate(inj):
        tc = s * seg_ticks + int(round(p["tc_h"] * tk))
        a = np.searchsorted(t, tc - int(tol_sec * tk), "left")
        out[s] = a < len(t) and t[a] <= tc + int(tol_sec * tk)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--segments", type=int, default=338)
    ap.add_argument("--slides", type=int, default=100000)
    ap.add_argument("--dtype", default="bf16", choices=["f32", "bf16", "f16"])
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--no-flat", action="store_true")
    ap.add_argument("--no-injections", action="store_true")
    ap.add_argument("--save-subset", default=None, help="npz path: triggers of a template subset + GPU counts")
    ap.add_argument("--subset-every", type=int, default=100, help="the subset: every this-many-th template")
    args = ap.parse_args()
    import torch
    import synth
    from . import autotune, hs, search, workload
    from .proposer import Proposer

    fs, f_low = workload.FS, workload.F_LOW
    n = int(256 * fs)
    n_seg = args.segments
    ctx = hs.Context(0)
    dev = ctx.device
    pool = mp.get_context("spawn").Pool(args.workers, initializer=synth.single_threaded)
    t0 = time.perf_counter()
    # run-level PSD of each detector from its first segment (the noise is stationary)
    first = [_segment_job((det, 0, n, fs, f_low, workload.GLITCH_RATE, None))[2] for det in (0, 1)]
    psds = [hs.hs_welch_psd(ctx, torch.as_tensor(x, device=dev), fs, int(4 * fs)) for x in first]
    fm1, fm2 = workload.bank_masses(30000, 0)
    cm1, cm2 = workload.bank_masses(1500, 1)
    fine_h, fine_l = workload.make_banks(ctx, n, fs, f_low, fm1, fm2, psds, args.dtype)
    n1 = n // 4
    coarse_h, coarse_l = workload.make_banks(ctx, n1, fs / 4, f_low, cm1, cm2,
                                             [p[: n1 // 2 + 1].contiguous() for p in psds], args.dtype)
    prop = Proposer.load(dev)
    spec_tune = hs.hs_whiten(ctx, torch.as_tensor(first[0], device=dev), fs, f_low, psds[0])
    sched = autotune.tune_mf_schedule(ctx, spec_tune, n, fs, fine_h,
                                      torch.arange(0, 30000, 10, dtype=torch.int32, device=dev), 4.0)
    del spec_tune
    log(f"[day] banks ({args.dtype}) and schedule ready in {time.perf_counter() - t0:.1f} s: {sched['batch_mb']} MB")
    cfg = search.SearchConfig(fs=fs, f_low=f_low, n_slides=args.slides, step_sec=0.1, coinc_min_snr=7.0,
                              stage1_min_snr=min(prop.rho_low, 7.0), edges=EDGES, far_x_min=7.0, far_x_fit=8.0)
    T_day = n_seg * n / fs
    out = {"workload": f"{n_seg} x 2 segments of 256 s at 2048 Hz ({T_day / 3600:.2f} h per detector), noise + "
                       f"glitches 0.05/s; coarse 1500 @ 512 Hz, fine 30000 @ 2048 Hz ({args.dtype} storage); "
                       f"{args.slides} slides x 0.1 s over the day, 15 ms window, coincidences from network SNR 7",
           "schedule": {k: sched[k] for k in ("batch_mb", "tile", "pa_cols")}}

    # ---- the noise-only day: background ----------------------------------------------------------
    t0 = time.perf_counter()
    specs = whitened_day(ctx, pool, n_seg, n, fs, f_low, workload.GLITCH_RATE, psds)
    torch.cuda.synchronize()
    log(f"[day] noise day ready in {time.perf_counter() - t0:.1f} s")
    runs = {}
    for key in (("mlp",) if args.no_flat else ("mlp", "flat")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if key == "mlp":
            res = search.hierarchical_search(ctx, specs[0], specs[1], coarse_h, coarse_l, fine_h, fine_l, cfg,
                                             proposer=prop)
        else:
            res = search.flat_search(ctx, specs[0], specs[1], fine_h, fine_l, cfg)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        far = search.background_far(ctx, res, cfg)
        if far is not None:
            far.pop("far", None)          # the per-record FARs are not used here
        r = {"wall_s": round(wall, 2),
             "flat_equivalent_template_s_per_s": round(2 * 30000 * T_day / wall, 1),
             "template_applications": int(res.templates_filtered),
             "triggers": [int(res.trig_h.shape[0]), int(res.trig_l.shape[0])],
             "coincidences_kept": int(res.coincs.shape[0]),
             "background_days": round(res.t_b / 86400.0, 1),
             "bg_counts_7_8_9_10_12": [int(res.bg_counts[EDGES.index(x)]) for x in (7.0, 8.0, 9.0, 10.0, 12.0)]}
        if far is not None:
            r.update(alpha=round(far["alpha"], 4), beta=round(far["beta"], 4), fit_points=far["n_fit"],
                     rho_c_ifar_1yr=round(far["ifar_1yr"], 3), rho_c_ifar_10yr=round(far["ifar_10yr"], 3))
        if key == "mlp":
            r["followed_per_segment_mean"] = round(float(np.mean(res.followed)), 1)
        runs[key] = (res, far)
        out[key] = r
        log(f"[day] {key}: {json.dumps(r)}")
        if key == "mlp" and args.save_subset:
            # stage-2 triggers of every 100th template and the GPU's counts over exactly them
            sub = {}
            for det, tr in (("h", res.trig_h), ("l", res.trig_l)):
                rec = hs.as_records(tr, hs.TRIGGER)
                sel = rec["tmpl"] % args.subset_every == 0
                sub[det] = rec[sel]
            # the search's own coincidence geometry, in ticks
            tk = cfg.ticks_per_second
            geom = dict(n_slides=cfg.n_slides, step=int(round(cfg.step_sec * tk)),
                        window=int(round(cfg.coinc_window_sec * tk)), wrap=n_seg * search.timeline(cfg, n)[3],
                        cluster_w=int(round(cfg.cluster_sec * tk)))
            co, bg = hs.hs_timeslide_coinc(ctx, hs.to_device_records(sub["h"], dev), hs.to_device_records(sub["l"], dev),
                                           fine_h.n_tmpl, geom["n_slides"], geom["step"], geom["window"], geom["wrap"],
                                           geom["cluster_w"], np.asarray(EDGES, np.float32),
                                           min_snr_c=cfg.coinc_min_snr)
            c = hs.as_records(co, hs.COINC)
            np.savez(args.save_subset, trig_h=sub["h"], trig_l=sub["l"], coincs=c, bg_counts=bg,
                     edges=np.asarray(EDGES, np.float32), ticks_per_second=tk, min_snr_c=cfg.coinc_min_snr, **geom)
            log(f"[day] subset of {len(sub['h'])} + {len(sub['l'])} triggers, {len(c)} coincidences saved")
        runs[key] = (None, far)           # only the fit is needed from here on
        del res
        torch.cuda.empty_cache()
    out["speedup_vs_flat"] = round(out["flat"]["wall_s"] / out["mlp"]["wall_s"], 3) if "flat" in out else None

    # ---- the injection day: sensitivity at each pipeline's IFAR thresholds ----------------------------
    if not args.no_injections:
        del specs
        torch.cuda.empty_cache()
        inj = injections_of_day(n_seg, n, fs, workload.MC_RANGE, workload.Q_RANGE)
        t0 = time.perf_counter()
        specs = whitened_day(ctx, pool, n_seg, n, fs, f_low, workload.GLITCH_RATE, psds, inj)
        log(f"[day] injection day ready in {time.perf_counter() - t0:.1f} s")
        zcfg = search.SearchConfig(**{**cfg.__dict__, "n_slides": 0})
        rho = np.array([p["net_snr"] for p in inj])
        w = rho ** -4.0                          # uniform-in-volume weight of a network SNR drawn uniformly
        det = {}
        for key, (_, far) in runs.items():
            if key == "mlp":
                res = search.hierarchical_search(ctx, specs[0], specs[1], coarse_h, coarse_l, fine_h, fine_l, zcfg,
                                                 proposer=prop)
            else:
                res = search.flat_search(ctx, specs[0], specs[1], fine_h, fine_l, zcfg)
            d = {"found_rho_c_8": int(found_above(res, inj, 8.0, n, cfg).sum())}
            if far is not None:
                for lab, x in (("1yr", far["ifar_1yr"]), ("10yr", far["ifar_10yr"])):
                    f = found_above(res, inj, x, n, cfg)
                    d["detected_ifar_" + lab] = int(f.sum())
                    d["vt_weight_ifar_" + lab] = float(np.sum(w[f]) / np.sum(w))
            det[key] = d
            del res
            torch.cuda.empty_cache()
            log(f"[day] injections {key}: {json.dumps(d)}")
        out["injections"] = {"n": n_seg, "network_snr": "uniform 6-20, one per segment", **det}
        if "flat" in det:
            for lab in ("1yr", "10yr"):
                k = "vt_weight_ifar_" + lab
                if k in det["mlp"] and k in det["flat"] and det["flat"][k] > 0:
                    out["injections"]["vt_ratio_mlp_vs_flat_ifar_" + lab] = round(det["mlp"][k] / det["flat"][k], 4)
    pool.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
