"""Whole searches at the benchmark's shapes against the oracle's pipelines.

Two detectors x 256 s at 2048 Hz of coloured noise with sine-Gaussian glitches (0.05/s) and one
injection; stage 2 and the flat search at N = 2^19 (pass B with N1 = 1024), stage 1 at 2^17 and
512 Hz (N1 = 256), the benchmark's filter schedule (192 MB batches, 128-thread pass B, 64-column
pass A), chi-square re-weighting from rho 5.5, 16 stage-1 slides of 15 s and 2,000 background
slides of 0.1 s with the 15 ms window, background counts on the benchmark's 81 edges.  The banks
are cut down (80 coarse, 400 fine templates, chirp mass 1.4-10) so the oracle finishes in about a
minute.  Every step is compared under the tolerance rule of ``search_compare``; the coincidence
step is also re-run by the oracle on the GPU's own triggers, where it must agree exactly
(records and background counts)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import DELTA, analytic_psd, loud
from search_compare import check_followed, check_stage, compare_coincs, exact_coinc, oracle_series

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N, FS, F_LOW = 2 ** 19, 2048.0, 20.0
N_FINE, N_COARSE = 400, 80
DSTAT = 1e-3           # network-SNR tolerance after re-weighting (rho 1e-4, chi-square ~2e-4)
HI = 6.0               # coincidences at or above this network SNR are compared one by one


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def world():
    import torch
    from paper_2309_00019_amd import hs, search, workload
    _say("full-size set-up")
    ctx = hs.Context(0)
    hs.hs_set_mf_batch_bytes(ctx, 192 << 20)
    hs.hs_set_mf_tile(ctx, 128)
    hs.hs_set_mf_pa_cols(ctx, 64)
    fm1, fm2 = synth.bank_by_tau0(N_FINE, 1.4, 10.0, 1.0, 4.0, synth.rng(81, 0, 0, synth.BANK))
    cm1, cm2 = synth.bank_by_tau0(N_COARSE, 1.4, 10.0, 1.0, 4.0, synth.rng(81, 1, 0, synth.BANK))
    fine = synth.taylorf2_bank(fm1, fm2, N, FS, F_LOW)
    coarse = synth.taylorf2_bank(cm1, cm2, N // 4, FS / 4, F_LOW)
    t = 150
    inj = lambda tc, ph: [dict(m1=fm1[t], m2=fm2[t], t_c=tc, phi_c=ph, snr=11.0)]
    sh = synth.make_strain(81, 0, 0, N, FS, F_LOW, glitch_rate=0.05, injections=loud(inj(131.0, 0.4), N, FS, F_LOW))[0]
    sl = synth.make_strain(81, 1, 0, N, FS, F_LOW, glitch_rate=0.05, injections=loud(inj(131.006, 2.0), N, FS, F_LOW))[0]
    psd = analytic_psd(N, FS)
    d = ctx.device
    psd_d = torch.as_tensor(psd, device=d)
    n1 = N // 4
    fine_d, = workload.make_banks(ctx, N, FS, F_LOW, fm1, fm2, [psd_d])
    coarse_d, = workload.make_banks(ctx, n1, FS / 4, F_LOW, cm1, cm2, [psd_d[: n1 // 2 + 1].contiguous()])
    spec_h = hs.hs_whiten(ctx, torch.as_tensor(sh, device=d), FS, F_LOW, psd_d)[None]
    spec_l = hs.hs_whiten(ctx, torch.as_tensor(sl, device=d), FS, F_LOW, psd_d)[None]
    cfg = search.SearchConfig(fs=FS, f_low=F_LOW)
    st = [oracle.strain_fft(x, FS) for x in (sh, sl)]
    w = dict(ctx=ctx, fine=fine, coarse=coarse, sh=sh, sl=sl, psd=psd, fine_d=fine_d, coarse_d=coarse_d,
             spec_h=spec_h, spec_l=spec_l, cfg=cfg, st=st, inj_tick=int(131.0 * 51200))
    yield w
    torch.cuda.synchronize()
    ctx.close()


def _oracle_kw(cfg):
    return dict(n_slides=cfg.n_slides, step_sec=cfg.step_sec, coinc_window_sec=cfg.coinc_window_sec,
                cluster_sec=cfg.cluster_sec, edges=cfg.edges, chisq_rho_min=cfg.chisq_rho_min)


def _series(w, n, fs, bank):
    return [oracle_series([w["st"][det]], [w["psd"]], n, fs, F_LOW, bank) for det in (0, 1)]


def _check_stage(w, hs, g_raw, g_rw, o_trig, n, fs, bank, thr, cfg, only=None):
    return check_stage(hs, g_raw, g_rw, o_trig, _series(w, n, fs, bank), thr, DELTA["f32"], DSTAT,
                       int(round(cfg.window_sec * fs)), N * 25, int(round(cfg.ticks_per_second / fs)),
                       cfg.chisq_rho_min, only, _say)


def _exact_coinc(res_coincs, res_bg, g_cols, n_slides, step, cfg, wrap):
    from paper_2309_00019_amd import hs
    tk = cfg.ticks_per_second
    return exact_coinc(hs, res_coincs, res_bg, g_cols, n_slides, step, int(round(cfg.coinc_window_sec * tk)), wrap,
                       int(round(cfg.cluster_sec * tk)), cfg.edges if res_bg is not None else [], tk)


def test_flat_search_full_size_matches_oracle(world):
    from paper_2309_00019_amd import hs, search
    w, cfg = world, world["cfg"]
    _say("flat search at full size: GPU")
    res = search.flat_search(w["ctx"], w["spec_h"], w["spec_l"], w["fine_d"], w["fine_d"], cfg)
    _say("flat search at full size: oracle")
    ref = oracle.flat_search([w["sh"]], [w["sl"]], [w["psd"]], [w["psd"]], FS, F_LOW, w["fine"], **_oracle_kw(cfg))
    fragile, g_cols = _check_stage(w, hs, (res.raw["h"], res.raw["l"]), (res.trig_h, res.trig_l),
                                   (ref["trig_h"], ref["trig_l"]), N, FS, w["fine"], cfg.thr2, cfg)
    wrap = N * 25
    step = int(round(cfg.step_sec * cfg.ticks_per_second))
    n_c = _exact_coinc(res.coincs, res.bg_counts, g_cols, cfg.n_slides, step, cfg, wrap)
    o_cols = [dict(tmpl=np.asarray(t["tmpl"], np.int64), tick=np.asarray(t["tick"], np.int64), snr=t["snr"])
              for t in (ref["trig_h"], ref["trig_l"])]
    n_ex = compare_coincs(hs.as_records(res.coincs, hs.COINC), ref["coinc"]["coincs"], g_cols, o_cols, fragile,
                          cfg.n_slides, step, int(round(cfg.coinc_window_sec * 51200)), wrap,
                          int(round(cfg.cluster_sec * 51200)), HI, DSTAT, cfg.edges, res.bg_counts,
                          ref["coinc"]["bg_counts"])
    _say(f"  {n_c} coincidences over 2,000 slides (exact on the GPU's triggers); {n_ex} exempt differences "
         f"against the oracle's chain; background counts {list(res.bg_counts[::20])} vs "
         f"{list(ref['coinc']['bg_counts'][::20])}")
    assert n_c > 10000 and n_ex <= 0.01 * n_c
    c = hs.as_records(res.coincs, hs.COINC)
    z = c[(c["slide"] == 0) & (c["snr_c"] >= 8.0)]
    assert np.any(np.abs(z["tick_h"] - w["inj_tick"]) <= 5120)


def _fragile_rows(ref, coarse, cfg, prop):
    """Stage-1 coincidences whose cell selection float32 rounding could change (oracle inputs)."""
    if prop is None:
        return np.zeros(len(ref["coinc1"]["coincs"]["tmpl"]), bool)
    P = oracle.proposer
    model, q_edges, p_cum, rho_low, p_low = prop
    cc = ref["coinc1"]["coincs"]
    x = P.features(cc, ref["stage1_h"], ref["stage1_l"], coarse.mchirp, coarse.q,
                   int(round(cfg.t_sh1_sec * cfg.ticks_per_second)), N * 25, cfg.ticks_per_second, 8)
    if not len(x):
        return np.zeros(0, bool)
    prob = P.softmax(P.forward(model, x)[0])
    out = np.zeros(len(x), bool)
    for i in range(len(x)):
        pc = p_cum if np.float32(x[i, 2]) >= np.float32(cfg.rho1) else p_low
        ps = np.sort(prob[i])[::-1]
        cs = np.cumsum(ps)
        k = int(np.searchsorted(cs, pc)) if cs[-1] >= pc else 63
        near_stop = abs(cs[min(k, 63)] - pc) < 1e-4 or (k > 0 and abs(cs[k - 1] - pc) < 1e-4)
        near_tie = k < 63 and abs(ps[k] - ps[k + 1]) < 1e-5
        out[i] = near_stop or near_tie
    return out


@pytest.mark.parametrize("use_proposer", [False, True])
def test_hierarchical_search_full_size_matches_oracle(world, use_proposer):
    from paper_2309_00019_amd import hs, search
    from paper_2309_00019_amd.proposer import Proposer
    w, cfg = world, world["cfg"]
    prop = oprop = None
    if use_proposer:
        prop = Proposer.load(w["ctx"].device)
        oprop = (prop.model.cpu().numpy().astype(np.float64), tuple(prop.q_edges), prop.p_cum, prop.rho_low,
                 prop.p_cum_low)
    _say(f"hierarchical search at full size (proposer={use_proposer}): GPU")
    res = search.hierarchical_search(w["ctx"], w["spec_h"], w["spec_l"], w["coarse_d"], w["coarse_d"], w["fine_d"],
                                     w["fine_d"], cfg, proposer=prop)
    _say("  oracle")
    ref = oracle.hierarchical_search([w["sh"]], [w["sl"]], [w["psd"]], [w["psd"]], FS, F_LOW, w["coarse"], w["fine"],
                                     n_sh1=cfg.n_sh1, t_sh1_sec=cfg.t_sh1_sec, rho1=cfg.rho1, proposer=oprop,
                                     **_oracle_kw(cfg))
    wrap = N * 25
    win, cw = int(round(cfg.coinc_window_sec * 51200)), int(round(cfg.cluster_sec * 51200))
    # stage 1: triggers at 2^17, coincidences over the 16 long slides
    n1 = N // 4
    _say("  stage 1")
    frag1, g1 = _check_stage(w, hs, (res.raw["h1"], res.raw["l1"]), res.stage1_trig,
                             (ref["stage1_h"], ref["stage1_l"]), n1, FS / 4, w["coarse"], cfg.thr1, cfg)
    step1 = int(round(cfg.t_sh1_sec * cfg.ticks_per_second))
    _exact_coinc(res.stage1_coincs, None, g1, cfg.n_sh1, step1, cfg, wrap)
    o1 = [dict(tmpl=np.asarray(t["tmpl"], np.int64), tick=np.asarray(t["tick"], np.int64), snr=t["snr"])
          for t in (ref["stage1_h"], ref["stage1_l"])]
    gc1 = hs.as_records(res.stage1_coincs, hs.COINC)
    oc1 = ref["coinc1"]["coincs"]
    lo1 = min(cfg.rho1, prop.rho_low) if prop else cfg.rho1
    ex1 = compare_coincs(gc1, oc1, g1, o1, frag1, cfg.n_sh1, step1, win, wrap, cw, 6.0, DSTAT)
    # the followed fine templates; a difference must come from a fragile stage-1 coincidence
    fg = set(res.fine_ids[0].cpu().numpy().tolist())
    fo = set(np.asarray(ref["fine_ids"][0]).tolist())
    _say(f"  {len(gc1)} stage-1 coincidences ({ex1} exempt differences); followed {len(fg)} (oracle {len(fo)})")
    rows = _fragile_rows(ref, w["coarse"], cfg, oprop) if fg != fo else None
    check_followed(fg, fo, gc1, oc1, (cfg.rho1, lo1), DSTAT, w["coarse"].mchirp, w["fine"].mchirp, cfg.mc_frac, rows)
    both = fg & fo
    # stage 2 on the followed templates
    _say("  stage 2")
    frag2, g2 = _check_stage(w, hs, (res.raw["h"], res.raw["l"]), (res.trig_h, res.trig_l),
                             (ref["trig_h"], ref["trig_l"]), N, FS, w["fine"], cfg.thr2, cfg, lambda s: both)
    for det, tr in ((0, res.raw["h"]), (1, res.raw["l"])):
        r = hs.as_records(tr, hs.TRIGGER)
        frag2[det] |= {(int(a), int(b)) for a, b in zip(r["tmpl"], r["tick"]) if int(a) not in both}
        o = (ref["trig_h"], ref["trig_l"])[det]
        frag2[det] |= {(int(a), int(b)) for a, b in zip(o["tmpl"], o["tick"]) if int(a) not in both}
    step = int(round(cfg.step_sec * cfg.ticks_per_second))
    n_c = _exact_coinc(res.coincs, res.bg_counts, g2, cfg.n_slides, step, cfg, wrap)
    o2 = [dict(tmpl=np.asarray(t["tmpl"], np.int64), tick=np.asarray(t["tick"], np.int64), snr=t["snr"])
          for t in (ref["trig_h"], ref["trig_l"])]
    n_ex = compare_coincs(hs.as_records(res.coincs, hs.COINC), ref["coinc"]["coincs"], g2, o2, frag2, cfg.n_slides,
                          step, win, wrap, cw, HI, DSTAT, cfg.edges, res.bg_counts, ref["coinc"]["bg_counts"])
    _say(f"  {n_c} stage-2 coincidences over 2,000 slides (exact on the GPU's triggers); {n_ex} exempt "
         f"differences against the oracle's chain; background {list(res.bg_counts[::20])} vs "
         f"{list(ref['coinc']['bg_counts'][::20])}")
    assert n_ex <= 0.01 * max(n_c, 1) + 3
