"""Blocks of overlapping 512 s segments at N = 2^20 (the paper's segment length) against the
oracle: the per-block PSD, and the flat and plain hierarchical searches over the segments of a
1,024 s block, each segment keeping only its valid region (144 s / 16 s pads, 352 s stride) and
the valid regions laid end to end as the timeline.  Compared under the tolerance rule of
``search_compare``; coincidences also exactly on the GPU's own triggers."""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import DELTA, loud
from oracle import segments as S
from search_compare import check_followed, check_stage, cols, compare_coincs, exact_coinc, oracle_series

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N, FS, F_LOW = 2 ** 20, 2048.0, 20.0
PAD_LO, PAD_HI = 144 * 2048, 16 * 2048
BLOCK = 2 ** 21


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def world():
    import torch
    from paper_2309_00019_amd import hs, search, workload
    _say("block of overlapping segments: set-up")
    ctx = hs.Context(0)
    g = synth.rng(82, 0, 0, synth.BANK)
    fm1, fm2 = synth.bank_by_tau0(40, 1.4, 10.0, 1.0, 4.0, g)
    cm1, cm2 = synth.bank_by_tau0(12, 1.4, 10.0, 1.0, 4.0, synth.rng(82, 1, 0, synth.BANK))
    t = 20
    starts = S.segment_starts(BLOCK, N, PAD_LO, PAD_HI)
    assert len(starts) == 2
    # the injection lies where the two segments overlap, inside the second one's valid region
    t_inj = (starts[1] + PAD_LO + 10 * 2048) / FS
    assert starts[0] + N - PAD_HI <= t_inj * FS < starts[0] + N
    inj = lambda dt, ph: [dict(m1=fm1[t], m2=fm2[t], t_c=t_inj + dt, phi_c=ph, snr=12.0)]
    bh = synth.make_strain(82, 0, 0, BLOCK, FS, F_LOW, glitch_rate=0.05, injections=loud(inj(0.0, 0.4), BLOCK, FS, F_LOW))[0]
    bl = synth.make_strain(82, 1, 0, BLOCK, FS, F_LOW, glitch_rate=0.05, injections=loud(inj(0.005, 1.9), BLOCK, FS, F_LOW))[0]
    d = ctx.device
    # per-block PSD: the GPU's Welch over the whole block on the block's grid, every 2nd bin is the
    # segment grid; against the oracle's block PSD on the segment grid
    psds = []
    for b in (bh, bl):
        gp = hs.hs_welch_psd(ctx, torch.as_tensor(b, device=d), FS, 8192).cpu().numpy()[::BLOCK // N]
        op = S.block_psd(b, FS, 8192, N)
        assert np.allclose(gp, op, rtol=1e-9, atol=0)
        psds.append(op)
    fine = synth.taylorf2_bank(fm1, fm2, N, FS, F_LOW)
    coarse = synth.taylorf2_bank(cm1, cm2, N // 4, FS / 4, F_LOW)
    pd = [torch.as_tensor(p, device=d) for p in psds]
    fine_h, fine_l = workload.make_banks(ctx, N, FS, F_LOW, fm1, fm2, pd)
    n1 = N // 4
    coarse_h, coarse_l = workload.make_banks(ctx, n1, FS / 4, F_LOW, cm1, cm2, [p[: n1 // 2 + 1].contiguous() for p in pd])
    segs = [[b[st:st + N] for st in starts] for b in (bh, bl)]
    specs = [torch.stack([hs.hs_whiten(ctx, torch.as_tensor(x, device=d), FS, F_LOW, pd[k]) for x in segs[k]])
             for k in (0, 1)]
    cfg = search.SearchConfig(fs=FS, f_low=F_LOW, pad_lo_sec=144.0, pad_hi_sec=16.0, n_slides=200, step_sec=0.1,
                              n_sh1=8, t_sh1_sec=15.0, rho1=6.5, chisq_rho_min=5.5,
                              edges=tuple(round(6.0 + 0.25 * i, 2) for i in range(17)))
    st = [[oracle.strain_fft(x, FS) for x in segs[k]] for k in (0, 1)]
    w = dict(ctx=ctx, fine=fine, coarse=coarse, segs=segs, psds=psds, fine_d=(fine_h, fine_l),
             coarse_d=(coarse_h, coarse_l), specs=specs, cfg=cfg, st=st, starts=starts,
             inj_tick=int(round((t_inj * FS - PAD_LO) * 25)))
    yield w
    torch.cuda.synchronize()
    ctx.close()


def _okw(cfg):
    return dict(n_slides=cfg.n_slides, step_sec=cfg.step_sec, edges=cfg.edges, chisq_rho_min=cfg.chisq_rho_min,
                pad_lo=PAD_LO, pad_hi=PAD_HI)


def _stage(w, hs, g_raw, g_rw, o_trig, n, fs, bank, thr, cfg, only=None):
    n_seg = len(w["starts"])
    ser = [oracle_series(w["st"][k], [w["psds"][k]] * n_seg, n, fs, F_LOW, bank) for k in (0, 1)]
    decim = N // n
    return check_stage(hs, g_raw, g_rw, o_trig, ser, thr, DELTA["f32"], 1e-3, int(round(cfg.window_sec * fs)),
                       (N - PAD_LO - PAD_HI) * 25, 25 * decim, cfg.chisq_rho_min, only, _say, PAD_LO // decim)


def test_flat_search_over_overlapping_segments_matches_oracle(world):
    from paper_2309_00019_amd import hs, search
    w, cfg = world, world["cfg"]
    _say("flat search over a block: GPU")
    res = search.flat_search(w["ctx"], w["specs"][0], w["specs"][1], *w["fine_d"], cfg)
    _say("  oracle")
    n_seg = len(w["starts"])
    ref = oracle.flat_search(w["segs"][0], w["segs"][1], [w["psds"][0]] * n_seg, [w["psds"][1]] * n_seg, FS, F_LOW,
                             w["fine"], **_okw(cfg))
    frag, gt = _stage(w, hs, (res.raw["h"], res.raw["l"]), (res.trig_h, res.trig_l), (ref["trig_h"], ref["trig_l"]),
                      N, FS, w["fine"], cfg.thr2, cfg)
    wrap = n_seg * (N - PAD_LO - PAD_HI) * 25
    exact_coinc(hs, res.coincs, res.bg_counts, gt, cfg.n_slides, 5120, 768, wrap, 51200, cfg.edges, 51200)
    c = hs.as_records(res.coincs, hs.COINC)
    n_ex = compare_coincs(c, ref["coinc"]["coincs"], gt, [cols(t) for t in (ref["trig_h"], ref["trig_l"])], frag,
                          cfg.n_slides, 5120, 768, wrap, 51200, 6.0, 1e-3, cfg.edges, res.bg_counts,
                          ref["coinc"]["bg_counts"])
    _say(f"  {len(c)} coincidences, {n_ex} exempt differences; background {list(res.bg_counts[::4])}")
    for tr in (res.trig_h, res.trig_l):
        r = hs.as_records(tr, hs.TRIGGER)
        assert np.all((r["tick"] >= 0) & (r["tick"] < wrap))
    z = c[(c["slide"] == 0) & (c["snr_c"] >= 10.0)]
    assert len(z) == 1 and abs(int(z["tick_h"][0]) - w["inj_tick"]) <= 5120


def test_hierarchical_search_over_overlapping_segments_matches_oracle(world):
    from paper_2309_00019_amd import hs, search
    w, cfg = world, world["cfg"]
    _say("hierarchical search over a block: GPU")
    res = search.hierarchical_search(w["ctx"], w["specs"][0], w["specs"][1], *w["coarse_d"], *w["fine_d"], cfg)
    _say("  oracle")
    n_seg = len(w["starts"])
    ref = oracle.hierarchical_search(w["segs"][0], w["segs"][1], [w["psds"][0]] * n_seg, [w["psds"][1]] * n_seg, FS,
                                     F_LOW, w["coarse"], w["fine"], n_sh1=cfg.n_sh1, t_sh1_sec=cfg.t_sh1_sec,
                                     rho1=cfg.rho1, **_okw(cfg))
    share = (N - PAD_LO - PAD_HI) * 25
    wrap = n_seg * share
    frag1, g1 = _stage(w, hs, (res.raw["h1"], res.raw["l1"]), res.stage1_trig, (ref["stage1_h"], ref["stage1_l"]),
                       N // 4, FS / 4, w["coarse"], cfg.thr1, cfg)
    step1 = int(round(cfg.t_sh1_sec * 51200))
    exact_coinc(hs, res.stage1_coincs, None, g1, cfg.n_sh1, step1, 768, wrap, 51200, [], 51200)
    c1 = hs.as_records(res.stage1_coincs, hs.COINC)
    r1 = ref["coinc1"]["coincs"]
    compare_coincs(c1, r1, g1, [cols(t) for t in (ref["stage1_h"], ref["stage1_l"])], frag1, cfg.n_sh1, step1, 768,
                   wrap, 51200, 5.5, 1e-3)
    both = []
    for s in range(n_seg):
        fg = set(res.fine_ids[s].cpu().numpy().tolist())
        fo = set(np.asarray(ref["fine_ids"][s]).tolist())
        check_followed(fg, fo, c1, r1, (cfg.rho1,), 1e-3, w["coarse"].mchirp, w["fine"].mchirp)
        both.append(fg & fo)
    _say(f"  followed per segment {[len(b) for b in both]}")
    assert sum(len(b) for b in both) > 0
    frag2, g2 = _stage(w, hs, (res.raw["h"], res.raw["l"]), (res.trig_h, res.trig_l), (ref["trig_h"], ref["trig_l"]),
                       N, FS, w["fine"], cfg.thr2, cfg, lambda s: both[s])
    for det, (gtr, otr) in enumerate(((res.raw["h"], ref["trig_h"]), (res.raw["l"], ref["trig_l"]))):
        r = hs.as_records(gtr, hs.TRIGGER)
        for a, b in list(zip(r["tmpl"], r["tick"])) + list(zip(otr["tmpl"], otr["tick"])):
            if int(a) not in both[int(b) // share]:
                frag2[det].add((int(a), int(b)))
    exact_coinc(hs, res.coincs, res.bg_counts, g2, cfg.n_slides, 5120, 768, wrap, 51200, cfg.edges, 51200)
    compare_coincs(hs.as_records(res.coincs, hs.COINC), ref["coinc"]["coincs"], g2,
                   [cols(t) for t in (ref["trig_h"], ref["trig_l"])], frag2, cfg.n_slides, 5120, 768, wrap, 51200, 6.0,
                   1e-3, cfg.edges, res.bg_counts, ref["coinc"]["bg_counts"])
