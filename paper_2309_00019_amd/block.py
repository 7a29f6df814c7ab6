"""A paper-shaped block through the searches: overlapping 512 s segments and the Eq. (8) cost model.

Sec. V: the data come in blocks, each cut into overlapping 512 s segments (N = 2^20 at 2048 Hz;
stage 1 at 512 Hz, N = 2^18).  Here one block of 2^23 samples (4,096 s) per detector holds 11
segments at a 352 s stride, each keeping its valid region (144 s / 16 s pads), with the PSD
estimated once per block (Welch over the whole block).  The flat search, the plain hierarchy and
the hierarchy with the learned proposer run over the block; stage 1 is also timed on its own,
which gives the per-template cost of stage 2 relative to the flat search, i.e. the gamma of
Eq. (8), measured rather than assumed, and Eq. (8)'s predicted speed-up beside the measured one.

    python -m paper_2309_00019_amd.block [--dtype bf16] [--steps 2]
"""
import argparse
import json
import multiprocessing as mp
import sys
import time

import numpy as np

CFG = 6                       # seed family of this workload
BLOCK = 2 ** 23
N = 2 ** 20
PAD_LO_SEC, PAD_HI_SEC = 144.0, 16.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _block_job(args):
    import synth
    det, fs, f_low, glitch = args
    return det, synth.make_strain(CFG, det, 0, BLOCK, fs, f_low, glitch_rate=glitch)[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtype", default="bf16", choices=["f32", "bf16", "f16"])
    ap.add_argument("--steps", type=int, default=2)
    args = ap.parse_args()
    import torch
    import synth
    from . import autotune, hs, search, workload
    from .proposer import Proposer

    fs, f_low = workload.FS, workload.F_LOW
    ctx = hs.Context(0)
    dev = ctx.device
    cfg = search.SearchConfig(fs=fs, f_low=f_low, pad_lo_sec=PAD_LO_SEC, pad_hi_sec=PAD_HI_SEC)
    plo, phi = int(PAD_LO_SEC * fs), int(PAD_HI_SEC * fs)
    stride = N - plo - phi
    starts = np.arange(0, BLOCK - N + 1, stride)
    n_seg = len(starts)
    with mp.get_context("spawn").Pool(2, initializer=synth.single_threaded) as pool:
        blocks = dict(pool.map(_block_job, [(d, fs, f_low, workload.GLITCH_RATE) for d in (0, 1)]))
    t0 = time.perf_counter()
    # one PSD per block: Welch over the block on its own grid; every 8th bin is the segment grid
    psds = []
    for d in (0, 1):
        p = hs.hs_welch_psd(ctx, torch.as_tensor(blocks[d], device=dev), fs, int(4 * fs))
        psds.append(p[:: BLOCK // N].contiguous())
    fm1, fm2 = workload.bank_masses(30000, 0)
    cm1, cm2 = workload.bank_masses(1500, 1)
    fine_h, fine_l = workload.make_banks(ctx, N, fs, f_low, fm1, fm2, psds, args.dtype)
    n1 = N // 4
    coarse_h, coarse_l = workload.make_banks(ctx, n1, fs / 4, f_low, cm1, cm2,
                                             [p[: n1 // 2 + 1].contiguous() for p in psds], args.dtype)
    prop = Proposer.load(dev)
    specs = []
    for d in (0, 1):
        x = torch.as_tensor(blocks[d], device=dev)
        specs.append(torch.stack([hs.hs_whiten(ctx, x[st:st + N], fs, f_low, psds[d]) for st in starts]))
    sched = autotune.tune_mf_schedule(ctx, specs[0][0], N, fs, fine_h,
                                      torch.arange(0, 30000, 10, dtype=torch.int32, device=dev), 4.0)
    torch.cuda.synchronize()
    log(f"[block] {n_seg} segments per detector, banks ({args.dtype}) and schedule ready in "
        f"{time.perf_counter() - t0:.1f} s ({sched['batch_mb']} MB)")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / args.steps, r

    w_s1, _ = timed(lambda: search.stage1(ctx, specs[0], specs[1], coarse_h, coarse_l, cfg, with_chisq=True))
    w_mlp, r_mlp = timed(lambda: search.hierarchical_search(ctx, specs[0], specs[1], coarse_h, coarse_l, fine_h,
                                                            fine_l, cfg, proposer=prop))
    w_hier, r_hier = timed(lambda: search.hierarchical_search(ctx, specs[0], specs[1], coarse_h, coarse_l, fine_h,
                                                              fine_l, cfg))
    w_flat, r_flat = timed(lambda: search.flat_search(ctx, specs[0], specs[1], fine_h, fine_l, cfg))
    T = N / fs
    apps_flat = 2 * n_seg * 30000
    out = {"workload": f"one block of {BLOCK / fs:.0f} s per detector (noise + glitches 0.05/s), {n_seg} overlapping "
                       f"segments of 512 s (stride {stride / fs:.0f} s, valid region [{PAD_LO_SEC:.0f}, "
                       f"{T - PAD_HI_SEC:.0f}) s), per-block Welch PSD; coarse 1500 @ 512 Hz (N = 2^18), fine 30000 "
                       f"@ 2048 Hz (N = 2^20), {args.dtype} storage; 2000 slides x 0.1 s",
           "schedule": {k: sched[k] for k in ("batch_mb", "tile", "pa_cols")},
           "flat_s": round(w_flat, 3), "stage1_s": round(w_s1, 3)}
    for key, w, r in (("mlp", w_mlp, r_mlp), ("plain", w_hier, r_hier)):
        apps2 = int(sum(r.followed)) * 2
        # gamma: cost of a stage-2 application (everything after stage 1, per template and segment)
        # relative to a flat one (the whole flat search per template and segment)
        gamma = ((w - w_s1) / apps2) / (w_flat / apps_flat)
        out[key] = {"s": round(w, 3), "speedup_vs_flat": round(w_flat / w, 3),
                    "flat_equivalent_template_s_per_s": round(apps_flat * T / w, 1),
                    "followed_per_segment": [int(c) for c in r.followed],
                    "gamma_measured": round(gamma, 3),
                    "eq8_gamma_1": round(search.speedup_eq8(n_seg, 30000, 1500, apps2 // 2, fs, fs / 4, T, 1.0), 3),
                    "eq8_gamma_measured": round(search.speedup_eq8(n_seg, 30000, 1500, apps2 // 2, fs, fs / 4, T,
                                                                   gamma), 3)}
        log(f"[block] {key}: {json.dumps(out[key])}")
    out["flat_equivalent_template_s_per_s_flat"] = round(apps_flat * T / w_flat, 1)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
