"""Train the learned follow-up proposer on injections the pipeline itself generates.

Usage: python -m paper_2309_00019_amd.train_proposer [--train 50000] [--val 5000] [--out PATH]

For each synthetic realisation (two detectors x 256 s of noise + glitches with several
injections, network SNR 6-20) stage 1 runs on the GPU exactly as in the search (coarse bank at
512 Hz, threshold 3.5, chi-square re-weighting, zero-lag coincidence); the loudest stage-1
coincidence within 0.1 s of an injection with network SNR >= rho1 gives one training sample:
its 16 features (hs_proposer_features) and, as the target, the neighbourhood cell of the
injected (Mc, q).  The MLP is trained with Adam (hs_mlp_train_step); P is then the smallest
value on a grid whose selected cells contain the injected cell for at least ``--hit`` of the
held-out injections.  The plain +-frac chirp-mass rule, which the cells partition, is reported
beside it as the yardstick.  Host workers only generate the synthetic strain.
"""
import argparse
import json
import multiprocessing as mp
import sys
import time

import numpy as np

N_SAMPLES = 2 ** 19
P_GRID = (0.5, 0.7, 0.8, 0.9, 0.95, 0.97, 0.98, 0.99, 0.995, 0.998, 0.999)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def collect(ctx, pool, rs, per_seg, coarse_h, coarse_l, psd_h, psd_l, cfg, label):
    """Stage-1 samples of the injections of realisations rs: (features, labels, info)."""
    import torch
    import synth
    from . import hs, search, proposer, workload
    dev = ctx.device
    tk = cfg.ticks_per_second
    cmc = coarse_h.mchirp.cpu().numpy()
    feats, labels, info = [], [], []
    n_inj = 0
    t0 = time.perf_counter()
    t_gpu = 0.0
    jobs = workload.realisation_jobs(rs, per_seg, N_SAMPLES)
    for k, (r, (sh, sl, ip)) in enumerate(pool.imap(synth.realisation_job, jobs, chunksize=2)):
        tg = time.perf_counter()
        spec_h = hs.hs_whiten(ctx, torch.as_tensor(sh, device=dev), workload.FS, workload.F_LOW, psd_h)[None]
        spec_l = hs.hs_whiten(ctx, torch.as_tensor(sl, device=dev), workload.FS, workload.F_LOW, psd_l)[None]
        th, tl, c1 = search.stage1(ctx, spec_h, spec_l, coarse_h, coarse_l, cfg, with_chisq=True)
        f = search.stage1_features(ctx, th, tl, c1, coarse_h, 1, N_SAMPLES, cfg).cpu().numpy()
        rec = hs.as_records(c1, hs.COINC)
        n_inj += per_seg
        for j in range(per_seg):
            tc = int(round(ip["tc_h"][j] * tk))
            sel = np.nonzero((rec["slide"] == 0) & (np.abs(rec["tick_h"] - tc) <= int(0.1 * tk)) &
                             (rec["stat"].astype(np.float64) >= cfg.rho1 ** 2))[0]
            if len(sel) == 0:
                continue
            i = sel[np.argmax(rec["stat"][sel])]
            mc_c = cmc[rec["tmpl"][i]]
            feats.append(f[i])
            labels.append(proposer.cell_labels([mc_c], [ip["mchirp"][j]], [ip["q"][j]], cfg.mc_frac,
                                               proposer.Q_EDGES)[0])
            info.append((ip["mchirp"][j], ip["q"][j], ip["net_snr"][j], mc_c,
                         abs(ip["mchirp"][j] - mc_c) <= cfg.mc_frac * mc_c))
        t_gpu += time.perf_counter() - tg
        if (k + 1) % 200 == 0:
            log(f"[{label}] {k + 1}/{len(rs)} realisations, {len(labels)} samples of {n_inj} injections, "
                f"{time.perf_counter() - t0:.0f} s ({t_gpu:.0f} s in stage 1)")
    return np.asarray(feats, np.float32), np.asarray(labels, np.int32), np.asarray(info), n_inj


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=50000, help="training injections")
    ap.add_argument("--stop", type=int, default=5000, help="early-stopping injections")
    ap.add_argument("--val", type=int, default=5000, help="held-out injections (P and the reported rates)")
    ap.add_argument("--per-seg", type=int, default=8, help="injections per 256 s realisation")
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=5e-5)
    ap.add_argument("--hit", type=float, default=0.99, help="held-out hit rate that sets P")
    ap.add_argument("--rho-low", type=float, default=6.75,
                    help="lower follow-up threshold of the second tier (set end to end on tuning injections)")
    ap.add_argument("--p-low", type=float, default=0.5, help="P of the second tier")
    ap.add_argument("--out", default=None)
    ap.add_argument("--data", default=None, help="save the collected samples here (npz); with --reuse, load them")
    ap.add_argument("--reuse", action="store_true")
    ap.add_argument("--train-seed0", type=int, default=10000,
                    help="first training realisation seed (the early-stopping and held-out sets use 40000.. and "
                         "20000..; keep the training range clear of them)")
    args = ap.parse_args()
    # host workers are spawned (fresh interpreters that never load the GPU runtime)
    import synth
    pool = mp.get_context("spawn").Pool(args.workers, initializer=synth.single_threaded)
    import torch
    from . import hs, search, proposer, workload
    t_start = time.perf_counter()
    ctx = hs.Context(0)
    dev = ctx.device
    n = N_SAMPLES
    cfg = search.SearchConfig(fs=workload.FS, f_low=workload.F_LOW, n_sh1=0)
    bg = workload.background_strains(n)
    L = int(4 * workload.FS)
    psd_h = hs.hs_welch_psd(ctx, torch.as_tensor(bg[0], device=dev), workload.FS, L)
    psd_l = hs.hs_welch_psd(ctx, torch.as_tensor(bg[1], device=dev), workload.FS, L)
    n1, fs1 = n // cfg.decim, workload.FS / cfg.decim
    cm1, cm2 = workload.bank_masses(1500, 1)
    coarse_h, coarse_l = workload.make_banks(ctx, n1, fs1, workload.F_LOW, cm1, cm2,
                                             [psd_h[: n1 // 2 + 1].contiguous(), psd_l[: n1 // 2 + 1].contiguous()])
    ps = args.per_seg
    keys = ("xt", "yt", "it", "nt", "xs", "ys", "is_", "ns", "xv", "yv", "iv", "nv")
    if args.reuse and args.data:
        z = np.load(args.data, allow_pickle=False)
        xt, yt, it, nt, xs, ys, is_, ns, xv, yv, iv, nv = (z[k] for k in keys)
        nt, ns, nv = int(nt), int(ns), int(nv)
    else:
        # disjoint seed ranges: training train_seed0.., early stopping 40000.., held-out 20000..
        r_train = [args.train_seed0 + r for r in range(-(-args.train // ps))]
        lo, hi = r_train[0], r_train[-1]
        for a, b in ((40000, 40000 + -(-args.stop // ps)), (20000, 20000 + -(-args.val // ps))):
            if lo < b and a <= hi:
                raise SystemExit(f"training realisations {lo}..{hi} overlap the range {a}..{b - 1}")
        r_stop = [40000 + r for r in range(-(-args.stop // ps))]
        r_val = [20000 + r for r in range(-(-args.val // ps))]
        xt, yt, it, nt = collect(ctx, pool, r_train, ps, coarse_h, coarse_l, psd_h, psd_l, cfg, "train")
        xs, ys, is_, ns = collect(ctx, pool, r_stop, ps, coarse_h, coarse_l, psd_h, psd_l, cfg, "stop")
        xv, yv, iv, nv = collect(ctx, pool, r_val, ps, coarse_h, coarse_l, psd_h, psd_l, cfg, "val")
        if args.data:
            np.savez(args.data, **dict(zip(keys, (xt, yt, it, nt, xs, ys, is_, ns, xv, yv, iv, nv))))
    pool.close()
    log(f"[data] train {len(yt)} samples of {nt} injections, early stopping {len(ys)} of {ns}, "
        f"held-out {len(yv)} of {nv}")
    t_train = time.perf_counter()
    model, hist, best_epoch = proposer.train(ctx, xt, yt, epochs=args.epochs, lr=args.lr, lr_final=args.lr_final,
                                             log=log, stop=(xs, ys))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    table = []
    for p in P_GRID:
        hit, cells = proposer.selection_stats(ctx, model, xv, yv, p)
        table.append((p, hit, cells))
        log(f"[val] P={p}: injected cell selected for {hit:.4f}, mean cells {cells:.2f} of 64")
    ok = [row for row in table if row[1] >= args.hit]
    p_cum, hit, cells = ok[0] if ok else table[-1]
    plain_hit = float(np.mean(iv[:, 4])) if len(iv) else float("nan")
    meta = dict(n_train=len(yt), n_val=len(yv), train_injections=nt, val_injections=nv, epochs=args.epochs,
                best_epoch=best_epoch, n_stop=len(ys),
                lr=args.lr, lr_final=args.lr_final, val_hit=hit, val_loss=proposer.mean_loss(ctx, model, xv, yv), val_mean_cells=cells, val_plain_hit=plain_hit,
                loss_first=hist[0], loss_last=hist[-1], train_seconds=t_train,
                seeds=f"realisations: training {args.train_seed0}.., early stopping 40000.., held-out 20000.. (cfg 2)",
                p_table=json.dumps([list(map(float, r)) for r in table]))
    prop = proposer.Proposer(model, p_cum, proposer.Q_EDGES, cfg.mc_frac, meta, args.rho_low, args.p_low)
    prop.save(args.out or proposer.DEFAULT_PATH)
    log(f"[done] P={p_cum} hit {hit:.4f} (plain rule {plain_hit:.4f}), {cells:.2f} cells, "
        f"{time.perf_counter() - t_start:.0f} s total")
    print(json.dumps({k: (float(v) if isinstance(v, (np.floating, float)) else v) for k, v in meta.items()}))
    ctx.close()


if __name__ == "__main__":
    main()
