"""Matched-filter schedule autotuner.

The two-pass filter stages a batch of templates' N-point intermediates between pass A and
pass B.  Small batches leave the GPU under-filled at the kernel boundaries and pay each launch's
ramp and tail more often; larger ones than the best have also measured slower.  Pass B's tile (the
rows of the intermediate one workgroup transforms) trades LDS per workgroup against the number
of workgroups; pass A's tile (the columns one workgroup transforms) sets the width of the
pieces in which each row of the intermediate is written.  The best setting depends on N, the
bank's band lengths and the candidate volume, so it is measured per transform length: the filter runs on a sample of
the real bank and data for each candidate (device time from events on the library's stream),
first over the batch budgets at the default tiles, then over the pass-B tiles at the best budget,
then over the pass-A tiles, and the fastest is set on the context.  No knob changes the results
(same candidates, same values).
"""
import torch

from . import hs

BUDGETS_MB = (64, 96, 128, 160, 192, 256)
TILES = (64, 128, 256)          # pass-B threads per workgroup
PA_COLS = (16, 32, 64)          # pass-A columns per workgroup


def _time(ctx, spec, n, fs, bank, tmpl_ids, thr, reps):
    hs.hs_matched_filter(ctx, spec, n, fs, bank, tmpl_ids, thr)          # warm-up (scratch growth)
    best = float("inf")
    for _ in range(reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record(ctx.stream)
        hs.hs_matched_filter(ctx, spec, n, fs, bank, tmpl_ids, thr)
        e.record(ctx.stream)
        e.synchronize()
        best = min(best, s.elapsed_time(e) * 1e3 / tmpl_ids.numel())
    return round(best, 4)


def tune_mf_batch(ctx: hs.Context, spec, n: int, fs: float, bank, tmpl_ids, thr: float, budgets_mb=BUDGETS_MB,
                  reps: int = 3):
    """Times hs_matched_filter over tmpl_ids for each budget (at the context's tile), sets the
    fastest on ctx and returns (best_mb, {mb: microseconds per template})."""
    table = {}
    for mb in budgets_mb:
        hs.hs_set_mf_batch_bytes(ctx, int(mb) << 20)
        table[int(mb)] = _time(ctx, spec, n, fs, bank, tmpl_ids, thr, reps)
    best_mb = min(table, key=table.get)
    hs.hs_set_mf_batch_bytes(ctx, best_mb << 20)
    return best_mb, table


def tune_mf_schedule(ctx: hs.Context, spec, n: int, fs: float, bank, tmpl_ids, thr: float, budgets_mb=BUDGETS_MB,
                     tiles=TILES, pa_cols=PA_COLS, reps: int = 3):
    """Batch budget, then pass-B tile, then pass-A tile; sets all three on ctx and returns
    {"batch_mb", "tile", "pa_cols", "budgets": {mb: us/template}, "tiles": {threads: us/template},
    "pa_tiles": {columns: us/template}}; the result is also recorded as the context's schedule for
    length n (hs.apply_mf_schedule sets it before every filter call at that n)."""
    ctx.mf_schedules.pop(int(n), None)
    hs.hs_set_mf_tile(ctx, 128)
    hs.hs_set_mf_pa_cols(ctx, 64)
    best_mb, budgets = tune_mf_batch(ctx, spec, n, fs, bank, tmpl_ids, thr, budgets_mb, reps)
    table = {}
    for t in tiles:
        hs.hs_set_mf_tile(ctx, int(t))
        table[int(t)] = budgets[best_mb] if t == 128 else _time(ctx, spec, n, fs, bank, tmpl_ids, thr, reps)
    best_t = min(table, key=table.get)
    hs.hs_set_mf_tile(ctx, best_t)
    pa_table = {}
    for c in pa_cols:
        hs.hs_set_mf_pa_cols(ctx, int(c))
        pa_table[int(c)] = table[best_t] if c == 64 else _time(ctx, spec, n, fs, bank, tmpl_ids, thr, reps)
    best_c = min(pa_table, key=pa_table.get)
    hs.hs_set_mf_pa_cols(ctx, best_c)
    ctx.mf_schedules[int(n)] = (best_mb << 20, best_t, best_c)
    return {"batch_mb": best_mb, "tile": best_t, "pa_cols": best_c, "budgets": budgets, "tiles": table,
            "pa_tiles": pa_table}
