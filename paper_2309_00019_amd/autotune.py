"""Matched-filter schedule autotuner.

The two-pass filter stages a batch of templates' N-point intermediates between pass A and
pass B.  Small batches leave the GPU under-filled at the kernel boundaries; large ones push the
intermediate out of the 256 MB Infinity Cache before pass B reads it back.  The best budget
depends on N, the bank's band lengths and the candidate volume, so it is measured: the filter
runs on a sample of the real bank and data for each candidate budget (device time from events
on the library's stream) and the fastest is set on the context.
"""
import numpy as np
import torch

from . import hs

BUDGETS_MB = (64, 96, 128, 160, 192, 256)


def tune_mf_batch(ctx: hs.Context, spec, n: int, fs: float, bank, tmpl_ids, thr: float, budgets_mb=BUDGETS_MB,
                  reps: int = 3):
    """Times hs_matched_filter over tmpl_ids for each budget, sets the fastest on ctx and returns
    (best_mb, {mb: microseconds per template})."""
    table = {}
    for mb in budgets_mb:
        hs.hs_set_mf_batch_bytes(ctx, int(mb) << 20)
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
        table[int(mb)] = round(best, 4)
    best_mb = min(table, key=table.get)
    hs.hs_set_mf_batch_bytes(ctx, best_mb << 20)
    return best_mb, table
