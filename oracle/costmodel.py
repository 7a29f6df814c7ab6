"""Matched-filter cost model of Sec. V, Eq. (8) (oracle).

The cost of one template applied to one segment of N = f t_seg samples is
kappa N log N (Cooley-Tukey FFT count); the speed-up of the two-stage search
over the flat search is

  N_seg N_flat O_flat / (N_seg N_stage1 O_coarse + N_stage2 gamma O_flat),
  O_x = kappa f_x t_seg log(f_x t_seg),

where gamma accounts for per-segment overhead when a segment sees few
templates.  kappa and the base of the logarithm cancel.
"""
import math


def speedup_eq8(n_seg: int, n_flat: int, n_stage1: int, n_stage2: int, f_flat: float,
                f_coarse: float, t_seg: float, gamma: float = 1.0) -> float:
    def cost(f):
        n = f * t_seg
        return n * math.log(n)
    return n_seg * n_flat * cost(f_flat) / (n_seg * n_stage1 * cost(f_coarse) + n_stage2 * gamma * cost(f_flat))
