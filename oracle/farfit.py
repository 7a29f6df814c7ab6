"""Background tail fit and extrapolated false-alarm rate (oracle, float64) -- TEST
INFRASTRUCTURE (see the package docstring).

Sec. IV: the cumulative number of background coincidences n_b(Lambda) (time-slid, foreground
excluded) falls linearly on a logarithmic scale for large Lambda, so for Lambda >~ 8 it is
replaced by the least-squares line of Eq. (7), log n_b = alpha + beta Lambda, and the FAR of a
foreground event follows from Eq. (6) with the counted background below the fit range and the
fitted one above.  Readings taken where the text is silent:

* Lambda is the network SNR rho_c of the coincidence (see ``coinc``); counts are taken on the
  grid of edges x_e as n_b(x_e) = #{background survivors with float64(stat) >= float64(x_e)^2}.
* The fit uses the edges with x_e >= x_min and n_b(x_e) > 0 (log of zero is undefined), natural
  logarithm, ordinary least squares with equal weights; at least two such edges are needed.
* Hybrid FAR of a foreground coincidence with statistic rho (stat = rho^2):
    rho <  x_fit : (1 + #{background stat >= stat}) / T_b        (Eq. (6), counted)
    rho >= x_fit : exp(alpha + beta rho) / T_b                     (Eq. (7), the fitted expected
                                                                    count per background time)
  The fitted count is an expectation and may fall below one event, which is what lets the
  extrapolation reach inverse FARs longer than the background time T_b.
* The statistic at which the fitted FAR equals 1 / ifar: x = (log(T_b / ifar) - alpha) / beta.
"""
import math

import numpy as np


def cumulative_counts(bg_stat, edges) -> np.ndarray:
    """n_b(x_e) for every edge (bg_stat: float32 stat = rho_c^2 of background survivors)."""
    s = np.asarray(bg_stat).astype(np.float64)
    return np.array([int(np.sum(s >= float(e) ** 2)) for e in np.asarray(edges, np.float32).astype(np.float64)],
                    np.int64)


def tail_fit(edges, counts, x_min: float):
    """(alpha, beta, n_used) of log n_b = alpha + beta x over the edges >= x_min with n_b > 0."""
    x = np.asarray(edges, np.float32).astype(np.float64)
    n = np.asarray(counts, np.int64)
    sel = (x >= float(np.float32(x_min))) & (n > 0)
    if sel.sum() < 2:
        raise ValueError("tail fit needs two edges with counts above x_min")
    xs, ys = x[sel], np.log(n[sel].astype(np.float64))
    xm, ym = xs.mean(), ys.mean()
    beta = float(np.sum((xs - xm) * (ys - ym)) / np.sum((xs - xm) ** 2))
    alpha = float(ym - beta * xm)
    return alpha, beta, int(sel.sum())


def far(fg_stat, bg_stat, t_b: float, alpha: float, beta: float, x_fit: float) -> np.ndarray:
    """Hybrid FAR (per second) of each foreground stat (float32 rho_c^2)."""
    fg = np.asarray(fg_stat, np.float32)
    bg = np.asarray(bg_stat, np.float32)
    out = np.empty(len(fg))
    xf = float(np.float32(x_fit))
    for i, s in enumerate(fg):
        rho = math.sqrt(float(s))
        if rho < xf:
            out[i] = (1.0 + float(np.sum(bg >= s))) / t_b
        else:
            out[i] = math.exp(alpha + beta * rho) / t_b
    return out


def ifar_threshold(alpha: float, beta: float, t_b: float, ifar: float) -> float:
    """Statistic at which the fitted FAR equals 1 / ifar (same time unit as t_b)."""
    return (math.log(t_b / ifar) - alpha) / beta
