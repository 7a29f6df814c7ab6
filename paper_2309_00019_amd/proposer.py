"""Learned follow-up proposer: model container, training loop and the choice of P.

The neighbourhood of a followed coarse template (|Mc_f - Mc_c| <= frac Mc_c, the chirp-mass
reading of Sec. III) is split into 64 cells (16 bins of the relative chirp-mass offset u in
[-1, 1] times 4 mass-ratio bins); an MLP scores the cells from 16 features of the stage-1
coincidence and the search re-filters only the smallest set of top cells whose probabilities
sum to at least ``p_cum``.  All arithmetic runs in libhs (hs_proposer_features, hs_mlp_*,
hs_followup_cells); this module holds the model, batches the training data and reads the
validation statistics.
"""
import os
from dataclasses import dataclass, field

import numpy as np
import torch

from . import hs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "proposer_model.npz")
Q_EDGES = (1.75, 2.5, 3.25)     # quartiles of the bank's uniform q in [1, 4]
LAYERS = [(16, 128), (128, 128), (128, 128), (128, 64)]


@dataclass
class Proposer:
    """Model and operating point: coincidences with rho_c >= rho1 (the stage-1 threshold) keep
    the cells of cumulative probability p_cum; weaker ones down to rho_low keep those of
    p_cum_low (rho_low = rho1 gives a single tier)."""
    model: torch.Tensor                      # device float32 [hs.MLP_MODEL]
    p_cum: float = 0.99
    q_edges: tuple = Q_EDGES
    frac: float = 0.05
    meta: dict = field(default_factory=dict)
    rho_low: float = 6.75
    p_cum_low: float = 0.5

    @classmethod
    def load(cls, device, path: str = DEFAULT_PATH) -> "Proposer":
        z = np.load(path, allow_pickle=False)
        meta = {k[5:]: z[k].item() if z[k].ndim == 0 else z[k] for k in z.files if k.startswith("meta_")}
        extra = {k: float(z[k]) for k in ("rho_low", "p_cum_low") if k in z.files}
        return cls(torch.as_tensor(z["model"].astype(np.float32), device=device), float(z["p_cum"]),
                   tuple(float(v) for v in z["q_edges"]), float(z["frac"]), meta, **extra)

    def save(self, path: str = DEFAULT_PATH):
        extra = {"meta_" + k: np.asarray(v) for k, v in self.meta.items()}
        np.savez(path, model=self.model.detach().cpu().numpy(), p_cum=np.float64(self.p_cum),
                 q_edges=np.asarray(self.q_edges, np.float64), frac=np.float64(self.frac),
                 rho_low=np.float64(self.rho_low), p_cum_low=np.float64(self.p_cum_low), **extra)


def cell_labels(coarse_mc, true_mc, true_q, frac: float, q_edges) -> np.ndarray:
    """Training targets: the cell of the injected (Mc, q) in the neighbourhood of the coarse
    template that found it (the cell rule of hs_followup_cells; u clamped into [-1, 1], so an
    injection outside the neighbourhood is labelled with the nearest edge bin)."""
    coarse_mc = np.asarray(coarse_mc, np.float64)
    u = (np.asarray(true_mc, np.float64) - coarse_mc) / (frac * coarse_mc)
    ib = np.clip(np.floor((np.clip(u, -1.0, 1.0) + 1.0) * 8.0), 0, 15).astype(np.int64)
    iq = sum((np.asarray(true_q, np.float64) >= e).astype(np.int64) for e in q_edges)
    return (4 * ib + iq).astype(np.int32)


def init_model(x_train: np.ndarray, seed: int) -> np.ndarray:
    """He-normal weights, zero biases, input normalisation from the training features."""
    g = np.random.default_rng(seed)
    mu = x_train.mean(axis=0)
    sd = x_train.std(axis=0)
    m = [mu, 1.0 / np.where(sd > 1e-12, sd, 1.0)]
    for k, j in LAYERS:
        m.append(g.normal(0.0, np.sqrt(2.0 / k), k * j))
        m.append(np.zeros(j))
    out = np.concatenate(m).astype(np.float32)
    assert out.size == hs.MLP_MODEL
    return out


def mean_loss(ctx: hs.Context, model: torch.Tensor, x: np.ndarray, y: np.ndarray) -> float:
    """Mean softmax cross-entropy of the model on (x, y) (logits from hs_mlp_forward)."""
    z = hs.hs_mlp_forward(ctx, model, torch.as_tensor(np.ascontiguousarray(x, np.float32), device=ctx.device))
    z = z.cpu().numpy().astype(np.float64)
    z -= z.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z).sum(axis=1))
    return float(np.mean(lse - z[np.arange(len(y)), np.asarray(y, np.int64)]))


def train(ctx: hs.Context, x: np.ndarray, y: np.ndarray, epochs: int = 40, batch: int = 512, lr: float = 1e-3,
          seed: int = 0, log=None, lr_final: float = None, stop=None):
    """Adam on the softmax cross-entropy (hs_mlp_train_step), shuffled mini-batches; the learning
    rate decays geometrically from lr to lr_final over the epochs.  With ``stop`` = (x, y) the
    model of the epoch with the lowest loss on that set is returned (early stopping)."""
    dev = ctx.device
    model = torch.as_tensor(init_model(x, seed), device=dev)
    m = torch.zeros(hs.MLP_PARAMS, dtype=torch.float32, device=dev)
    v = torch.zeros_like(m)
    xd = torch.as_tensor(np.ascontiguousarray(x, np.float32), device=dev)
    yd = torch.as_tensor(np.ascontiguousarray(y, np.int32), device=dev)
    g = np.random.default_rng(seed + 1)
    t, history = 0, []
    decay = (lr_final / lr) ** (1.0 / max(1, epochs - 1)) if lr_final else 1.0
    best = (float("inf"), None, -1)
    for ep in range(epochs):
        order = torch.as_tensor(g.permutation(len(x)), device=dev)
        xs, ys = xd[order].contiguous(), yd[order].contiguous()
        tot = 0.0
        lr_ep = lr * decay ** ep
        for b0 in range(0, len(x), batch):
            t += 1
            tot += hs.hs_mlp_train_step(ctx, model, m, v, t, lr_ep, xs[b0:b0 + batch], ys[b0:b0 + batch]) * \
                min(batch, len(x) - b0)
        history.append(tot / len(x))
        extra = ""
        if stop is not None:
            ls = mean_loss(ctx, model, stop[0], stop[1])
            if ls < best[0]:
                best = (ls, model.clone(), ep + 1)
            extra = f", early-stopping set {ls:.4f}"
        if log:
            log(f"[train] epoch {ep + 1}/{epochs} lr {lr_ep:.2e} loss {history[-1]:.4f}{extra}")
    if stop is not None:
        if log:
            log(f"[train] keeping epoch {best[2]} (early-stopping loss {best[0]:.4f})")
        return best[1], history, best[2]
    return model, history, epochs


def selection_stats(ctx: hs.Context, model: torch.Tensor, x: np.ndarray, y: np.ndarray, p_cum: float):
    """(fraction of samples whose labelled cell is selected, mean number of selected cells)."""
    xd = torch.as_tensor(np.ascontiguousarray(x, np.float32), device=ctx.device)
    masks = hs.hs_mlp_propose(ctx, model, xd, p_cum).cpu().numpy().view(np.uint64)
    hit = (masks >> np.asarray(y, np.uint64)) & np.uint64(1)
    cells = np.array([bin(int(mk)).count("1") for mk in masks])
    return float(hit.mean()), float(cells.mean())
