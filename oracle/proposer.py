"""Learned follow-up proposer (oracle, float64) -- TEST INFRASTRUCTURE (see the package docstring).

Sec. III re-filters, for every followed stage-1 coincidence, the whole fine-bank neighbourhood of
its coarse template; the neighbourhood reading used throughout is |Mc_f - Mc_c| <= frac Mc_c.  The
proposer layered on top splits that neighbourhood into 64 cells and re-filters only the cells a
small multilayer perceptron (MLP) ranks as likely to hold the signal:

* cell of fine template f for coarse template c (only for f inside the neighbourhood):
    u  = (Mc_f - Mc_c) / (frac Mc_c)           in [-1, 1]   (float64, operations in this order)
    ib = min(15, max(0, floor((u + 1) * 8)))   16 equal bins of the relative chirp-mass offset
    iq = number of the 3 mass-ratio edges <= q_f   4 mass-ratio bins
    cell = 4 ib + iq
* 16 features of a coincidence (k = its slide, p = 8 chi-square bins, Sec. II / Eq. (4)):
    0 rho~_H, 1 rho~_L, 2 rho_c (the coincidence's network SNR of re-weighted SNRs),
    3 (chi2_r,H + chi2_r,L) / 2,
    4..11 (X_H,l + X_L,l) / (2 (2p - 2) / p), X_l = p |z_l - z / p|^2 the per-bin terms of the
          chi-square (their sum over l is chi2; each has mean (2p - 2) / p in Gaussian noise),
    12 Mc of the coarse template, 13 q = m1 / m2 >= 1 of the coarse template,
    14 delta t = circ(tick_H - tick_L - k step) / ticks_per_second   (seconds),
    15 delta phi = phi_H - phi_L wrapped into (-pi, pi].
  Triggers whose chi-square was not evaluated (rho below the chi-square threshold) contribute 0.
* MLP: h0 = (x - mu) * inv_std;  h_i = relu(h_{i-1} W_i + b_i) for i = 1..3 (width 128);
  logits = h3 W4 + b4 (64 cells).  Trained with the mean softmax cross-entropy against the cell
  of the injected parameters, by Adam (Kingma & Ba 2015, Algorithm 1).
* Selection: cells sorted by softmax probability (descending; equal probabilities by lower cell
  index); the smallest leading set whose cumulative probability reaches P is followed (all 64
  cells if the sum never reaches P).  All 64 cells give back the plain neighbourhood rule.
  Two tiers: coincidences with rho_c >= rho_split use P, weaker ones (followed down to a lower
  threshold) use a smaller P_low.

Model layout (float32 in the library, float64 here): one flat vector
  [mu (16), inv_std (16), W1 (16 x 128), b1, W2 (128 x 128), b2, W3 (128 x 128), b3, W4 (128 x 64), b4]
with each W stored row-major as [input][output]; the 43,456 values after the first 32 are the
trained parameters.
"""
import math

import numpy as np

N_FEATURES = 16
N_CELLS = 64
WIDTH = 128
N_NORM = 2 * N_FEATURES
LAYERS = [(N_FEATURES, WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH), (WIDTH, N_CELLS)]
N_PARAMS = sum(k * j + j for k, j in LAYERS)          # 43,456 trained values
N_MODEL = N_NORM + N_PARAMS


def unpack(model):
    """(mu, inv_std, [(W, b)] * 4) views of a flat model vector."""
    model = np.asarray(model, np.float64)
    assert model.shape == (N_MODEL,)
    mu, inv_std = model[:N_FEATURES], model[N_FEATURES:N_NORM]
    off, layers = N_NORM, []
    for k, j in LAYERS:
        W = model[off:off + k * j].reshape(k, j)
        off += k * j
        b = model[off:off + j]
        off += j
        layers.append((W, b))
    return mu, inv_std, layers


def forward(model, x):
    """Logits [n, 64] and the activations h0..h3 (for the backward pass)."""
    mu, inv_std, layers = unpack(model)
    h = (np.asarray(x, np.float64) - mu) * inv_std
    acts = [h]
    for i, (W, b) in enumerate(layers):
        z = h @ W + b
        h = np.maximum(z, 0.0) if i < len(layers) - 1 else z
        acts.append(h)
    return acts[-1], acts[:-1]


def softmax(logits):
    z = np.asarray(logits, np.float64)
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(model, x, labels):
    """Mean softmax cross-entropy over the batch and its gradient with respect to the 43,456
    trained parameters (flat, model layout without the first 32 values), by backpropagation."""
    logits, acts = forward(model, x)
    labels = np.asarray(labels, np.int64)
    n = len(labels)
    p = softmax(logits)
    loss = float(np.mean(-np.log(p[np.arange(n), labels])))
    dz = p.copy()
    dz[np.arange(n), labels] -= 1.0
    dz /= n
    _, _, layers = unpack(model)
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        a = acts[i]
        grads[i] = (a.T @ dz, dz.sum(axis=0))
        if i > 0:
            dz = (dz @ W.T) * (acts[i] > 0.0)
    return loss, np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam_step(theta, m, v, g, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) at step t >= 1; returns (theta, m, v)."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return np.asarray(theta, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def select_cells(logits, p_cum: float, rho_c=None, rho_split: float = None, p_cum_low: float = None):
    """uint64 cell masks: smallest set of most probable cells with cumulative probability >=
    p_cum.  Two tiers: with rho_c (float32 feature 2 of each row) and rho_split given, rows with
    rho_c < rho_split use p_cum_low instead."""
    p = softmax(logits)
    out = np.zeros(len(p), np.uint64)
    for i in range(len(p)):
        pc = p_cum
        if rho_split is not None and float(np.float32(rho_c[i])) < float(np.float32(rho_split)):
            pc = p_cum_low
        order = sorted(range(N_CELLS), key=lambda c: (-p[i, c], c))
        acc, mask = 0.0, 0
        for c in order:
            mask |= 1 << c
            acc += p[i, c]
            if acc >= pc:
                break
        out[i] = np.uint64(mask)
    return out


def cell_index(mc_c: float, mc_f: float, q_f: float, frac: float, q_edges) -> int:
    """Cell of fine template (mc_f, q_f) in the neighbourhood of a coarse template with chirp
    mass mc_c, or -1 outside the neighbourhood."""
    mc_c, mc_f, q_f = float(mc_c), float(mc_f), float(q_f)
    if not abs(mc_f - mc_c) <= frac * mc_c:
        return -1
    u = (mc_f - mc_c) / (frac * mc_c)
    ib = min(15, max(0, int(math.floor((u + 1.0) * 8.0))))
    iq = sum(1 for e in q_edges if float(e) <= q_f)
    return 4 * ib + iq


def followup_cells(coincs, rho_min: float, coarse_mchirp, fine_mchirp, fine_q, q_edges, frac: float,
                   seg_ticks: int, n_seg: int, masks):
    """As ``followup.followup_templates`` but each selected coincidence i only contributes the fine
    templates of its neighbourhood whose cell bit is set in masks[i] (masks indexed like coincs)."""
    stat = np.asarray(coincs["stat"]).astype(np.float64)
    sel = np.nonzero(stat >= float(rho_min) ** 2)[0]
    per_seg = [set() for _ in range(n_seg)]
    for c in sel:
        mc = float(coarse_mchirp[int(coincs["tmpl"][c])])
        mask = int(masks[c])
        nb = [f for f in range(len(fine_mchirp))
              if (ci := cell_index(mc, fine_mchirp[f], fine_q[f], frac, q_edges)) >= 0 and (mask >> ci) & 1]
        for s in {int(coincs["tick_h"][c]) // seg_ticks, int(coincs["tick_l"][c]) // seg_ticks}:
            if 0 <= s < n_seg:
                per_seg[s].update(nb)
    return [np.asarray(sorted(s), dtype=np.int64) for s in per_seg]


def features(coincs, trig_h, trig_l, coarse_mchirp, coarse_q, step: int, wrap: int, ticks_per_second: int,
             p: int = 8):
    """[n, 16] features of the coincidences.  trig_* are dicts of arrays with tmpl, tick, snr,
    phase, chisq (chi2_r) and bins ([n_trig, p] per-bin chi-square terms); the trigger of each
    coincidence is the one with the coincidence's template and tick (tick_L unshifted)."""
    def index(tr):
        return {(int(a), int(b)): i for i, (a, b) in enumerate(zip(tr["tmpl"], tr["tick"]))}
    ih, il = index(trig_h), index(trig_l)
    n = len(coincs["tmpl"])
    out = np.zeros((n, N_FEATURES), np.float64)
    norm = 2.0 * (2.0 * p - 2.0) / p
    for c in range(n):
        t = int(coincs["tmpl"][c])
        a = ih[(t, int(coincs["tick_h"][c]))]
        b = il[(t, int(coincs["tick_l"][c]))]
        out[c, 0] = float(coincs["snr_h"][c])
        out[c, 1] = float(coincs["snr_l"][c])
        out[c, 2] = float(coincs["snr_c"][c])
        out[c, 3] = (float(trig_h["chisq"][a]) + float(trig_l["chisq"][b])) / 2.0
        for l in range(p):
            out[c, 4 + l] = (float(trig_h["bins"][a][l]) + float(trig_l["bins"][b][l])) / norm
        out[c, 12] = float(coarse_mchirp[t])
        out[c, 13] = float(coarse_q[t])
        d = int(coincs["tick_h"][c]) - int(coincs["tick_l"][c]) - int(coincs["slide"][c]) * int(step)
        d = (d + wrap // 2) % wrap - wrap // 2
        out[c, 14] = d / float(ticks_per_second)
        dp = float(trig_h["phase"][a]) - float(trig_l["phase"][b])
        dp = math.remainder(dp, 2.0 * math.pi)      # into [-pi, pi]
        out[c, 15] = math.pi if dp == -math.pi else dp
    return out
