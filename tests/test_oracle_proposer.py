"""Pins of the learned follow-up proposer's oracle: the chi-square bin terms, the features, the
MLP forward/backward, Adam, the cell selection and the cell follow-up rule."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import proposer as P


def _random_model(seed, scale=0.3):
    g = np.random.default_rng(seed)
    m = g.normal(0.0, scale, P.N_MODEL)
    m[:P.N_FEATURES] = g.normal(0.0, 1.0, P.N_FEATURES)              # mu
    m[P.N_FEATURES:P.N_NORM] = g.uniform(0.5, 2.0, P.N_FEATURES)     # inv_std
    return m


def test_layout_has_43456_trained_parameters():
    assert P.N_PARAMS == 16 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 64 + 64 == 43456
    mu, inv_std, layers = P.unpack(np.arange(P.N_MODEL, dtype=np.float64))
    assert mu[0] == 0 and inv_std[0] == 16 and layers[0][0][0, 1] == 33 and layers[3][1][-1] == P.N_MODEL - 1


def test_forward_closed_form_single_path():
    # one path: h1[0] = relu((x0 - mu0) * s0), copied through two identity units, into logit 5
    m = np.zeros(P.N_MODEL)
    m[0], m[P.N_FEATURES] = 1.5, 2.0
    mu, inv_std, L = P.unpack(m)       # views into m
    L[0][0][0, 0] = 1.0
    L[1][0][0, 0] = 1.0
    L[2][0][0, 0] = 1.0
    L[3][0][0, 5] = 3.0
    L[3][1][7] = -0.25
    x = np.zeros((3, 16))
    x[:, 0] = [0.0, 2.0, 4.0]
    logits, _ = P.forward(m, x)
    want5 = 3.0 * np.maximum((x[:, 0] - 1.5) * 2.0, 0.0)
    assert np.allclose(logits[:, 5], want5, rtol=0, atol=1e-15)
    assert np.all(logits[:, 7] == -0.25)
    assert np.count_nonzero(logits) == 3 + 1 + 1   # logit 7 everywhere, logit 5 where x0 > mu0


def test_zero_model_loss_is_log64_and_bias_gradient_is_closed_form():
    m = np.zeros(P.N_MODEL)
    m[P.N_FEATURES:P.N_NORM] = 1.0
    x = np.random.default_rng(1).normal(size=(10, 16))
    labels = np.arange(10) * 6 % 64
    loss, g = P.loss_and_grad(m, x, labels)
    assert abs(loss - math.log(64.0)) < 1e-14
    gb4 = g[-64:]
    want = np.full(64, 1.0 / 64.0)
    for c in labels:
        want[c] -= 1.0 / 10.0
    assert np.allclose(gb4, want, atol=1e-15)
    assert np.all(g[:-64] == 0.0)      # zero weights block every other path


def test_gradient_matches_central_finite_differences():
    m = _random_model(2)
    g_ = np.random.default_rng(3)
    x = g_.normal(size=(7, 16))
    labels = g_.integers(0, 64, 7)
    _, grad = P.loss_and_grad(m, x, labels)
    # check every layer's weights and biases at random coordinates
    idx = np.concatenate([g_.integers(0, 16 * 128, 12), 16 * 128 + g_.integers(0, 128, 4),
                          2176 + g_.integers(0, 128 * 128, 12), 43456 - 64 + g_.integers(0, 64, 6),
                          43456 - 64 - 8192 + g_.integers(0, 8192, 6)])
    h = 1e-6
    for i in idx:
        mp, mm = m.copy(), m.copy()
        mp[P.N_NORM + i] += h
        mm[P.N_NORM + i] -= h
        fd = (P.loss_and_grad(mp, x, labels)[0] - P.loss_and_grad(mm, x, labels)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(grad[i])), (i, fd, grad[i])


def test_adam_first_step_moves_each_parameter_by_lr_against_its_gradient_sign():
    g = np.array([3.0, -0.5, 1e-3, -2e4])
    th, m, v = P.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-5)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_second_step_by_hand():
    # scalar: g1 = 2, g2 = -1, lr = 0.1
    th, m, v = P.adam_step(np.zeros(1), np.zeros(1), np.zeros(1), np.array([2.0]), 1, 0.1)
    th, m, v = P.adam_step(th, m, v, np.array([-1.0]), 2, 0.1)
    m2 = 0.9 * 0.2 + 0.1 * -1.0             # 0.08
    v2 = 0.999 * 0.004 + 0.001 * 1.0        # 0.004996
    mh, vh = m2 / (1 - 0.81), v2 / (1 - 0.999 ** 2)
    th1 = -0.1 * (0.2 / 0.1) / (math.sqrt(0.004 / 0.001) + 1e-8)
    want = th1 - 0.1 * mh / (math.sqrt(vh) + 1e-8)
    assert abs(th[0] - want) < 1e-15 and abs(m[0] - m2) < 1e-16 and abs(v[0] - v2) < 1e-16


def test_select_cells_is_the_minimal_top_set():
    g = np.random.default_rng(4)
    logits = g.normal(0, 2.0, (40, 64))
    for pc in (0.0, 0.5, 0.9, 0.99):
        masks = P.select_cells(logits, pc)
        p = P.softmax(logits)
        for i in range(len(p)):
            sel = [c for c in range(64) if (int(masks[i]) >> c) & 1]
            ps = np.sort(p[i])[::-1]
            k = len(sel)
            assert p[i, sel].sum() >= pc or k == 64
            assert k == 1 or ps[:k - 1].sum() < pc               # nothing smaller reaches pc
            assert p[i, sel].min() >= ps[k - 1] - 1e-15           # the selected are the top k
    assert np.all(P.select_cells(logits, 2.0) == np.uint64(2 ** 64 - 1))


def test_two_tier_selection_is_the_per_row_single_tier_selection():
    g = np.random.default_rng(8)
    logits = g.normal(0, 2.0, (60, 64))
    rho = g.uniform(6.0, 8.0, 60).astype(np.float32)
    rho[:3] = np.float32(7.0)                                  # the split itself belongs to the upper tier
    got = P.select_cells(logits, 0.99, rho, 7.0, 0.5)
    hi, lo = P.select_cells(logits, 0.99), P.select_cells(logits, 0.5)
    assert np.array_equal(got, np.where(rho >= np.float32(7.0), hi, lo))
    assert np.all(got[:3] == hi[:3])


def test_select_cells_breaks_ties_by_lower_index():
    logits = np.zeros((1, 64))
    assert int(P.select_cells(logits, 3.0 / 64.0 - 1e-12)[0]) == 0b111


def test_cell_index_by_hand():
    e = (1.75, 2.5, 3.25)
    assert P.cell_index(2.0, 2.0, 1.0, 0.05, e) == 4 * 8 + 0
    # frac = 1/16 makes the window edges exact: 2 (1 -+ 1/16) = 1.875, 2.125
    assert P.cell_index(2.0, 1.875, 1.75, 0.0625, e) == 4 * 0 + 1
    assert P.cell_index(2.0, 2.125, 4.0, 0.0625, e) == 4 * 15 + 3       # u = 1 -> bin 16 -> 15
    assert P.cell_index(2.0, 2.125 + 2 ** -40, 2.0, 0.0625, e) == -1
    assert P.cell_index(2.0, 1.875 - 2 ** -40, 2.0, 0.0625, e) == -1
    # bin width 2 * 0.125 / 16 = 1/64: 1.875 + 3.5/64 is inside bin 3
    assert P.cell_index(2.0, 1.875 + 3.5 / 64, 3.0, 0.0625, e) == 4 * 3 + 2
    assert P.cell_index(2.0, 1.875 + 4.0 / 64, 3.25, 0.0625, e) == 4 * 4 + 3


def _coinc_fixture(seed):
    g = np.random.default_rng(seed)
    coarse_mc = np.sort(g.uniform(1.4, 10.0, 30))
    fine_m1, fine_m2 = synth.bank_by_tau0(400, 1.4, 10.0, 1.0, 4.0, g)
    fine_mc, _ = synth.mchirp_eta(fine_m1, fine_m2)
    fine_q = fine_m1 / fine_m2
    seg_ticks = 51200 * 64
    c = np.zeros(25, synth.COINC_DTYPE)
    c["tmpl"] = g.integers(0, 30, 25)
    c["tick_h"] = g.integers(0, 3 * seg_ticks, 25)
    c["tick_l"] = c["tick_h"] + g.integers(-seg_ticks // 2, seg_ticks // 2, 25)
    c["tick_l"] = np.clip(c["tick_l"], 0, 3 * seg_ticks - 1)
    c["stat"] = g.uniform(30.0, 80.0, 25).astype(np.float32)
    return c, coarse_mc, fine_mc, fine_q, seg_ticks


def test_followup_cells_with_every_cell_is_the_plain_rule():
    c, cmc, fmc, fq, st = _coinc_fixture(5)
    plain = oracle.followup_templates(c, 7.0, cmc, fmc, 0.05, st, 3)
    cells = P.followup_cells(c, 7.0, cmc, fmc, fq, (1.75, 2.5, 3.25), 0.05, st, 3,
                             np.full(len(c), 2 ** 64 - 1, np.uint64))
    assert all(np.array_equal(a, b) for a, b in zip(plain, cells))
    empty = P.followup_cells(c, 7.0, cmc, fmc, fq, (1.75, 2.5, 3.25), 0.05, st, 3, np.zeros(len(c), np.uint64))
    assert all(len(a) == 0 for a in empty)


def test_followup_cells_single_cell_brute_force():
    c, cmc, fmc, fq, st = _coinc_fixture(6)
    e = (1.75, 2.5, 3.25)
    g = np.random.default_rng(7)
    masks = np.array([np.uint64(1) << np.uint64(g.integers(0, 64)) for _ in range(len(c))], np.uint64)
    got = P.followup_cells(c, 7.0, cmc, fmc, fq, e, 0.05, st, 3, masks)
    for s in range(3):
        want = set()
        for i in range(len(c)):
            if not float(c["stat"][i]) >= 49.0:
                continue
            if s not in (int(c["tick_h"][i]) // st, int(c["tick_l"][i]) // st):
                continue
            mc = cmc[c["tmpl"][i]]
            cell = int(np.log2(float(masks[i])))
            for f in range(len(fmc)):
                if abs(fmc[f] - mc) > 0.05 * mc:
                    continue
                u = (fmc[f] - mc) / (0.05 * mc)
                ib = min(15, int((u + 1.0) * 8.0)) if u > -1.0 else 0
                iq = int(fq[f] >= 1.75) + int(fq[f] >= 2.5) + int(fq[f] >= 3.25)
                if 4 * ib + iq == cell:
                    want.add(f)
        assert set(got[s].tolist()) == want


def test_features_by_hand():
    tps = 51200
    th = dict(tmpl=np.array([3, 4]), tick=np.array([1000, 52000]), snr=np.float32([6.5, 7.0]),
              phase=np.float32([3.0, -1.0]), chisq=np.float32([1.5, 0.0]),
              bins=np.array([np.arange(8) * 0.5, np.zeros(8)], np.float32))
    tl = dict(tmpl=np.array([4, 4]), tick=np.array([51000, 62000]), snr=np.float32([5.0, 4.5]),
              phase=np.float32([-3.0, 0.5]), chisq=np.float32([0.0, 2.5]),
              bins=np.array([np.zeros(8), np.full(8, 1.75)], np.float32))
    c = np.zeros(1, synth.COINC_DTYPE)
    c["slide"], c["tmpl"], c["tick_h"], c["tick_l"] = 2, 4, 52000, 62000
    c["snr_h"], c["snr_l"], c["stat"], c["snr_c"] = 7.0, 4.5, 69.25, 8.3216584
    wrap, step = 5 * tps, 2 * tps + 100
    cmc = np.arange(10) * 0.5 + 1.0
    cq = np.arange(10) * 0.25 + 1.0
    f = P.features(c, th, tl, cmc, cq, step, wrap, tps)[0]
    assert f[0] == 7.0 and f[1] == 4.5 and f[2] == np.float64(np.float32(8.3216584))
    assert f[3] == (0.0 + 2.5) / 2
    assert np.allclose(f[4:12], (0.0 + 1.75) / (2 * 14 / 8))
    assert f[12] == 3.0 and f[13] == 2.0
    # 52000 - 62000 - 2 (102500) = -215000 -> circ into [-128000, 128000) -> 41000
    assert f[14] == 41000 / tps
    assert abs(f[15] - (-1.0 - 0.5)) < 1e-15
    # phase wrap: 3.0 - (-3.0) = 6.0 -> 6 - 2 pi
    c["tick_h"], c["tmpl"], c["slide"] = 1000, 3, 0
    th["tmpl"][0] = 3
    tl["tmpl"][0], tl["tick"][0] = 3, 51000
    c["tick_l"] = 51000
    f = P.features(c, th, tl, cmc, cq, step, wrap, tps)[0]
    assert abs(f[15] - (6.0 - 2 * math.pi)) < 1e-12
    assert f[3] == 0.75 and np.allclose(f[4:12], np.arange(8) * 0.5 / 3.5)
    assert f[14] == (1000 - 51000) / tps


def test_chisq_terms_sum_to_chisq_and_have_the_expected_mean_in_noise():
    n, fs, f_low = 8192, 512.0, 30.0
    b = synth.taylorf2_bank([12.0], [12.0], n, fs, f_low)
    h = b.spectrum(0)
    k = np.arange(n // 2 + 1)
    psd = np.empty(n // 2 + 1)
    psd[1:] = synth.aligo_psd_fit(k[1:] * fs / n)
    psd[0] = psd[1]
    k_lo, k_hi = oracle.band_edges(n, fs, f_low, b.kstart[0], b.k1[0])
    sig = oracle.template_sigma(h, psd, n, fs, k_lo, k_hi)
    e = oracle.chisq_bin_edges(h, psd, k_lo, k_hi, 8)
    terms = []
    for seed in range(10):
        s, _ = synth.make_strain(911, 0, seed, n, fs, f_low)
        st = oracle.strain_fft(s, fs)
        for m in range(0, n, 263):
            zl = oracle.chisq.bin_snrs(st, h, psd, n, fs, sig, m, e)
            t = oracle.chisq.chisq_terms(zl)
            c2, _ = oracle.chisq_at(st, h, psd, n, fs, sig, m, e)
            assert abs(t.sum() / 14.0 - c2) < 1e-12 * max(1.0, c2)
            terms.append(t)
    terms = np.asarray(terms)
    # each term p |z_l - z/p|^2 has mean (2p - 2)/p = 1.75 in Gaussian noise (z_l - z/p: complex
    # Gaussian with variance 2 (1/p)(1 - 1/p) in the sigma-normalised units)
    assert np.all(np.abs(terms.mean(axis=0) - 1.75) < 0.35)
    assert abs(terms.mean() - 1.75) < 0.1
