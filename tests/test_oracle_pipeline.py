"""Whole-chain self-consistency of the oracle (parity unpinned against the paper: the
paper's own search outcomes need data that is not available; this checks only that
a loud injection is found by both the flat and the hierarchical oracle searches)."""
import numpy as np

import oracle
import synth
from helpers import loud


def test_flat_and_hierarchical_find_a_loud_injection():
    n, fs, f_low = 2 ** 15, 2048.0, 20.0
    g = synth.rng(77, 0, 0, synth.BANK)
    m1, m2 = synth.bank_by_tau0(60, 4.0, 10.0, 1.0, 2.0, g)
    fine = synth.taylorf2_bank(m1, m2, n, fs, f_low)
    cm1, cm2 = m1[::6], m2[::6]
    coarse = synth.taylorf2_bank(cm1, cm2, n // 4, fs / 4, f_low)
    t = 30
    inj_h = dict(m1=m1[t], m2=m2[t], t_c=9.0, phi_c=0.3, snr=11.0)
    inj_l = dict(m1=m1[t], m2=m2[t], t_c=9.004, phi_c=1.3, snr=11.0)
    sh, _ = synth.make_strain(77, 0, 0, n, fs, f_low, injections=loud([inj_h], n, fs, f_low))
    sl, _ = synth.make_strain(77, 1, 0, n, fs, f_low, injections=loud([inj_l], n, fs, f_low))
    k = np.arange(n // 2 + 1)
    psd = np.empty(n // 2 + 1)
    psd[1:] = synth.aligo_psd_fit(k[1:] * fs / n)
    psd[0] = psd[1]
    flat = oracle.flat_search([sh], [sl], [psd], [psd], fs, f_low, fine, n_slides=20,
                              step_sec=0.1)
    hier = oracle.hierarchical_search([sh], [sl], [psd], [psd], fs, f_low, coarse, fine,
                                      n_sh1=2, t_sh1_sec=3.0, n_slides=20, step_sec=0.1)
    for res in (flat, hier):
        c = res["coinc"]["coincs"]
        zl = c["slide"] == 0
        hit = zl & (np.abs(c["tick_h"] - 9.0 * 51200) <= 0.1 * 51200) & (c["snr_c"] >= 8.0)
        assert np.any(hit)
    assert 0 < sum(len(x) for x in hier["fine_ids"]) < fine.n_tmpl


def test_proposer_with_every_cell_selected_reproduces_the_plain_hierarchy():
    from oracle import proposer as P
    n, fs, f_low = 2 ** 15, 2048.0, 20.0
    g = synth.rng(78, 0, 0, synth.BANK)
    m1, m2 = synth.bank_by_tau0(60, 4.0, 10.0, 1.0, 2.0, g)
    fine = synth.taylorf2_bank(m1, m2, n, fs, f_low)
    coarse = synth.taylorf2_bank(m1[::6], m2[::6], n // 4, fs / 4, f_low)
    t = 24
    sh, _ = synth.make_strain(78, 0, 0, n, fs, f_low, injections=loud([dict(m1=m1[t], m2=m2[t], t_c=7.0, phi_c=0.3, snr=10.0)], n, fs, f_low))
    sl, _ = synth.make_strain(78, 1, 0, n, fs, f_low, injections=loud([dict(m1=m1[t], m2=m2[t], t_c=7.003, phi_c=1.0, snr=10.0)], n, fs, f_low))
    k = np.arange(n // 2 + 1)
    psd = np.empty(n // 2 + 1)
    psd[1:] = synth.aligo_psd_fit(k[1:] * fs / n)
    psd[0] = psd[1]
    kw = dict(n_sh1=2, t_sh1_sec=3.0, n_slides=10, step_sec=0.1, rho1=6.0, chisq_rho_min=5.0)
    plain = oracle.hierarchical_search([sh], [sl], [psd], [psd], fs, f_low, coarse, fine, **kw)
    model = np.random.default_rng(9).normal(0, 0.1, P.N_MODEL)
    every = oracle.hierarchical_search([sh], [sl], [psd], [psd], fs, f_low, coarse, fine,
                                       proposer=(model, (1.75, 2.5, 3.25), 2.0), **kw)
    assert sum(len(x) for x in plain["fine_ids"]) > 0
    assert all(np.array_equal(a, b) for a, b in zip(plain["fine_ids"], every["fine_ids"]))
    one = oracle.hierarchical_search([sh], [sl], [psd], [psd], fs, f_low, coarse, fine,
                                     proposer=(model, (1.75, 2.5, 3.25), 0.0), **kw)
    assert all(set(b.tolist()) <= set(a.tolist()) for a, b in zip(plain["fine_ids"], one["fine_ids"]))
