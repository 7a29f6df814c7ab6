"""The allocation-free matched filter (hs_matched_filter_noalloc) against hs_matched_filter.

Both run the same kernels; the allocation-free call keeps its scratch in a fixed device array
and computes its twiddles on the device, so candidates must agree to the FP32 tolerance rule:
identical (template, sample) sets outside the threshold band thr (1 +- 1e-4), rho within 1e-4
relative (in practice ~1e-7), and the oracle's rule on sampled templates.  Two calls in a row,
the second smaller, show that what the first leaves in the shared array does not leak."""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import DELTA, analytic_psd, check_candidates, device_bank

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2309_00019_amd import hs
    c = hs.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _case(ctx, n, fs, n_tmpl, seed):
    import torch
    from paper_2309_00019_amd import hs, workload
    f_low = workload.F_LOW
    fm1, fm2 = workload.bank_masses(30000, 0)
    pick = np.linspace(0, 29999, n_tmpl).astype(np.int64)
    bank = synth.taylorf2_bank(fm1[pick], fm2[pick], n, fs, f_low)
    s, _ = synth.make_strain(seed, 0, 0, n, fs, f_low, glitch_rate=0.05)
    psd = analytic_psd(n, fs)
    psd_d = torch.as_tensor(psd, device=ctx.device)
    pb = device_bank(ctx, bank, psd_d, f_low)
    spec = hs.hs_whiten(ctx, torch.as_tensor(s, device=ctx.device), fs, f_low, psd_d)
    ids = torch.arange(bank.n_tmpl, dtype=torch.int32, device=ctx.device)
    return bank, s, psd, pb, spec, ids


def _compare(a, b, thr, delta):
    """a, b: candidate records of the same call through the two entry points."""
    ka = {(int(t), int(m)): r for t, m, r in zip(a["tpos"], a["m"], a["rho2"])}
    kb = {(int(t), int(m)): r for t, m, r in zip(b["tpos"], b["m"], b["rho2"])}
    assert len(ka) == len(a) and len(kb) == len(b), "duplicate candidates"
    lo, hi = (thr * (1 - delta)) ** 2, (thr * (1 + delta)) ** 2
    for k in set(ka) ^ set(kb):
        r = ka.get(k, kb.get(k))
        assert lo <= r < hi, (k, r)
    common = sorted(set(ka) & set(kb))
    ra = np.array([ka[k] for k in common], np.float64)
    rb = np.array([kb[k] for k in common], np.float64)
    err = float(np.max(np.abs(np.sqrt(ra / rb) - 1.0))) if common else 0.0
    assert err <= delta, err
    return len(set(ka) ^ set(kb)), err


def test_noalloc_matches_matched_filter_on_two_calls_in_a_row(ctx):
    import torch
    from paper_2309_00019_amd import hs, workload
    thr = 4.0
    # call 1: N = 2^19 at 2048 Hz, 40 templates of the benchmark's fine bank; the capacity leaves
    # room for a few templates' intermediates per batch, so the call runs several batches
    # call 2: N = 2^17 at 512 Hz, 12 templates, a smaller capacity
    for n, fs, n_tmpl, cap, seed in ((2 ** 19, 2048.0, 40, 1_200_000, 31), (2 ** 17, 512.0, 12, 200_000, 32)):
        _say(f"noalloc n={n} templates={n_tmpl} cap={cap}")
        bank, s, psd, pb, spec, ids = _case(ctx, n, fs, n_tmpl, seed)
        ref = hs.as_records(hs.hs_matched_filter(ctx, spec, n, fs, pb, ids, thr), hs.CANDIDATE)
        cand = torch.full((cap, 4), -1, dtype=torch.int32, device=ctx.device)
        cnt = hs.hs_matched_filter_noalloc(ctx, spec, n, fs, pb, ids, thr, cand)
        got = hs.as_records(cand[:cnt], hs.CANDIDATE)
        assert cnt > 1000 and len(ref) > 1000
        ndiff, err = _compare(got, ref, thr, DELTA["f32"])
        _say(f"  {cnt} candidates ({len(ref)} through hs_matched_filter), {ndiff} in the threshold band differ, "
             f"max rho difference {err:.2e}")
        assert np.all((got["tpos"] >= 0) & (got["tpos"] < n_tmpl) & (got["m"] >= 0) & (got["m"] < n))
        # the oracle's rule on sampled templates (first, middle, last)
        st = oracle.strain_fft(s, fs)
        for t in (0, n_tmpl // 2, n_tmpl - 1):
            a, b = oracle.band_edges(n, fs, workload.F_LOW, bank.kstart[t], bank.k1[t])
            z = oracle.snr_series(st, bank.spectrum(t), psd, n, fs, a, b)
            sel = got["tpos"] == t
            assert check_candidates(got["m"][sel], got["rho2"][sel], z, thr, DELTA["f32"]) < DELTA["f32"]


def test_noalloc_reports_overflow_and_rejects_sizes_beyond_its_scratch(ctx):
    import torch
    from paper_2309_00019_amd import hs
    n, fs, thr = 2 ** 17, 512.0, 4.0
    _say("noalloc overflow and size limit")
    bank, s, psd, pb, spec, ids = _case(ctx, n, fs, 6, 33)
    total = hs.hs_matched_filter(ctx, spec, n, fs, pb, ids, thr).shape[0]
    assert total > 100
    small = torch.empty((total // 3, 4), dtype=torch.int32, device=ctx.device)
    with pytest.raises(hs.HsError) as e:
        hs.hs_matched_filter_noalloc(ctx, spec, n, fs, pb, ids, thr, small)
    assert e.value.status == hs.HS_EOVERFLOW and e.value.required == total
    # a capacity whose candidate lists alone exceed the fixed scratch is refused before any work
    huge = torch.empty((3_000_000, 4), dtype=torch.int32, device=ctx.device)
    with pytest.raises(hs.HsError) as e:
        hs.hs_matched_filter_noalloc(ctx, spec, n, fs, pb, ids, thr, huge)
    assert e.value.status == hs.HS_EINVAL and "scratch" in str(e.value)
    # and the next call with a fitting capacity is unaffected
    cand = torch.empty((total + 10, 4), dtype=torch.int32, device=ctx.device)
    assert hs.hs_matched_filter_noalloc(ctx, spec, n, fs, pb, ids, thr, cand) == total
