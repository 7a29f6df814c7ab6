"""Thin ctypes binding of libhs (``include/hs.h``): argument marshalling only.

Every function has the name of the C entry point it calls.  Device buffers are
PyTorch tensors (memory and streams only); all computation happens in the HIP
kernels of libhs.  If the shared library is missing the import fails loudly --
there is no fallback.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhs.so")

HS_OK, HS_EINVAL, HS_ENOMEM, HS_EOVERFLOW, HS_EDEVICE = 0, -1, -2, -3, -4
HS_F32, HS_BF16, HS_F16 = 0, 1, 2
DTYPES = {"f32": HS_F32, "bf16": HS_BF16, "f16": HS_F16}
ELEM_BYTES = {HS_F32: 8, HS_BF16: 4, HS_F16: 4}

CANDIDATE = np.dtype([("tpos", "<i4"), ("m", "<i4"), ("rho2", "<f4"), ("phase", "<f4")])
TRIGGER = np.dtype([("seg", "<i4"), ("tmpl", "<i4"), ("tick", "<i8"), ("snr", "<f4"), ("phase", "<f4")])
COINC = np.dtype([("slide", "<i4"), ("tmpl", "<i4"), ("tick_h", "<i8"), ("tick_l", "<i8"),
                  ("snr_h", "<f4"), ("snr_l", "<f4"), ("stat", "<f4"), ("snr_c", "<f4")])
EXPORTS = ["hs_create", "hs_destroy", "hs_last_error", "hs_abi_version", "hs_welch_psd", "hs_whiten",
           "hs_prepare_bank", "hs_matched_filter", "hs_snr_series", "hs_cluster_triggers",
           "hs_chisq", "hs_chisq_at_peaks", "hs_timeslide_coinc", "hs_followup", "hs_proposer_features", "hs_mlp_forward",
           "hs_mlp_train_step", "hs_mlp_propose", "hs_followup_cells", "hs_far_fit", "hs_far",
           "hs_far_threshold", "hs_set_mf_batch_bytes", "hs_get_mf_batch_bytes", "hs_set_mf_tile", "hs_get_mf_tile",
           "hs_set_mf_pa_cols", "hs_get_mf_pa_cols", "hs_matched_filter_noalloc"]
MLP_FEATURES, MLP_CELLS, MLP_PARAMS = 16, 64, 43456
MLP_MODEL = 32 + MLP_PARAMS


class HsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Bank(ctypes.Structure):
    _fields_ = [("n_tmpl", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_int64),
                ("fs", ctypes.c_double), ("offset", ctypes.c_void_p), ("k0", ctypes.c_void_p),
                ("k_lo", ctypes.c_void_p), ("k_hi", ctypes.c_void_p), ("spectra", ctypes.c_void_p),
                ("rho2_scale", ctypes.c_void_p), ("chisq_bins", ctypes.c_int32),
                ("chisq_edges", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libhs.so not found at {path}: build it with `python paper_2309_00019_amd/build.py` (or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P, I32, I64, D, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    sig = {
        "hs_create": [ctypes.POINTER(P), ctypes.c_int, P],
        "hs_destroy": [P],
        "hs_last_error": [],
        "hs_abi_version": [],
        "hs_welch_psd": [P, P, I64, D, I64, P],
        "hs_whiten": [P, P, I64, D, D, P, P],
        "hs_prepare_bank": [P, I64, D, D, P, I32, P, P, P, P, P, I32, P, P, P, P, P, I32, P],
        "hs_matched_filter": [P, P, I64, D, ctypes.POINTER(_Bank), P, I32, F, P, I64, ctypes.POINTER(I64)],
        "hs_matched_filter_noalloc": [P, P, I64, D, ctypes.POINTER(_Bank), P, I32, F, P, I64, ctypes.POINTER(I64)],
        "hs_snr_series": [P, P, I64, D, ctypes.POINTER(_Bank), P, I32, P],
        "hs_cluster_triggers": [P, P, I64, I64, P, I32, I64, I64, I64, I32, I64, I64, P, I64, ctypes.POINTER(I64)],
        "hs_chisq": [P, P, I64, D, ctypes.POINTER(_Bank), P, I64, I64, I64, F, P, P, P],
        "hs_chisq_at_peaks": [P, P, I64, D, ctypes.POINTER(_Bank), P, I64, I64, I64, F, P, P, P],
        "hs_timeslide_coinc": [P, P, I64, P, I64, I32, I64, I64, I64, I64, I64, F, P, I32, P, P, I64,
                               ctypes.POINTER(I64)],
        "hs_followup": [P, P, I64, F, P, I32, P, I32, D, I64, I32, P, P],
        "hs_proposer_features": [P, P, I64, P, I64, P, P, P, I64, P, P, I32, I64, P, P, I32, I64, I64, I64, P],
        "hs_mlp_forward": [P, P, P, I64, P],
        "hs_mlp_train_step": [P, P, P, P, I64, F, P, P, I64, P, ctypes.POINTER(F)],
        "hs_mlp_propose": [P, P, P, I64, F, F, F, P],
        "hs_followup_cells": [P, P, I64, F, P, I32, P, P, I32, D, P, P, I64, I32, P, P],
        "hs_far_fit": [P, P, I32, F, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I32)],
        "hs_far": [P, P, I64, D, D, D, F, P],
        "hs_far_threshold": [D, D, D, D],
        "hs_set_mf_batch_bytes": [P, I64],
        "hs_get_mf_batch_bytes": [P],
        "hs_set_mf_tile": [P, I32],
        "hs_get_mf_tile": [P],
        "hs_set_mf_pa_cols": [P, I32],
        "hs_get_mf_pa_cols": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = {"hs_last_error": ctypes.c_char_p, "hs_far_threshold": ctypes.c_double,
                      "hs_get_mf_batch_bytes": ctypes.c_int64, "hs_get_mf_tile": ctypes.c_int32,
                      "hs_get_mf_pa_cols": ctypes.c_int32}.get(name, ctypes.c_int)
    _lib = lib
    return lib


def _check(status, what=""):
    if status != HS_OK:
        msg = _lib.hs_last_error().decode(errors="replace")
        raise HsError(status, f"{what}: {msg}" if what else msg)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return ctypes.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(int(t))


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """hs_ctx bound to one device and the current (or given) torch stream."""

    def __init__(self, device: int = 0, stream=None):
        load_library()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(_lib.hs_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream)), "hs_create")
        self.handle = h
        # matched-filter schedule per transform length n: (batch bytes, pass-B threads, pass-A
        # columns), applied before each filter call at that n (the autotuner fills it)
        self.mf_schedules = {}
        # largest candidate fraction (x 1.25) seen per threshold: sizes later candidate buffers
        self.cand_fraction = {}

    def close(self):
        if getattr(self, "handle", None):
            _lib.hs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PreparedBank:
    """Device arrays of a prepared bank (see hs_bank in hs.h)."""

    def __init__(self, n, fs, dtype, offset, k0, k_lo, k_hi, spectra, rho2_scale, sigma, mchirp=None,
                 chisq_bins=0, chisq_edges=None):
        self.n, self.fs, self.dtype = int(n), float(fs), int(dtype)
        self.offset, self.k0, self.k_lo, self.k_hi = offset, k0, k_lo, k_hi
        self.spectra, self.rho2_scale, self.sigma, self.mchirp = spectra, rho2_scale, sigma, mchirp
        self.chisq_bins, self.chisq_edges = int(chisq_bins), chisq_edges

    @property
    def n_tmpl(self):
        return int(self.offset.numel())

    def struct(self) -> _Bank:
        return _Bank(self.n_tmpl, self.dtype, self.n, self.fs, _ptr(self.offset), _ptr(self.k0),
                     _ptr(self.k_lo), _ptr(self.k_hi), _ptr(self.spectra), _ptr(self.rho2_scale),
                     self.chisq_bins, _ptr(self.chisq_edges))

    @staticmethod
    def allocate(n, fs, dtype, offset, k0, total_elems, device, chisq_bins=0):
        """Empty bank with the given layout (offset/k0 host arrays)."""
        T = len(offset)
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        spectra = torch.empty(int(total_elems) * ELEM_BYTES[dt], dtype=torch.uint8, device=device)
        edges = torch.empty((T, chisq_bins + 1), dtype=torch.int32, device=device) if chisq_bins else None
        return PreparedBank(n, fs, dt,
                            torch.as_tensor(np.asarray(offset, np.int64), device=device),
                            torch.as_tensor(np.asarray(k0, np.int32), device=device),
                            torch.empty(T, dtype=torch.int32, device=device),
                            torch.empty(T, dtype=torch.int32, device=device),
                            spectra,
                            torch.empty(T, dtype=torch.float32, device=device),
                            torch.empty(T, dtype=torch.float64, device=device),
                            chisq_bins=chisq_bins, chisq_edges=edges)


def mf_batch_templates(n: int, n_ids: int, ctx: "Context" = None) -> int:
    """Templates per pass-A/pass-B launch in hs_matched_filter (same rule as the library)."""
    if ctx is not None:
        sch = ctx.mf_schedules.get(int(n))
        budget = sch[0] if sch is not None else hs_get_mf_batch_bytes(ctx)
    else:
        try:
            mb = int(os.environ.get("HS_MF_BATCH_MB", "0") or 0)
        except ValueError:
            mb = 0
        budget = (mb << 20) if 1 <= mb <= (1 << 16) else (128 << 20)
    return max(1, min(65535, n_ids, budget // (n * 8)))


def apply_mf_schedule(ctx: "Context", n: int):
    """Sets the context's matched-filter schedule for length n, when one was recorded for it."""
    sch = ctx.mf_schedules.get(int(n))
    if sch is None:
        return
    b, t, c = sch
    if _lib.hs_get_mf_batch_bytes(ctx.handle) != b:
        _check(_lib.hs_set_mf_batch_bytes(ctx.handle, int(b)), "hs_set_mf_batch_bytes")
    if _lib.hs_get_mf_tile(ctx.handle) != t:
        _check(_lib.hs_set_mf_tile(ctx.handle, int(t)), "hs_set_mf_tile")
    if _lib.hs_get_mf_pa_cols(ctx.handle) != c:
        _check(_lib.hs_set_mf_pa_cols(ctx.handle, int(c)), "hs_set_mf_pa_cols")


def hs_set_mf_batch_bytes(ctx: "Context", nbytes: int):
    _check(_lib.hs_set_mf_batch_bytes(ctx.handle, int(nbytes)), "hs_set_mf_batch_bytes")


def hs_get_mf_batch_bytes(ctx: "Context") -> int:
    return int(_lib.hs_get_mf_batch_bytes(ctx.handle))


def hs_set_mf_tile(ctx: "Context", pass_b_threads: int):
    _check(_lib.hs_set_mf_tile(ctx.handle, int(pass_b_threads)), "hs_set_mf_tile")


def hs_get_mf_tile(ctx: "Context") -> int:
    return int(_lib.hs_get_mf_tile(ctx.handle))


def hs_set_mf_pa_cols(ctx: "Context", cols: int):
    _check(_lib.hs_set_mf_pa_cols(ctx.handle, int(cols)), "hs_set_mf_pa_cols")


def hs_get_mf_pa_cols(ctx: "Context") -> int:
    return int(_lib.hs_get_mf_pa_cols(ctx.handle))


def hs_abi_version() -> int:
    return load_library().hs_abi_version()


def hs_welch_psd(ctx: Context, strain, fs: float, seg_len: int, out=None):
    _dev(strain, torch.float32, "strain")
    n = strain.numel()
    out = torch.empty(n // 2 + 1, dtype=torch.float64, device=strain.device) if out is None else out
    _dev(out, torch.float64, "psd_out")
    _check(_lib.hs_welch_psd(ctx.handle, _ptr(strain), n, fs, seg_len, _ptr(out)), "hs_welch_psd")
    return out


def hs_whiten(ctx: Context, strain, fs: float, f_low: float, psd, out=None):
    _dev(strain, torch.float32, "strain")
    _dev(psd, torch.float64, "psd")
    n = strain.numel()
    if psd.numel() < n // 2 + 1:
        raise ValueError("psd must have n/2+1 bins")
    out = torch.empty(n // 2, dtype=torch.complex64, device=strain.device) if out is None else out
    _dev(out, torch.complex64, "spec_out")
    _check(_lib.hs_whiten(ctx.handle, _ptr(strain), n, fs, f_low, _ptr(psd), _ptr(out)), "hs_whiten")
    return out


def hs_prepare_bank(ctx: Context, n: int, fs: float, f_low: float, psd, raw, offset, k0, kstart, k1,
                    dtype="f32", bank: PreparedBank = None, t0: int = 0, elem0: int = 0, chisq_bins: int = 8):
    """Prepare templates into ``bank`` (allocated with the same layout as ``raw``).

    ``raw`` complex64 device tensor; offset/k0/kstart/k1 device tensors relative to ``raw``.
    With ``bank`` given, the templates land at template index ``t0`` and spectra element
    ``elem0`` of that bank (chunked preparation of a large bank).
    """
    _dev(psd, torch.float64, "psd")
    _dev(raw, torch.complex64, "raw")
    T = offset.numel()
    if bank is None:
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        bank = PreparedBank(n, fs, dt, offset.clone(), k0.clone(),
                            torch.empty(T, dtype=torch.int32, device=raw.device),
                            torch.empty(T, dtype=torch.int32, device=raw.device),
                            torch.empty(raw.numel() * ELEM_BYTES[dt], dtype=torch.uint8, device=raw.device),
                            torch.empty(T, dtype=torch.float32, device=raw.device),
                            torch.empty(T, dtype=torch.float64, device=raw.device),
                            chisq_bins=chisq_bins,
                            chisq_edges=torch.empty((T, chisq_bins + 1), dtype=torch.int32, device=raw.device)
                            if chisq_bins else None)
    eb = ELEM_BYTES[bank.dtype]
    pb = bank.chisq_bins
    edges_ptr = ctypes.c_void_p(bank.chisq_edges.data_ptr() + 4 * (pb + 1) * t0) if pb else None
    sp = bank.spectra.data_ptr() + elem0 * eb
    _check(_lib.hs_prepare_bank(ctx.handle, n, fs, f_low, _ptr(psd), T, _ptr(raw), _ptr(offset), _ptr(k0),
                                _ptr(kstart), _ptr(k1), bank.dtype, ctypes.c_void_p(sp),
                                ctypes.c_void_p(bank.k_lo.data_ptr() + 4 * t0),
                                ctypes.c_void_p(bank.k_hi.data_ptr() + 4 * t0),
                                ctypes.c_void_p(bank.rho2_scale.data_ptr() + 4 * t0),
                                ctypes.c_void_p(bank.sigma.data_ptr() + 8 * t0), pb, edges_ptr), "hs_prepare_bank")
    return bank


def hs_matched_filter(ctx: Context, spec, n: int, fs: float, bank: PreparedBank, tmpl_ids, thr: float,
                      cap: int = None, cand=None):
    """Returns an int32 [n_cand, 4] device tensor of hs_candidate records (view with as_records)."""
    _dev(spec, torch.complex64, "spec")
    _dev(tmpl_ids, torch.int32, "tmpl_ids")
    apply_mf_schedule(ctx, n)
    n_ids = tmpl_ids.numel()
    if cap is None:
        # Rayleigh tail e^{-thr^2/2} per sample, with head-room for loud glitches; a glitch that rings
        # every template can exceed it, which costs a second pass, so the context remembers the
        # largest fraction of candidates per (template, sample) seen at this threshold
        frac = min(1.0, 8.0 * np.exp(-thr * thr / 2.0))
        frac = max(frac, ctx.cand_fraction.get(float(thr), 0.0))
        cap = int(n_ids * n * frac) + 65536
    bs = bank.struct()
    for _ in range(2):
        if cand is None or cand.shape[0] < cap:
            cand = torch.empty((cap, 4), dtype=torch.int32, device=spec.device)
        cnt = ctypes.c_int64(0)
        st = _lib.hs_matched_filter(ctx.handle, _ptr(spec), n, fs, ctypes.byref(bs), _ptr(tmpl_ids), n_ids,
                                    float(thr), _ptr(cand), cand.shape[0], ctypes.byref(cnt))
        if n_ids:
            seen = 1.25 * cnt.value / (n_ids * n)
            if seen > ctx.cand_fraction.get(float(thr), 0.0):
                ctx.cand_fraction[float(thr)] = min(1.0, seen)
        if st == HS_EOVERFLOW:
            cap = int(cnt.value)
            cand = None
            continue
        _check(st, "hs_matched_filter")
        return cand[: cnt.value]
    raise HsError(HS_EOVERFLOW, "hs_matched_filter: overflow after resize")


MF_NOALLOC_SCRATCH_BYTES = 64 << 20


def hs_matched_filter_noalloc(ctx: Context, spec, n: int, fs: float, bank: PreparedBank, tmpl_ids, thr: float, cand):
    """hs_matched_filter into a caller-allocated candidate buffer (device int32 [cap, 4]) through the
    allocation-free entry point; returns the candidate count.  A count above cap raises HsError
    (HS_EOVERFLOW) with the required count in ``HsError.required``."""
    _dev(spec, torch.complex64, "spec")
    _dev(tmpl_ids, torch.int32, "tmpl_ids")
    _dev(cand, torch.int32, "cand")
    if cand.dim() != 2 or cand.shape[1] != 4:
        raise ValueError("cand must be an int32 [cap, 4] tensor of hs_candidate records")
    bs = bank.struct()
    cnt = ctypes.c_int64(0)
    st = _lib.hs_matched_filter_noalloc(ctx.handle, _ptr(spec), n, fs, ctypes.byref(bs), _ptr(tmpl_ids),
                                        tmpl_ids.numel(), float(thr), _ptr(cand), cand.shape[0], ctypes.byref(cnt))
    if st == HS_EOVERFLOW:
        err = HsError(st, "hs_matched_filter_noalloc: " + _lib.hs_last_error().decode(errors="replace"))
        err.required = int(cnt.value)
        raise err
    _check(st, "hs_matched_filter_noalloc")
    return int(cnt.value)


def hs_snr_series(ctx: Context, spec, n: int, fs: float, bank: PreparedBank, tmpl_ids, out=None):
    _dev(spec, torch.complex64, "spec")
    _dev(tmpl_ids, torch.int32, "tmpl_ids")
    n_ids = tmpl_ids.numel()
    out = torch.empty((n_ids, n), dtype=torch.complex64, device=spec.device) if out is None else out
    bs = bank.struct()
    _check(_lib.hs_snr_series(ctx.handle, _ptr(spec), n, fs, ctypes.byref(bs), _ptr(tmpl_ids), n_ids, _ptr(out)),
           "hs_snr_series")
    return out


def hs_cluster_triggers(ctx: Context, cand, n: int, tmpl_ids, window: int, seg: int = 0, seg_t0: int = 0,
                        ticks_per_sample: int = 1, cap: int = None, valid=None):
    """Returns an int32 [n_trig, 6] device tensor of hs_trigger records; valid = (m_lo, m_hi)
    restricts the peaks to that part of the segment (default: all of it)."""
    m_lo, m_hi = (0, n) if valid is None else (int(valid[0]), int(valid[1]))
    _dev(cand, torch.int32, "cand")
    _dev(tmpl_ids, torch.int32, "tmpl_ids")
    n_cand = cand.shape[0]
    if cap is None:
        cap = min(n_cand, tmpl_ids.numel() * (n // max(window, 1) + 2)) + 16
    for _ in range(2):
        out = torch.empty((max(cap, 1), 6), dtype=torch.int32, device=cand.device)
        cnt = ctypes.c_int64(0)
        st = _lib.hs_cluster_triggers(ctx.handle, _ptr(cand), n_cand, n, _ptr(tmpl_ids), tmpl_ids.numel(), window,
                                      m_lo, m_hi, seg, seg_t0, ticks_per_sample, _ptr(out), cap, ctypes.byref(cnt))
        if st == HS_EOVERFLOW:
            cap = int(cnt.value)
            continue
        _check(st, "hs_cluster_triggers")
        return out[: cnt.value]
    raise HsError(HS_EOVERFLOW, "hs_cluster_triggers: overflow after resize")


def hs_chisq(ctx: Context, spec, n: int, fs: float, bank: PreparedBank, trig, seg_t0: int = 0,
             ticks_per_sample: int = 1, rho_min: float = 0.0, out=None, bins: bool = False, at_peaks: bool = False):
    """Returns (float32 [n_trig] chi2_r, int32 [n_trig, 6] triggers with snr re-weighted by Eq. (4))
    and, with bins=True, a third item: float32 [n_trig, p] per-bin chi-square terms.
    at_peaks=True calls hs_chisq_at_peaks (triggers must carry the filter's own rho and arg z)."""
    _dev(spec, torch.complex64, "spec")
    _dev(trig, torch.int32, "trig")
    n_trig = trig.shape[0]
    chi = torch.empty(n_trig, dtype=torch.float32, device=trig.device)
    out = torch.empty_like(trig) if out is None else out
    b = torch.empty((n_trig, max(1, bank.chisq_bins)), dtype=torch.float32, device=trig.device) if bins else None
    bs = bank.struct()
    fn = _lib.hs_chisq_at_peaks if at_peaks else _lib.hs_chisq
    _check(fn(ctx.handle, _ptr(spec), n, fs, ctypes.byref(bs), _ptr(trig), n_trig, seg_t0,
              ticks_per_sample, float(rho_min), _ptr(chi), _ptr(out), _ptr(b)),
           "hs_chisq_at_peaks" if at_peaks else "hs_chisq")
    return (chi, out, b) if bins else (chi, out)


def hs_timeslide_coinc(ctx: Context, trig_h, trig_l, n_tmpl: int, n_slides: int, step: int, window: int,
                       wrap: int, cluster_w: int, edges, cap: int = None, min_snr_c: float = 0.0):
    """Returns (int32 [n, 10] device tensor of hs_coinc records, int64 numpy background counts).
    min_snr_c > 0: coincidences with network SNR below it are not formed (exact at and above it)."""
    _dev(trig_h, torch.int32, "trig_h")
    _dev(trig_l, torch.int32, "trig_l")
    edges = np.ascontiguousarray(edges, dtype=np.float32)
    bg = np.zeros(len(edges), np.int64)
    if cap is None:
        # at most one survivor per (slide, cluster window); grown on overflow beyond 4 M records
        cap = min((n_slides + 1) * (wrap // cluster_w + 2), 1 << 22)
    for _ in range(2):
        out = torch.empty((max(cap, 1), 10), dtype=torch.int32, device=trig_h.device)
        cnt = ctypes.c_int64(0)
        st = _lib.hs_timeslide_coinc(ctx.handle, _ptr(trig_h), trig_h.shape[0], _ptr(trig_l), trig_l.shape[0],
                                     n_tmpl, n_slides, step, window, wrap, cluster_w, float(min_snr_c), _ptr(edges),
                                     len(edges), _ptr(bg), _ptr(out), cap, ctypes.byref(cnt))
        if st == HS_EOVERFLOW:
            cap = int(cnt.value)
            continue
        _check(st, "hs_timeslide_coinc")
        return out[: cnt.value], bg
    raise HsError(HS_EOVERFLOW, "hs_timeslide_coinc: overflow after resize")


def hs_followup(ctx: Context, coincs, rho_min: float, coarse_mchirp, fine_mchirp, frac: float, seg_ticks: int,
                n_seg: int):
    """Returns (int32 [n_seg, n_fine] device tensor, host list of per-segment counts)."""
    _dev(coincs, torch.int32, "coincs")
    _dev(coarse_mchirp, torch.float64, "coarse_mchirp")
    _dev(fine_mchirp, torch.float64, "fine_mchirp")
    n_fine = fine_mchirp.numel()
    ids = torch.empty((n_seg, n_fine), dtype=torch.int32, device=coincs.device)
    counts = np.zeros(n_seg, np.int32)
    _check(_lib.hs_followup(ctx.handle, _ptr(coincs), coincs.shape[0], float(rho_min), _ptr(coarse_mchirp),
                            coarse_mchirp.numel(), _ptr(fine_mchirp), n_fine, float(frac), seg_ticks, n_seg,
                            _ptr(ids), _ptr(counts)), "hs_followup")
    return ids, counts.tolist()


def hs_proposer_features(ctx: Context, coincs, trig_h, chisq_h, bins_h, trig_l, chisq_l, bins_l, seg_ticks: int,
                         coarse_mchirp, coarse_q, step: int, wrap: int, ticks_per_second: int, out=None):
    """float32 [n_c, 16] features of the coincidences (see hs.h)."""
    _dev(coincs, torch.int32, "coincs")
    for t, nm in ((trig_h, "trig_h"), (trig_l, "trig_l")):
        _dev(t, torch.int32, nm)
    for t, nm in ((chisq_h, "chisq_h"), (chisq_l, "chisq_l"), (bins_h, "bins_h"), (bins_l, "bins_l")):
        _dev(t, torch.float32, nm)
    _dev(coarse_mchirp, torch.float64, "coarse_mchirp")
    _dev(coarse_q, torch.float64, "coarse_q")
    n_c = coincs.shape[0]
    out = torch.empty((n_c, MLP_FEATURES), dtype=torch.float32, device=coincs.device) if out is None else out
    p = bins_h.shape[1] if bins_h.dim() == 2 else 0
    _check(_lib.hs_proposer_features(ctx.handle, _ptr(coincs), n_c, _ptr(trig_h), trig_h.shape[0], _ptr(chisq_h),
                                     _ptr(bins_h), _ptr(trig_l), trig_l.shape[0], _ptr(chisq_l), _ptr(bins_l), p,
                                     seg_ticks, _ptr(coarse_mchirp), _ptr(coarse_q), coarse_mchirp.numel(), step,
                                     wrap, ticks_per_second, _ptr(out)), "hs_proposer_features")
    return out


def hs_mlp_forward(ctx: Context, model, x, out=None):
    _dev(model, torch.float32, "model")
    _dev(x, torch.float32, "x")
    out = torch.empty((x.shape[0], MLP_CELLS), dtype=torch.float32, device=x.device) if out is None else out
    _check(_lib.hs_mlp_forward(ctx.handle, _ptr(model), _ptr(x), x.shape[0], _ptr(out)), "hs_mlp_forward")
    return out


def hs_mlp_train_step(ctx: Context, model, adam_m, adam_v, t: int, lr: float, x, labels, grad_out=None) -> float:
    """One Adam step of the softmax cross-entropy; updates model, adam_m, adam_v in place and
    returns the batch loss before the update."""
    _dev(model, torch.float32, "model")
    _dev(adam_m, torch.float32, "adam_m")
    _dev(adam_v, torch.float32, "adam_v")
    _dev(x, torch.float32, "x")
    _dev(labels, torch.int32, "labels")
    loss = ctypes.c_float(0.0)
    _check(_lib.hs_mlp_train_step(ctx.handle, _ptr(model), _ptr(adam_m), _ptr(adam_v), int(t), float(lr), _ptr(x),
                                  _ptr(labels), x.shape[0], _ptr(grad_out), ctypes.byref(loss)), "hs_mlp_train_step")
    return float(loss.value)


def hs_mlp_propose(ctx: Context, model, x, p_cum: float, rho_split: float = float("-inf"), p_cum_low: float = None,
                   out=None):
    """uint64 cell masks [n] (returned as an int64 device tensor with the same bits); rows with
    x[:, 2] < rho_split use p_cum_low."""
    _dev(model, torch.float32, "model")
    _dev(x, torch.float32, "x")
    out = torch.empty(x.shape[0], dtype=torch.int64, device=x.device) if out is None else out
    p_low = p_cum if p_cum_low is None else p_cum_low
    _check(_lib.hs_mlp_propose(ctx.handle, _ptr(model), _ptr(x), x.shape[0], float(p_cum), float(rho_split),
                               float(p_low), _ptr(out)), "hs_mlp_propose")
    return out


def hs_followup_cells(ctx: Context, coincs, rho_min: float, coarse_mchirp, fine_mchirp, fine_q, frac: float, q_edges,
                      cell_mask, seg_ticks: int, n_seg: int):
    """As hs_followup with per-coincidence cell masks (int64 device tensor of uint64 bits)."""
    _dev(coincs, torch.int32, "coincs")
    _dev(coarse_mchirp, torch.float64, "coarse_mchirp")
    _dev(fine_mchirp, torch.float64, "fine_mchirp")
    _dev(fine_q, torch.float64, "fine_q")
    _dev(cell_mask, torch.int64, "cell_mask")
    qe = np.ascontiguousarray(q_edges, dtype=np.float64)
    if qe.shape != (3,):
        raise ValueError("q_edges must hold 3 values")
    n_fine = fine_mchirp.numel()
    ids = torch.empty((n_seg, n_fine), dtype=torch.int32, device=coincs.device)
    counts = np.zeros(n_seg, np.int32)
    _check(_lib.hs_followup_cells(ctx.handle, _ptr(coincs), coincs.shape[0], float(rho_min), _ptr(coarse_mchirp),
                                  coarse_mchirp.numel(), _ptr(fine_mchirp), _ptr(fine_q), n_fine, float(frac), _ptr(qe),
                                  _ptr(cell_mask), seg_ticks, n_seg, _ptr(ids), _ptr(counts)), "hs_followup_cells")
    return ids, counts.tolist()


def hs_far_fit(edges, counts, x_min: float):
    """(alpha, beta, n_used) of the Eq. (7) tail fit (host arrays)."""
    e = np.ascontiguousarray(edges, dtype=np.float32)
    c = np.ascontiguousarray(counts, dtype=np.int64)
    a, b, m = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    _check(_lib.hs_far_fit(_ptr(e), _ptr(c), len(e), float(x_min), ctypes.byref(a), ctypes.byref(b), ctypes.byref(m)),
           "hs_far_fit")
    return a.value, b.value, m.value


def hs_far(ctx: Context, coincs, t_b: float, alpha: float, beta: float, x_fit: float, out=None):
    """float64 [n] hybrid FAR of the zero-lag records (-1 for background records)."""
    _dev(coincs, torch.int32, "coincs")
    out = torch.empty(coincs.shape[0], dtype=torch.float64, device=coincs.device) if out is None else out
    _check(_lib.hs_far(ctx.handle, _ptr(coincs), coincs.shape[0], float(t_b), float(alpha), float(beta), float(x_fit),
                       _ptr(out)), "hs_far")
    return out


def hs_far_threshold(alpha: float, beta: float, t_b: float, ifar: float) -> float:
    return float(_lib.hs_far_threshold(float(alpha), float(beta), float(t_b), float(ifar)))


def as_records(t, dtype) -> np.ndarray:
    """Copy a device record tensor to a numpy structured array."""
    a = t.detach().cpu().contiguous().numpy()
    return a.view(np.uint8).reshape(-1).view(dtype)


def to_device_records(rec: np.ndarray, device) -> torch.Tensor:
    """Upload a numpy structured array of 4-byte-multiple records as an int32 [n, k] tensor."""
    rec = np.ascontiguousarray(rec)
    k = rec.dtype.itemsize // 4
    raw = rec.view(np.uint8).reshape(-1).view(np.int32).reshape(len(rec), k)
    return torch.as_tensor(raw.copy(), device=device)
