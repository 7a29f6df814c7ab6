"""TaylorF2 template banks, band-packed on the circular frequency grid of one segment.

Placement (the paper does not give its method): templates uniform in the
Newtonian chirp time tau0 ~ Mc^(-5/3) between the chirp-mass bounds and uniform
in mass ratio q = m1/m2 in [q_min, q_max], drawn from the seeded bank stream;
component spins are zero.  Spectra come from ``taylorf2.c`` (3.5PN SPA phase,
f^-7/6 amplitude, ISCO cut), built with gcc on first use.

Storage: template t covers bins [k0[t], k1[t]] at ``data[offset[t] + k - k0[t]]``
(complex64).  k0 is ``kstart`` rounded down to a multiple of 64 so each band
starts on an aligned bin, bins in [k0, kstart) are zero, kstart = ceil(f_start/df)
and k1 = min(floor(f_isco/df), N/2 - 1).  Offsets are multiples of 64 elements.
"""
import ctypes
import os
import subprocess
import sys
from dataclasses import dataclass

import numpy as np

MSUN_SEC = 4.925490947641267e-06
ALIGN = 64

_here = os.path.dirname(os.path.abspath(__file__))
_so_path = os.path.join(_here, "_taylorf2.so")
_lib = None


def build_generator(force: bool = False) -> str:
    """Compile ``taylorf2.c`` into ``_taylorf2.so`` (gcc, OpenMP)."""
    src = os.path.join(_here, "taylorf2.c")
    if force or not os.path.exists(_so_path) or os.path.getmtime(_so_path) < os.path.getmtime(src):
        tmp = _so_path + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src, "-lm"])
        os.replace(tmp, _so_path)
    return _so_path


def _load():
    global _lib
    if _lib is None:
        build_generator()
        lib = ctypes.CDLL(_so_path)
        P = ctypes.c_void_p
        lib.synth_taylorf2.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_double, P, P, P, P, P]
        lib.synth_taylorf2.restype = None
        _lib = lib
    return _lib


def mchirp_eta(m1, m2):
    m1 = np.asarray(m1, np.float64)
    m2 = np.asarray(m2, np.float64)
    mt = m1 + m2
    eta = m1 * m2 / (mt * mt)
    return mt * eta ** 0.6, eta


def f_isco(m1, m2):
    """Schwarzschild ISCO gravitational-wave frequency (Hz)."""
    mt = (np.asarray(m1, np.float64) + np.asarray(m2, np.float64)) * MSUN_SEC
    return 1.0 / (6.0 ** 1.5 * np.pi * mt)


def tau0(mchirp, f0):
    """Newtonian chirp time from f0 (s)."""
    return 5.0 / 256.0 * (np.pi * f0) ** (-8.0 / 3.0) * (np.asarray(mchirp) * MSUN_SEC) ** (-5.0 / 3.0)


def masses_from_mchirp_q(mchirp, q):
    """Component masses (m1 >= m2) from chirp mass and q = m1/m2 >= 1."""
    mchirp = np.asarray(mchirp, np.float64)
    q = np.asarray(q, np.float64)
    eta = q / (1.0 + q) ** 2
    mt = mchirp / eta ** 0.6
    m1 = mt * q / (1.0 + q)
    m2 = mt / (1.0 + q)
    return m1, m2


@dataclass
class Bank:
    """Band-packed template spectra plus their parameters (host, numpy)."""
    n: int                 # FFT length of the segment the spectra live on
    fs: float              # sample rate (Hz)
    f_start: float         # first non-zero frequency of every template (Hz)
    m1: np.ndarray         # float64 [T]
    m2: np.ndarray         # float64 [T]
    offset: np.ndarray     # int64 [T]
    k0: np.ndarray         # int32 [T] first stored bin (aligned)
    kstart: np.ndarray     # int32 [T] first non-zero bin
    k1: np.ndarray         # int32 [T] last stored bin (inclusive)
    data: np.ndarray       # complex64 [total]

    @property
    def n_tmpl(self) -> int:
        return len(self.m1)

    @property
    def mchirp(self) -> np.ndarray:
        return mchirp_eta(self.m1, self.m2)[0]

    @property
    def q(self) -> np.ndarray:
        return self.m1 / self.m2

    def spectrum(self, t: int) -> np.ndarray:
        """Full one-sided spectrum of template t on bins 0..n/2 (complex128, zero outside its band)."""
        out = np.zeros(self.n // 2 + 1, dtype=np.complex128)
        L = int(self.k1[t]) - int(self.k0[t]) + 1
        out[self.k0[t]:self.k1[t] + 1] = self.data[self.offset[t]:self.offset[t] + L]
        return out

    def subset(self, idx) -> "Bank":
        """A new bank holding templates ``idx`` (re-packed)."""
        idx = np.asarray(idx, dtype=np.int64)
        lens = (self.k1[idx].astype(np.int64) - self.k0[idx] + 1)
        padded = (lens + ALIGN - 1) // ALIGN * ALIGN
        off = np.zeros(len(idx), np.int64)
        off[1:] = np.cumsum(padded)[:-1]
        data = np.zeros(int(padded.sum()), np.complex64)
        for j, t in enumerate(idx):
            data[off[j]:off[j] + lens[j]] = self.data[self.offset[t]:self.offset[t] + lens[j]]
        return Bank(self.n, self.fs, self.f_start, self.m1[idx].copy(), self.m2[idx].copy(), off,
                    self.k0[idx].copy(), self.kstart[idx].copy(), self.k1[idx].copy(), data)


def bank_layout(m1, m2, n: int, fs: float, f_start: float):
    """Band edges and aligned offsets for a set of templates."""
    df = fs / n
    kstart = np.full(len(m1), int(np.ceil(f_start / df - 1e-9)), dtype=np.int32)
    k1 = np.minimum(np.floor(f_isco(m1, m2) / df), n // 2 - 1).astype(np.int32)
    if np.any(k1 < kstart):
        raise ValueError("template ISCO below the start frequency")
    k0 = (kstart // ALIGN * ALIGN).astype(np.int32)
    lens = k1.astype(np.int64) - k0 + 1
    padded = (lens + ALIGN - 1) // ALIGN * ALIGN
    offset = np.zeros(len(m1), np.int64)
    offset[1:] = np.cumsum(padded)[:-1]
    return k0, kstart, k1, offset, int(padded.sum())


def taylorf2_bank(m1, m2, n: int, fs: float, f_start: float, tc=None, phic=None, out=None) -> Bank:
    """Generate TaylorF2 spectra for component masses (m1, m2) on an n-point grid at fs."""
    m1 = np.ascontiguousarray(m1, np.float64)
    m2 = np.ascontiguousarray(m2, np.float64)
    T = len(m1)
    tc = np.zeros(T) if tc is None else np.ascontiguousarray(np.broadcast_to(tc, (T,)), np.float64)
    phic = np.zeros(T) if phic is None else np.ascontiguousarray(np.broadcast_to(phic, (T,)), np.float64)
    k0, kstart, k1, offset, total = bank_layout(m1, m2, n, fs, f_start)
    if out is None:
        data = np.zeros(total, np.complex64)
    else:
        data = out[:total]
    lib = _load()
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    lib.synth_taylorf2(T, ptr(m1), ptr(m2), ptr(tc), ptr(phic), fs / n,
                       ptr(k0), ptr(kstart), ptr(k1), ptr(offset), ptr(data))
    return Bank(n, fs, f_start, m1, m2, offset, k0, kstart, k1, data)


def bank_by_tau0(n_tmpl: int, mc_min: float, mc_max: float, q_min: float, q_max: float,
                 gen: np.random.Generator, f_ref: float = 20.0, sort: bool = True):
    """Random placement uniform in tau0(f_ref) and q; returns (m1, m2) sorted by chirp mass."""
    t_hi = tau0(mc_min, f_ref)
    t_lo = tau0(mc_max, f_ref)
    t = gen.uniform(t_lo, t_hi, n_tmpl)
    q = gen.uniform(q_min, q_max, n_tmpl)
    mc = (t / (5.0 / 256.0 * (np.pi * f_ref) ** (-8.0 / 3.0))) ** (-3.0 / 5.0) / MSUN_SEC
    m1, m2 = masses_from_mchirp_q(mc, q)
    if sort:
        o = np.argsort(mc, kind="stable")
        m1, m2 = m1[o], m2[o]
    return m1, m2


def equal_mass_bank(masses):
    m = np.asarray(masses, np.float64)
    return m.copy(), m.copy()
