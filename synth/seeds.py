"""Seed streams: one independent PCG64 generator per (config, detector, segment, stream)."""
import numpy as np

NOISE, GLITCH, INJECT, BANK, TRIG = 0, 1, 2, 3, 4


def rng(cfg: int, det: int, seg: int, stream: int) -> np.random.Generator:
    """Generator for one (config, detector, segment, stream) tuple."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg, det, seg, stream])))
