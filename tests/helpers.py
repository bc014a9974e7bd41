"""Shared test helpers: error metrics and GPU availability."""

from __future__ import annotations

import numpy as np


def rel_rms_per_channel(got, want) -> np.ndarray:
    """Per-channel ||got - want|| / ||want|| over time (axis 0); channels whose
    reference is identically zero report the absolute RMS error instead."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    num = np.sqrt(np.sum((got - want) ** 2, axis=0))
    den = np.sqrt(np.sum(want ** 2, axis=0))
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def max_rel_rms(got, want) -> float:
    r = rel_rms_per_channel(got, want)
    return float(r.max()) if r.size else 0.0


def pole_margin(sos) -> float:
    """1 - max |pole| over the sections of an SOS array."""
    m = 0.0
    for r in np.asarray(sos, dtype=np.float64):
        a0 = r[3]
        roots = np.roots([1.0, r[4] / a0, r[5] / a0]) if r[5] != 0 else np.array([-r[4] / a0])
        m = max(m, float(np.max(np.abs(roots))))
    return 1.0 - m


def tolerance_for(sos) -> float:
    """1e-5 relative RMS per channel, 1e-4 when a pole lies within 1e-3 of the unit circle."""
    return 1e-4 if pole_margin(sos) < 1e-3 else 1e-5


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False
