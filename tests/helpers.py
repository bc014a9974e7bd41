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


def assert_within_ulps(a, b, ulps: int = 2, max_fraction: float = 1e-3, floor_rel: float = 1e-10):
    """FP32 arrays [n_t, n_ch] equal up to `ulps` units in the last place, with
    differing elements rare.  This is the run-to-run spread of the FP64 carry:
    its rounding depends on which predecessor records a segment composed, so
    two runs differ by FP64 rounding of the state, i.e. by ~1e-13 of the
    channel's scale in the output.  Near a zero crossing that is many ulps of
    the sample itself, so each channel also gets an absolute allowance of
    `floor_rel` times its largest magnitude (still far below one FP32 ulp of
    the channel's typical sample)."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    assert a.shape == b.shape
    ulp = np.spacing(np.maximum(np.abs(a), np.abs(b))).astype(np.float64)
    d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    scale = np.max(np.abs(a.astype(np.float64)), axis=0, keepdims=True) if a.ndim == 2 and a.size \
        else np.max(np.abs(a.astype(np.float64)), initial=0.0)
    bound = ulps * ulp + floor_rel * scale
    assert np.all(d <= bound), float(np.max(d / bound))
    assert np.mean(d > 0) <= max_fraction
