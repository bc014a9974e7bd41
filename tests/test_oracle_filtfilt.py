"""Pins of the oracle's zero-phase (forward-backward) filtering of a window.

* library special case: scipy's sosfilt forward from rest, then over the
  reversed result from rest (no padding);
* zero phase and squared magnitude: a steady sinusoid comes out in phase with
  amplitude |H(f)|^2, |H| from scipy's sosfreqz;
* an impulse far from both edges gives an output symmetric about it.
"""

import numpy as np
import pytest

import oracle

signal = pytest.importorskip("scipy.signal")


@pytest.mark.parametrize("order,btype,f1,f2,fs", [
    (4, "bandpass", 1.0, 50.0, 500.0),
    (8, "bandpass", 1.0, 100.0, 1500.0),
    (5, "lowpass", 30.0, 0.0, 200.0),
])
def test_matches_scipy_forward_backward(order, btype, f1, f2, fs):
    sos = oracle.butter_sos(order, btype, f1, f2, fs)
    x = np.random.default_rng(order).standard_normal((3000, 4))
    y = oracle.sos_filtfilt(sos, x)
    ref = signal.sosfilt(sos, signal.sosfilt(sos, x, axis=0)[::-1], axis=0)[::-1]
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("f0", [5.0, 20.0, 45.0])
def test_zero_phase_and_squared_gain(f0):
    fs = 500.0
    sos = oracle.butter_sos(4, "bandpass", 2.0, 60.0, fs)
    n = 40_000
    t = np.arange(n) / fs
    x = np.sin(2 * np.pi * f0 * t)[:, None]
    y = oracle.sos_filtfilt(sos, x)[:, 0]
    mid = slice(n // 3, 2 * n // 3)
    A = np.stack([np.sin(2 * np.pi * f0 * t[mid]), np.cos(2 * np.pi * f0 * t[mid])], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, y[mid], rcond=None)
    _, h = signal.sosfreqz(sos, worN=[f0], fs=fs)
    assert abs(b) <= 1e-7 * abs(a)  # no phase shift
    assert a == pytest.approx(abs(h[0]) ** 2, rel=1e-7)


def test_impulse_response_is_symmetric():
    sos = oracle.butter_sos(6, "bandpass", 5.0, 80.0, 1000.0)
    n, n0 = 20_001, 10_000
    x = np.zeros((n, 1))
    x[n0, 0] = 1.0
    y = oracle.sos_filtfilt(sos, x)[:, 0]
    k = np.arange(1, 3000)
    np.testing.assert_allclose(y[n0 + k], y[n0 - k], rtol=0, atol=1e-12 * np.abs(y).max())
    assert np.abs(y[n0]) == np.abs(y).max()
