"""Pins for the oracle's Butterworth bilinear design (paper: bandpass / lowpass /
highpass wrappers of the stateful IIR operator, Section 3.4; the design method
itself is the textbook bilinear transform with pre-warping, the paper being
silent on it).

The oracle is checked against facts that do not come from it:
  * the closed-form magnitude of a bilinear Butterworth filter,
        |H|^2 = 1 / (1 + R(W)^(2N)),  W = 2 fs tan(w / 2),
    with R = W/Wc (LP), Wc/W (HP), (W^2 - W0^2)/(B W) (BP), B W/(W^2 - W0^2) (BS);
  * -3.01 dB exactly at every band edge;
  * the first-order lowpass in closed form;
  * scipy.signal.butter as an independent library special case.
"""

import math

import numpy as np
import pytest


def sos_response(sos, f, fs):
    """H(e^{jw}) of an SOS cascade evaluated directly from its rows."""
    q = np.exp(-2j * np.pi * np.asarray(f, dtype=np.float64) / fs)
    h = np.ones_like(q)
    for b0, b1, b2, a0, a1, a2 in sos:
        h *= (b0 + b1 * q + b2 * q * q) / (a0 + a1 * q + a2 * q * q)
    return h


def butter_mag2(f, fs, N, btype, f1, f2=0.0):
    W = 2 * fs * np.tan(np.pi * np.asarray(f, dtype=np.float64) / fs)
    W1 = 2 * fs * math.tan(math.pi * f1 / fs)
    if btype == "lowpass":
        R = W / W1
    elif btype == "highpass":
        R = W1 / W
    else:
        W2 = 2 * fs * math.tan(math.pi * f2 / fs)
        W0sq, B = W1 * W2, W2 - W1
        R = (W * W - W0sq) / (B * W)
        if btype == "bandstop":
            R = 1.0 / R
    return 1.0 / (1.0 + R ** (2 * N))


CASES = [
    # order, btype, f1, f2, fs
    (4, "bandpass", 1.0, 50.0, 500.0),        # small workload
    (8, "bandpass", 1.0, 100.0, 1500.0),      # 6000-channel workload
    (16, "highpass", 0.5, 0.0, 10_000.0),     # near-unit-circle stress
    (5, "lowpass", 40.0, 0.0, 1000.0),
    (1, "lowpass", 10.0, 0.0, 100.0),
    (3, "highpass", 10.0, 0.0, 100.0),
    (2, "bandpass", 3.0, 40.0, 100.0),        # odd prototype, wide band (two real poles)
    (10, "bandpass", 20.0, 3000.0, 10_000.0),
    (6, "bandpass", 2.0, 40.0, 100.0),
    (6, "bandstop", 10.0, 20.0, 100.0),
    (4, "bandstop", 50.0, 120.0, 1000.0),
]


@pytest.mark.parametrize("order,btype,f1,f2,fs", CASES)
def test_closed_form_magnitude(orc, order, btype, f1, f2, fs):
    sos = orc.butter_sos(order, btype, f1, f2, fs)
    assert sos.shape == ((order + 1) // 2, 6)
    N = order // 2 if btype in ("bandpass", "bandstop") else order
    f = np.linspace(0.0, fs / 2, 3001)[1:-1]
    got = np.abs(sos_response(sos, f, fs)) ** 2
    want = butter_mag2(f, fs, N, btype, f1, f2)
    # 1e-9 absolute on |H|^2 (near-unit-circle designs lose a few digits in the poles)
    assert np.max(np.abs(got - want)) < 1e-9


@pytest.mark.parametrize("order,btype,f1,f2,fs", CASES)
def test_minus_3db_at_edges_and_unit_passband(orc, order, btype, f1, f2, fs):
    sos = orc.butter_sos(order, btype, f1, f2, fs)
    edges = [f1] if btype in ("lowpass", "highpass") else [f1, f2]
    h = np.abs(sos_response(sos, edges, fs))
    assert np.allclose(h, 1 / math.sqrt(2), rtol=0, atol=1e-9)
    if btype == "lowpass":
        ref = [0.0]
    elif btype == "highpass":
        ref = [fs / 2]
    elif btype == "bandpass":
        W1, W2 = (2 * fs * math.tan(math.pi * f / fs) for f in (f1, f2))
        ref = [fs / math.pi * math.atan(math.sqrt(W1 * W2) / (2 * fs))]
    else:
        ref = [0.0, fs / 2]
    assert np.allclose(np.abs(sos_response(sos, ref, fs)), 1.0, atol=1e-9)


@pytest.mark.parametrize("order,btype,f1,f2,fs", CASES)
def test_stable_and_sections(orc, order, btype, f1, f2, fs):
    import scipy.signal as ss

    sos = orc.butter_sos(order, btype, f1, f2, fs)
    assert np.all(sos[:, 3] == 1.0)
    z, p, k = ss.sos2zpk(sos)
    assert np.all(np.abs(p) < 1.0)
    # sections are ordered from best damped to least damped (closest pole last)
    radii = [np.max(np.abs(np.roots([1.0, r[4], r[5]]))) if r[5] != 0 else abs(r[4]) for r in sos]
    assert all(radii[i] <= radii[i + 1] + 1e-12 for i in range(len(radii) - 1))


def test_first_order_lowpass_closed_form(orc):
    fs, fc = 1000.0, 37.0
    K = math.tan(math.pi * fc / fs)
    sos = orc.butter_sos(1, "lowpass", fc, 0.0, fs)
    assert sos.shape == (1, 6)
    np.testing.assert_allclose(sos[0, :2], [K / (1 + K), K / (1 + K)], rtol=1e-14)
    assert sos[0, 2] == 0.0 and sos[0, 5] == 0.0
    np.testing.assert_allclose(sos[0, 4], (K - 1) / (K + 1), rtol=1e-14)


@pytest.mark.parametrize("order,btype,f1,f2,fs", CASES)
def test_matches_scipy_transfer_function(orc, order, btype, f1, f2, fs):
    import scipy.signal as ss

    sos = orc.butter_sos(order, btype, f1, f2, fs)
    N = order // 2 if btype in ("bandpass", "bandstop") else order
    wn = [f1, f2] if btype in ("bandpass", "bandstop") else f1
    ref = ss.butter(N, wn, btype, fs=fs, output="sos")
    f = np.linspace(0.0, fs / 2, 2049)
    h1, h2 = sos_response(sos, f, fs), sos_response(ref, f, fs)
    assert np.max(np.abs(h1 - h2)) < 1e-9
    z1, p1, k1 = ss.sos2zpk(sos)
    z2, p2, k2 = ss.sos2zpk(ref)
    np.testing.assert_allclose(np.sort_complex(p1), np.sort_complex(p2), atol=1e-9)
    assert abs(k1 - k2) <= 1e-9 * abs(k2)


@pytest.mark.parametrize("args", [
    (0, "lowpass", 10.0, 0.0, 100.0),
    (3, "bandpass", 1.0, 10.0, 100.0),      # odd band order
    (4, "bandpass", 10.0, 1.0, 100.0),      # f1 >= f2
    (4, "lowpass", 60.0, 0.0, 100.0),       # above Nyquist
    (4, "lowpass", 0.0, 0.0, 100.0),
    (4, "highpass", 10.0, 0.0, -1.0),
])
def test_invalid_arguments(orc, args):
    with pytest.raises(orc.OracleError):
        orc.butter_sos(*args)


def test_near_unit_circle_config_pole_distance(orc):
    import scipy.signal as ss

    sos = orc.butter_sos(16, "highpass", 0.5, 0.0, 10_000.0)
    _, p, _ = ss.sos2zpk(sos)
    d = 1 - np.abs(p).max()
    assert 1e-5 < d < 1e-3
