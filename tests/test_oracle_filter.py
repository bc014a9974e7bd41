"""Pins for the oracle's stateful DF2T cascade (the paper's stateful IIR-SOS
operator: chunks in, equal-length outputs out, state carried so that chunked
processing has no boundary discontinuities; Section 3.4 and Section 6.2).

Facts used, none taken from the oracle itself:
  * closed-form impulse responses (one pole: p^n; all-pole biquad:
    r^n sin((n+1) theta) / sin(theta));
  * steady-state gain and phase on pure sinusoids against H(e^{jw}) evaluated
    from the coefficients;
  * brute-force convolution with the impulse response obtained from the
    partial-fraction expansion of the transfer function;
  * bitwise chunked == one-shot, for every split including single samples and
    empty chunks;
  * scipy.signal.sosfilt with carried zi;
  * an extended-precision run of the same recurrence bounding the oracle's
    own double-precision error on near-unit-circle poles.
"""

import numpy as np
import pytest


def one_pole(p):
    return np.array([[1.0, 0.0, 0.0, 1.0, -p, 0.0]])


@pytest.mark.parametrize("p", [0.5, 0.999, 0.9999, -0.7])
def test_one_pole_impulse_response(orc, p):
    n = 20_000
    x = np.zeros((n, 1))
    x[0, 0] = 1.0
    y, zf = orc.sos_filter(one_pole(p), x)
    want = p ** np.arange(n, dtype=np.float64)
    np.testing.assert_allclose(y[:, 0], want, rtol=1e-11, atol=1e-300)
    np.testing.assert_allclose(zf[0, 0, 0], p * want[-1], rtol=1e-11, atol=1e-300)


@pytest.mark.parametrize("r,theta", [(0.9, 0.3), (0.999, 0.01), (0.95, 2.5)])
def test_all_pole_biquad_impulse_response(orc, r, theta):
    sos = np.array([[1.0, 0.0, 0.0, 1.0, -2 * r * np.cos(theta), r * r]])
    n = 5000
    x = np.zeros((n, 1))
    x[0, 0] = 1.0
    y, _ = orc.sos_filter(sos, x)
    k = np.arange(n, dtype=np.float64)
    want = r ** k * np.sin((k + 1) * theta) / np.sin(theta)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(y[:, 0] - want)) < 1e-11 * scale


def test_numerator_taps_feed_forward(orc):
    # FIR-only section: y[n] = b0 x[n] + b1 x[n-1] + b2 x[n-2]
    sos = np.array([[0.3, -1.7, 2.5, 1.0, 0.0, 0.0]])
    rng = np.random.default_rng(3)
    x = rng.standard_normal((300, 4))
    y, _ = orc.sos_filter(sos, x)
    want = 0.3 * x.copy()
    want[1:] += -1.7 * x[:-1]
    want[2:] += 2.5 * x[:-2]
    np.testing.assert_allclose(y, want, rtol=1e-13, atol=1e-13)


def sos_response(sos, f, fs):
    q = np.exp(-2j * np.pi * np.asarray(f, dtype=np.float64) / fs)
    h = np.ones_like(q)
    for b0, b1, b2, a0, a1, a2 in sos:
        h = h * (b0 + b1 * q + b2 * q * q) / (a0 + a1 * q + a2 * q * q)
    return h


@pytest.mark.parametrize("order,btype,f1,f2,fs,freqs", [
    (4, "bandpass", 1.0, 50.0, 500.0, [0.7, 5.0, 20.0, 50.0, 125.0]),
    (8, "bandpass", 1.0, 100.0, 1500.0, [1.5, 10.0, 100.0, 300.0]),
    (5, "lowpass", 40.0, 0.0, 1000.0, [10.0, 40.0, 100.0]),
])
def test_steady_state_sinusoid_gain_and_phase(orc, order, btype, f1, f2, fs, freqs):
    sos = orc.butter_sos(order, btype, f1, f2, fs)
    import scipy.signal as ss

    _, p, _ = ss.sos2zpk(sos)
    settle = int(np.ceil(40.0 / (1 - np.abs(p).max())))
    for f in freqs:
        period = fs / f
        n_per = int(np.ceil(4000 / period))
        n_fit = int(round(n_per * period))
        # choose a fit window holding an integer number of periods (up to rounding)
        n = settle + n_fit
        t = np.arange(n, dtype=np.float64)
        x = np.sin(2 * np.pi * f / fs * t)[:, None]
        y, _ = orc.sos_filter(sos, x)
        tt = t[settle:]
        A = np.stack([np.sin(2 * np.pi * f / fs * tt), np.cos(2 * np.pi * f / fs * tt)], axis=1)
        coef, *_ = np.linalg.lstsq(A, y[settle:, 0], rcond=None)
        amp = np.hypot(coef[0], coef[1])
        phase = np.arctan2(coef[1], coef[0])
        h = sos_response(sos, [f], fs)[0]
        assert abs(amp - abs(h)) < 1e-8
        if abs(h) > 1e-3:
            d = np.angle(np.exp(1j * (phase - np.angle(h))))
            assert abs(d) < 1e-6


def test_brute_force_convolution_with_partial_fraction_response(orc):
    import scipy.signal as ss

    sos = orc.butter_sos(4, "bandpass", 2.0, 40.0, 250.0)  # max|p| ~ 0.95
    b, a = ss.sos2tf(sos)
    r, p, kdir = ss.residuez(b, a)
    assert np.abs(p).max() <= 0.99
    M = int(np.ceil(np.log(1e-17) / np.log(np.abs(p).max())))
    n = np.arange(M)
    h = np.real(np.sum(r[:, None] * p[:, None] ** n[None, :], axis=0))
    for i, kd in enumerate(np.atleast_1d(kdir)):
        h[i] += np.real(kd)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((200, 3))
    y, _ = orc.sos_filter(sos, x)
    want = np.zeros_like(x)
    for t in range(x.shape[0]):
        k = np.arange(min(t + 1, M))
        want[t] = np.sum(h[k, None] * x[t - k], axis=0)
    assert np.max(np.abs(y - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("splits", [
    [1000],
    [1, 1, 1, 997],
    [0, 333, 0, 333, 334],
    [999, 1],
    [17] * 58 + [14],
])
def test_chunked_equals_one_shot_bitwise(orc, splits):
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((sum(splits), 5))
    y1, z1 = orc.sos_filter(sos, x)
    zi = np.zeros_like(z1)
    outs = []
    t0 = 0
    for n in splits:
        y, zi = orc.sos_filter(sos, x[t0:t0 + n], zi)
        outs.append(y)
        t0 += n
    y2 = np.concatenate(outs, axis=0)
    assert np.array_equal(y1, y2)
    assert np.array_equal(z1, zi)


def test_matches_scipy_sosfilt_with_state(orc):
    import scipy.signal as ss

    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3000, 6))
    zi0 = rng.standard_normal((6, sos.shape[0], 2)) * 0.1
    y, zf = orc.sos_filter(sos, x, zi0)
    # scipy's zi layout: [n_sections, ..., 2] along the filtered axis
    yr, zr = ss.sosfilt(sos, x, axis=0, zi=np.transpose(zi0, (1, 2, 0)).copy())
    np.testing.assert_allclose(y, yr, rtol=0, atol=1e-12 * np.max(np.abs(yr)))
    np.testing.assert_allclose(zf, np.transpose(zr, (2, 0, 1)), rtol=0, atol=1e-12 * np.max(np.abs(zr)))


def test_oracle_error_bound_near_unit_circle(orc):
    """Extended-precision run of the same loop bounds the FP64 oracle's own error
    on the near-unit-circle highpass with a large slow drift."""
    sos = orc.butter_sos(16, "highpass", 0.5, 0.0, 10_000.0)
    rng = np.random.default_rng(1)
    n = 40_000
    t = np.arange(n) / 10_000.0
    x = rng.standard_normal((n, 2)) + 100 * np.sin(2 * np.pi * 0.1 * t[:, None] + np.array([0.3, 2.0]))
    y, _ = orc.sos_filter(sos, x)
    y_ld, _ = orc.sos_filter(sos, x, extended=True)
    rel = np.linalg.norm(y - y_ld, axis=0) / np.linalg.norm(y_ld, axis=0)
    # the extended run is a different computation (64-bit significands), so
    # the bound is not vacuous: the two runs must differ
    assert np.finfo(np.longdouble).nmant > np.finfo(np.float64).nmant
    assert np.all(rel > 1e-14), rel
    assert np.all(rel < 1e-7), rel


def test_in_place(orc):
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((500, 3))
    y, _ = orc.sos_filter(sos, x)
    z = np.zeros((3, sos.shape[0], 2))
    buf = x.copy()
    lib = orc.lib()
    lib.oracle_sos_filter(orc._ptr(np.ascontiguousarray(sos)), sos.shape[0], orc._ptr(buf), orc._ptr(buf),
                          3, 500, orc._ptr(z))
    assert np.array_equal(buf, y)
