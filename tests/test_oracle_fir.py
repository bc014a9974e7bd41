"""Pins of the oracle's realtime FIR with carried history (Table 1's FIR row).

* impulse response equals the taps; a step gives the running sums of the taps;
* library special case: scipy's lfilter(h, 1, x) on the whole record;
* chunked == one-shot bit for bit over splits shorter and longer than the
  history, including empty and one-sample chunks;
* the carried history is the last M - 1 samples.
"""

import numpy as np
import pytest

import oracle

signal = pytest.importorskip("scipy.signal")


@pytest.mark.parametrize("M", [1, 2, 17, 64])
def test_impulse_and_step(M):
    h = np.random.default_rng(M).standard_normal(M)
    x = np.zeros(200)
    x[0] = 1.0
    y = oracle.Fir(h, 1).process(x)[:, 0]
    np.testing.assert_array_equal(y[:M], h)
    assert np.all(y[M:] == 0.0)
    y = oracle.Fir(h, 1).process(np.ones(200))[:, 0]
    np.testing.assert_allclose(y[:M], np.cumsum(h), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("M", [5, 64])
def test_matches_scipy_lfilter(M):
    rng = np.random.default_rng(3)
    h = rng.standard_normal(M)
    x = rng.standard_normal((1000, 4))
    np.testing.assert_allclose(oracle.Fir(h, 4).process(x), signal.lfilter(h, [1.0], x, axis=0), rtol=1e-12,
                               atol=1e-12)


@pytest.mark.parametrize("splits", [[1000], [1, 2, 3, 994], [0, 10, 0, 990], [63, 1, 936], [500, 500]])
def test_chunked_equals_one_shot_and_history(splits):
    rng = np.random.default_rng(4)
    M = 64
    h = rng.standard_normal(M)
    x = rng.standard_normal((sum(splits), 3))
    one = oracle.Fir(h, 3).process(x)
    f = oracle.Fir(h, 3)
    parts, t = [], 0
    for n in splits:
        parts.append(f.process(x[t:t + n]))
        t += n
    np.testing.assert_array_equal(np.concatenate(parts), one)
    np.testing.assert_array_equal(f.hist, x[-(M - 1):])


@pytest.mark.parametrize("M,splits", [(1, [3000]), (64, [1, 1000, 1999]), (256, [255, 0, 2745]), (1024, [1023, 1977])])
def test_matches_overlap_add_convolution(M, splits):
    """FFT filtering (Table 1's overlap-add row) computes the same linear
    convolution: scipy's oaconvolve of the whole record, cut at the record's
    length, equals the oracle fed chunk by chunk (the history carried), within
    FP64 transform rounding."""
    rng = np.random.default_rng(M)
    h = rng.standard_normal(M)
    x = rng.standard_normal((sum(splits), 3))
    ref = signal.oaconvolve(x, h[:, None], axes=0)[:x.shape[0]]
    f, parts, t = oracle.Fir(h, 3), [], 0
    for n in splits:
        parts.append(f.process(x[t:t + n]))
        t += n
    got = np.concatenate(parts)
    scale = np.sqrt(M) * np.max(np.abs(x))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)
