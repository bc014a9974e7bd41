"""Pins of the oracle's stateful exponential-average operators (running-mean
removal and running AGC, Table 1's running mean / AGC rows).

* closed forms: constant input (both modes), unit impulse (running mean);
* brute-force weighted sums m_t = sum_j c (1 - c)^(t - j) x_j on small inputs;
* AGC is invariant to a positive gain on its input;
* chunked == one-shot, bit for bit, over splits with empty and one-sample
  chunks.
"""

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n_win", [1, 4, 300])
def test_demean_constant_and_impulse(n_win):
    c = 1.0 / n_win
    t = np.arange(2000)
    y = oracle.Ema(1, n_win, "demean").process(np.full(2000, 3.0))[:, 0]
    # y = x - m cancels as m -> x: the error scale is that of x
    np.testing.assert_allclose(y, 3.0 * (1 - c) ** (t + 1), rtol=1e-12, atol=3.0 * 1e-14)
    x = np.zeros(2000)
    x[0] = 1.0
    y = oracle.Ema(1, n_win, "demean").process(x)[:, 0]
    assert y[0] == pytest.approx(1 - c, rel=1e-15)
    np.testing.assert_allclose(y[1:], -c * (1 - c) ** t[1:], rtol=1e-12, atol=1e-300)  # no cancellation


@pytest.mark.parametrize("a", [2.5, -0.75])
def test_agc_constant_input(a):
    n_win, n = 50, 3000
    c = 1.0 / n_win
    t = np.arange(n)
    y = oracle.Ema(1, n_win, "agc").process(np.full(n, a))[:, 0]
    np.testing.assert_allclose(y, np.sign(a) / np.sqrt(1 - (1 - c) ** (t + 1)), rtol=1e-12)


@pytest.mark.parametrize("mode", ["demean", "agc"])
def test_brute_force_sums(mode):
    rng = np.random.default_rng(1)
    n_win, n = 7, 60
    c = 1.0 / n_win
    x = rng.standard_normal((n, 3))
    e = x if mode == "demean" else x * x
    w = c * (1 - c) ** np.arange(n)
    avg = np.stack([[np.dot(w[:t + 1][::-1], e[:t + 1, k]) for k in range(3)] for t in range(n)])
    ref = x - avg if mode == "demean" else x / np.sqrt(avg)
    np.testing.assert_allclose(oracle.Ema(3, n_win, mode).process(x), ref, rtol=1e-12, atol=1e-14)


def test_agc_gain_invariance():
    x = np.random.default_rng(2).standard_normal((4000, 5))
    a = oracle.Ema(5, 200, "agc").process(x)
    b = oracle.Ema(5, 200, "agc").process(x * 37.0)
    np.testing.assert_allclose(a, b, rtol=1e-12)


@pytest.mark.parametrize("mode", ["demean", "agc"])
def test_chunked_equals_one_shot(mode):
    x = np.random.default_rng(3).standard_normal((5000, 4))
    one = oracle.Ema(4, 250, mode).process(x)
    e = oracle.Ema(4, 250, mode)
    parts, t = [], 0
    for n in [0, 1, 1999, 0, 3000]:
        parts.append(e.process(x[t:t + n]))
        t += n
    np.testing.assert_array_equal(np.concatenate(parts), one)
