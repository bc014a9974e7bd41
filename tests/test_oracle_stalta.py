"""Pins for the oracle's recursive STA/LTA characteristic (energy-detector
monitor of Section 3.4; definition: exponential recursive STA/LTA on the
squared filter output, warm-up of nlta samples, cf = 0 where lta = 0).

Facts used:
  * constant energy E: sta_t = E (1 - (1-cs)^(t+1)), lta_t = E (1 - (1-cl)^(t+1));
  * unit impulse at t = 0: cf_t = (cs/cl) ((1-cs)/(1-cl))^t;
  * nsta == nlta gives cf == 1 after warm-up;
  * brute-force direct sums sta_t = sum_j cs (1-cs)^(t-j) e_j;
  * warm-up mask exactly at the global index nlta, across chunk boundaries;
  * chunked == one-shot bit for bit.
"""

import numpy as np
import pytest


def test_constant_energy_closed_form(orc):
    nsta, nlta, n = 30, 300, 2000
    amp = 1.7
    y = np.full((n, 2), amp)
    y[:, 1] = -amp
    cf, st, g = orc.stalta(y, nsta, nlta)
    t = np.arange(n, dtype=np.float64)
    cs, cl = 1.0 / nsta, 1.0 / nlta
    E = amp * amp
    sta = E * (1 - (1 - cs) ** (t + 1))
    lta = E * (1 - (1 - cl) ** (t + 1))
    want = np.where(t >= nlta, sta / lta, 0.0)
    np.testing.assert_allclose(cf[:, 0], want, rtol=1e-12, atol=0)
    np.testing.assert_allclose(cf[:, 1], want, rtol=1e-12, atol=0)
    np.testing.assert_allclose(st[0], [sta[-1], lta[-1]], rtol=1e-12)
    assert g == n


def test_impulse_closed_form(orc):
    nsta, nlta, n = 7, 50, 400
    y = np.zeros((n, 1))
    y[0, 0] = 1.0
    cf, _, _ = orc.stalta(y, nsta, nlta)
    cs, cl = 1.0 / nsta, 1.0 / nlta
    t = np.arange(n, dtype=np.float64)
    want = np.where(t >= nlta, (cs / cl) * ((1 - cs) / (1 - cl)) ** t, 0.0)
    np.testing.assert_allclose(cf[:, 0], want, rtol=1e-11, atol=1e-300)


def test_equal_windows_give_unit_ratio(orc):
    rng = np.random.default_rng(4)
    y = rng.standard_normal((1000, 3))
    cf, _, _ = orc.stalta(y, 100, 100)
    assert np.all(cf[:100] == 0.0)
    np.testing.assert_allclose(cf[100:], 1.0, rtol=1e-13)


def test_brute_force_direct_sums(orc):
    rng = np.random.default_rng(9)
    n, nsta, nlta = 150, 5, 40
    y = rng.standard_normal((n, 2))
    cf, _, _ = orc.stalta(y, nsta, nlta)
    cs, cl = 1.0 / nsta, 1.0 / nlta
    e = y * y
    for t in range(n):
        j = np.arange(t + 1)
        sta = np.sum(cs * (1 - cs) ** (t - j)[:, None] * e[: t + 1], axis=0)
        lta = np.sum(cl * (1 - cl) ** (t - j)[:, None] * e[: t + 1], axis=0)
        want = sta / lta if t >= nlta else np.zeros(2)
        np.testing.assert_allclose(cf[t], want, rtol=1e-12, atol=0)


def test_zero_energy_gives_zero(orc):
    y = np.zeros((500, 2))
    y[300:, 1] = 1.0
    cf, _, _ = orc.stalta(y, 10, 100)
    assert np.all(cf[:, 0] == 0.0)
    assert np.all(cf[:300, 1] == 0.0)
    assert np.all(cf[300:, 1] > 0.0)


@pytest.mark.parametrize("splits", [[1000], [299, 2, 699], [1] * 10 + [990], [0, 500, 0, 500]])
def test_chunked_equals_one_shot_and_warmup_across_chunks(orc, splits):
    rng = np.random.default_rng(12)
    y = rng.standard_normal((sum(splits), 4))
    nsta, nlta = 30, 300
    cf1, st1, g1 = orc.stalta(y, nsta, nlta)
    st, g, outs, t0 = None, 0, [], 0
    for n in splits:
        cf, st, g = orc.stalta(y[t0:t0 + n], nsta, nlta, st, g)
        outs.append(cf)
        t0 += n
    cf2 = np.concatenate(outs, axis=0)
    assert np.array_equal(cf1, cf2)
    assert np.array_equal(st1, st) and g1 == g
    assert np.all(cf1[:nlta] == 0.0) and np.all(cf1[nlta:] > 0.0)


def test_stream_helper_matches_stages(orc):
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    rng = np.random.default_rng(13)
    x = rng.standard_normal((10_000, 8))
    y1, _ = orc.sos_filter(sos, x)
    cf1, _, _ = orc.stalta(y1, 250, 2500)
    s = orc.Stream(sos, 8, 250, 2500)
    parts = [s.process(x[i:i + 1000]) for i in range(0, 10_000, 1000)]
    assert np.array_equal(np.concatenate([p[0] for p in parts]), y1)
    assert np.array_equal(np.concatenate([p[1] for p in parts]), cf1)


def test_window_rounding():
    import oracle

    assert oracle.window_samples(0.5, 500.0) == 250
    assert oracle.window_samples(5.0, 500.0) == 2500
    assert oracle.window_samples(0.2, 1500.0) == 300
    assert oracle.window_samples(2.0, 1500.0) == 3000
