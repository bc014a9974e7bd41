"""Pins of the oracle's two-threshold trigger (the monitor of Section 3.4:
cf in, time-channel events out).

* a hand-worked sequence, events derived from the definition on paper;
* an independent derivation of the same events by searching (first sample
  above `on` after the previous close, then the first later sample below
  `off`), written without a state machine;
* invariants every event list must satisfy (non-overlapping, the opening
  sample above `on`, the closing sample below `off`, nothing in between below
  `off`, nothing between events above `on`);
* chunked = one-shot for every split, including empty and one-sample chunks,
  with events that straddle chunk boundaries;
* NaN never opens or closes an event.
"""

import numpy as np
import pytest

import oracle


def _search_events(cf, on, off, t_open=None):
    """Events of one channel by searching: no state machine."""
    cf = np.asarray(cf, dtype=np.float32)
    on, off = np.float32(on), np.float32(off)
    ev, t = [], 0
    n = len(cf)
    if t_open is not None:  # an event carried in open
        below = np.nonzero(cf < off)[0]
        if len(below) == 0:
            return ev, t_open
        ev.append((t_open, int(below[0])))
        t = int(below[0]) + 1
    while t < n:
        above = np.nonzero(cf[t:] > on)[0]
        if len(above) == 0:
            return ev, None
        s = t + int(above[0])
        below = np.nonzero(cf[s + 1:] < off)[0]
        if len(below) == 0:
            return ev, s
        e = s + 1 + int(below[0])
        ev.append((s, e))
        t = e + 1
    return ev, None


def test_hand_worked_sequence():
    # on = 2.5, off = 1.0: 3 > 2.5 opens at t = 2, 0.5 < 1 closes at t = 4;
    # 1.5 and 0.2 are ignored while closed/open respectively as they cross
    # nothing; 4 > 2.5 opens at t = 6 and 0.1 < 1 closes at t = 8.
    cf = np.array([0.0, 2.0, 3.0, 1.5, 0.5, 0.2, 4.0, 4.0, 0.1], dtype=np.float32)
    ev = oracle.Trigger(1, 2.5, 1.0).process(cf)
    assert ev.tolist() == [[0, 2, 4], [0, 6, 8]]


def test_equal_to_threshold_does_not_cross():
    # strict comparisons: cf == on does not open, cf == off does not close
    cf = np.array([2.5, 3.0, 1.0, 1.0, 0.99, 2.5], dtype=np.float32)
    ev = oracle.Trigger(1, 2.5, 1.0).process(cf)
    assert ev.tolist() == [[0, 1, 4]]


def test_square_pulses():
    n = 1000
    cf = np.zeros((n, 3), dtype=np.float32)
    edges = {0: [(10, 20), (500, 501)], 1: [], 2: [(0, 999)]}
    for c, runs in edges.items():
        for a, b in runs:
            cf[a:b, c] = 10.0
    tr = oracle.Trigger(3, 5.0, 1.0)
    ev = tr.process(cf)
    assert ev.tolist() == [[0, 10, 20], [0, 500, 501], [2, 0, 999]]
    assert tr.open.tolist() == [0, 0, 0]


def _random_cf(rng, n_t, n_ch):
    # a smooth positive process that crosses both thresholds often
    w = rng.standard_normal((n_t, n_ch)).cumsum(axis=0) * 0.3
    return (2.0 + np.sin(np.arange(n_t)[:, None] / 17.0 + rng.uniform(0, 6, n_ch)) * 1.5 + 0.2 * w).astype(np.float32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_search_derivation_and_invariants(seed):
    rng = np.random.default_rng(seed)
    n_t, n_ch = 3000, 7
    on, off = 3.0, 1.2
    cf = _random_cf(rng, n_t, n_ch)
    tr = oracle.Trigger(n_ch, on, off)
    ev = tr.process(cf)
    assert len(ev) > 10
    for c in range(n_ch):
        mine = [tuple(e[1:]) for e in ev if e[0] == c]
        ref, still_open = _search_events(cf[:, c], on, off)
        assert mine == ref
        assert bool(tr.open[c]) == (still_open is not None)
        if still_open is not None:
            assert tr.t_on[c] == still_open
        prev_end = -1
        for s, e in mine:
            assert s < e and s > prev_end - 1
            assert cf[s, c] > np.float32(on) and cf[e, c] < np.float32(off)
            assert np.all(cf[s + 1:e, c] >= np.float32(off))
            assert np.all(cf[prev_end + 1:s, c] <= np.float32(on))
            prev_end = e


@pytest.mark.parametrize("splits", [[3000], [1, 2999], [0, 1000, 0, 2000], [7] * 428 + [4], [1499, 1501]])
def test_chunked_equals_one_shot(splits):
    rng = np.random.default_rng(5)
    n_ch = 5
    cf = _random_cf(rng, sum(splits), n_ch)
    one = oracle.Trigger(n_ch, 3.0, 1.2).process(cf)
    tr = oracle.Trigger(n_ch, 3.0, 1.2)
    parts, t = [], 0
    for n in splits:
        parts.append(tr.process(cf[t:t + n]))
        t += n
    chunked = np.concatenate(parts) if parts else np.zeros((0, 3), np.int64)
    key = lambda a: sorted(map(tuple, a.tolist()))
    assert key(chunked) == key(one)
    assert tr.g == sum(splits)


def test_nan_never_crosses():
    cf = np.array([np.nan, 5.0, np.nan, np.nan, 0.0, np.nan], dtype=np.float32)
    ev = oracle.Trigger(1, 2.0, 1.0).process(cf)
    assert ev.tolist() == [[0, 1, 4]]
