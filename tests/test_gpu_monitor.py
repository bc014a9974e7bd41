"""GPU: the monitor chain in one pass (filark_monitor_process: SOS cascade,
STA/LTA, two-threshold trigger) against the same chain as two calls
(filark_sos_stalta_process, then filark_trigger_process on its cf) and
against the oracle.

Against the two calls: y and cf bit for bit where written, the three carried
states bit for bit, the events equal as sorted sets (their order in the list
depends on timing in both paths).  Against the oracle: the oracle's cf
(FP64, rounded to FP32) through the oracle's trigger gives the reference
events; where the GPU's FP32 cf and the oracle's straddle a threshold the
events may differ, so the bar there is the cf bar (1e-5 per-channel relative
RMS) plus the count of events within 1 % of the oracle's.  Shapes: ragged
channel groups, chunks of one row, chunks spanning several 1536-row
windows, y and cf written or not, 8- and 16-channel groups.
"""

import numpy as np
import pytest

from tests.helpers import max_rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_20132_amd as F

    F.lib()
    return F


def _orc():
    import oracle

    return oracle


def _sorted(ev):
    a = np.asarray(ev, dtype=np.int64).reshape(-1, 3)
    return a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))]


def _objects(F, sos, n_ch, nsta, nlta, on, off, tile):
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
    if tile is not None:
        st.set_tile(*tile)
        sl.set_tile(*tile)
    return st, sl, F.Trigger(n_ch, on, off)


def _chain(F, sos, x, splits, nsta, nlta, on, off, fused, write_y, write_cf, tile=None):
    n_t, n_ch = x.shape
    st, sl, tr = _objects(F, sos, n_ch, nsta, nlta, on, off, tile)
    cap = n_t * n_ch // 4 + 16
    ev = torch.full((cap, 3), -7, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    y = torch.full_like(x, -1.0) if write_y else None
    cf = torch.full_like(x, -1.0) if (write_cf or not fused) else None
    t0 = 0
    for n in splits:
        xs = x[t0:t0 + n]
        ys = y[t0:t0 + n] if y is not None else None
        cs = cf[t0:t0 + n] if cf is not None else None
        if fused:
            F.monitor_process(st, sl, tr, xs, ev, count, y=ys, cf=cs)
        else:
            F.sos_stalta_process(st, sl, xs, y=ys, cf=cs, write_y=write_y)
            tr.process(cs, ev, count)
        t0 += n
    torch.cuda.synchronize()
    st.check()
    k = int(count.item())
    return (y, cf, _sorted(ev[:min(k, cap)].cpu().numpy()), k, st.get_state(), sl.get_state(), tr.get_state())


@pytest.mark.parametrize("n_ch,splits,write_y,write_cf,tile", [
    (37, [3000, 1, 1499, 1536], True, True, None),
    (200, [1500] * 4, False, False, None),
    (96, [700, 5000], True, False, None),
    (65, [100] * 20, False, True, (48, 4, 8)),
])
def test_monitor_matches_two_calls(F, n_ch, splits, write_y, write_cf, tile):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    nsta, nlta, on, off = 30, 300, 2.0, 1.2
    g = torch.Generator(device="cuda").manual_seed(n_ch)
    n_t = sum(splits)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    x[n_t // 3:n_t // 3 + 200] *= 6.0  # an energetic stretch: events on every channel
    a = _chain(F, sos, x, splits, nsta, nlta, on, off, True, write_y, write_cf, tile)
    b = _chain(F, sos, x, splits, nsta, nlta, on, off, False, write_y, write_cf, tile)
    if write_y:
        np.testing.assert_array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    if write_cf:
        np.testing.assert_array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
    np.testing.assert_array_equal(a[2], b[2])
    assert a[3] == b[3] and a[3] > 0
    np.testing.assert_array_equal(a[4], b[4])
    for u, v in zip(a[5], b[5]):
        np.testing.assert_array_equal(u, v)
    for u, v in zip(a[6], b[6]):
        np.testing.assert_array_equal(u, v)


def test_monitor_against_oracle(F):
    orc = _orc()
    sos = orc.butter_sos(4, "bandpass", 2.0, 40.0, 500.0)
    n_ch, nsta, nlta, on, off = 24, 25, 250, 2.5, 1.3
    splits = [1000, 1000, 2500]
    n_t = sum(splits)
    g = torch.Generator(device="cuda").manual_seed(9)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    x[1800:1900] *= 8.0
    x[3300:3350] *= 10.0
    y, cf, ev, k, _, _, _ = _chain(F, sos, x, splits, nsta, nlta, on, off, True, True, True)
    xh = x.cpu().numpy().astype(np.float64)
    yo, _ = orc.sos_filter(sos, xh)
    co, _, _ = orc.stalta(yo, nsta, nlta)
    assert max_rel_rms(y.cpu().numpy(), yo) <= 1e-5
    assert max_rel_rms(cf.cpu().numpy(), co) <= 1e-5
    # the oracle's trigger on the GPU's cf: exactly the GPU's events
    tro = orc.Trigger(n_ch, on, off)
    oev = tro.process(cf.cpu().numpy())
    np.testing.assert_array_equal(ev, _sorted(oev))
    # on the oracle's own cf (rounded to FP32): the same events up to threshold straddles
    tro2 = orc.Trigger(n_ch, on, off)
    oev2 = tro2.process(co.astype(np.float32))
    assert k > 0 and abs(len(oev2) - k) <= max(1, k // 100)


def test_monitor_errors(F):
    orc = _orc()
    sos = orc.butter_sos(4, "lowpass", 10.0, 0.0, 100.0)
    st, sl, tr = _objects(F, sos, 16, 5, 50, 2.0, 1.0, None)
    x = torch.zeros((40, 16), device="cuda")
    ev = torch.zeros((8, 3), dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    F.monitor_process(st, sl, tr, x[:0], ev, count)  # no rows: nothing happens
    with pytest.raises(F.FilarkError):  # another channel count
        F.monitor_process(st, sl, F.Trigger(17, 2.0, 1.0), x, ev, count)
    st.set_tile(64, 4, 8)
    sl.set_tile(64, 4, 8)
    with pytest.raises(F.FilarkError):  # 64-row blocks
        F.monitor_process(st, sl, tr, x, ev, count)
