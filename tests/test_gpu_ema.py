"""GPU parity of the stateful exponential-average operators (running-mean
removal, running AGC) against the oracle on the exact FP32 input (upcast).
Bar: per-channel relative RMS <= 1e-5.  Shapes: one sample, ragged channel
groups, chunks shorter and longer than a 1536-row window, empty chunks, an
input with a large offset (the running mean's cancellation); state carried
and set from the oracle; in place; the full 6000 x 90,000 record sampled.
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


def _run(F, x, splits, mode, win_s, fs):
    n_ch = x.shape[1]
    e = F.Ema(n_ch, win_s, fs, mode)
    ys, t0 = [], 0
    for n in splits:
        ys.append(e.process(x[t0:t0 + n].contiguous()))
        t0 += n
    torch.cuda.synchronize()
    return torch.cat(ys).cpu().numpy(), e


@pytest.mark.parametrize("mode", ["demean", "agc"])
@pytest.mark.parametrize("n_ch,splits,offset", [
    (1, [1, 2, 300], 0.0),
    (9, [1536, 1, 1535, 0, 1537], 0.0),
    (65, [100] * 20, 50.0),
    (300, [5000, 777], 1000.0),
])
def test_ema_matches_oracle(F, mode, n_ch, splits, offset):
    orc = _orc()
    g = torch.Generator(device="cuda").manual_seed(40 + n_ch)
    x = torch.randn((sum(splits), n_ch), generator=g, device="cuda", dtype=torch.float32) + offset
    win_s, fs = 0.5, 500.0
    y, e = _run(F, x, splits, mode, win_s, fs)
    o = orc.Ema(n_ch, orc.window_samples(win_s, fs), mode)
    yo = o.process(x.cpu().numpy().astype(np.float64))
    assert max_rel_rms(y, yo) <= 1e-5
    np.testing.assert_allclose(e.get_state(), o.avg, rtol=1e-9)


@pytest.mark.parametrize("mode", ["demean", "agc"])
def test_ema_state_set_and_in_place(F, mode):
    orc = _orc()
    n_ch = 33
    g = torch.Generator(device="cuda").manual_seed(8)
    x = torch.randn((3000, n_ch), generator=g, device="cuda", dtype=torch.float32)
    xh = x.cpu().numpy().astype(np.float64)
    o = orc.Ema(n_ch, 100, mode)
    o.process(xh[:1000])
    e = F.Ema(n_ch, 0.2, 500.0, mode)  # 100 samples
    e.set_state(o.avg)
    buf = x[1000:].clone()
    e.process(buf, buf)
    torch.cuda.synchronize()
    assert max_rel_rms(buf.cpu().numpy(), o.process(xh[1000:])) <= 1e-5


def test_ema_full_size_sampled(F):
    import synth

    orc = _orc()
    w = synth.make_config2(device="cuda")
    x = w.x
    n_t, n_ch = x.shape
    e = F.Ema(n_ch, 2.0, w.fs, "agc")
    y = torch.empty_like(x)
    for a in range(0, n_t, w.chunk):
        e.process(x[a:a + w.chunk], y[a:a + w.chunk])
    torch.cuda.synchronize()
    cols = [0, 7, 8, 2999, 5998, 5999]
    tc = torch.as_tensor(cols, device="cuda")
    yo = orc.Ema(len(cols), orc.window_samples(2.0, w.fs), "agc").process(x[:, tc].double().cpu().numpy())
    assert max_rel_rms(y[:, tc].cpu().numpy(), yo) <= 1e-5


def test_ema_argument_errors(F):
    with pytest.raises(F.FilarkError):
        F.Ema(4, 0.0, 100.0, "agc")
    e = F.Ema(4, 1.0, 100.0, "demean")
    with pytest.raises(F.FilarkError) as ex:
        e.process(torch.zeros((10, 5), device="cuda"))
    assert ex.value.status == F.ESHAPE
