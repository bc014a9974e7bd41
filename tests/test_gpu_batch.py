"""GPU tests of the batched multi-stream launch: every stream's output equals
its own per-stream call bit for bit (same kernel body, same tile) and the
oracle within the tolerance; states carry across chunks; HIP-graph replays
advance the states like launches; completion stamps are ordered."""

import numpy as np
import pytest

from tests.helpers import max_rel_rms, tolerance_for

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


# (n_ch, n_t, order, f1, f2, fs, group): uneven channels, chunks, orders, groups
STREAMS = [
    (37, 1500, 2, 1.0, 20.0, 100.0, 8),
    (300, 777, 4, 3.0, 100.0, 500.0, 4),
    (130, 3333, 6, 2.0, 300.0, 1500.0, 16),
    (64, 1, 8, 5.0, 2000.0, 10000.0, 64),
    (520, 2100, 10, 1.0, 400.0, 1500.0, 8),
]


def _make(F, orc, block=64, waves=4):
    sts, soss = [], []
    for n_ch, n_t, order, f1, f2, fs, group in STREAMS:
        sos = orc.butter_sos(order, "bandpass", f1, f2, fs)
        st = F.SOSState(sos, n_ch)
        st.set_tile(block, waves, group)
        sts.append(st)
        soss.append(sos)
    return sts, soss


def _inputs(seed, scale=1):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return [torch.randn((max(1, n_t * scale), n_ch), generator=g, device="cuda", dtype=torch.float32)
            for n_ch, n_t, *_ in STREAMS]


def test_batch_equals_per_stream_calls_and_oracle(F):
    orc = _orc()
    sts, soss = _make(F, orc)
    ref_sts, _ = _make(F, orc)
    xs = _inputs(1)
    ys = [torch.empty_like(x) for x in xs]
    b = F.Batch(sts)
    b.bind(xs, ys)
    b.launch()
    refs = [st.process(x) for st, x in zip(ref_sts, xs)]
    torch.cuda.synchronize()
    for i, (y, r, x, sos) in enumerate(zip(ys, refs, xs, soss)):
        assert torch.equal(y, r), f"stream {i} differs from its per-stream call"
        yo, zo = orc.sos_filter(sos, x.cpu().numpy())
        assert max_rel_rms(y.cpu().numpy(), yo) <= tolerance_for(sos)
        np.testing.assert_array_equal(sts[i].get_state(), ref_sts[i].get_state())
    st_ = b.stamps()
    start, ends = int(st_[-1]), st_[:-1].astype(np.int64)
    assert np.all(ends > start)


def test_batch_carries_state_over_chunks(F):
    orc = _orc()
    sts, soss = _make(F, orc)
    b = F.Batch(sts)
    chunks = [_inputs(10 + k) for k in range(3)]
    outs = []
    for xs in chunks:
        ys = [torch.empty_like(x) for x in xs]
        b.bind(xs, ys)
        b.launch()
        outs.append(ys)
    torch.cuda.synchronize()
    for i, sos in enumerate(soss):
        x = torch.cat([c[i] for c in chunks]).cpu().numpy()
        y = torch.cat([o[i] for o in outs]).cpu().numpy()
        yo, zo = orc.sos_filter(sos, x)
        assert max_rel_rms(y, yo) <= tolerance_for(sos)
        np.testing.assert_allclose(sts[i].get_state(), zo, rtol=1e-6, atol=1e-6 * np.abs(zo).max())


def test_batch_graph_replays_advance_state(F):
    """Capture one launch; each replay, with eager work in between, must equal
    the per-stream calls on objects advanced the same way."""
    orc = _orc()
    sts, _ = _make(F, orc)
    ref_sts, _ = _make(F, orc)
    xs = _inputs(20)
    ys = [torch.empty_like(x) for x in xs]
    b = F.Batch(sts)
    b.bind(xs, ys)
    b.launch()  # warm-up outside the capture
    for st, x in zip(ref_sts, xs):
        st.process(x)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.launch(stream=s)
    torch.cuda.synchronize()
    # the capture enqueued nothing: states are where the warm-up left them
    for rep in range(3):
        g.replay()
        refs = [st.process(x) for st, x in zip(ref_sts, xs)]
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, (y, r) in enumerate(zip(ys, refs)):
            assert torch.equal(y, r), f"replay {rep}: stream {i} differs"


def test_batch_argument_errors(F):
    orc = _orc()
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    a, c = F.SOSState(sos, 64), F.SOSState(sos, 64)
    c.set_tile(32, 4, 8)
    with pytest.raises(F.FilarkError) as e:
        F.Batch([a, c])  # blocks differ
    assert e.value.status == F.EINVAL
    with pytest.raises(F.FilarkError):
        F.Batch([a, a])  # the same state twice
    b = F.Batch([a])
    with pytest.raises(F.FilarkError):
        b.launch()  # not bound
    x = torch.zeros((10, 65), device="cuda")
    with pytest.raises(F.FilarkError) as e:
        b.bind([x], [torch.empty_like(x)])
    assert e.value.status == F.ESHAPE


def test_autotuner_picks_and_caches(F, tmp_path):
    from paper_2605_20132_amd.autotune import GROUPS, Autotuner

    orc = _orc()
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    path = str(tmp_path / "tiles.json")
    t = Autotuner(path, block=64, waves=4, reps=2)
    gsel = t.group_for(sos, 3000, 1000)
    assert gsel in GROUPS
    t2 = Autotuner(path, block=64, waves=4)
    assert t2.group_for(sos, 3000, 1000) == gsel  # from the cache, no measurement


def test_tile_change_after_bind_is_refused_until_bound_again(F):
    """A tile change rebuilds a state's tables, which a bound batch names:
    the next launch is refused until the batch is bound again, and a bind
    refuses a state whose block or waves no longer match the batch's."""
    orc = _orc()
    sts, soss = _make(F, orc)
    xs = _inputs(5)
    ys = [torch.empty_like(x) for x in xs]
    b = F.Batch(sts)
    b.bind(xs, ys)
    b.launch()
    torch.cuda.synchronize()
    sts[1].set_tile(64, 4, 8)  # group only: allowed per stream, but the tables are new
    with pytest.raises(F.FilarkError):
        b.launch()
    b.bind(xs, ys)
    b.launch()
    torch.cuda.synchronize()
    sts[2].set_tile(48, 4, 16)  # block differs from the batch's
    with pytest.raises(F.FilarkError):
        b.bind(xs, ys)
    b.close()
