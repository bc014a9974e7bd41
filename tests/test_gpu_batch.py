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


def _make(F, orc, block=48, waves=4):
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
    # a second launch (the queue counters cleared themselves at the end of the
    # first): its start follows every completion of the first, and its own
    # completions follow its start
    b.launch()
    st2 = b.stamps()
    start2, ends2 = int(st2[-1]), st2[:-1].astype(np.int64)
    assert start2 > int(ends.max())
    assert np.all(ends2 > start2)


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


def test_autotuner_picks_applies_and_caches(F, tmp_path):
    """filark_autotune through the Python caller: the chosen tile is applied
    to the state, written to the JSON cache and reused from it."""
    import json

    from paper_2605_20132_amd.autotune import Autotuner

    orc = _orc()
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    path = str(tmp_path / "tiles.json")
    st = F.SOSState(sos, 3000)
    block, waves, group = Autotuner(path, block=48, waves=4).tune(st, 1000)
    assert (block, waves) == (48, 4) and group in (4, 8, 16, 32, 64)
    assert st.tile() == (block, waves, group)
    table = json.load(open(path))
    assert len(table) == 1 and list(table.values())[0]["group"] == group
    # a free search (block and waves too) adds an entry of its own
    b2, w2, g2 = F.tune_tile(st, 1000, cache=path)
    assert b2 in (32, 48, 64) and w2 in (2, 4, 8) and st.tile() == (b2, w2, g2)
    assert len(json.load(open(path))) == 2
    st2 = F.SOSState(sos, 3000)
    assert Autotuner(path, block=48, waves=4).tune(st2, 1000) == (block, waves, group)  # from the cache
    assert st2.tile() == (block, waves, group)
    st.close()
    st2.close()


def test_batch_capture_replays(F):
    """The batch-owned graph (filark_batch_capture): each launch after the
    capture replays it, with eager work in between, and must equal the
    per-stream calls on objects advanced the same way; a bind drops it."""
    orc = _orc()
    sts, _ = _make(F, orc)
    ref_sts, _ = _make(F, orc)
    xs = _inputs(30)
    ys = [torch.empty_like(x) for x in xs]
    b = F.Batch(sts)
    b.bind(xs, ys)
    b.capture()
    for rep in range(3):
        b.launch()
        refs = [st.process(x) for st, x in zip(ref_sts, xs)]
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, (y, r) in enumerate(zip(ys, refs)):
            assert torch.equal(y, r), f"replay {rep}: stream {i} differs"
    xs2 = _inputs(31)
    ys2 = [torch.empty_like(x) for x in xs2]
    b.bind(xs2, ys2)  # drops the graph: the next launch runs the new binding
    b.launch()
    refs = [st.process(x) for st, x in zip(ref_sts, xs2)]
    torch.cuda.synchronize()
    for y, r in zip(ys2, refs):
        assert torch.equal(y, r)


def test_drawn_twelve_stream_table_against_oracle(F):
    """The uneven 12-stream table of the batched benchmark (channel counts
    500 .. 20,000, rates 100 Hz .. 10 kHz, chunks 0.25-2 s, orders 2-10), each
    stream's group chosen by the autotuner, two chunks in a row through one
    captured batch: sampled channels of every stream (first, middle, last and
    five drawn) against the oracle run over both chunks."""
    import synth
    from paper_2605_20132_amd.autotune import Autotuner

    orc = _orc()
    specs = synth.draw_batched_streams()
    tuner = Autotuner(None, block=48, waves=8)
    sts, soss, xs1, xs2 = [], [], [], []
    for sp in specs:
        sos = orc.butter_sos(sp.order, "bandpass", sp.f1, sp.f2, sp.fs)
        st = F.SOSState(sos, sp.n_ch)
        tuner.tune(st, sp.n_t)
        sts.append(st)
        soss.append(sos)
        xs1.append(synth.pink_noise(sp.n_t, sp.n_ch, seed=sp.seed, device="cuda"))
        xs2.append(synth.pink_noise(sp.n_t, sp.n_ch, seed=sp.seed + 7, device="cuda"))
    ys1 = [torch.empty_like(x) for x in xs1]
    ys2 = [torch.empty_like(x) for x in xs2]
    b1, b2 = F.Batch(sts), F.Batch(sts)
    b1.bind(xs1, ys1)
    b2.bind(xs2, ys2)
    b1.capture()
    b2.capture()
    b1.launch()
    b2.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for i, (sp, sos) in enumerate(zip(specs, soss)):
        cols = sorted(set([0, sp.n_ch // 2, sp.n_ch - 1] + list(rng.integers(0, sp.n_ch, 5))))
        x = torch.cat([xs1[i][:, cols], xs2[i][:, cols]]).double().cpu().numpy()
        y = torch.cat([ys1[i][:, cols], ys2[i][:, cols]]).double().cpu().numpy()
        yo, _ = orc.sos_filter(sos, x)
        err = max_rel_rms(y, yo)
        assert err <= tolerance_for(sos), (i, sp, err)


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
    sts[1].set_tile(48, 4, 8 if STREAMS[1][6] != 8 else 16)  # group only: allowed per stream, but new tables
    with pytest.raises(F.FilarkError):
        b.launch()
    b.bind(xs, ys)
    b.launch()
    torch.cuda.synchronize()
    sts[2].set_tile(64, 4, 16)  # block differs from the batch's
    with pytest.raises(F.FilarkError):
        b.bind(xs, ys)
    b.close()
