"""GPU parity of the realtime FIR with carried history against the oracle, on
the exact FP32 input the GPU saw (upcast).

Bar: element by element, |y_gpu - y_oracle| <= (M + 2) 2^-24 sum_k |h_k| |x_{t-k}|
(+ 1e-37), the rounding bound of M FP32 FMAs after rounding the taps to FP32;
the bound itself comes from the oracle run on |h| and |x|.  Beyond parity:
chunked == one-shot bit for bit on the GPU (every output takes its taps in
one fixed order), every tile gives the same bits, the carried history is the
last M - 1 input rows exactly, and state set/get round-trips.
Shapes: one sample, chunks shorter than the history, ragged channel groups
and row blocks, tap counts that are and are not multiples of the 32-tap
chunk, and a million-channel record split over several launch windows.
"""

import numpy as np
import pytest

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


def _taps(M, kind, seed):
    if kind == "random":
        return np.random.default_rng(seed).standard_normal(M)
    # windowed-sinc lowpass at a quarter of the sample rate
    n = np.arange(M) - (M - 1) / 2
    return 0.5 * np.sinc(0.5 * n) * np.hamming(M) if M > 1 else np.ones(1)


def _check(y, x, h, orc, hist=None):
    """y (GPU, [n_t, n_ch]) against the oracle on x (float32 numpy) from the
    given starting history, within the FMA rounding bound."""
    n_ch = x.shape[1]
    f = orc.Fir(h, n_ch)
    fa = orc.Fir(np.abs(h), n_ch)
    if hist is not None:
        f.hist[:] = hist
        fa.hist[:] = np.abs(hist)
    xd = x.astype(np.float64)
    ref = f.process(xd)
    bound = (len(h) + 2) * 2.0 ** -24 * fa.process(np.abs(xd)) + 1e-37
    err = np.abs(y.astype(np.float64) - ref)
    assert np.all(err <= bound), f"max err/bound {np.max(err / bound):.3g}"
    return f


@pytest.mark.parametrize("n_ch,n_t", [(1, 1), (7, 100), (65, 129), (130, 1537), (300, 5000)])
@pytest.mark.parametrize("M,kind", [(1, "random"), (2, "random"), (17, "sinc"), (32, "random"), (33, "sinc"),
                                    (64, "random"), (101, "sinc")])
def test_fir_matches_oracle(F, n_ch, n_t, M, kind):
    orc = _orc()
    h = _taps(M, kind, M)
    g = torch.Generator(device="cuda").manual_seed(400 + n_ch + M)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    f = F.Fir(h, n_ch)
    y = f.process(x)
    torch.cuda.synchronize()
    of = _check(y.cpu().numpy(), x.cpu().numpy(), h, orc)
    if M > 1:
        np.testing.assert_array_equal(f.get_state(), of.hist.astype(np.float32))
    f.close()


@pytest.mark.parametrize("rows", [16, 32, 48])
@pytest.mark.parametrize("M", [1, 32, 33, 64, 65, 200])
def test_rows_per_wave_match_oracle_and_each_other(F, rows, M):
    """Every rows-per-wave kernel (unrolled up to 64 taps, looped beyond)
    against the oracle, ragged in rows and channels, through a chunk shorter
    than the history, and bit for bit against the default tile."""
    orc = _orc()
    h = _taps(M, "random", 40 + M)
    n_ch, n_t = 150, 1000
    g = torch.Generator(device="cuda").manual_seed(600 + M)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    f = F.Fir(h, n_ch)
    f.set_tile(rows, 1, 2)
    cut = max(1, M // 3)
    y = torch.cat([f.process(x[:cut].contiguous()), f.process(x[cut:].contiguous())])
    ref = F.Fir(h, n_ch).process(x)
    torch.cuda.synchronize()
    _check(y.cpu().numpy(), x.cpu().numpy(), h, orc)
    assert torch.equal(y, ref)


@pytest.mark.parametrize("M", [63, 65, 96, 128, 129, 1024])
def test_long_filters_and_kernel_switch(F, M):
    """Tap counts on both sides of the unrolled kernel's limit (64 taps) up to
    the maximum, over ragged shapes, in two chunks."""
    orc = _orc()
    h = _taps(M, "sinc", M)
    n_ch, n_t = 97, 2 * M + 333
    g = torch.Generator(device="cuda").manual_seed(500 + M)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    f = F.Fir(h, n_ch)
    y = torch.cat([f.process(x[:M // 2 + 1].contiguous()), f.process(x[M // 2 + 1:].contiguous())])
    torch.cuda.synchronize()
    of = _check(y.cpu().numpy(), x.cpu().numpy(), h, orc)
    np.testing.assert_array_equal(f.get_state(), of.hist.astype(np.float32))


@pytest.mark.parametrize("M", [2, 64, 101])
def test_chunked_equals_one_shot_bitwise(F, M):
    n_ch, n_t = 200, 3000
    h = _taps(M, "random", 7)
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    one = F.Fir(h, n_ch).process(x)
    f = F.Fir(h, n_ch)
    parts, t = [], 0
    for n in [0, 1, 5, M - 1, 0, 700, 1, 1]:
        parts.append(f.process(x[t:t + n].contiguous()))
        t += n
    parts.append(f.process(x[t:].contiguous()))
    torch.cuda.synchronize()
    assert torch.equal(torch.cat(parts), one)
    np.testing.assert_array_equal(f.get_state(), x[n_t - (M - 1):].cpu().numpy())


@pytest.mark.parametrize("rows,waves,order", [(16, 1, 0), (16, 4, 1), (32, 1, 1), (32, 8, 0), (16, 8, 1), (32, 4, 1),
                                               (32, 1, 2), (16, 2, 2), (32, 4, 2), (48, 1, 2), (48, 4, 0),
                                               (48, 2, 1), (0, 1, 2), (0, 3, 0)])
def test_every_tile_gives_the_same_bits(F, rows, waves, order):
    n_ch, n_t, M = 129, 2051, 64
    h = _taps(M, "sinc", 0)
    g = torch.Generator(device="cuda").manual_seed(12)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    ref = F.Fir(h, n_ch)
    a = [ref.process(x[:1000].contiguous()), ref.process(x[1000:].contiguous())]
    f = F.Fir(h, n_ch)
    f.set_tile(rows, waves, order)
    b = [f.process(x[:1000].contiguous()), f.process(x[1000:].contiguous())]
    torch.cuda.synchronize()
    assert torch.equal(torch.cat(a), torch.cat(b))
    np.testing.assert_array_equal(f.get_state(), ref.get_state())


@pytest.mark.parametrize("order", [0, 1, 2])
def test_orders_on_few_channel_groups(F, order):
    """1 to 9 channel groups of 64 (fewer groups than XCDs for order 2)."""
    orc = _orc()
    h = _taps(64, "random", 9)
    for n_ch in (1, 64, 130, 513):
        g = torch.Generator(device="cuda").manual_seed(n_ch)
        x = torch.randn((777, n_ch), generator=g, device="cuda", dtype=torch.float32)
        f = F.Fir(h, n_ch)
        f.set_tile(32, 1, order)
        y = f.process(x)
        torch.cuda.synchronize()
        _check(y.cpu().numpy(), x.cpu().numpy(), h, orc)


@pytest.mark.parametrize("M,n_ch,chunk", [(64, 300, 500), (101, 70, 40), (33, 65, 1)])
def test_graph_replays_carry_history(F, M, n_ch, chunk):
    """One call captured in a HIP graph, replayed over successive chunks with
    eager work in between: every replay equals an eager object's call on the
    same chunk bit for bit, and the carried history follows (chunks shorter
    than the history included)."""
    h = _taps(M, "random", 21)
    g0 = torch.Generator(device="cuda").manual_seed(22)
    x = torch.randn((6 * chunk, n_ch), generator=g0, device="cuda", dtype=torch.float32)
    f, ref = F.Fir(h, n_ch), F.Fir(h, n_ch)
    xs, ys = torch.empty((chunk, n_ch), device="cuda"), torch.empty((chunk, n_ch), device="cuda")
    xs.copy_(x[:chunk])
    f.process(xs, ys)  # warm-up outside the capture
    r0 = ref.process(x[:chunk].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(ys, r0)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            f.process(xs, ys, stream=s)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(f.get_state(), ref.get_state())  # the capture ran nothing
    for i in range(1, 6):
        xs.copy_(x[i * chunk:(i + 1) * chunk])
        g.replay()
        r = ref.process(x[i * chunk:(i + 1) * chunk].contiguous())
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(ys, r), f"replay {i}"
        np.testing.assert_array_equal(f.get_state(), ref.get_state())


def test_state_set_continues_a_stream(F):
    orc = _orc()
    n_ch, M = 70, 40
    h = _taps(M, "random", 3)
    rng = np.random.default_rng(5)
    hist = rng.standard_normal((M - 1, n_ch)).astype(np.float32)
    f = F.Fir(h, n_ch)
    f.set_state(hist)
    np.testing.assert_array_equal(f.get_state(), hist)
    x = torch.from_numpy(rng.standard_normal((500, n_ch)).astype(np.float32)).cuda()
    y = f.process(x)
    torch.cuda.synchronize()
    _check(y.cpu().numpy(), x.cpu().numpy(), h, orc, hist=hist.astype(np.float64))
    # a chunk shorter than the history keeps the newest old rows in front
    f.set_state(hist)
    x2 = torch.from_numpy(rng.standard_normal((10, n_ch)).astype(np.float32)).cuda()
    f.process(x2)
    np.testing.assert_array_equal(f.get_state(), np.concatenate([hist[10:], x2.cpu().numpy()]))


def test_errors(F):
    h = _taps(16, "random", 1)
    f = F.Fir(h, 8)
    x = torch.zeros((100, 8), device="cuda")
    with pytest.raises(F.FilarkError):
        f.process(x, x)  # in place: neighbouring outputs read the same inputs
    with pytest.raises(F.FilarkError):
        f.process(torch.zeros((100, 9), device="cuda"))
    with pytest.raises(F.FilarkError):
        f.set_tile(64, 4)
    with pytest.raises(F.FilarkError):
        f.set_tile(32, 4, 3)
    with pytest.raises(F.FilarkError):
        F.Fir(np.ones(64), 1 << 23)  # rows of 32 MiB: the taps' reach does not fit a launch


@pytest.mark.parametrize("M", [64, 100])
def test_long_window_default_tile_matches_fixed_tiles(F, M):
    """A 9000-row call (48-row waves by default at 64 taps, 32-row waves at
    100) against fixed 32- and 48-row tiles bit for bit and the oracle on
    sampled channels."""
    orc = _orc()
    h = _taps(M, "sinc", 3)
    n_ch, n_t = 200, 9000
    g = torch.Generator(device="cuda").manual_seed(700 + M)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    y = F.Fir(h, n_ch).process(x)
    for rows in (32, 48):
        f = F.Fir(h, n_ch)
        f.set_tile(rows, 1, 2)
        assert torch.equal(f.process(x), y)
    torch.cuda.synchronize()
    cols = [0, 63, 64, 199]
    _check(y[:, cols].cpu().numpy(), x[:, cols].cpu().numpy(), h, orc)


def test_channel_limit_for_64_taps(F):
    """The largest channel count 64 taps allow (launch windows of 96 rows):
    a 100-row record in two chunks against the oracle on sampled channels."""
    orc = _orc()
    n_ch, M = 1_760_232, 64
    h = _taps(M, "sinc", 5)
    g = torch.Generator(device="cuda").manual_seed(14)
    x = torch.randn((100, n_ch), generator=g, device="cuda", dtype=torch.float32)
    f = F.Fir(h, n_ch)
    y = torch.cat([f.process(x[:30].contiguous()), f.process(x[30:].contiguous())])
    torch.cuda.synchronize()
    cols = np.array([0, 64, n_ch // 2, n_ch - 1])
    idx = torch.from_numpy(cols).cuda()
    _check(y.index_select(1, idx).cpu().numpy(), x.index_select(1, idx).cpu().numpy(), h, orc)
    with pytest.raises(F.FilarkError):
        f.set_tile(32, 2, 2)  # a second wave per workgroup needs 96 rows more
    del x, y
    torch.cuda.empty_cache()


def test_million_channels_over_several_launch_windows(F):
    """1,000,003 channels x 700 rows in two chunks: every launch window is a
    few hundred rows, so windows meet inside both chunks; sampled channels
    (each group edge, the ragged last group) against the oracle."""
    orc = _orc()
    n_ch, M = 1_000_003, 64
    h = _taps(M, "sinc", 0)
    g = torch.Generator(device="cuda").manual_seed(13)
    x = torch.randn((700, n_ch), generator=g, device="cuda", dtype=torch.float32)
    f = F.Fir(h, n_ch)
    y = torch.cat([f.process(x[:300].contiguous()), f.process(x[300:].contiguous())])
    torch.cuda.synchronize()
    cols = np.array([0, 1, 63, 64, 65, 500_000, 999_935, 999_936, n_ch - 2, n_ch - 1])
    idx = torch.from_numpy(cols).cuda()
    xs = x.index_select(1, idx).cpu().numpy()
    ys = y.index_select(1, idx).cpu().numpy()
    _check(ys, xs, h, orc)
    st = f.get_state()
    np.testing.assert_array_equal(st[:, cols], xs[700 - (M - 1):])
    del x, y
    torch.cuda.empty_cache()
