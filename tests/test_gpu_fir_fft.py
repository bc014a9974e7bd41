"""GPU parity of the FIR's FFT method (overlap-save blocks of 2049 - M rows
from 2048-row windows, Table 1's overlap-add row) against the oracle's direct
convolution on the exact FP32 input the GPU saw (upcast).

Bar.  The FFT path rounds differently from the direct sum, so the bar is an
FFT error bound rather than the FMA bound of the direct kernel.  For one
block of one channel, with x_w the block's 2048-row window (history rows
included, zeros past the chunk) and H the taps' unnormalised 2048-point
spectrum, the exact circular convolution has 2-norm at most max|H| ||x_w||_2
(Parseval).  A radix-2-equivalent FFT of n points in precision u with
twiddles accurate to u has relative 2-norm error at most log2(n) eta / (1 -
log2(n) eta), eta = u + gamma_4 (sqrt 2 + u) < 7u (Higham, Accuracy and
Stability of Numerical Algorithms, Thm 24.2).  Forward and inverse 1024-point
transforms (10 levels each), plus the unpacking, the product with H rounded
to FP32 and the repacking (under 16u together), give

    || y_gpu - y_exact ||_2 over the block's rows  <=  (2 * 10 * 7 + 16) u max|H| ||x_w||_2,

u = 2^-24, checked block by block and channel by channel.  Beyond parity:
the carried history is the last M - 1 input rows exactly (a copy), shared
with the direct method, so a stream can switch methods between calls.
Shapes: one sample, ragged channel groups (not multiples of 8), ragged last
blocks, chunks shorter than the history, 1 to 1024 taps.
"""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_FFT = 2048
C_BOUND = 2 * 10 * 7 + 16


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
    n = np.arange(M) - (M - 1) / 2
    return 0.5 * np.sinc(0.5 * n) * np.hamming(M) if M > 1 else np.ones(1)


def _check(y, x, h, hist=None):
    """y (GPU, [n_t, n_ch]) against the oracle from history `hist` (zeros by
    default), block by block within the FFT bound; returns the oracle object
    (its history is the exact new state)."""
    orc = _orc()
    n_t, n_ch = x.shape
    M = len(h)
    h32 = h.astype(np.float32).astype(np.float64)  # the taps the GPU applies
    f = orc.Fir(h32, n_ch)
    hm = M - 1
    if hist is None:
        hist = np.zeros((hm, n_ch))
    f.hist[:] = hist
    xd = x.astype(np.float64)
    ref = f.process(xd)
    maxH = np.max(np.abs(np.fft.fft(h32, N_FFT)))
    full = np.concatenate([hist, xd, np.zeros((N_FFT, n_ch))])  # row t of the chunk at t + hm
    B = N_FFT - hm
    err = (y.astype(np.float64) - ref)
    worst = 0.0
    for t0 in range(0, n_t, B):
        t1 = min(n_t, t0 + B)
        win = full[t0:t0 + N_FFT]
        bound = C_BOUND * 2.0 ** -24 * maxH * np.linalg.norm(win, axis=0) + 1e-37
        e = np.linalg.norm(err[t0:t1], axis=0)
        worst = max(worst, float(np.max(e / bound)))
        assert np.all(e <= bound), f"block at row {t0}: max err/bound {np.max(e / bound):.3g}"
    return f, worst


@pytest.mark.parametrize("n_ch,n_t", [(1, 1), (7, 100), (13, 2049), (300, 5000)])
@pytest.mark.parametrize("M,kind", [(1, "random"), (2, "random"), (64, "sinc"), (256, "random"), (1023, "sinc"),
                                    (1024, "random")])
def test_fft_matches_oracle(F, n_ch, n_t, M, kind):
    h = _taps(M, kind, M)
    g = torch.Generator(device="cuda").manual_seed(900 + n_ch + M)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    f = F.Fir(h, n_ch)
    f.set_method("fft")
    y = f.process(x)
    torch.cuda.synchronize()
    of, _ = _check(y.cpu().numpy(), x.cpu().numpy(), h)
    if M > 1:
        np.testing.assert_array_equal(f.get_state(), of.hist.astype(np.float32))
    f.close()


@pytest.mark.parametrize("M", [2, 64, 1024])
def test_fft_chunked_carries_history(F, M):
    """Chunks of 0, 1, a few, M - 1 and several blocks' rows: each chunk
    against the oracle continued from the previous chunk's history, and the
    history after each call the exact last M - 1 rows."""
    n_ch = 45
    h = _taps(M, "sinc", 1)
    g = torch.Generator(device="cuda").manual_seed(31 + M)
    sizes = [0, 1, 5, M - 1, 0, 3 * N_FFT + 17, 1, 700]
    x = torch.randn((sum(sizes), n_ch), generator=g, device="cuda", dtype=torch.float32)
    f = F.Fir(h, n_ch)
    f.set_method("fft")
    hist = np.zeros((M - 1, n_ch))
    t = 0
    for n in sizes:
        xc = x[t:t + n].contiguous()
        y = f.process(xc)
        torch.cuda.synchronize()
        if n:
            of, _ = _check(y.cpu().numpy(), xc.cpu().numpy(), h, hist)
            hist = of.hist.copy()
        np.testing.assert_array_equal(f.get_state(), hist.astype(np.float32))
        t += n


def test_method_switch_shares_the_history(F):
    """direct -> fft -> direct: the FFT call leaves the same history as the
    direct one would, so the third call's output equals a direct-only
    object's bit for bit."""
    M, n_ch = 128, 77
    h = _taps(M, "random", 2)
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((3000, n_ch), generator=g, device="cuda", dtype=torch.float32)
    cuts = [(0, 1000), (1000, 2500), (2500, 3000)]
    ref = F.Fir(h, n_ch)
    yr = [ref.process(x[a:b].contiguous()) for a, b in cuts]
    f = F.Fir(h, n_ch)
    y0 = f.process(x[0:1000].contiguous())
    f.set_method("fft")
    y1 = f.process(x[1000:2500].contiguous())
    f.set_method("direct")
    y2 = f.process(x[2500:3000].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(y0, yr[0])
    assert torch.equal(y2, yr[2])
    _check(y1.cpu().numpy(), x[1000:2500].cpu().numpy(), h, x[1000 - (M - 1):1000].double().cpu().numpy())
    np.testing.assert_array_equal(f.get_state(), ref.get_state())


def test_fft_graph_replays_carry_history(F):
    """The FFT call captured in a HIP graph, replayed over successive chunks
    with eager work in between: every replay equals an eager FFT object's
    call bit for bit (the same kernels on the same bits)."""
    M, n_ch, chunk = 200, 40, 3000
    h = _taps(M, "sinc", 0)
    g0 = torch.Generator(device="cuda").manual_seed(23)
    x = torch.randn((5 * chunk, n_ch), generator=g0, device="cuda", dtype=torch.float32)
    f, ref = F.Fir(h, n_ch), F.Fir(h, n_ch)
    f.set_method("fft")
    ref.set_method("fft")
    xs, ys = torch.empty((chunk, n_ch), device="cuda"), torch.empty((chunk, n_ch), device="cuda")
    xs.copy_(x[:chunk])
    f.process(xs, ys)
    r0 = ref.process(x[:chunk].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(ys, r0)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            f.process(xs, ys, stream=s)
    torch.cuda.synchronize()
    for i in range(1, 5):
        xs.copy_(x[i * chunk:(i + 1) * chunk])
        g.replay()
        r = ref.process(x[i * chunk:(i + 1) * chunk].contiguous())
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(ys, r), f"replay {i}"
        np.testing.assert_array_equal(f.get_state(), ref.get_state())


def test_fft_many_channels_sampled(F):
    """100,003 channels x 6000 rows (ragged last group and block) in two
    chunks, sampled channels at group edges against the oracle."""
    M, n_ch = 512, 100_003
    h = _taps(M, "sinc", 4)
    g = torch.Generator(device="cuda").manual_seed(17)
    x = torch.randn((6000, n_ch), generator=g, device="cuda", dtype=torch.float32)
    f = F.Fir(h, n_ch)
    f.set_method("fft")
    y = torch.cat([f.process(x[:2500].contiguous()), f.process(x[2500:].contiguous())])
    torch.cuda.synchronize()
    cols = np.array([0, 7, 8, 50_000, 99_999, 100_000, n_ch - 1])
    idx = torch.from_numpy(cols).cuda()
    xs = x.index_select(1, idx).cpu().numpy()
    ys = y.index_select(1, idx).cpu().numpy()
    _check(ys, xs, h)
    np.testing.assert_array_equal(f.get_state()[:, cols], xs[6000 - (M - 1):])
    del x, y
    torch.cuda.empty_cache()


def test_fft_errors(F):
    import ctypes

    f = F.Fir(_taps(1024, "sinc", 0), 1)
    f.set_method("fft")
    with pytest.raises(KeyError):
        f.set_method("overlap")
    x = torch.zeros((4, 1), device="cuda")
    # 65536 blocks of 1025 rows: refused on the host before any access
    n_t = 65536 * 1025
    st = F.lib().filark_fir_process(f._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr() + (1 << 40)),
                                    ctypes.c_int64(1), ctypes.c_int64(n_t), None)
    assert st != 0
    assert math.isfinite(float(f.process(x).sum()))
