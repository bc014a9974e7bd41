"""GPU parity of the fused SOS + STA/LTA forward path against the FP64 oracle.

Every GPU result is compared element by element with the oracle run on the
exact FP32 input the GPU saw (upcast to FP64), using the oracle's own SOS
array for both sides.  Bar: per-channel relative RMS <= 1e-5 (1e-4 when a
pole lies within 1e-3 of the unit circle); GPU chunked vs GPU one-shot
<= 1e-6.  Shapes cover several workgroup tiles, ragged channel groups and
ragged time blocks, single-sample and empty chunks.
"""

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


def _oracle():
    import oracle

    return oracle


def run_gpu_chunks(F, sos, x, splits, nsta=None, nlta=None, fs=None, write_y=True, mode="fused"):
    n_t, n_ch = x.shape
    st = F.SOSState(sos, n_ch) if mode in ("fused", "sos") else None
    sl = F.StaLtaState(nsta / fs, nlta / fs, fs, n_ch) if mode in ("fused", "stalta") else None
    ys, cfs = [], []
    t0 = 0
    for n in splits:
        xc = x[t0:t0 + n].contiguous()
        if mode == "fused":
            y, cf = F.sos_stalta_process(st, sl, xc, write_y=write_y)
            ys.append(y)
            cfs.append(cf)
        elif mode == "sos":
            ys.append(st.process(xc))
        else:
            cfs.append(sl.process(xc))
        t0 += n
    torch.cuda.synchronize()
    if st is not None:
        st.check()
    if sl is not None:
        sl.check()
    y = torch.cat(ys).cpu().numpy() if ys and ys[0] is not None else None
    cf = torch.cat(cfs).cpu().numpy() if cfs else None
    return y, cf, st, sl


def test_config1_fused_chunked_matches_oracle(F):
    import synth

    orc = _oracle()
    w = synth.make_config1(device="cuda")
    sos = orc.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
    nsta, nlta = orc.window_samples(w.sta_s, w.fs), orc.window_samples(w.lta_s, w.fs)
    x = w.x
    y, cf, st, sl = run_gpu_chunks(F, sos, x, [w.chunk] * (x.shape[0] // w.chunk), nsta, nlta, w.fs)
    xh = x.cpu().numpy().astype(np.float64)
    s = orc.Stream(sos, x.shape[1], nsta, nlta)
    yo, cfo = s.process(xh)
    tol = tolerance_for(sos)
    ey, ec = max_rel_rms(y, yo), max_rel_rms(cf, cfo)
    print(f"config1: y rel-RMS {ey:.3e}  cf rel-RMS {ec:.3e}  tol {tol:g}")
    assert ey <= tol and ec <= tol
    assert np.all(cf[:nlta] == 0.0)
    # carried states after the record match the oracle's
    z = st.get_state()
    np.testing.assert_allclose(z, s.zi, rtol=1e-6, atol=1e-6 * np.abs(s.zi).max())
    slst, g = sl.get_state()
    assert g == x.shape[0]
    np.testing.assert_allclose(slst, s.st, rtol=1e-5)


def test_chunked_equals_one_shot_on_gpu(F):
    import synth

    orc = _oracle()
    w = synth.make_config1(device="cuda")
    sos = orc.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
    nsta, nlta = 250, 2500
    y1, cf1, _, _ = run_gpu_chunks(F, sos, w.x, [w.x.shape[0]], nsta, nlta, w.fs)
    y2, cf2, _, _ = run_gpu_chunks(F, sos, w.x, [1000] * 10, nsta, nlta, w.fs)
    y3, cf3, _, _ = run_gpu_chunks(F, sos, w.x, [1, 0, 127, 4000, 1, 5871], nsta, nlta, w.fs)
    for a, b in [(y1, y2), (y1, y3), (cf1, cf2), (cf1, cf3)]:
        assert max_rel_rms(b, a) <= 1e-6


@pytest.mark.parametrize("n_ch,splits", [
    (1, [1, 2, 3, 300]),
    (63, [129, 0, 1000]),
    (65, [31, 33, 4099]),
    (130, [1, 127, 128, 129, 255, 257]),
    (200, [5000]),
])
@pytest.mark.parametrize("order,btype,f1,f2,fs", [
    (8, "bandpass", 1.0, 100.0, 1500.0),
    (2, "lowpass", 30.0, 0.0, 200.0),
    (6, "bandpass", 2.0, 40.0, 100.0),
    (16, "bandpass", 5.0, 400.0, 2000.0),
    (5, "highpass", 3.0, 0.0, 500.0),
])
def test_ragged_shapes_and_orders(F, n_ch, splits, order, btype, f1, f2, fs):
    orc = _oracle()
    g = torch.Generator(device="cuda").manual_seed(1000 + n_ch + order)
    n_t = sum(splits)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    sos = orc.butter_sos(order, btype, f1, f2, fs)
    nsta, nlta = 20, 200
    y, cf, _, _ = run_gpu_chunks(F, sos, x, splits, nsta, nlta, fs)
    s = orc.Stream(sos, n_ch, nsta, nlta)
    yo, cfo = s.process(x.cpu().numpy().astype(np.float64))
    tol = tolerance_for(sos)
    assert max_rel_rms(y, yo) <= tol
    assert max_rel_rms(cf, cfo) <= tol


@pytest.mark.parametrize("order", [4, 8, 16])
def test_general_numerators(F, order):
    """Sections whose numerators are not [1, b1, 1] after the first take the
    general section step: moving gain between sections (the same transfer
    function) must still give the oracle's result, for every tile block."""
    orc = _oracle()
    sos = orc.butter_sos(order, "bandpass", 2.0, 80.0, 1000.0).copy()
    sos[0, :3] *= 4.0
    sos[1, :3] *= 0.25  # b0 = b2 = 0.25 in section 2
    g = torch.Generator(device="cuda").manual_seed(77 + order)
    n_ch, splits = 70, [600, 1, 1399]
    x = torch.randn((sum(splits), n_ch), generator=g, device="cuda", dtype=torch.float32)
    s = orc.Stream(sos, n_ch, 20, 200)
    yo, cfo = s.process(x.cpu().numpy().astype(np.float64))
    for block in (32, 48, 64):
        st = F.SOSState(sos, n_ch)
        sl = F.StaLtaState(20 / 1000.0, 200 / 1000.0, 1000.0, n_ch)
        st.set_tile(block, 4, 8)
        sl.set_tile(block, 4, 8)
        ys, cfs, t0 = [], [], 0
        for n in splits:
            y, cf = F.sos_stalta_process(st, sl, x[t0:t0 + n].contiguous())
            ys.append(y)
            cfs.append(cf)
            t0 += n
        torch.cuda.synchronize()
        st.check()
        assert max_rel_rms(torch.cat(ys).cpu().numpy(), yo) <= tolerance_for(sos)
        assert max_rel_rms(torch.cat(cfs).cpu().numpy(), cfo) <= tolerance_for(sos)


@pytest.mark.parametrize("n_ch,splits", [(64, [1000, 1000, 1]), (100, [7, 700, 77])])
def test_sos_only_and_stalta_only_entries(F, n_ch, splits):
    orc = _oracle()
    g = torch.Generator(device="cuda").manual_seed(7)
    n_t = sum(splits)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    y, _, _, _ = run_gpu_chunks(F, sos, x, splits, mode="sos")
    yo, _ = orc.sos_filter(sos, x.cpu().numpy())
    assert max_rel_rms(y, yo) <= 1e-5
    # STA/LTA alone on an already filtered FP32 signal
    yin = torch.from_numpy(yo.astype(np.float32)).cuda()
    _, cf, _, _ = run_gpu_chunks(F, None, yin, splits, 25, 250, 500.0, mode="stalta")
    cfo, _, _ = orc.stalta(yin.cpu().numpy().astype(np.float64), 25, 250)
    assert max_rel_rms(cf, cfo) <= 1e-5


def test_in_place_and_without_y(F):
    orc = _oracle()
    g = torch.Generator(device="cuda").manual_seed(8)
    x = torch.randn((3000, 96), generator=g, device="cuda", dtype=torch.float32)
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    yo, _ = orc.sos_filter(sos, x.cpu().numpy())
    buf = x.clone()
    st = F.SOSState(sos, 96)
    st.process(buf, out=buf)
    torch.cuda.synchronize()
    assert max_rel_rms(buf.cpu().numpy(), yo) <= 1e-5
    _, cf_a, _, _ = run_gpu_chunks(F, sos, x, [1500, 1500], 300, 3000, 1500.0, write_y=False)
    _, cf_b, _, _ = run_gpu_chunks(F, sos, x, [1500, 1500], 300, 3000, 1500.0, write_y=True)
    assert np.array_equal(cf_a, cf_b)


def test_state_set_from_oracle_and_resume(F):
    """Snapshot/restore: a fresh state object loaded with the oracle's state at
    a chunk boundary continues exactly like the uninterrupted run."""
    orc = _oracle()
    g = torch.Generator(device="cuda").manual_seed(9)
    n_ch = 70
    x = torch.randn((4000, n_ch), generator=g, device="cuda", dtype=torch.float32)
    xh = x.cpu().numpy().astype(np.float64)
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    s = orc.Stream(sos, n_ch, 30, 300)
    s.process(xh[:1700])
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(30 / 1500.0, 300 / 1500.0, 1500.0, n_ch)
    st.set_state(s.zi)
    sl.set_state(s.st, s.g)
    y, cf = F.sos_stalta_process(st, sl, x[1700:].contiguous())
    torch.cuda.synchronize()
    yo, cfo = s.process(xh[1700:])
    assert max_rel_rms(y.cpu().numpy(), yo) <= 1e-5
    assert max_rel_rms(cf.cpu().numpy(), cfo) <= 1e-5
    z = st.get_state()
    np.testing.assert_allclose(z, s.zi, rtol=1e-6, atol=1e-6 * np.abs(s.zi).max())
    # a GPU snapshot restored into another object continues bit for bit (the
    # snapshot is exact FP64 and the kernels are deterministic)
    st2 = F.SOSState(sos, n_ch)
    st2.set_state(z)
    sl2 = F.StaLtaState(30 / 1500.0, 300 / 1500.0, 1500.0, n_ch)
    a, c = sl.get_state()
    sl2.set_state(a, c)
    more = torch.randn((500, n_ch), generator=g, device="cuda", dtype=torch.float32)
    y1, cf1 = F.sos_stalta_process(st, sl, more)
    y2, cf2 = F.sos_stalta_process(st2, sl2, more)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y1.cpu().numpy(), y2.cpu().numpy())
    np.testing.assert_array_equal(cf1.cpu().numpy(), cf2.cpu().numpy())


def test_near_unit_circle_highpass(F):
    import synth

    orc = _oracle()
    w = synth.make_config3(device="cuda", n_ch=96, n_t=30_000)
    sos = orc.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
    assert tolerance_for(sos) == 1e-4
    y, _, _, _ = run_gpu_chunks(F, sos, w.x, [10_000] * 3, mode="sos")
    yo, _ = orc.sos_filter(sos, w.x.cpu().numpy())
    e = max_rel_rms(y, yo)
    print(f"near-unit-circle highpass: y rel-RMS {e:.3e}")
    assert e <= 1e-4


def test_run_to_run_reproducibility(F):
    """Carries never cross workgroups and every reduction has a fixed order,
    so two runs give identical bits."""
    orc = _oracle()
    g = torch.Generator(device="cuda").manual_seed(10)
    x = torch.randn((6000, 500), generator=g, device="cuda", dtype=torch.float32)
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    a = run_gpu_chunks(F, sos, x, [1500] * 4, 300, 3000, 1500.0)
    b = run_gpu_chunks(F, sos, x, [1500] * 4, 300, 3000, 1500.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2].get_state(), b[2].get_state())
    sa, ga = a[3].get_state()
    sb, gb = b[3].get_state()
    assert np.array_equal(sa, sb) and ga == gb == 6000


def test_shape_errors(F):
    orc = _oracle()
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    st = F.SOSState(sos, 64)
    x = torch.zeros((10, 65), device="cuda")
    with pytest.raises(F.FilarkError) as e:
        st.process(x)
    assert e.value.status == F.ESHAPE
    st.process(torch.zeros((0, 64), device="cuda"))  # empty chunk is a no-op
    with pytest.raises(F.FilarkError):
        F.SOSState(np.array([[1.0, 0, 0, 1.0, -2.0, 1.0]]), 4)  # double pole at z = 1


@pytest.mark.parametrize("block", [32, 48, 64])
@pytest.mark.parametrize("waves", [1, 3, 8])
@pytest.mark.parametrize("group", [4, 8, 16, 64])
def test_tile_shapes(F, block, waves, group):
    """Every tile shape gives the oracle's result (ragged channels, chunks
    shorter and longer than a window, which then runs as several launches)."""
    orc = _oracle()
    g = torch.Generator(device="cuda").manual_seed(11 + block + waves + group)
    n_ch, splits = 131, [1, 700, 1999, 2]
    x = torch.randn((sum(splits), n_ch), generator=g, device="cuda", dtype=torch.float32)
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(30 / 1500.0, 300 / 1500.0, 1500.0, n_ch)
    st.set_tile(block, waves, group)
    sl.set_tile(block, waves, group)
    assert st.tile() == (block, waves, group) and sl.tile() == (block, waves, group)
    ys, cfs, t0 = [], [], 0
    for n in splits:
        y, cf = F.sos_stalta_process(st, sl, x[t0:t0 + n].contiguous())
        ys.append(y)
        cfs.append(cf)
        t0 += n
    torch.cuda.synchronize()
    st.check()
    sl.check()
    s = orc.Stream(sos, n_ch, 30, 300)
    yo, cfo = s.process(x.cpu().numpy().astype(np.float64))
    assert max_rel_rms(torch.cat(ys).cpu().numpy(), yo) <= 1e-5
    assert max_rel_rms(torch.cat(cfs).cpu().numpy(), cfo) <= 1e-5
    np.testing.assert_allclose(st.get_state(), s.zi, rtol=1e-6, atol=1e-6 * np.abs(s.zi).max())
    slst, gg = sl.get_state()
    assert gg == sum(splits)
    np.testing.assert_allclose(slst, s.st, rtol=1e-6)


def test_tile_shape_errors(F):
    orc = _oracle()
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    st = F.SOSState(sos, 64)
    sl = F.StaLtaState(0.1, 1.0, 500.0, 64)
    for b, w, gr in [(16, 4, 8), (64, 0, 8), (64, 9, 8), (40, 2, 8), (64, 2, 3), (64, 2, 128)]:
        with pytest.raises(F.FilarkError) as e:
            st.set_tile(b, w, gr)
        assert e.value.status == F.EINVAL
    st.set_tile(32, 2, 8)
    with pytest.raises(F.FilarkError) as e:  # fused call needs equal shapes
        F.sos_stalta_process(st, sl, torch.zeros((10, 64), device="cuda"))
    assert e.value.status == F.EINVAL
