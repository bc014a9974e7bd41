"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (default tiles, one call per chunk, state carried).

* 6000 ch x 90,000 samples, 60 chunks of 1500, fused SOS (8th-order 1-100 Hz
  bandpass) + STA/LTA 0.2 s / 2 s: y, cf and the final states of sampled
  channels (both ends of the channel range, group boundaries, random ones)
  against the oracle run on those channels' exact FP32 input.
* 2000 ch x 100,000 samples at 10 kHz, 10 chunks of 10,000 (several windows
  per chunk), 16th-order highpass at 0.5 Hz (poles within 1e-3 of the unit
  circle, tolerance 1e-4): sampled channels against the oracle.
* 6000 ch x 30,000 samples, 10 chunks of 3000: forward with per-chunk device
  checkpoints, then the adjoint chunk by chunk in reverse, loss mean
  (cf - target)^2 with the target the oracle's cf of the filter designed at
  (1.05 f1, 0.95 f2); dL/dx of every channel and dL/dtheta against the
  oracle's reference gradient over the whole record.
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

    oracle.set_num_threads(max(1, min(16, len(__import__("os").sched_getaffinity(0)))))
    return oracle


def _sample_channels(n_ch, seed, n_random=10):
    rng = np.random.default_rng(seed)
    fixed = [0, 1, 7, 8, 9, n_ch // 2, n_ch - 2, n_ch - 1]
    return sorted(set(fixed) | set(int(c) for c in rng.choice(n_ch, n_random, replace=False)))


def test_config2_full_size_fused(F):
    import synth

    orc = _oracle()
    w = synth.make_config2(device="cuda")
    x = w.x
    n_t, n_ch = x.shape
    assert (n_t, n_ch, w.chunk) == (90_000, 6000, 1500)
    sos = orc.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
    nsta, nlta = orc.window_samples(w.sta_s, w.fs), orc.window_samples(w.lta_s, w.fs)
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(w.sta_s, w.lta_s, w.fs, n_ch)
    y = torch.empty_like(x)
    cf = torch.empty_like(x)
    for a in range(0, n_t, w.chunk):
        F.sos_stalta_process(st, sl, x[a:a + w.chunk], y[a:a + w.chunk], cf[a:a + w.chunk])
    torch.cuda.synchronize()
    st.check()
    sl.check()
    cols = _sample_channels(n_ch, 1)
    xs = x[:, cols].cpu().numpy()
    yo, zo = orc.sos_filter(sos, xs)
    cfo, slo, go = orc.stalta(yo, nsta, nlta)
    ey = max_rel_rms(y[:, cols].cpu().numpy(), yo)
    ec = max_rel_rms(cf[:, cols].cpu().numpy(), cfo)
    print(f"6000 x 90000 fused: y {ey:.2e} cf {ec:.2e} on {len(cols)} channels")
    assert ey <= tolerance_for(sos)
    assert ec <= 1e-5
    z = st.get_state()[cols]
    np.testing.assert_allclose(z, zo, rtol=1e-6, atol=1e-6 * np.abs(zo).max())
    s, g = sl.get_state()
    assert g == go == n_t
    np.testing.assert_allclose(s[cols], slo, rtol=1e-6)


def test_config3_full_size_near_unit_circle(F):
    import synth

    orc = _oracle()
    w = synth.make_config3(device="cuda")
    x = w.x
    n_t, n_ch = x.shape
    assert (n_t, n_ch, w.chunk) == (100_000, 2000, 10_000)
    sos = orc.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
    assert sos.shape[0] == 8 and tolerance_for(sos) == 1e-4
    st = F.SOSState(sos, n_ch)
    y = torch.empty_like(x)
    for a in range(0, n_t, w.chunk):
        st.process(x[a:a + w.chunk], y[a:a + w.chunk])
    torch.cuda.synchronize()
    st.check()
    cols = _sample_channels(n_ch, 2)
    yo, zo = orc.sos_filter(sos, x[:, cols].cpu().numpy())
    e = max_rel_rms(y[:, cols].cpu().numpy(), yo)
    print(f"2000 x 100000 highpass K=8: y {e:.2e} on {len(cols)} channels")
    assert e <= 1e-4


def test_config5_full_size_forward_adjoint(F):
    import synth

    orc = _oracle()
    w = synth.make_config5(device="cuda")
    x = w.x
    n_t, n_ch = x.shape
    assert (n_t, n_ch, w.chunk) == (30_000, 6000, 3000)
    sos = orc.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
    nsta, nlta = orc.window_samples(w.sta_s, w.fs), orc.window_samples(w.lta_s, w.fs)
    xh = x.cpu().numpy().astype(np.float64)
    # target: the oracle's cf of the filter designed at (1.05 f1, 0.95 f2)
    sos_t = orc.butter_sos(w.order, w.btype, 1.05 * w.f1, 0.95 * w.f2, w.fs)
    tgt_h, _, _ = orc.stalta(orc.sos_filter(sos_t, xh)[0], nsta, nlta)
    tgt = torch.from_numpy(tgt_h.astype(np.float32)).to("cuda")
    scale = 1.0 / (n_ch * n_t)

    K = sos.shape[0]
    tq = tgt.cpu().numpy().astype(np.float64)  # the exact target the GPU saw
    _, ogx, ogs, _ = orc.stalta_grad(sos, xh, tq, nsta, nlta, scale)
    # both ways into the adjoint: state checkpoints per chunk, and the
    # forward's tape (the path the benchmark times)
    for path in ("checkpoints", "tape"):
        st = F.SOSState(sos, n_ch)
        sl = F.StaLtaState(w.sta_s, w.lta_s, w.fs, n_ch)
        cks = []
        for a in range(0, n_t, w.chunk):
            if path == "tape":
                cks.append(F.sos_stalta_process_tape(st, sl, x[a:a + w.chunk])[2])
            else:
                cks.append((st.save(), sl.save()))
                F.sos_stalta_process(st, sl, x[a:a + w.chunk], write_y=False)
        gx = torch.empty_like(x)
        adj = torch.zeros((2 * K + 2, n_ch), dtype=torch.float64, device="cuda")
        gs = torch.zeros((K, 5), dtype=torch.float64, device="cuda")
        for i in reversed(range(len(cks))):
            a = i * w.chunk
            if path == "tape":
                F.sos_stalta_adjoint_tape(st, sl, cks[i], x[a:a + w.chunk], tgt[a:a + w.chunk], gx[a:a + w.chunk],
                                          adj, gs, mode="mse", scale=scale)
            else:
                st.load(cks[i][0])
                sl.load(cks[i][1])
                F.sos_stalta_adjoint(st, sl, x[a:a + w.chunk], tgt[a:a + w.chunk], gx[a:a + w.chunk], adj, gs,
                                     mode="mse", scale=scale)
        torch.cuda.synchronize()
        st.check()
        ex = max_rel_rms(gx.cpu().numpy(), ogx)
        es = float(np.linalg.norm(gs.cpu().numpy() - ogs) / np.linalg.norm(ogs))
        print(f"6000 x 30000 fwd+adjoint ({path}): dL/dx {ex:.2e} dL/dtheta {es:.2e}")
        assert ex <= 1e-5
        assert es <= 1e-5
        st.close()
        sl.close()
        del cks, gx
