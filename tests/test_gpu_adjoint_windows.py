"""GPU: several adjoint windows in one launch against one launch per window.

With the default adjoint tile and a Butterworth-shaped cascade the full
windows of a chunk run in one launch of the several-window kernel (the
adjoint state passes between windows in LDS, the next window's input is
prefetched into LDS).  Its arithmetic, and the order of it, is that of one
launch per window, so dL/dx, the adjoint state and the coefficient
gradients must be bit-identical for every cap on windows per launch
(filark_adjoint_windows_set: 1 = one launch per window, 2 = runs of two,
0 = no cap), on the tape path and on the checkpoint path, and within the
oracle's gradient bars (1e-5 relative, as the other adjoint tests).
Shapes: chunks of whole windows, with a partial last window, of one window
and just over one; 24 to 1003 channels (a ragged last channel group);
cascades of 2 to 8 sections (the several-window kernel takes 2 to 4).
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


def _adjoint(F, sos, x, tgt, nsta, nlta, mode, scale, tape, cap, splits):
    n_t, n_ch = x.shape
    K = sos.shape[0]
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
    st.set_adjoint_windows(cap)
    saved = []
    for a, b in splits:
        if tape:
            saved.append(F.sos_stalta_process_tape(st, sl, x[a:b].contiguous())[2])
        else:
            saved.append((st.save(), sl.save()))
            F.sos_stalta_process(st, sl, x[a:b].contiguous(), write_y=False)
    gx = torch.empty_like(x)
    adj = torch.zeros((2 * K + 2, n_ch), dtype=torch.float64, device="cuda")
    gs = torch.zeros((K, 5), dtype=torch.float64, device="cuda")
    for (a, b), sv in reversed(list(zip(splits, saved))):
        ga = torch.empty((b - a, n_ch), dtype=torch.float32, device="cuda")
        if tape:
            F.sos_stalta_adjoint_tape(st, sl, sv, x[a:b].contiguous(), tgt[a:b].contiguous(), ga, adj, gs,
                                      mode=mode, scale=scale)
        else:
            st.load(sv[0])
            sl.load(sv[1])
            F.sos_stalta_adjoint(st, sl, x[a:b].contiguous(), tgt[a:b].contiguous(), ga, adj, gs, mode=mode,
                                 scale=scale)
        gx[a:b] = ga
    torch.cuda.synchronize()
    st.check()
    return gx.cpu().numpy(), adj.cpu().numpy(), gs.cpu().numpy()


@pytest.mark.parametrize("tape", [True, False])
@pytest.mark.parametrize("n_ch,splits", [
    (24, [(0, 2048)]),                 # four whole windows
    (37, [(0, 2600)]),                 # five whole windows and a partial one
    (1003, [(0, 1537), (1537, 3584)]),  # three windows and one row; four whole windows
    (64, [(0, 512), (512, 1024)]),     # one window per chunk
])
def test_windows_per_launch_bit_identical(F, tape, n_ch, splits):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    nsta, nlta = 30, 300
    n_t = splits[-1][1]
    g = torch.Generator(device="cuda").manual_seed(n_ch + n_t)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    tgt = torch.rand((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32) * 3.0
    scale = 1.0 / x.numel()
    ref = _adjoint(F, sos, x, tgt, nsta, nlta, "mse", scale, tape, 1, splits)
    for cap in (2, 0):
        got = _adjoint(F, sos, x, tgt, nsta, nlta, "mse", scale, tape, cap, splits)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
    # the oracle's one-shot gradient, on every channel or on sampled ones
    cols = np.arange(n_ch) if n_ch < 100 else np.array([0, 7, 8, 500, n_ch - 1])
    gx, adj, gs = ref
    xh = x.cpu().numpy().astype(np.float64)[:, cols]
    th = tgt.cpu().numpy().astype(np.float64)[:, cols]
    _, ogx, ogs, oadj = orc.stalta_grad(sos, xh, th, nsta, nlta, scale)
    assert max_rel_rms(gx[:, cols], ogx) <= 1e-5
    assert float(np.max(np.abs(adj.T[cols] - oadj)) / np.max(np.abs(oadj))) <= 1e-6
    if len(cols) == n_ch:
        assert float(np.linalg.norm(gs - ogs) / np.linalg.norm(ogs)) <= 1e-5


@pytest.mark.parametrize("order,btype,f1,f2,fs", [
    (4, "lowpass", 30.0, 0.0, 200.0),       # 2 sections
    (6, "bandpass", 2.0, 60.0, 500.0),      # 3 sections
    (10, "bandpass", 2.0, 60.0, 500.0),     # 5 sections: one launch per window (the cap is moot)
    (16, "bandpass", 5.0, 400.0, 2000.0),   # 8 sections: likewise
])
def test_windows_per_launch_other_orders(F, order, btype, f1, f2, fs):
    """The several-window kernel for the other section counts it is built
    for (2 to 4; longer cascades run one launch per window): bit for bit
    against one launch per window, and the oracle's bars."""
    orc = _orc()
    sos = orc.butter_sos(order, btype, f1, f2, fs)
    n_ch, nsta, nlta = 29, 15, 150
    splits = [(0, 3 * 512 + 100)]
    n_t = splits[-1][1]
    g = torch.Generator(device="cuda").manual_seed(order)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    tgt = torch.rand((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32) * 3.0
    scale = 1.0 / x.numel()
    for tape in (True, False):
        ref = _adjoint(F, sos, x, tgt, nsta, nlta, "mse", scale, tape, 1, splits)
        got = _adjoint(F, sos, x, tgt, nsta, nlta, "mse", scale, tape, 0, splits)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
    gx, adj, gs = ref
    xh = x.cpu().numpy().astype(np.float64)
    th = tgt.cpu().numpy().astype(np.float64)
    _, ogx, ogs, oadj = orc.stalta_grad(sos, xh, th, nsta, nlta, scale)
    assert max_rel_rms(gx, ogx) <= 1e-5
    assert float(np.linalg.norm(gs - ogs) / np.linalg.norm(ogs)) <= 1e-5
    assert float(np.max(np.abs(adj.T - oadj)) / np.max(np.abs(oadj))) <= 1e-6


def test_windows_per_launch_grad_mode(F):
    """dL/dcf handed in (mode grad) instead of a target: several windows per
    launch against one per window, bit for bit."""
    orc = _orc()
    sos = orc.butter_sos(6, "bandpass", 2.0, 40.0, 500.0)
    n_ch, n_t = 40, 3000
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    dcf = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    splits = [(0, n_t)]
    ref = _adjoint(F, sos, x, dcf, 20, 200, "grad", 1.0, True, 1, splits)
    got = _adjoint(F, sos, x, dcf, 20, 200, "grad", 1.0, True, 0, splits)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    xh = x.cpu().numpy().astype(np.float64)
    y, _ = orc.sos_filter(sos, xh)
    # dL/dcf = dcf: the gradient of sum(dcf * cf); the oracle's gradient of
    # that linear loss comes from its mse form with the target cf - dcf / 2
    ocf, _, _ = orc.stalta(y, 20, 200)
    th = ocf - 0.5 * dcf.cpu().numpy().astype(np.float64)
    _, ogx, ogs, _ = orc.stalta_grad(sos, xh, th, 20, 200, 1.0)
    assert max_rel_rms(ref[0], ogx) <= 1e-5
    assert float(np.linalg.norm(ref[2] - ogs) / np.linalg.norm(ogs)) <= 1e-5


def test_windows_cap_rejects_negative(F):
    orc = _orc()
    st = F.SOSState(orc.butter_sos(4, "lowpass", 10.0, 0.0, 100.0), 8)
    with pytest.raises(F.FilarkError):
        st.set_adjoint_windows(-1)
