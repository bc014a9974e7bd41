"""GPU parity of the adjoint with a tape (the forward records the state at
every adjoint window start; the adjoint reads it instead of rerunning a
forward pass or restoring checkpoints).

Bars as for the plain adjoint (gradient tolerance reading: 1e-5 relative):
dL/dx per-channel relative RMS <= 1e-5 and the coefficient gradient relative
L2 <= 1e-5 against the oracle's one-shot gradient, the adjoint state handed
back within 1e-6 of its scale; the forward's cf within 1e-5 (per-channel
relative RMS) of the oracle's.  Against the plain adjoint path on the same
data: the tape's forward runs 64-row blocks where the plain forward runs
48-row blocks, so the chunk states differ by the rounding of the block scan
(measured 1e-8 of the state's scale for this bandpass, whose 1 Hz poles sit
close to the unit circle); the end state, the coefficient gradients and the
adjoint state are held to 1e-6 of their scale and dL/dx to 2e-7 per-channel
relative RMS: tighter than the oracle bars, which remain the parity bar.
Shapes: 24 to 4100 channels (ragged channel groups), chunks shorter than one
adjoint window, of one row, longer than the tape forward's 2048-row launch
window, and ragged.
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


def _run(F, x, tgt, sos, nsta, nlta, splits, scale, tape: bool):
    n_t, n_ch = x.shape
    K = sos.shape[0]
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
    cf = torch.empty_like(x)
    saved = []
    for a, b in splits:
        if tape:
            _, _, tp = F.sos_stalta_process_tape(st, sl, x[a:b].contiguous(), cf=cf[a:b])
            saved.append(tp)
        else:
            saved.append((st.save(), sl.save()))
            F.sos_stalta_process(st, sl, x[a:b].contiguous(), cf=cf[a:b], write_y=False)
    zend = st.get_state()
    gx = torch.empty_like(x)
    adj = torch.zeros((2 * K + 2, n_ch), dtype=torch.float64, device="cuda")
    gs = torch.zeros((K, 5), dtype=torch.float64, device="cuda")
    for (a, b), sv in reversed(list(zip(splits, saved))):
        ga = torch.empty((b - a, n_ch), dtype=torch.float32, device="cuda")
        if tape:
            z_before = st.get_state()
            F.sos_stalta_adjoint_tape(st, sl, sv, x[a:b].contiguous(), tgt[a:b].contiguous(), ga, adj, gs,
                                      mode="mse", scale=scale)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(st.get_state(), z_before)  # the objects' state is not used
        else:
            st.load(sv[0])
            sl.load(sv[1])
            F.sos_stalta_adjoint(st, sl, x[a:b].contiguous(), tgt[a:b].contiguous(), ga, adj, gs, mode="mse",
                                 scale=scale)
        gx[a:b] = ga
    torch.cuda.synchronize()
    st.check()
    return cf.cpu().numpy(), zend, gx.cpu().numpy(), adj.cpu().numpy().T, gs.cpu().numpy()


@pytest.mark.parametrize("n_ch,splits", [
    (24, [(0, 1000), (1000, 1001), (1001, 2600), (2600, 3100)]),
    (37, [(0, 300), (300, 2348), (2348, 2350), (2350, 5000)]),
    (4100, [(0, 2048), (2048, 3000), (3000, 4500)]),
])
def test_tape_chain_matches_oracle_and_plain_adjoint(F, n_ch, splits):
    orc = _orc()
    nsta, nlta = 30, 300
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    n_t = splits[-1][1]
    g = torch.Generator(device="cuda").manual_seed(n_ch)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    tgt = torch.rand((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32) * 3.0
    scale = 1.0 / x.numel()
    cf, zend, gx, adj, gs = _run(F, x, tgt, sos, nsta, nlta, splits, scale, True)
    _, zend0, gx0, adj0, gs0 = _run(F, x, tgt, sos, nsta, nlta, splits, scale, False)
    # the oracle on every channel for small cases, else on sampled channels
    cols = np.arange(n_ch) if n_ch < 100 else np.array([0, 15, 16, 2047, n_ch - 1])
    xh = x.cpu().numpy().astype(np.float64)[:, cols]
    th = tgt.cpu().numpy().astype(np.float64)[:, cols]
    y, zo = orc.sos_filter(sos, xh)
    ocf, _, _ = orc.stalta(y, nsta, nlta)
    assert max_rel_rms(cf[:, cols], ocf) <= 1e-5
    np.testing.assert_allclose(zend[cols], zo, rtol=0, atol=1e-6 * np.max(np.abs(zo)))
    _, ogx, ogs, oadj = orc.stalta_grad(sos, xh, th, nsta, nlta, scale)
    assert max_rel_rms(gx[:, cols], ogx) <= 1e-5
    ea = float(np.max(np.abs(adj[cols] - oadj)) / np.max(np.abs(oadj)))
    assert ea <= 1e-6
    if len(cols) == n_ch:
        assert float(np.linalg.norm(gs - ogs) / np.linalg.norm(ogs)) <= 1e-5
    # against the plain path on the same data, every channel
    assert max_rel_rms(gx, gx0) <= 2e-7
    assert float(np.linalg.norm(gs - gs0) / np.linalg.norm(gs0)) <= 1e-6
    assert float(np.max(np.abs(adj - adj0)) / np.max(np.abs(adj0))) <= 1e-6
    np.testing.assert_allclose(zend, zend0, rtol=0, atol=1e-6 * np.max(np.abs(zend0)))


def _sos(kind):
    orc = _orc()
    if kind == "bp8":
        return orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    if kind == "gain_moved":  # later sections no longer [1, b1, 1]: the general section step
        sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0).copy()
        sos[0, :3] *= 8.0
        sos[2, :3] *= 0.125
        return sos
    if kind == "hp5":  # odd order: a first-order section among second-order ones
        return orc.butter_sos(5, "highpass", 3.0, 0.0, 500.0)
    return orc.butter_sos(2, "lowpass", 30.0, 0.0, 200.0)  # one section


@pytest.mark.parametrize("kind", ["gain_moved", "hp5", "lp2"])
def test_tape_chain_other_cascades(F, kind):
    """The tape path for the other kernel variants: general numerators, a
    first-order section (the rebuild's per-section test), one section; full
    and partial windows, against the oracle's one-shot gradient."""
    orc = _orc()
    sos = _sos(kind)
    n_ch, nsta, nlta = 29, 15, 150
    splits = [(0, 1024), (1024, 1030), (1030, 2200)]
    n_t = splits[-1][1]
    g = torch.Generator(device="cuda").manual_seed(77)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    tgt = torch.rand((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32) * 3.0
    scale = 1.0 / x.numel()
    cf, zend, gx, adj, gs = _run(F, x, tgt, sos, nsta, nlta, splits, scale, True)
    xh = x.cpu().numpy().astype(np.float64)
    th = tgt.cpu().numpy().astype(np.float64)
    y, zo = orc.sos_filter(sos, xh)
    ocf, _, _ = orc.stalta(y, nsta, nlta)
    assert max_rel_rms(cf, ocf) <= 1e-5
    _, ogx, ogs, oadj = orc.stalta_grad(sos, xh, th, nsta, nlta, scale)
    assert max_rel_rms(gx, ogx) <= 1e-5
    assert float(np.linalg.norm(gs - ogs) / np.linalg.norm(ogs)) <= 1e-5
    assert float(np.max(np.abs(adj - oadj)) / np.max(np.abs(oadj))) <= 1e-6


def test_tape_bytes_and_errors(F):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    n_ch = 10
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(20.0, 200.0, 1.0, n_ch)
    slot = (2 * 4 + 3) * n_ch * 8
    for n_t, n_win in ((1, 1), (512, 1), (513, 2), (3000, 6)):
        assert F.adjoint_tape_bytes(st, sl, n_t) == n_win * slot
    x = torch.zeros((100, n_ch), device="cuda")
    with pytest.raises(F.FilarkError):  # a tape too small
        F.sos_stalta_process_tape(st, sl, x, tape=torch.empty(10, dtype=torch.uint8, device="cuda"))
    # a tape written with 512-row windows, read after the adjoint tile moved
    # to 256-row windows: twice the slots are needed, so it is refused
    x2 = torch.zeros((1000, n_ch), device="cuda")
    _, _, tp = F.sos_stalta_process_tape(st, sl, x2)
    assert tp.numel() == 2 * slot
    st.set_adjoint_tile(8, 4, 8)
    sl.set_adjoint_tile(8, 4, 8)
    with pytest.raises(F.FilarkError):
        F.sos_stalta_adjoint_tape(st, sl, tp, x2, x2)
    st.set_adjoint_tile(16, 4, 8)
    sl.set_adjoint_tile(16, 4, 8)
    # 384-row adjoint windows do not divide the tape's 2048-row launch windows
    st.set_adjoint_tile(16, 3, 8)
    sl.set_adjoint_tile(16, 3, 8)
    with pytest.raises(F.FilarkError):
        F.adjoint_tape_bytes(st, sl, 1000)
    # 256-row windows do
    st.set_adjoint_tile(8, 4, 8)
    sl.set_adjoint_tile(8, 4, 8)
    assert F.adjoint_tape_bytes(st, sl, 1000) == 4 * slot
    # empty chunks: nothing is written or read, the state stays
    assert F.adjoint_tape_bytes(st, sl, 0) == 0
    tape = torch.full((slot,), 7, dtype=torch.uint8, device="cuda")
    z0 = st.get_state()
    F.sos_stalta_process_tape(st, sl, torch.zeros((0, n_ch), device="cuda"), tape=tape)
    gx, adj, gs = F.sos_stalta_adjoint_tape(st, sl, tape, torch.zeros((0, n_ch), device="cuda"),
                                            torch.zeros((0, n_ch), device="cuda"))
    torch.cuda.synchronize()
    assert bool((tape == 7).all()) and not adj.any() and not gs.any()
    np.testing.assert_array_equal(st.get_state(), z0)


def test_tape_step_in_a_graph(F):
    """A whole forward + adjoint step on the tape path (state reset, forward
    with tapes over every chunk, adjoint chain) captured in a HIP graph after
    one eager step, replayed three times with eager work in between: every
    replay equals the eager step bit for bit."""
    orc = _orc()
    sos = _sos("bp8")
    n_ch, nsta, nlta = 40, 30, 300
    splits = [(0, 1000), (1000, 2100), (2100, 2600)]
    n_t, K = splits[-1][1], sos.shape[0]
    g = torch.Generator(device="cuda").manual_seed(91)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    tgt = torch.rand((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
    z0, s0 = st.save(), sl.save()
    tapes = [torch.empty(F.adjoint_tape_bytes(st, sl, b - a), dtype=torch.uint8, device="cuda") for a, b in splits]
    cf, gx = torch.empty_like(x), torch.empty_like(x)
    adj = torch.zeros((2 * K + 2, n_ch), dtype=torch.float64, device="cuda")
    gs = torch.zeros((K, 5), dtype=torch.float64, device="cuda")

    def step(stream=None):
        st.load(z0, stream=stream)
        sl.load(s0, stream=stream)
        for i, (a, b) in enumerate(splits):
            F.sos_stalta_process_tape(st, sl, x[a:b], tape=tapes[i], cf=cf[a:b], stream=stream)
        adj.zero_()
        gs.zero_()
        for i in reversed(range(len(splits))):
            a, b = splits[i]
            F.sos_stalta_adjoint_tape(st, sl, tapes[i], x[a:b], tgt[a:b], gx[a:b], adj, gs, mode="mse",
                                      scale=1.0 / x.numel(), stream=stream)

    step()
    torch.cuda.synchronize()
    ref = (cf.clone(), gx.clone(), adj.clone(), gs.clone())
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            step(stream=s)
    torch.cuda.synchronize()
    for r in range(3):
        cf.zero_()
        gx.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for got, want in zip((cf, gx, adj, gs), ref):
            assert torch.equal(got, want), f"replay {r}"
    _, ogx, ogs, _ = orc.stalta_grad(sos, x.cpu().numpy().astype(np.float64),
                                     tgt.cpu().numpy().astype(np.float64), nsta, nlta, 1.0 / x.numel())
    assert max_rel_rms(gx.cpu().numpy(), ogx) <= 1e-5
    assert float(np.linalg.norm(gs.cpu().numpy() - ogs) / np.linalg.norm(ogs)) <= 1e-5
