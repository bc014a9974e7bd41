"""GPU parity of the adjoint (reverse-mode) kernel against the oracle's
reference gradient.

The oracle runs on the exact FP32 inputs the GPU saw, upcast, from the same
checkpointed forward state and the same handed-in adjoint state.  Bars
(gradient tolerance reading: 1e-5 relative): dL/dx per-channel relative RMS
<= 1e-5; the coefficient gradient vector relative L2 <= 1e-5; the adjoint
state handed back within 1e-6 of its scale.
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


def _adj_to_oracle(adj_gpu, n_sec):
    """[2K+2, n_ch] device layout -> the oracle's [n_ch, 2K+2]."""
    return adj_gpu.T.copy()


def _chunk_case(F, n_ch, n_pre, n_t, sos, nsta, nlta, seed, mode, tile=None):
    """One chunk after a prefix of n_pre samples: forward state from the oracle,
    random handed-in adjoint, GPU adjoint vs oracle gradient."""
    orc = _orc()
    g = torch.Generator(device="cuda").manual_seed(seed)
    xall = torch.randn((n_pre + n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    x = xall[n_pre:].contiguous()
    xh = xall.cpu().numpy().astype(np.float64)
    s = orc.Stream(sos, n_ch, nsta, nlta)
    if n_pre:
        s.process(xh[:n_pre])
    zi0, st0, g0 = s.zi.copy(), s.st.copy(), s.g
    K = sos.shape[0]
    rng = np.random.default_rng(seed)
    adj_in = rng.standard_normal((n_ch, 2 * K + 2)) * 1e-3
    if mode == "grad":
        gq = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32) * 1e-3
        scale = 1.0
    else:
        gq = torch.rand((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32) * 4.0
        scale = 1.0 / (n_ch * n_t)
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
    if tile is not None:
        st.set_adjoint_tile(*tile)
        sl.set_adjoint_tile(*tile)
    st.set_state(zi0)
    sl.set_state(st0, g0)
    adj = torch.tensor(adj_in.T.copy(), device="cuda")
    gx, adj, gsos = F.sos_stalta_adjoint(st, sl, x, gq, adj=adj, mode=mode, scale=scale)
    torch.cuda.synchronize()
    st.check()
    # the forward states are left as they were
    np.testing.assert_array_equal(st.get_state(), zi0)
    # oracle
    gqh = gq.cpu().numpy().astype(np.float64)
    if mode == "grad":
        _, ogx, ogs, oadj = _grad_mode_oracle(orc, sos, xh[n_pre:], gqh, nsta, nlta, zi0, st0, g0, adj_in)
    else:
        _, ogx, ogs, oadj = orc.stalta_grad(sos, xh[n_pre:], gqh, nsta, nlta, scale, zi0, st0, g0, adj_in)
    return gx.cpu().numpy(), adj.cpu().numpy().T, gsos.cpu().numpy(), ogx, oadj, ogs


def _grad_mode_oracle(orc, sos, x, gcf, nsta, nlta, zi0, st0, g0, adj_in):
    """dL/dcf given: the oracle's MSE gradient with target cf - gcf / 2 and
    scale 1 has q = 2 (cf - target) = gcf exactly where cf is live."""
    y, _ = orc.sos_filter(sos, x, zi0)
    cf, _, _ = orc.stalta(y, nsta, nlta, st0, g0)
    tgt = cf - gcf / 2.0
    return orc.stalta_grad(sos, x, tgt, nsta, nlta, 1.0, zi0, st0, g0, adj_in)


def _check(gx, adj, gs, ogx, oadj, ogs, tol=1e-5):
    ex = max_rel_rms(gx, ogx)
    es = float(np.linalg.norm(gs - ogs) / np.linalg.norm(ogs))
    ea = float(np.max(np.abs(adj - oadj)) / np.max(np.abs(oadj)))
    print(f"dL/dx rel-RMS {ex:.2e}  dL/dtheta rel-L2 {es:.2e}  adjoint state {ea:.2e}")
    assert ex <= tol
    assert es <= tol
    assert ea <= 1e-6


@pytest.mark.parametrize("mode", ["grad", "mse"])
def test_adjoint_one_chunk_matches_oracle(F, mode):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    _check(*_chunk_case(F, 37, 700, 1300, sos, 20, 200, 21, mode))


@pytest.mark.parametrize("order,btype,f1,f2,fs", [
    (2, "lowpass", 30.0, 0.0, 200.0),
    (5, "highpass", 3.0, 0.0, 500.0),
    (16, "bandpass", 5.0, 400.0, 2000.0),
])
def test_adjoint_orders(F, order, btype, f1, f2, fs):
    orc = _orc()
    sos = orc.butter_sos(order, btype, f1, f2, fs)
    _check(*_chunk_case(F, 70, 300, 900, sos, 15, 150, 22, "mse"))


@pytest.mark.parametrize("tile", [(8, 8, 8), (16, 4, 8), (8, 2, 4), (8, 1, 64), (16, 8, 16), (8, 3, 32)])
def test_adjoint_tiles(F, tile):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    _check(*_chunk_case(F, 45, 400, 777, sos, 20, 200, 23, "mse", tile=tile))


def test_adjoint_general_numerators(F):
    """Gain moved between sections (same transfer function, later sections no
    longer [1, b1, 1]): the general section step of the adjoint kernel."""
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0).copy()
    sos[0, :3] *= 8.0
    sos[2, :3] *= 0.125
    _check(*_chunk_case(F, 41, 500, 1200, sos, 20, 200, 29, "mse"))


def test_adjoint_short_and_warmup_chunks(F):
    """Chunks shorter than one block, and chunks that straddle the warm-up."""
    orc = _orc()
    sos = orc.butter_sos(4, "bandpass", 1.0, 50.0, 500.0)
    for n_pre, n_t in [(250, 1), (250, 5), (0, 300), (180, 50)]:
        _check(*_chunk_case(F, 9, n_pre, n_t, sos, 20, 200, 24 + n_t, "mse"))


def test_chunked_adjoint_chain_equals_oracle_one_shot(F):
    """Forward with device checkpoints, then the chunks last to first,
    carrying the adjoint state: the one-shot reference gradient."""
    orc = _orc()
    n_ch, nsta, nlta = 24, 30, 300
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    g = torch.Generator(device="cuda").manual_seed(31)
    x = torch.randn((3100, n_ch), generator=g, device="cuda", dtype=torch.float32)
    tgt = torch.rand((3100, n_ch), generator=g, device="cuda", dtype=torch.float32) * 3.0
    scale = 1.0 / x.numel()
    splits = [(0, 1000), (1000, 1001), (1001, 2600), (2600, 3100)]
    st = F.SOSState(sos, n_ch)
    sl = F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
    cks = []
    for a, b in splits:
        cks.append((st.save(), sl.save()))
        F.sos_stalta_process(st, sl, x[a:b].contiguous(), write_y=False)
    gx = torch.empty_like(x)
    adj = torch.zeros((2 * sos.shape[0] + 2, n_ch), dtype=torch.float64, device="cuda")
    gs = torch.zeros((sos.shape[0], 5), dtype=torch.float64, device="cuda")
    for (a, b), (cz, cs) in reversed(list(zip(splits, cks))):
        st.load(cz)
        sl.load(cs)
        ga = torch.empty((b - a, n_ch), dtype=torch.float32, device="cuda")
        F.sos_stalta_adjoint(st, sl, x[a:b].contiguous(), tgt[a:b].contiguous(), ga, adj, gs, mode="mse",
                             scale=scale)
        gx[a:b] = ga
    torch.cuda.synchronize()
    _, ogx, ogs, oadj = orc.stalta_grad(sos, x.cpu().numpy().astype(np.float64),
                                        tgt.cpu().numpy().astype(np.float64), nsta, nlta, scale)
    _check(gx.cpu().numpy(), adj.cpu().numpy().T, gs.cpu().numpy(), ogx, oadj, ogs)


def test_autograd_function_matches_oracle(F):
    from paper_2605_20132_amd.autograd import sos_stalta_cf, sos_to_theta

    orc = _orc()
    n_ch, nsta, nlta, chunk = 19, 25, 250, 700
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    g = torch.Generator(device="cuda").manual_seed(41)
    x = torch.randn((2500, n_ch), generator=g, device="cuda", dtype=torch.float32).requires_grad_(True)
    theta = torch.tensor(sos_to_theta(sos), requires_grad=True)
    tgt = torch.rand((2500, n_ch), generator=g, device="cuda", dtype=torch.float32) * 2.0
    cf = sos_stalta_cf(x, theta, nsta, nlta, chunk)
    loss = torch.mean((cf.double() - tgt.double()) ** 2)
    loss.backward()
    ol, ogx, ogs, _ = orc.stalta_grad(sos, x.detach().cpu().numpy().astype(np.float64),
                                      tgt.cpu().numpy().astype(np.float64), nsta, nlta, 1.0 / x.numel())
    assert loss.item() == pytest.approx(ol, rel=1e-5)
    assert max_rel_rms(x.grad.cpu().numpy(), ogx) <= 1e-5
    assert float(np.linalg.norm(theta.grad.numpy() - ogs) / np.linalg.norm(ogs)) <= 1e-5


def test_adjoint_is_deterministic(F):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    a = _chunk_case(F, 100, 400, 1500, sos, 20, 200, 51, "mse")
    b = _chunk_case(F, 100, 400, 1500, sos, 20, 200, 51, "mse")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
