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


def _check(gx, adj, gs, ogx, oadj, ogs, tol=1e-5, tol_state=1e-6):
    ex = max_rel_rms(gx, ogx)
    es = float(np.linalg.norm(gs - ogs) / np.linalg.norm(ogs))
    ea = float(np.max(np.abs(adj - oadj)) / np.max(np.abs(oadj)))
    print(f"dL/dx rel-RMS {ex:.2e}  dL/dtheta rel-L2 {es:.2e}  adjoint state {ea:.2e}")
    assert ex <= tol
    assert es <= tol
    assert ea <= tol_state


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


def _chain_case(F, n_ch, nsta, nlta, splits, seed, raw=False):
    """Forward with device checkpoints over the splits, then the chunks last
    to first carrying the adjoint state, against the one-shot reference."""
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    n_t = splits[-1][1]
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    tgt = torch.rand((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32) * 3.0
    scale = 1.0 / x.numel()
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
    if raw:
        return gx.cpu().numpy(), adj.cpu().numpy().T, gs.cpu().numpy(), x.cpu().numpy(), tgt.cpu().numpy(), sos
    _, ogx, ogs, oadj = orc.stalta_grad(sos, x.cpu().numpy().astype(np.float64),
                                        tgt.cpu().numpy().astype(np.float64), nsta, nlta, scale)
    return gx.cpu().numpy(), adj.cpu().numpy().T, gs.cpu().numpy(), ogx, oadj, ogs


def test_chunked_adjoint_chain_equals_oracle_one_shot(F):
    _check(*_chain_case(F, 24, 30, 300, [(0, 1000), (1000, 1001), (1001, 2600), (2600, 3100)], 31))


# One- to three-sample STA windows with one- and four-sample LTA windows, the
# STA window both shorter and longer than the LTA window.  A one-sample
# window has a zero decay: the STA (or LTA) equals the current energy.
SHORT_WINDOWS = [(1, 1), (1, 4), (2, 1), (2, 4), (3, 1), (3, 4)]


def _state_tol(nsta, nlta):
    """Bar for the adjoint state handed back.  With a one-sample LTA window
    (and a longer STA window) cf = sta / y^2, and the gradient terms grow like
    1 / y^5 where y crosses zero; the GPU's block-scan y and the oracle's
    sequential y differ by FP64 rounding of the order of 1e-13 of the
    channel's scale, which at the smallest |y| of the data is ~1e-6 of y and
    is amplified five-fold in the few samples that dominate every gradient.
    Those cases are held to the gradient bar (1e-5) throughout."""
    return 1e-5 if nlta == 1 and nsta > 1 else 1e-6


# The grad-mode reference passes dL/dcf to the oracle as target = cf - g / 2,
# which keeps g only to the rounding of cf.  A one-sample LTA window makes cf
# the ratio of the STA to the current energy, up to ~1e9 near zero crossings
# of y, where that subtraction loses g (1e-3) entirely; so grad mode runs on
# the four-sample LTA window only, MSE mode on every pair.
@pytest.mark.parametrize("nsta,nlta,mode", [(s, l, "mse") for s, l in SHORT_WINDOWS] +
                         [(s, l, "grad") for s, l in SHORT_WINDOWS if l == 4])
def test_adjoint_short_windows_one_chunk(F, nsta, nlta, mode):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    out = _chunk_case(F, 21, 40, 1100, sos, nsta, nlta, 60 + 7 * nsta + nlta, mode)
    assert all(np.all(np.isfinite(a)) for a in out[:3])
    _check(*out, tol_state=_state_tol(nsta, nlta))


def test_adjoint_equal_one_sample_windows_chunked(F):
    """nsta = nlta = 1: sta and lta are both the current energy, so cf = 1
    wherever it is live and the exact gradient is zero; the oracle's and the
    GPU's values are rounding noise of different arithmetic, so they are not
    compared with each other.  Bound: the STA/LTA step's two terms at a row
    are 2 q / y each (they cancel), and the GPU holds them in FP32, so the
    residue is at most a few FP32 ulps of them; the Butterworth bandpass's
    gain is at most 1, so each channel's dL/dx stays within 2^-21 of the
    norm of those terms."""
    orc = _orc()
    gx, adj, gs, x, tgt, sos = _chain_case(F, 13, 1, 1, [(0, 3), (3, 700), (700, 701), (701, 2100)], 78, raw=True)
    assert np.all(np.isfinite(gx)) and np.all(np.isfinite(adj)) and np.all(np.isfinite(gs))
    y, _ = orc.sos_filter(sos, x.astype(np.float64))
    q = np.where(np.arange(len(y))[:, None] >= 1, 2.0 * (1.0 - tgt) / x.size, 0.0)
    terms = np.sqrt(np.sum((2.0 * q / np.where(y != 0, y, np.inf)) ** 2, axis=0))
    assert np.all(np.linalg.norm(gx, axis=0) <= 2.0 ** -21 * terms)


@pytest.mark.parametrize("nsta,nlta", [w for w in SHORT_WINDOWS if w != (1, 1)])
def test_adjoint_short_windows_chunked(F, nsta, nlta):
    out = _chain_case(F, 13, nsta, nlta, [(0, 3), (3, 700), (700, 701), (701, 2100)], 70 + 7 * nsta + nlta)
    assert all(np.all(np.isfinite(a)) for a in out[:3])
    _check(*out, tol_state=_state_tol(nsta, nlta))


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
