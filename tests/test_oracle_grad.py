"""Pins for the oracle's reference gradient (reverse mode through the DF2T
cascade and the recursive STA/LTA; the paper gives no gradient, the
definition is the derivative of the forward loops).

Facts used, each independent of the routine under test:
  * central finite differences of the forward oracle in FP64 (every
    coefficient, random input positions, random directions on all of x),
    Richardson-extrapolated and taken at the step where the estimate has
    settled: with poles this close to the unit circle the loss bends so
    sharply in a1, a2 that a plain central difference at h = 1e-6 |theta| is
    off by 1e-2 (the error falls as h^2: the step is wrong, not the gradient),
    while for the small numerator gain b0 such a step is all rounding;
  * the transpose identity <H v, w> = <v, H^T w> for the linear cascade;
  * the closed-form adjoint of a one-pole section, x_bar_t = sum_k p^k w_(t+k);
  * an independent autodiff (torch float64 on the CPU through a plain
    per-sample loop);
  * chunks processed last-to-first with checkpoints and the adjoint carry
    give the one-shot gradient.
Loss (reading for the differentiation workload): mean over (channel, sample)
of (cf - cf_target)^2, the target being cf of the same input filtered with
the band edges moved to (1.05 f1, 0.95 f2).
"""

import numpy as np
import pytest

import synth


def _case(orc, n_ch=16, n_t=2000, nsta=20, nlta=200, seed=5):
    x = synth.pink_noise(n_t, n_ch, seed=seed).double().numpy()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    sos_t = orc.butter_sos(8, "bandpass", 1.05, 95.0, 1500.0)
    y_t, _ = orc.sos_filter(sos_t, x)
    tgt, _, _ = orc.stalta(y_t, nsta, nlta)
    return x, sos, tgt, 1.0 / (n_ch * n_t)


def _loss(orc, sos, x, tgt, nsta, nlta, scale):
    return orc.stalta_loss(sos, x, tgt, nsta, nlta, scale)


def _fd(f, h):
    """Central difference of f(s) at s = 0, Richardson-extrapolated in h."""
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def _fd_settled(f, scale):
    """The Richardson difference at the step where it has settled: over steps
    scale * 10^-m, the one whose estimate agrees best with the next smaller
    step (truncation falls and rounding grows as the step shrinks)."""
    hs = [scale * 10.0 ** (-m) for m in range(2, 10)]
    est = [_fd(f, h) for h in hs]
    gaps = [abs(est[m] - est[m + 1]) for m in range(len(est) - 1)]
    gaps = [g if np.isfinite(g) else np.inf for g in gaps]  # large steps can leave the stable region
    m = int(np.argmin(gaps))
    return est[m]


def _coef_fd(orc, sos, x, tgt, nsta, nlta, scale, k, i):
    r, col = _coef_index(k, i)

    def f(d):
        sp = sos.copy()
        sp[r, col] += d
        return _loss(orc, sp, x, tgt, nsta, nlta, scale)

    return _fd_settled(f, max(abs(sos[r, col]), 1e-3))


def _coef_index(k, i):
    """(b0, b1, b2, a1, a2) of section k -> (row, column) of the sos array."""
    return k, (0, 1, 2, 4, 5)[i]


def test_coefficient_gradient_matches_central_differences(orc):
    nsta, nlta = 20, 200
    x, sos, tgt, scale = _case(orc, nsta=nsta, nlta=nlta)
    loss, gx, gsos, _ = orc.stalta_grad(sos, x, tgt, nsta, nlta, scale)
    assert loss == pytest.approx(_loss(orc, sos, x, tgt, nsta, nlta, scale), rel=1e-12)
    fd = np.zeros_like(gsos)
    for k in range(sos.shape[0]):
        for i in range(5):
            fd[k, i] = _coef_fd(orc, sos, x, tgt, nsta, nlta, scale, k, i)
    rel = np.linalg.norm(gsos - fd) / np.linalg.norm(fd)
    print(f"coefficient gradient vs FD: rel L2 {rel:.2e}")
    assert rel < 1e-6
    # every individual coefficient is checked, not only the vector norm
    np.testing.assert_allclose(gsos, fd, rtol=1e-4, atol=1e-6 * np.abs(fd).max())


def test_input_gradient_matches_central_differences(orc):
    nsta, nlta = 20, 200
    x, sos, tgt, scale = _case(orc, nsta=nsta, nlta=nlta)
    _, gx, _, _ = orc.stalta_grad(sos, x, tgt, nsta, nlta, scale)
    rng = np.random.default_rng(7)
    n_t, n_ch = x.shape
    pts = [(int(rng.integers(0, n_t)), int(rng.integers(0, n_ch))) for _ in range(256)]
    fd, an = [], []
    for t, c in pts:
        def f(d, t=t, c=c):
            xp = x.copy()
            xp[t, c] += d
            return _loss(orc, sos, xp, tgt, nsta, nlta, scale)

        fd.append(_fd(f, 1e-3 * max(1.0, abs(x[t, c]))))
        an.append(gx[t, c])
    fd, an = np.array(fd), np.array(an)
    rel = np.linalg.norm(an - fd) / np.linalg.norm(fd)
    print(f"input gradient vs FD at 256 points: rel L2 {rel:.2e}")
    assert rel < 1e-6
    # random directional derivatives over all of x
    for _ in range(8):
        v = rng.standard_normal(x.shape)
        dd = _fd(lambda d: _loss(orc, sos, x + d * v, tgt, nsta, nlta, scale), 1e-4)
        assert np.sum(gx * v) == pytest.approx(dd, rel=1e-6)


def test_gradient_with_the_differentiation_workload_windows(orc):
    """STA 300 / LTA 3000 samples: the record must outlast the warm-up."""
    nsta, nlta = 300, 3000
    x, sos, tgt, scale = _case(orc, n_ch=4, n_t=5000, nsta=nsta, nlta=nlta, seed=9)
    _, gx, gsos, _ = orc.stalta_grad(sos, x, tgt, nsta, nlta, scale)
    assert np.abs(gx[:, 0]).max() > 0
    for k, i in [(0, 0), (1, 3), (3, 4), (2, 1)]:
        fd = _coef_fd(orc, sos, x, tgt, nsta, nlta, scale, k, i)
        assert gsos[k, i] == pytest.approx(fd, rel=1e-5)


def test_cascade_transpose_identity(orc):
    rng = np.random.default_rng(3)
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    v = rng.standard_normal((3000, 5))
    w = rng.standard_normal((3000, 5))
    hv, _ = orc.sos_filter(sos, v)
    htw, _, _ = orc.sos_vjp(sos, rng.standard_normal((3000, 5)), w)  # H^T does not depend on x
    lhs, rhs = np.sum(hv * w), np.sum(v * htw)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_one_pole_adjoint_closed_form(orc):
    p = 0.93
    sos = np.array([[1.0, 0.0, 0.0, 1.0, -p, 0.0]])
    rng = np.random.default_rng(4)
    n = 400
    w = rng.standard_normal((n, 1))
    gx, gs, _ = orc.sos_vjp(sos, rng.standard_normal((n, 1)), w)
    want = np.array([sum(p ** k * w[t + k, 0] for k in range(n - t)) for t in range(n)])
    np.testing.assert_allclose(gx[:, 0], want, rtol=1e-12, atol=1e-12)


def test_vjp_coefficients_match_differences_of_a_linear_functional(orc):
    rng = np.random.default_rng(6)
    sos = orc.butter_sos(6, "bandpass", 2.0, 40.0, 100.0)
    x = rng.standard_normal((1500, 3))
    w = rng.standard_normal((1500, 3))
    _, gs, _ = orc.sos_vjp(sos, x, w)
    for k in range(sos.shape[0]):
        for i in range(5):
            r, col = _coef_index(k, i)

            def f(d):
                sp = sos.copy()
                sp[r, col] += d
                return np.sum(orc.sos_filter(sp, x)[0] * w)

            fd = _fd(f, 1e-6)
            assert gs[k, i] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(gs).max())


def test_gradient_matches_torch_autodiff(orc):
    torch = pytest.importorskip("torch")
    nsta, nlta = 10, 100
    n_t, n_ch = 600, 6
    x, sos, tgt, scale = _case(orc, n_ch=n_ch, n_t=n_t, nsta=nsta, nlta=nlta, seed=11)
    loss, gx, gsos, _ = orc.stalta_grad(sos, x, tgt, nsta, nlta, scale)
    # independent reference: a plain per-sample loop under torch.autograd
    xt = torch.tensor(x, requires_grad=True)
    th = torch.tensor(sos[:, [0, 1, 2, 4, 5]].copy(), requires_grad=True)
    z1 = [torch.zeros(n_ch, dtype=torch.float64) for _ in range(sos.shape[0])]
    z2 = [torch.zeros(n_ch, dtype=torch.float64) for _ in range(sos.shape[0])]
    sta = torch.zeros(n_ch, dtype=torch.float64)
    lta = torch.zeros(n_ch, dtype=torch.float64)
    cs, cl = 1.0 / nsta, 1.0 / nlta
    tot = torch.zeros((), dtype=torch.float64)
    tg = torch.tensor(tgt)
    for t in range(n_t):
        v = xt[t]
        for k in range(sos.shape[0]):
            b0, b1, b2, a1, a2 = th[k]
            yk = b0 * v + z1[k]
            z1[k] = b1 * v - a1 * yk + z2[k]
            z2[k] = b2 * v - a2 * yk
            v = yk
        sta = (1 - cs) * sta + cs * v * v
        lta = (1 - cl) * lta + cl * v * v
        cf = sta / lta if t >= nlta else torch.zeros(n_ch, dtype=torch.float64)
        tot = tot + scale * torch.sum((cf - tg[t]) ** 2)
    tot.backward()
    assert loss == pytest.approx(tot.item(), rel=1e-12)
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(gx).max())
    np.testing.assert_allclose(gsos, th.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(gsos).max())


def test_chunked_gradient_equals_one_shot(orc):
    nsta, nlta = 20, 200
    x, sos, tgt, scale = _case(orc, n_ch=7, n_t=2500, nsta=nsta, nlta=nlta, seed=12)
    loss1, gx1, gs1, a1 = orc.stalta_grad(sos, x, tgt, nsta, nlta, scale)
    splits = [0, 1, 700, 701, 1999, 2500]
    # forward with checkpoints
    s = orc.Stream(sos, x.shape[1], nsta, nlta)
    ck = []
    for a, b in zip(splits[:-1], splits[1:]):
        ck.append((s.zi.copy(), s.st.copy(), s.g))
        s.process(x[a:b])
    # backward, last chunk first, carrying the adjoint state
    adj = None
    gx = np.empty_like(x)
    gs = np.zeros_like(gs1)
    loss = 0.0
    for (a, b), (zi, st, g) in reversed(list(zip(zip(splits[:-1], splits[1:]), ck))):
        l, g_x, g_s, adj = orc.stalta_grad(sos, x[a:b], tgt[a:b], nsta, nlta, scale, zi, st, g, adj)
        gx[a:b] = g_x
        gs += g_s
        loss += l
    assert np.array_equal(gx, gx1)
    assert np.array_equal(adj, a1)
    np.testing.assert_allclose(gs, gs1, rtol=1e-12)
    assert loss == pytest.approx(loss1, rel=1e-13)
