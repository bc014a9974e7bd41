"""GPU parity of zero-phase (forward-backward) filtering of a window against
the oracle, on the exact FP32 input the GPU saw (upcast).  Bar: per-channel
relative RMS <= 1e-5 (1e-4 with a pole within 1e-3 of the unit circle).
Shapes: one sample, windows shorter and longer than one 1536-row launch
window (the backward pass then walks the windows last to first), ragged
channel groups; in place; the state object's carried state untouched.
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


def _orc():
    import oracle

    return oracle


@pytest.mark.parametrize("n_ch,n_t", [(1, 1), (7, 100), (65, 1536), (130, 1537), (300, 5000), (9, 4609)])
@pytest.mark.parametrize("order,btype,f1,f2,fs", [
    (8, "bandpass", 1.0, 100.0, 1500.0),
    (2, "lowpass", 30.0, 0.0, 200.0),
    (5, "highpass", 3.0, 0.0, 500.0),
    (16, "bandpass", 5.0, 400.0, 2000.0),
])
def test_filtfilt_matches_oracle(F, n_ch, n_t, order, btype, f1, f2, fs):
    orc = _orc()
    sos = orc.butter_sos(order, btype, f1, f2, fs)
    g = torch.Generator(device="cuda").manual_seed(300 + n_ch + order)
    x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
    st = F.SOSState(sos, n_ch)
    y = st.filtfilt(x)
    torch.cuda.synchronize()
    st.check()
    yo = orc.sos_filtfilt(sos, x.cpu().numpy().astype(np.float64))
    assert max_rel_rms(y.cpu().numpy(), yo) <= tolerance_for(sos)


def test_filtfilt_in_place_and_state_untouched(F):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    n_ch = 40
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((3100, n_ch), generator=g, device="cuda", dtype=torch.float32)
    xh = x.cpu().numpy().astype(np.float64)
    st = F.SOSState(sos, n_ch)
    st.process(x[:500].contiguous())  # some carried state
    z0 = st.get_state()
    buf = x.clone()
    st.filtfilt(buf, buf)
    torch.cuda.synchronize()
    assert max_rel_rms(buf.cpu().numpy(), orc.sos_filtfilt(sos, xh)) <= 1e-5
    np.testing.assert_array_equal(st.get_state(), z0)


def test_filtfilt_general_numerators_and_errors(F):
    orc = _orc()
    sos = orc.butter_sos(8, "bandpass", 2.0, 80.0, 1000.0).copy()
    sos[0, :3] *= 4.0
    sos[1, :3] *= 0.25
    g = torch.Generator(device="cuda").manual_seed(6)
    x = torch.randn((2000, 33), generator=g, device="cuda", dtype=torch.float32)
    st = F.SOSState(sos, 33)
    y = st.filtfilt(x)
    torch.cuda.synchronize()
    assert max_rel_rms(y.cpu().numpy(), orc.sos_filtfilt(sos, x.cpu().numpy().astype(np.float64))) <= 1e-5
    st.set_tile(64, 3, 8)
    with pytest.raises(F.FilarkError):
        st.filtfilt(x)  # zero-phase filtering runs on 48-sample blocks
