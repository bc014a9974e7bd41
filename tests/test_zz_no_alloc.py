"""The allocation-free zero-phase entry point (filark_sos_filtfilt_noalloc)
against the allocating one (filark_sos_filtfilt), both called through the C
ABI: the same kernels from the same zero work state, so the outputs must be
equal bit for bit, on two calls in a row (the second smaller, so a stale
larger work state would show), with the state object's carried state left
alone; sizes beyond the fixed scratch are refused before any work."""

import ctypes

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


def _call(F, fn, st, x, out):
    s = torch.cuda.current_stream()
    rc = fn(st.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), x.shape[1], x.shape[0],
            ctypes.c_void_p(s.cuda_stream))
    assert rc == F.OK, F.lib().filark_last_error().decode()


def test_noalloc_equals_filtfilt_on_two_calls(F):
    import oracle

    sos = oracle.butter_sos(8, "bandpass", 1.0, 100.0, 1500.0)
    L = F.lib()
    g = torch.Generator(device="cuda").manual_seed(77)
    for n_ch, n_t in [(6000, 4000), (997, 1537)]:  # 2 * 4 * 6000 = 48000 <= 131072
        st = F.SOSState(sos, n_ch)
        z0 = st.get_state()
        x = torch.randn((n_t, n_ch), generator=g, device="cuda", dtype=torch.float32)
        a = torch.empty_like(x)
        b = torch.full_like(x, float("nan"))
        _call(F, L.filark_sos_filtfilt, st, x, a)
        _call(F, L.filark_sos_filtfilt_noalloc, st, x, b)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
        np.testing.assert_array_equal(st.get_state(), z0)
        st.close()


def test_noalloc_refuses_more_than_its_scratch(F):
    import oracle

    sos = oracle.butter_sos(16, "highpass", 0.5, 0.0, 10_000.0)  # 8 sections: at most 8192 channels
    L = F.lib()
    st = F.SOSState(sos, 8193)
    x = torch.zeros((10, 8193), device="cuda", dtype=torch.float32)
    y = torch.zeros_like(x)
    s = torch.cuda.current_stream()
    rc = L.filark_sos_filtfilt_noalloc(st.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       8193, 10, ctypes.c_void_p(s.cuda_stream))
    assert rc == F.EINVAL and b"131072" in L.filark_last_error()
    st.close()
    st = F.SOSState(sos, 8192)
    x = torch.randn((300, 8192), device="cuda", dtype=torch.float32)
    a, b = torch.empty_like(x), torch.empty_like(x)
    _call(F, L.filark_sos_filtfilt, st, x, a)
    _call(F, L.filark_sos_filtfilt_noalloc, st, x, b)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    st.close()
