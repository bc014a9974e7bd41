"""The C-ABI library loads on a machine without a GPU and exports every entry
point the header declares; host-only calls (filter design, argument checks
that fail before anything is enqueued) behave as documented."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "filark.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(filark_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def F():
    import paper_2605_20132_amd as F

    if not os.path.exists(F.LIB_PATH):
        pytest.fail("libfilark.so is not built (python -m paper_2605_20132_amd.build)")
    F.lib()
    return F


def test_header_declares_the_binding_exports(F):
    assert set(declared_symbols()) == set(F.EXPORTS)


def test_every_declared_symbol_is_exported(F):
    lib = ctypes.CDLL(F.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_version_and_error_strings(F):
    assert F.version()
    assert isinstance(F.lib().filark_last_error(), bytes)


@pytest.mark.parametrize("order,btype,f1,f2,fs", [
    (8, "bandpass", 1.0, 100.0, 1500.0),
    (4, "bandpass", 1.0, 50.0, 500.0),
    (16, "highpass", 0.5, 0.0, 10_000.0),
    (5, "lowpass", 30.0, 0.0, 200.0),
    (6, "bandstop", 45.0, 55.0, 500.0),
    (1, "highpass", 3.0, 0.0, 100.0),
])
def test_library_design_matches_oracle(F, orc, order, btype, f1, f2, fs):
    """The library's own Butterworth design (independent code) gives the
    oracle's sections, row for row."""
    a = F.sos_design(order, btype, f1, f2, fs)
    b = orc.butter_sos(order, btype, f1, f2, fs)
    assert a.shape == b.shape
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("args", [
    (3, "bandpass", 1.0, 50.0, 500.0),   # odd band order
    (4, "bandpass", 50.0, 1.0, 500.0),   # f1 > f2
    (4, "lowpass", 300.0, 0.0, 500.0),   # above Nyquist
    (0, "lowpass", 10.0, 0.0, 500.0),    # order 0
    (65, "lowpass", 10.0, 0.0, 500.0),   # order above the limit
])
def test_design_argument_errors(F, args):
    with pytest.raises(F.FilarkError) as e:
        F.sos_design(*args)
    assert e.value.status == F.EINVAL


def test_null_and_range_errors_without_gpu(F):
    L = F.lib()
    vp = ctypes.c_void_p
    assert L.filark_sos_process(vp(0), vp(0), vp(0), 4, 4, vp(0)) == F.EINVAL
    assert L.filark_stalta_process(vp(0), vp(0), vp(0), 4, 4, vp(0)) == F.EINVAL
    assert L.filark_sos_stalta_process(vp(0), vp(0), vp(0), vp(0), vp(0), 4, 4, vp(0)) == F.EINVAL
    assert L.filark_tile_set(vp(0), 0, 64, 4, 8, vp(0)) == F.EINVAL
    assert L.filark_sos_destroy(vp(0)) == F.OK
    assert L.filark_stalta_destroy(vp(0)) == F.OK
    sos = np.array([[1.0, 0.0, 0.0, 1.0, -0.5, 0.0]])
    h = vp()
    D = ctypes.POINTER(ctypes.c_double)
    # n_sec out of range and bad flags are rejected before any device call
    assert L.filark_sos_init(ctypes.byref(h), sos.ctypes.data_as(D), 0, 4, 0, vp(0)) == F.EINVAL
    assert L.filark_sos_init(ctypes.byref(h), sos.ctypes.data_as(D), 1, 4, 7, vp(0)) == F.EINVAL
    assert L.filark_sos_init(ctypes.byref(h), sos.ctypes.data_as(D), 9, 4, 0, vp(0)) == F.EINVAL
    assert L.filark_stalta_init(ctypes.byref(h), -1.0, 1.0, 100.0, 4, vp(0)) == F.EINVAL
    # trigger: thresholds, channel count and null handles
    assert L.filark_trigger_init(ctypes.byref(h), 1.0, 2.0, 4, vp(0)) == F.EINVAL  # off > on
    assert L.filark_trigger_init(ctypes.byref(h), float("nan"), 1.0, 4, vp(0)) == F.EINVAL
    assert L.filark_trigger_init(ctypes.byref(h), 2.0, 1.0, 0, vp(0)) == F.EINVAL
    assert L.filark_trigger_init(None, 2.0, 1.0, 4, vp(0)) == F.EINVAL
    assert L.filark_trigger_process(vp(0), vp(0), 4, 4, vp(0), 0, vp(0), vp(0)) == F.EINVAL
    assert L.filark_trigger_destroy(vp(0)) == F.OK
    # FIR: tap count, non-finite taps, channel count, null handles
    taps = np.ones(4)
    assert L.filark_fir_init(ctypes.byref(h), taps.ctypes.data_as(D), 0, 4, vp(0)) == F.EINVAL
    assert L.filark_fir_init(ctypes.byref(h), np.ones(1025).ctypes.data_as(D), 1025, 4, vp(0)) == F.EINVAL
    assert L.filark_fir_init(ctypes.byref(h), np.array([1.0, np.nan]).ctypes.data_as(D), 2, 4, vp(0)) == F.EINVAL
    assert L.filark_fir_init(ctypes.byref(h), np.array([1.0, 1e39]).ctypes.data_as(D), 2, 4, vp(0)) == F.EINVAL
    assert L.filark_fir_init(ctypes.byref(h), taps.ctypes.data_as(D), 4, 0, vp(0)) == F.EINVAL
    assert L.filark_fir_init(ctypes.byref(h), None, 4, 4, vp(0)) == F.EINVAL
    assert L.filark_fir_init(None, taps.ctypes.data_as(D), 4, 4, vp(0)) == F.EINVAL
    # one channel past the launch-window limit for 64 taps (2 x 64 + 81 + 96 rows
    # of n_ch floats must stay below 2 GiB): refused before any allocation
    assert L.filark_fir_init(ctypes.byref(h), np.ones(64).ctypes.data_as(D), 64, 1_760_233, vp(0)) == F.EINVAL
    assert L.filark_fir_process(vp(0), vp(0), vp(0), 4, 4, vp(0)) == F.EINVAL
    assert L.filark_fir_set_tile(vp(0), 32, 4, 0) == F.EINVAL
    assert L.filark_fir_state_get(vp(0), vp(0), vp(0)) == F.EINVAL
    assert L.filark_fir_destroy(vp(0)) == F.OK
    assert L.filark_last_error()


def test_unstable_sections_rejected_on_host(F):
    L = F.lib()
    h = ctypes.c_void_p()
    D = ctypes.POINTER(ctypes.c_double)
    for row in ([1.0, 0.0, 0.0, 1.0, -2.0, 1.0],     # double pole at z = 1
                [1.0, 0.0, 0.0, 1.0, 0.0, -1.0],     # poles at +-1
                [1.0, 0.0, 0.0, 1.0, -1.0, 1.0001]):  # complex pair just outside
        sos = np.array([row])
        assert L.filark_sos_init(ctypes.byref(h), sos.ctypes.data_as(D), 1, 4, 0, ctypes.c_void_p(0)) \
            == F.EUNSTABLE
