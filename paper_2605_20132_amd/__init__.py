"""Python binding of libfilark (stateful chunked SOS + STA/LTA on MI355X).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libfilark.so``; PyTorch supplies device memory and streams.  There is no
CPU fallback: if the library is missing or a call fails, an exception is
raised.

Layout: FP32 CUDA tensors of shape ``[n_t, n_ch]`` (time-major, channel
contiguous).  Calls are asynchronous on the given (default: current) stream.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfilark.so")

OK, EINVAL, ESHAPE, ENOMEM, EHIP, EUNSTABLE, ETIMEOUT = range(7)
BTYPES = {"lowpass": 0, "highpass": 1, "bandpass": 2, "bandstop": 3}
STATE_SOS, STATE_STALTA, TILE_SOS_ADJOINT, TILE_STALTA_ADJOINT = 0, 1, 2, 3
ADJ_GRAD, ADJ_MSE = 0, 1

_lib = None

# Every symbol the C header declares; checked on load.
EXPORTS = (
    "filark_sos_design", "filark_sos_init", "filark_sos_process", "filark_stalta_init",
    "filark_stalta_process", "filark_sos_stalta_process", "filark_state_get", "filark_state_set",
    "filark_check", "filark_sos_destroy", "filark_stalta_destroy", "filark_last_error",
    "filark_version", "filark_tile_set", "filark_tile_get", "filark_adjoint_windows_set", "filark_state_bytes", "filark_state_save",
    "filark_state_load", "filark_sos_stalta_adjoint", "filark_adjoint_tape_bytes",
    "filark_sos_stalta_process_tape", "filark_sos_stalta_adjoint_tape", "filark_batch_create", "filark_batch_bind",
    "filark_batch_launch", "filark_batch_capture", "filark_autotune", "filark_batch_stamps", "filark_batch_destroy", "filark_trigger_init",
    "filark_trigger_process", "filark_monitor_process", "filark_trigger_state_get", "filark_trigger_state_set", "filark_trigger_destroy",
    "filark_sos_filtfilt", "filark_sos_filtfilt_noalloc", "filark_ema_init", "filark_ema_process", "filark_ema_state_get", "filark_ema_state_set",
    "filark_ema_destroy", "filark_fir_init", "filark_fir_set_tile", "filark_fir_set_method", "filark_fir_process", "filark_fir_state_get",
    "filark_fir_state_set", "filark_fir_destroy",
)


class FilarkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"filark status {status}: {msg}")
        self.status = status


def lib():
    """Load libfilark.so (built in-tree by ``paper_2605_20132_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FilarkError(EHIP, f"{LIB_PATH} is missing; build it with python -m paper_2605_20132_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    for name in EXPORTS:
        if not hasattr(L, name):
            raise FilarkError(EHIP, f"libfilark.so does not export {name}")
    D = ctypes.POINTER(ctypes.c_double)
    vp, i64, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.filark_sos_design.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, D, ctypes.POINTER(ctypes.c_int)]
    L.filark_sos_init.argtypes = [ctypes.POINTER(vp), D, ctypes.c_int, i64, ctypes.c_uint, vp]
    L.filark_sos_process.argtypes = [vp, vp, vp, i64, i64, vp]
    L.filark_sos_filtfilt.argtypes = [vp, vp, vp, i64, i64, vp]
    L.filark_sos_filtfilt_noalloc.argtypes = [vp, vp, vp, i64, i64, vp]
    L.filark_stalta_init.argtypes = [ctypes.POINTER(vp), ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     i64, vp]
    L.filark_stalta_process.argtypes = [vp, vp, vp, i64, i64, vp]
    L.filark_sos_stalta_process.argtypes = [vp, vp, vp, vp, vp, i64, i64, vp]
    L.filark_state_get.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t, vp]
    L.filark_state_set.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t, vp]
    L.filark_check.argtypes = [vp, ctypes.c_int, vp]
    ip = ctypes.POINTER(ctypes.c_int)
    L.filark_tile_set.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    L.filark_adjoint_windows_set.argtypes = [vp, ctypes.c_int]
    L.filark_tile_get.argtypes = [vp, ctypes.c_int, ip, ip, ip]
    L.filark_state_bytes.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.filark_state_save.argtypes = [vp, ctypes.c_int, vp, vp]
    L.filark_state_load.argtypes = [vp, ctypes.c_int, vp, vp]
    L.filark_sos_stalta_adjoint.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_double, vp, vp, vp, i64,
                                            i64, vp]
    L.filark_adjoint_tape_bytes.argtypes = [vp, vp, i64, ctypes.POINTER(ctypes.c_size_t)]
    L.filark_sos_stalta_process_tape.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, i64, i64, vp]
    L.filark_sos_stalta_adjoint_tape.argtypes = [vp, vp, vp, ctypes.c_size_t, vp, vp, ctypes.c_int, ctypes.c_double,
                                                 vp, vp, vp, i64, i64, vp]
    L.filark_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp), vp]
    L.filark_batch_bind.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64), vp]
    L.filark_batch_launch.argtypes = [vp, vp]
    L.filark_batch_capture.argtypes = [vp]
    L.filark_autotune.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ip, ip, ip, vp]
    L.filark_batch_stamps.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), vp]
    L.filark_batch_destroy.argtypes = [vp]
    L.filark_sos_destroy.argtypes = [vp]
    L.filark_stalta_destroy.argtypes = [vp]
    I64P = ctypes.POINTER(i64)
    L.filark_trigger_init.argtypes = [ctypes.POINTER(vp), ctypes.c_float, ctypes.c_float, i64, vp]
    L.filark_trigger_process.argtypes = [vp, vp, i64, i64, vp, i64, vp, vp]
    L.filark_monitor_process.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64, vp, i64, i64, vp]
    L.filark_trigger_state_get.argtypes = [vp, I64P, I64P, vp]
    L.filark_trigger_state_set.argtypes = [vp, I64P, i64, vp]
    L.filark_trigger_destroy.argtypes = [vp]
    L.filark_ema_init.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_double, ctypes.c_double, i64, vp]
    L.filark_ema_process.argtypes = [vp, vp, vp, i64, i64, vp]
    L.filark_ema_state_get.argtypes = [vp, D, vp]
    L.filark_ema_state_set.argtypes = [vp, D, vp]
    L.filark_ema_destroy.argtypes = [vp]
    L.filark_fir_init.argtypes = [ctypes.POINTER(vp), D, ctypes.c_int, i64, vp]
    L.filark_fir_set_tile.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.filark_fir_set_method.argtypes = [vp, ctypes.c_int, vp]
    L.filark_fir_process.argtypes = [vp, vp, vp, i64, i64, vp]
    L.filark_fir_state_get.argtypes = [vp, vp, vp]
    L.filark_fir_state_set.argtypes = [vp, vp, vp]
    L.filark_fir_destroy.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("filark_last_error", "filark_version"):
            getattr(L, name).restype = st
    L.filark_last_error.restype = ctypes.c_char_p
    L.filark_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise FilarkError(rc, lib().filark_last_error().decode())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev_f32(t, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2 \
            or not t.is_contiguous():
        raise FilarkError(EINVAL, f"{name} must be a contiguous float32 CUDA tensor [n_t, n_ch]")
    return ctypes.c_void_p(t.data_ptr())


def version() -> str:
    return lib().filark_version().decode()


def sos_design(order: int, btype: str, f1: float, f2: float = 0.0, fs: float = 1.0) -> np.ndarray:
    """Butterworth SOS by the bilinear transform, rows {b0 b1 b2 1 a1 a2}."""
    n_max = max(1, (int(order) + 1) // 2)
    out = np.zeros((n_max, 6), dtype=np.float64)
    n = ctypes.c_int(0)
    _check(lib().filark_sos_design(int(order), BTYPES[btype], float(f1), float(f2), float(fs),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(n)))
    return out[: n.value].copy()


class SOSState:
    """Stateful SOS cascade for ``n_ch`` channels (zero initial condition)."""

    def __init__(self, sos, n_ch: int, stream=None):
        self._h = ctypes.c_void_p()
        self.sos = np.ascontiguousarray(np.asarray(sos, dtype=np.float64))
        if self.sos.ndim != 2 or self.sos.shape[1] != 6:
            raise FilarkError(EINVAL, "sos must have shape [n_sec, 6]")
        self.n_ch = int(n_ch)
        self.n_sec = self.sos.shape[0]
        _check(lib().filark_sos_init(ctypes.byref(self._h),
                                     self.sos.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     self.n_sec, self.n_ch, 0, _stream(stream)))

    @property
    def handle(self):
        return self._h

    def process(self, x, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty_like(x)
        _check(lib().filark_sos_process(self._h, _dev_f32(x, "x"), _dev_f32(out, "out"), x.shape[1],
                                        x.shape[0], _stream(stream)))
        return out

    def filtfilt(self, x, out=None, stream=None):
        """Zero-phase filtering of a whole window (forward, then backward in
        time, each from rest); the carried state is not used or changed."""
        import torch

        if out is None:
            out = torch.empty_like(x)
        _check(lib().filark_sos_filtfilt(self._h, _dev_f32(x, "x"), _dev_f32(out, "out"), x.shape[1],
                                         x.shape[0], _stream(stream)))
        return out

    def filtfilt_noalloc(self, x, out, stream=None):
        """filtfilt() through the allocation-free entry point: the passes'
        state lives in a fixed per-GPU array (2 * sections * channels <=
        131072); `out` must be given.  Overlapping calls on one GPU race."""
        _check(lib().filark_sos_filtfilt_noalloc(self._h, _dev_f32(x, "x"), _dev_f32(out, "out"), x.shape[1],
                                                 x.shape[0], _stream(stream)))
        return out

    def get_state(self, stream=None) -> np.ndarray:
        buf = np.empty((self.n_ch, self.n_sec, 2), dtype=np.float64)
        _check(lib().filark_state_get(self._h, STATE_SOS, buf.ctypes.data, buf.nbytes, _stream(stream)))
        return buf

    def set_state(self, z, stream=None):
        buf = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        _check(lib().filark_state_set(self._h, STATE_SOS, buf.ctypes.data, buf.nbytes, _stream(stream)))

    def check(self, stream=None):
        _check(lib().filark_check(self._h, STATE_SOS, _stream(stream)))

    def set_tile(self, block: int, waves: int, group: int = 8, stream=None):
        """Tile shape: `block` samples per lane, `waves` per workgroup, `group`
        channels per workgroup."""
        _check(lib().filark_tile_set(self._h, STATE_SOS, int(block), int(waves), int(group), _stream(stream)))

    def tile(self):
        b, w, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().filark_tile_get(self._h, STATE_SOS, ctypes.byref(b), ctypes.byref(w), ctypes.byref(g)))
        return b.value, w.value, g.value

    def set_adjoint_tile(self, block: int, waves: int, group: int = 8, stream=None):
        _check(lib().filark_tile_set(self._h, TILE_SOS_ADJOINT, int(block), int(waves), int(group), _stream(stream)))

    def adjoint_tile(self):
        b, w, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().filark_tile_get(self._h, TILE_SOS_ADJOINT, ctypes.byref(b), ctypes.byref(w), ctypes.byref(g)))
        return b.value, w.value, g.value

    def set_adjoint_windows(self, max_windows: int):
        """Most adjoint windows per kernel launch (0: no limit, 1: one launch
        per window); results are bit-identical for every value."""
        _check(lib().filark_adjoint_windows_set(self._h, int(max_windows)))

    def state_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().filark_state_bytes(self._h, STATE_SOS, ctypes.byref(n)))
        return n.value

    def save(self, buf=None, stream=None):
        """Copy the device state into `buf` (a CUDA uint8 tensor; allocated if None)."""
        import torch

        if buf is None:
            buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device="cuda")
        if not buf.is_cuda or buf.numel() * buf.element_size() < self.state_bytes():
            raise FilarkError(EINVAL, "checkpoint buffer too small")
        _check(lib().filark_state_save(self._h, STATE_SOS, ctypes.c_void_p(buf.data_ptr()), _stream(stream)))
        return buf

    def load(self, buf, stream=None):
        if not buf.is_cuda or buf.numel() * buf.element_size() < self.state_bytes():
            raise FilarkError(EINVAL, "checkpoint buffer too small")
        _check(lib().filark_state_load(self._h, STATE_SOS, ctypes.c_void_p(buf.data_ptr()), _stream(stream)))

    def close(self):
        if self._h:
            lib().filark_sos_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StaLtaState:
    """Recursive STA/LTA state (windows in seconds, rounded to samples)."""

    def __init__(self, sta_s: float, lta_s: float, fs: float, n_ch: int, stream=None):
        self._h = ctypes.c_void_p()
        self.n_ch = int(n_ch)
        self.nsta = int(round(sta_s * fs))
        self.nlta = int(round(lta_s * fs))
        _check(lib().filark_stalta_init(ctypes.byref(self._h), float(sta_s), float(lta_s), float(fs),
                                        self.n_ch, _stream(stream)))

    @property
    def handle(self):
        return self._h

    def process(self, y, cf=None, stream=None):
        import torch

        if cf is None:
            cf = torch.empty_like(y)
        _check(lib().filark_stalta_process(self._h, _dev_f32(y, "y"), _dev_f32(cf, "cf"), y.shape[1],
                                           y.shape[0], _stream(stream)))
        return cf

    def get_state(self, stream=None):
        buf = np.empty(self.n_ch * 2 + 1, dtype=np.float64)
        _check(lib().filark_state_get(self._h, STATE_STALTA, buf.ctypes.data, buf.nbytes, _stream(stream)))
        counter = int(buf[-1:].view(np.int64)[0])
        return buf[:-1].reshape(self.n_ch, 2).copy(), counter

    def set_state(self, st, counter: int, stream=None):
        buf = np.empty(self.n_ch * 2 + 1, dtype=np.float64)
        buf[:-1] = np.asarray(st, dtype=np.float64).reshape(-1)
        buf[-1:] = np.array([int(counter)], dtype=np.int64).view(np.float64)
        _check(lib().filark_state_set(self._h, STATE_STALTA, buf.ctypes.data, buf.nbytes, _stream(stream)))

    def check(self, stream=None):
        _check(lib().filark_check(self._h, STATE_STALTA, _stream(stream)))

    def set_tile(self, block: int, waves: int, group: int = 8, stream=None):
        """Tile shape: `block` samples per lane, `waves` per workgroup, `group`
        channels per workgroup."""
        _check(lib().filark_tile_set(self._h, STATE_STALTA, int(block), int(waves), int(group), _stream(stream)))

    def tile(self):
        b, w, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().filark_tile_get(self._h, STATE_STALTA, ctypes.byref(b), ctypes.byref(w), ctypes.byref(g)))
        return b.value, w.value, g.value

    def set_adjoint_tile(self, block: int, waves: int, group: int = 8, stream=None):
        _check(lib().filark_tile_set(self._h, TILE_STALTA_ADJOINT, int(block), int(waves), int(group), _stream(stream)))

    def adjoint_tile(self):
        b, w, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().filark_tile_get(self._h, TILE_STALTA_ADJOINT, ctypes.byref(b), ctypes.byref(w), ctypes.byref(g)))
        return b.value, w.value, g.value

    def state_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().filark_state_bytes(self._h, STATE_STALTA, ctypes.byref(n)))
        return n.value

    def save(self, buf=None, stream=None):
        """Copy the device state into `buf` (a CUDA uint8 tensor; allocated if None)."""
        import torch

        if buf is None:
            buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device="cuda")
        if not buf.is_cuda or buf.numel() * buf.element_size() < self.state_bytes():
            raise FilarkError(EINVAL, "checkpoint buffer too small")
        _check(lib().filark_state_save(self._h, STATE_STALTA, ctypes.c_void_p(buf.data_ptr()), _stream(stream)))
        return buf

    def load(self, buf, stream=None):
        if not buf.is_cuda or buf.numel() * buf.element_size() < self.state_bytes():
            raise FilarkError(EINVAL, "checkpoint buffer too small")
        _check(lib().filark_state_load(self._h, STATE_STALTA, ctypes.c_void_p(buf.data_ptr()), _stream(stream)))

    def close(self):
        if self._h:
            lib().filark_stalta_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sos_stalta_process(sos: SOSState, sl: StaLtaState, x, y=None, cf=None, write_y: bool = True,
                       stream=None):
    """Fused chunk: y = SOS(x), cf = STA/LTA(y).  Returns (y or None, cf)."""
    import torch

    if cf is None:
        cf = torch.empty_like(x)
    if write_y and y is None:
        y = torch.empty_like(x)
    yp = _dev_f32(y, "y") if (write_y and y is not None) else ctypes.c_void_p(0)
    _check(lib().filark_sos_stalta_process(sos.handle, sl.handle, _dev_f32(x, "x"), yp, _dev_f32(cf, "cf"),
                                           x.shape[1], x.shape[0], _stream(stream)))
    return (y if write_y else None), cf


def sos_stalta_adjoint(sos: SOSState, sl: StaLtaState, x, g, gx=None, adj=None, gsos=None, mode: str = "grad",
                       scale: float = 1.0, stream=None):
    """Adjoint of the fused path over one chunk (states hold the chunk-start
    checkpoint).  mode "grad": g = dL/dcf; mode "mse": g = target cf and
    L = scale * sum (cf - g)^2.  adj [2K+2, n_ch] float64 carries the adjoint
    state (after the chunk in, before it out); gsos [K, 5] float64 is added to.
    Returns (gx, adj, gsos)."""
    import torch

    n_t, n_ch = x.shape
    K = sos.n_sec
    if gx is None:
        gx = torch.empty_like(x)
    if adj is None:
        adj = torch.zeros((2 * K + 2, n_ch), dtype=torch.float64, device=x.device)
    if gsos is None:
        gsos = torch.zeros((K, 5), dtype=torch.float64, device=x.device)
    for t, name in ((adj, "adj"), (gsos, "gsos")):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise FilarkError(EINVAL, f"{name} must be a contiguous float64 CUDA tensor")
    if adj.shape != (2 * K + 2, n_ch) or gsos.shape != (K, 5):
        raise FilarkError(EINVAL, "adj must be [2K+2, n_ch] and gsos [K, 5]")
    m = {"grad": ADJ_GRAD, "mse": ADJ_MSE}[mode]
    _check(lib().filark_sos_stalta_adjoint(sos.handle, sl.handle, _dev_f32(x, "x"), _dev_f32(g, "g"), m,
                                           float(scale), _dev_f32(gx, "gx"), ctypes.c_void_p(adj.data_ptr()),
                                           ctypes.c_void_p(gsos.data_ptr()), n_ch, n_t, _stream(stream)))
    return gx, adj, gsos


def adjoint_tape_bytes(sos: SOSState, sl: StaLtaState, n_t: int) -> int:
    """Bytes of the adjoint tape of one chunk of n_t rows."""
    n = ctypes.c_size_t()
    _check(lib().filark_adjoint_tape_bytes(sos.handle, sl.handle, int(n_t), ctypes.byref(n)))
    return int(n.value)


def sos_stalta_process_tape(sos: SOSState, sl: StaLtaState, x, tape=None, y=None, cf=None, stream=None):
    """The fused forward over one chunk that also records the chunk's adjoint
    tape (the forward state at every adjoint window start).  tape: a uint8
    CUDA tensor of adjoint_tape_bytes bytes (allocated if None).  Returns
    (y or None, cf, tape)."""
    import torch

    n_t, n_ch = x.shape
    if cf is None:
        cf = torch.empty_like(x)
    if tape is None:
        tape = torch.empty(adjoint_tape_bytes(sos, sl, n_t), dtype=torch.uint8, device=x.device)
    if not tape.is_cuda or not tape.is_contiguous():
        raise FilarkError(EINVAL, "tape must be a contiguous CUDA tensor")
    _check(lib().filark_sos_stalta_process_tape(sos.handle, sl.handle, _dev_f32(x, "x"),
                                                _dev_f32(y, "y") if y is not None else None, _dev_f32(cf, "cf"),
                                                ctypes.c_void_p(tape.data_ptr()), tape.numel() * tape.element_size(),
                                                n_ch, n_t, _stream(stream)))
    return y, cf, tape


def sos_stalta_adjoint_tape(sos: SOSState, sl: StaLtaState, tape, x, g, gx=None, adj=None, gsos=None,
                            mode: str = "grad", scale: float = 1.0, stream=None):
    """sos_stalta_adjoint from the chunk's tape (the objects' state is not
    used).  Returns (gx, adj, gsos)."""
    import torch

    n_t, n_ch = x.shape
    K = sos.n_sec
    if gx is None:
        gx = torch.empty_like(x)
    if adj is None:
        adj = torch.zeros((2 * K + 2, n_ch), dtype=torch.float64, device=x.device)
    if gsos is None:
        gsos = torch.zeros((K, 5), dtype=torch.float64, device=x.device)
    for t, name in ((adj, "adj"), (gsos, "gsos")):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise FilarkError(EINVAL, f"{name} must be a contiguous float64 CUDA tensor")
    if adj.shape != (2 * K + 2, n_ch) or gsos.shape != (K, 5):
        raise FilarkError(EINVAL, "adj must be [2K+2, n_ch] and gsos [K, 5]")
    if not tape.is_cuda or not tape.is_contiguous():
        raise FilarkError(EINVAL, "tape must be a contiguous CUDA tensor")
    m = {"grad": ADJ_GRAD, "mse": ADJ_MSE}[mode]
    _check(lib().filark_sos_stalta_adjoint_tape(sos.handle, sl.handle, ctypes.c_void_p(tape.data_ptr()),
                                                tape.numel() * tape.element_size(),
                                                _dev_f32(x, "x"), _dev_f32(g, "g"), m, float(scale),
                                                _dev_f32(gx, "gx"), ctypes.c_void_p(adj.data_ptr()),
                                                ctypes.c_void_p(gsos.data_ptr()), n_ch, n_t, _stream(stream)))
    return gx, adj, gsos


def tune_tile(st: SOSState, n_t: int, block: int = 0, waves: int = 0, cache: str | None = None, stream=None):
    """Time the tile candidates for st's filter and channel count on a chunk of
    n_t rows (filark_autotune), apply the fastest to st and return it as
    (block, waves, group); block / waves 0 are searched, else kept."""
    b, w, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().filark_autotune(st.handle, int(n_t), int(block), int(waves),
                                 cache.encode() if cache else None, ctypes.byref(b), ctypes.byref(w),
                                 ctypes.byref(g), _stream(stream)))
    return b.value, w.value, g.value


class Batch:
    """Many independent SOS streams filtered by one launch sequence (see
    filark_batch_* in include/filark.h).  Each stream keeps its SOSState;
    all states must share the tile's block and waves, the group may differ."""

    def __init__(self, states, stream=None):
        self.states = list(states)
        arr = (ctypes.c_void_p * len(self.states))(*[st.handle.value for st in self.states])
        self._h = ctypes.c_void_p()
        _check(lib().filark_batch_create(ctypes.byref(self._h), len(self.states), arr, _stream(stream)))
        self._bound = None

    def bind(self, xs, ys, stream=None):
        """One chunk per stream: xs[s], ys[s] float32 CUDA tensors [n_t_s, n_ch_s]."""
        n = len(self.states)
        if len(xs) != n or len(ys) != n:
            raise FilarkError(EINVAL, "need one input and one output per stream")
        ins = (ctypes.c_void_p * n)()
        outs = (ctypes.c_void_p * n)()
        nts = (ctypes.c_int64 * n)()
        for i, (x, y, st) in enumerate(zip(xs, ys, self.states)):
            if x.shape[1] != st.n_ch or y.shape != x.shape:
                raise FilarkError(ESHAPE, f"stream {i}: shapes do not match its state")
            ins[i] = _dev_f32(x, "x").value
            outs[i] = _dev_f32(y, "y").value
            nts[i] = x.shape[0]
        _check(lib().filark_batch_bind(self._h, ins, outs, nts, _stream(stream)))
        self._bound = (list(xs), list(ys))  # keep the buffers alive while bound

    def launch(self, stream=None):
        """One launch of the bound work (a replay of the captured graph after capture())."""
        _check(lib().filark_batch_launch(self._h, _stream(stream)))

    def capture(self):
        """Capture the launch sequence in a graph the batch owns; launch() then replays it."""
        _check(lib().filark_batch_capture(self._h))

    def stamps(self, stream=None) -> np.ndarray:
        """Per-stream completion ticks and, last, the start tick (100 MHz)."""
        out = np.zeros(len(self.states) + 1, dtype=np.uint64)
        _check(lib().filark_batch_stamps(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                         _stream(stream)))
        return out

    def close(self):
        if self._h:
            lib().filark_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def monitor_process(sos: SOSState, sl: StaLtaState, trig: "Trigger", x, events, count, y=None, cf=None,
                    stream=None):
    """The monitor chain in one pass (filark_monitor_process): x float32 CUDA
    [n_t, n_ch] through the cascade, the STA/LTA and the trigger; events int64
    CUDA [cap, 3] and count (one 64-bit CUDA element) as Trigger.process; y and
    cf (float32 CUDA [n_t, n_ch]) are written only when given.  Asynchronous."""
    import torch

    n_t, n_ch = x.shape
    if not (isinstance(events, torch.Tensor) and events.is_cuda and events.dtype == torch.int64
            and events.dim() == 2 and events.shape[1] == 3 and events.is_contiguous()):
        raise FilarkError(EINVAL, "events must be a contiguous int64 CUDA tensor [cap, 3]")
    if not (isinstance(count, torch.Tensor) and count.is_cuda and count.numel() == 1 and count.element_size() == 8):
        raise FilarkError(EINVAL, "count must be a one-element 64-bit CUDA tensor")
    yp = _dev_f32(y, "y") if y is not None else ctypes.c_void_p(0)
    cp = _dev_f32(cf, "cf") if cf is not None else ctypes.c_void_p(0)
    _check(lib().filark_monitor_process(sos.handle, sl.handle, trig._h, _dev_f32(x, "x"), yp, cp,
                                        ctypes.c_void_p(events.data_ptr()), events.shape[0],
                                        ctypes.c_void_p(count.data_ptr()), n_ch, n_t, _stream(stream)))


class Trigger:
    """Two-threshold trigger on cf (filark_trigger_* in include/filark.h):
    events (channel, t_on, t_off) of the chunks passed to process(), with the
    open events and the sample counter carried between calls."""

    def __init__(self, n_ch: int, on: float, off: float, stream=None):
        self.n_ch = int(n_ch)
        self._h = ctypes.c_void_p()
        _check(lib().filark_trigger_init(ctypes.byref(self._h), float(on), float(off), self.n_ch, _stream(stream)))

    def process(self, cf, events, count, stream=None):
        """cf: float32 CUDA [n_t, n_ch]; events: int64 CUDA [cap, 3]; count:
        uint64/int64 CUDA [1], advanced by the events of this chunk (stored at
        count + i while below cap).  Asynchronous."""
        import torch

        if cf.shape[1] != self.n_ch:
            raise FilarkError(ESHAPE, "cf channels do not match the trigger")
        if not (isinstance(events, torch.Tensor) and events.is_cuda and events.dtype == torch.int64
                and events.dim() == 2 and events.shape[1] == 3 and events.is_contiguous()):
            raise FilarkError(EINVAL, "events must be a contiguous int64 CUDA tensor [cap, 3]")
        if not (isinstance(count, torch.Tensor) and count.is_cuda and count.numel() == 1
                and count.element_size() == 8):
            raise FilarkError(EINVAL, "count must be a one-element 64-bit CUDA tensor")
        _check(lib().filark_trigger_process(self._h, _dev_f32(cf, "cf"), self.n_ch, cf.shape[0],
                                            ctypes.c_void_p(events.data_ptr()), events.shape[0],
                                            ctypes.c_void_p(count.data_ptr()), _stream(stream)))

    def get_state(self, stream=None):
        """(open_ton int64 [n_ch, 2] = (open flag, start of the open event), counter)."""
        ot = np.zeros((self.n_ch, 2), dtype=np.int64)
        g = ctypes.c_int64(0)
        _check(lib().filark_trigger_state_get(self._h, ot.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                              ctypes.byref(g), _stream(stream)))
        return ot, int(g.value)

    def set_state(self, open_ton, counter: int, stream=None):
        ot = np.ascontiguousarray(np.asarray(open_ton, dtype=np.int64).reshape(self.n_ch, 2))
        _check(lib().filark_trigger_state_set(self._h, ot.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                              int(counter), _stream(stream)))

    def close(self):
        if self._h:
            lib().filark_trigger_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


EMA_MODES = {"demean": 0, "agc": 1}


class Ema:
    """Stateful running-mean removal ("demean") or running AGC ("agc") over a
    win_s-second exponential average (filark_ema_* in include/filark.h)."""

    def __init__(self, n_ch: int, win_s: float, fs: float, mode: str, stream=None):
        self.n_ch = int(n_ch)
        self._h = ctypes.c_void_p()
        _check(lib().filark_ema_init(ctypes.byref(self._h), EMA_MODES[mode], float(win_s), float(fs), self.n_ch,
                                     _stream(stream)))

    def process(self, x, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty_like(x)
        _check(lib().filark_ema_process(self._h, _dev_f32(x, "x"), _dev_f32(out, "out"), x.shape[1], x.shape[0],
                                        _stream(stream)))
        return out

    def get_state(self, stream=None) -> np.ndarray:
        buf = np.zeros(self.n_ch, dtype=np.float64)
        _check(lib().filark_ema_state_get(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          _stream(stream)))
        return buf

    def set_state(self, avg, stream=None):
        buf = np.ascontiguousarray(np.asarray(avg, dtype=np.float64).reshape(self.n_ch))
        _check(lib().filark_ema_state_set(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          _stream(stream)))

    def close(self):
        if self._h:
            lib().filark_ema_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Fir:
    """Realtime FIR y[t] = sum_k h[k] x[t - k] with the last len(taps) - 1
    samples of every channel carried between calls (filark_fir_* in
    include/filark.h).  Input and output must not overlap."""

    def __init__(self, taps, n_ch: int, stream=None):
        h = np.ascontiguousarray(np.asarray(taps, dtype=np.float64).ravel())
        self.n_taps = int(h.size)
        self.n_ch = int(n_ch)
        self._h = ctypes.c_void_p()
        _check(lib().filark_fir_init(ctypes.byref(self._h), h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     self.n_taps, self.n_ch, _stream(stream)))

    def set_tile(self, rows: int, waves: int, order: int = 2):
        _check(lib().filark_fir_set_tile(self._h, int(rows), int(waves), int(order)))

    def set_method(self, method: str, stream=None):
        """'direct' (default) or 'fft' (FFT filtering in 2048-row windows,
        up to 1024 taps); the carried history is shared by both."""
        m = {"direct": 0, "fft": 1}[method]
        _check(lib().filark_fir_set_method(self._h, m, _stream(stream)))

    def process(self, x, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty_like(x)
        _check(lib().filark_fir_process(self._h, _dev_f32(x, "x"), _dev_f32(out, "out"), x.shape[1], x.shape[0],
                                        _stream(stream)))
        return out

    def get_state(self, stream=None) -> np.ndarray:
        buf = np.zeros((max(self.n_taps - 1, 0), self.n_ch), dtype=np.float32)
        _check(lib().filark_fir_state_get(self._h, buf.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return buf

    def set_state(self, hist, stream=None):
        buf = np.ascontiguousarray(np.asarray(hist, dtype=np.float32).reshape(max(self.n_taps - 1, 0), self.n_ch))
        _check(lib().filark_fir_state_set(self._h, buf.ctypes.data_as(ctypes.c_void_p), _stream(stream)))

    def close(self):
        if self._h:
            lib().filark_fir_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
