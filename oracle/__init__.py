"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never loads it and
shares no code with it.  See ``oracle.c`` for the definitions it follows.

Every function here takes and returns float64 numpy arrays in the time-major
layout ``[n_t, n_ch]``.

Parity status: design, filter and STA/LTA are pinned by closed forms, brute
force, invariants and library special cases in ``tests/test_oracle_*.py``;
the trigger, zero-phase filtering, running averages and the FIR by closed
forms, brute force and library special cases in their own test files;
the gradient routines are pinned by finite differences, the transpose
(dot-product) identity and an independent autodiff in
``tests/test_oracle_grad.py``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BTYPES = {"lowpass": 0, "highpass": 1, "bandpass": 2, "bandstop": 3}

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11",
               "-D_DEFAULT_SOURCE", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        I64 = ctypes.c_int64
        L.oracle_butter_sos.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, D, ctypes.POINTER(ctypes.c_int)]
        L.oracle_butter_sos.restype = ctypes.c_int
        for name in ("oracle_sos_filter", "oracle_sos_filter_ld"):
            f = getattr(L, name)
            f.argtypes = [D, ctypes.c_int, D, D, I64, I64, D]
            f.restype = None
        L.oracle_stalta.argtypes = [D, D, I64, I64, I64, I64, D, ctypes.POINTER(I64)]
        L.oracle_stalta.restype = None
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _register_grad(L)
        L.oracle_trigger.argtypes = [ctypes.POINTER(ctypes.c_float), I64, I64, ctypes.c_float, ctypes.c_float,
                                     ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(I64), I64,
                                     ctypes.POINTER(I64), I64]
        L.oracle_trigger.restype = I64
        L.oracle_sos_filtfilt.argtypes = [D, ctypes.c_int, D, D, I64, I64]
        L.oracle_sos_filtfilt.restype = None
        L.oracle_ema_op.argtypes = [D, D, I64, I64, I64, ctypes.c_int, D]
        L.oracle_ema_op.restype = None
        L.oracle_fir.argtypes = [D, ctypes.c_int, D, D, I64, I64, D]
        L.oracle_fir.restype = None
        _lib = L
    return _lib


def _register_grad(L):
    D = ctypes.POINTER(ctypes.c_double)
    I64 = ctypes.c_int64
    L.oracle_sos_stalta_grad.argtypes = [D, ctypes.c_int, D, D, I64, I64, I64, I64, I64, ctypes.c_double,
                                         D, D, D, D, D, D]
    L.oracle_sos_stalta_grad.restype = None
    L.oracle_sos_vjp.argtypes = [D, ctypes.c_int, D, D, I64, I64, D, D, D, D]
    L.oracle_sos_vjp.restype = None


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


class OracleError(RuntimeError):
    pass


def butter_sos(order: int, btype: str, f1: float, f2: float = 0.0, fs: float = 1.0) -> np.ndarray:
    """Butterworth SOS by the bilinear transform; rows {b0 b1 b2 1 a1 a2}."""
    n_max = (order + 1) // 2
    out = np.zeros((max(1, n_max), 6), dtype=np.float64)
    n = ctypes.c_int(0)
    rc = lib().oracle_butter_sos(int(order), BTYPES[btype], float(f1), float(f2), float(fs), _ptr(out),
                                 ctypes.byref(n))
    if rc != 0:
        raise OracleError(f"oracle_butter_sos failed with status {rc}")
    return out[: n.value].copy()


def sos_filter(sos, x, zi=None, extended: bool = False):
    """Run the DF2T cascade over x [n_t, n_ch]; returns (y, zf) with zf [n_ch, n_sec, 2]."""
    sos = _f64(sos)
    x = _f64(x)
    if x.ndim == 1:
        x = x[:, None]
    n_t, n_ch = x.shape
    n_sec = sos.shape[0]
    z = np.zeros((n_ch, n_sec, 2)) if zi is None else _f64(zi).copy()
    assert z.shape == (n_ch, n_sec, 2)
    y = np.empty_like(x)
    f = lib().oracle_sos_filter_ld if extended else lib().oracle_sos_filter
    f(_ptr(sos), n_sec, _ptr(x), _ptr(y), n_ch, n_t, _ptr(z))
    return y, z


def sos_filtfilt(sos, x) -> np.ndarray:
    """Zero-phase filtering of the window x [n_t, n_ch]: the cascade forward
    from rest, then backward in time from rest (oracle_sos_filtfilt)."""
    sos = _f64(sos)
    x = _f64(x)
    if x.ndim == 1:
        x = x[:, None]
    y = np.empty_like(x)
    lib().oracle_sos_filtfilt(_ptr(sos), sos.shape[0], _ptr(x), _ptr(y), x.shape[1], x.shape[0])
    return y


def stalta(y, nsta: int, nlta: int, st=None, g0: int = 0):
    """Recursive STA/LTA of y [n_t, n_ch]; returns (cf, st [n_ch, 2], g)."""
    y = _f64(y)
    if y.ndim == 1:
        y = y[:, None]
    n_t, n_ch = y.shape
    s = np.zeros((n_ch, 2)) if st is None else _f64(st).copy()
    cf = np.empty_like(y)
    g = ctypes.c_int64(int(g0))
    lib().oracle_stalta(_ptr(y), _ptr(cf), n_ch, n_t, int(nsta), int(nlta), _ptr(s), ctypes.byref(g))
    return cf, s, int(g.value)


def window_samples(seconds: float, fs: float) -> int:
    """Window length in samples: round(T * fs) (reading R4)."""
    return int(round(seconds * fs))


class Stream:
    """Chunked SOS + STA/LTA with carried state, the oracle's process(chunk, state)."""

    def __init__(self, sos, n_ch: int, nsta: int | None = None, nlta: int | None = None):
        self.sos = _f64(sos)
        self.n_ch = n_ch
        self.zi = np.zeros((n_ch, self.sos.shape[0], 2))
        self.nsta, self.nlta = nsta, nlta
        self.st = np.zeros((n_ch, 2))
        self.g = 0

    def process(self, x):
        y, self.zi = sos_filter(self.sos, x, self.zi)
        if self.nsta is None:
            return y, None
        cf, self.st, self.g = stalta(y, self.nsta, self.nlta, self.st, self.g)
        return y, cf


def stalta_grad(sos, x, tgt, nsta: int, nlta: int, scale: float, zi0=None, st0=None, g0: int = 0,
                adj=None):
    """Reverse-mode gradient of loss = scale * sum (cf - tgt)^2 over one chunk.

    x, tgt: [n_t, n_ch].  zi0 [n_ch, n_sec, 2], st0 [n_ch, 2], g0: the forward
    state at the chunk start (the checkpoint).  adj [n_ch, 2 n_sec + 2]: the
    adjoint of the state after the chunk (zero after the record's end).
    Returns (loss, gx [n_t, n_ch], gsos [n_sec, 5] for (b0, b1, b2, a1, a2),
    adj_before [n_ch, 2 n_sec + 2]).
    """
    sos = _f64(sos)
    x = _f64(x)
    tgt = _f64(tgt)
    n_t, n_ch = x.shape
    n_sec = sos.shape[0]
    z = np.zeros((n_ch, n_sec, 2)) if zi0 is None else _f64(zi0)
    st = np.zeros((n_ch, 2)) if st0 is None else _f64(st0)
    a = np.zeros((n_ch, 2 * n_sec + 2)) if adj is None else _f64(adj).copy()
    gx = np.empty_like(x)
    gsos = np.zeros((n_sec, 5))
    loss = np.zeros(1)
    lib().oracle_sos_stalta_grad(_ptr(sos), n_sec, _ptr(x), _ptr(tgt), n_ch, n_t, int(nsta), int(nlta),
                                 int(g0), float(scale), _ptr(z), _ptr(st), _ptr(a), _ptr(gx), _ptr(gsos),
                                 _ptr(loss))
    return float(loss[0]), gx, gsos, a


def sos_vjp(sos, x, gy, zi0=None, adjz=None):
    """(dy/dx)^T gy and sum gy . dy/dtheta of the cascade over one chunk.

    Returns (gx [n_t, n_ch], gsos [n_sec, 5], adjz_before [n_ch, n_sec, 2]).
    """
    sos = _f64(sos)
    x = _f64(x)
    gy = _f64(gy)
    n_t, n_ch = x.shape
    n_sec = sos.shape[0]
    z = np.zeros((n_ch, n_sec, 2)) if zi0 is None else _f64(zi0)
    a = np.zeros((n_ch, n_sec, 2)) if adjz is None else _f64(adjz).copy()
    gx = np.empty_like(x)
    gsos = np.zeros((n_sec, 5))
    lib().oracle_sos_vjp(_ptr(sos), n_sec, _ptr(x), _ptr(gy), n_ch, n_t, _ptr(z), _ptr(a), _ptr(gx),
                         _ptr(gsos))
    return gx, gsos, a


def stalta_loss(sos, x, tgt, nsta: int, nlta: int, scale: float) -> float:
    """loss = scale * sum (cf - tgt)^2 of one record from the zero state (forward only)."""
    y, _ = sos_filter(sos, x)
    cf, _, _ = stalta(y, nsta, nlta)
    return float(scale * np.sum((cf - _f64(tgt)) ** 2))


class Trigger:
    """Stateful two-threshold trigger on cf (oracle_trigger): process(cf32)
    takes a float32 chunk [n_t, n_ch] and returns its events as int64
    [n_events, 3] rows (channel, t_on, t_off), channel by channel in time
    order; the open flags, open-event starts and the global sample counter
    carry over to the next call."""

    def __init__(self, n_ch: int, on: float, off: float):
        self.n_ch = int(n_ch)
        self.on = np.float32(on)
        self.off = np.float32(off)
        self.open = np.zeros(self.n_ch, dtype=np.uint8)
        self.t_on = np.zeros(self.n_ch, dtype=np.int64)
        self.g = 0

    def process(self, cf) -> np.ndarray:
        cf = np.ascontiguousarray(np.asarray(cf, dtype=np.float32))
        if cf.ndim == 1:
            cf = cf[:, None]
        n_t, n_ch = cf.shape
        assert n_ch == self.n_ch
        def run(ev, cap):
            return lib().oracle_trigger(cf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n_ch, n_t, self.on,
                                        self.off, self.open.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                        self.t_on.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), self.g,
                                        ev.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cap)

        # count first (from a copy of the state), then store exactly that many
        o0, t0 = self.open.copy(), self.t_on.copy()
        n = run(np.zeros((1, 3), dtype=np.int64), 0)
        self.open[:], self.t_on[:] = o0, t0
        ev = np.zeros((max(1, n), 3), dtype=np.int64)
        assert run(ev, n) == n
        self.g += n_t
        return ev[:n].copy()


EMA_MODES = {"demean": 0, "agc": 1}


class Ema:
    """Stateful running-mean removal ("demean") or running AGC ("agc") with
    an n_win-sample exponential average (oracle_ema_op); the average carries
    over to the next call."""

    def __init__(self, n_ch: int, n_win: int, mode: str):
        self.n_ch, self.n_win, self.mode = int(n_ch), int(n_win), EMA_MODES[mode]
        self.avg = np.zeros(self.n_ch)

    def process(self, x) -> np.ndarray:
        x = _f64(x)
        if x.ndim == 1:
            x = x[:, None]
        y = np.empty_like(x)
        lib().oracle_ema_op(_ptr(x), _ptr(y), x.shape[1], x.shape[0], self.n_win, self.mode, _ptr(self.avg))
        return y


class Fir:
    """Realtime FIR y[t] = sum_k h[k] x[t - k] with the last M - 1 samples of
    every channel carried between calls (oracle_fir)."""

    def __init__(self, taps, n_ch: int):
        self.h = _f64(np.asarray(taps, dtype=np.float64).ravel())
        self.n_ch = int(n_ch)
        self.hist = np.zeros((max(0, len(self.h) - 1), self.n_ch))

    def process(self, x) -> np.ndarray:
        x = _f64(x)
        if x.ndim == 1:
            x = x[:, None]
        y = np.empty_like(x)
        hist = self.hist if self.hist.size else np.zeros((1, self.n_ch))
        lib().oracle_fir(_ptr(self.h), len(self.h), _ptr(x), _ptr(y), x.shape[1], x.shape[0], _ptr(hist))
        return y
