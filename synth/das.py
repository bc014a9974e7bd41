"""Seeded synthetic channel x time DAS records (time-major, FP32).

Layout: every record is a ``torch.float32`` tensor of shape ``[n_t, n_ch]``
(time-major, channel contiguous), the ``dims='nt_nc'`` convention of the
paper's binary tape (Section 3.5, streaming-aware I/O).

The paper measures its causal IIR on ocean-cable DAS files that are not
available here; these generators stand in for them with the shapes and
structure of the workloads: Gaussian or 1/f background noise, Ricker-wavelet
events with linear moveout across channels, and a slow drift.

Random numbers come from ``torch.Generator`` objects seeded with the given
integer, on the device the record is built on.  CPU and GPU generators are
different algorithms, so a record depends on (seed, device); consumers that
compare two implementations feed both the same materialised tensor.  Event
parameters (times, velocities, signs) are drawn on the host with numpy's
PCG64 and are device independent.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

RICKER_HALF_WINDOW_S = 0.1  # exp(-(pi f0 tau)^2) < 1e-16 beyond this at f0 = 20 Hz


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def white_noise(n_t: int, n_ch: int, seed: int, device="cpu", sigma: float = 1.0) -> torch.Tensor:
    """N(0, sigma^2) samples, float32 [n_t, n_ch]."""
    g = _gen(seed, device)
    x = torch.randn((n_t, n_ch), generator=g, device=device, dtype=torch.float32)
    if sigma != 1.0:
        x.mul_(sigma)
    return x


def pink_noise(n_t: int, n_ch: int, seed: int, device="cpu", block: int = 512) -> torch.Tensor:
    """1/f-coloured Gaussian noise, float32 [n_t, n_ch], unit variance per channel.

    White noise is shaped in the frequency domain by an f^(-1/2) amplitude
    (power ~ 1/f) with the DC bin zeroed, then each channel is scaled to
    sigma = 1.  Channels are processed in blocks to bound memory.
    """
    out = torch.empty((n_t, n_ch), device=device, dtype=torch.float32)
    g = _gen(seed, device)
    n_f = n_t // 2 + 1
    f = torch.arange(n_f, device=device, dtype=torch.float32)
    shape = torch.zeros_like(f)
    shape[1:] = f[1:].rsqrt()
    for c0 in range(0, n_ch, block):
        c1 = min(n_ch, c0 + block)
        w = torch.randn((n_t, c1 - c0), generator=g, device=device, dtype=torch.float32)
        spec = torch.fft.rfft(w, dim=0)
        spec.mul_(shape[:, None])
        col = torch.fft.irfft(spec, n=n_t, dim=0)
        col.sub_(col.mean(dim=0, keepdim=True))
        std = col.std(dim=0, keepdim=True).clamp_min(1e-30)
        out[:, c0:c1] = col / std
    return out


@dataclasses.dataclass
class Event:
    t0: float        # arrival time at channel 0 [s]
    velocity: float  # apparent velocity [m/s]
    sign: int        # +1: moveout toward higher channels, -1: toward lower
    amplitude: float
    f0: float        # Ricker peak frequency [Hz]


def draw_events(n_events: int, seed: int, t_max: float, v_lo: float, v_hi: float,
                amplitude: float = 5.0, f0: float = 20.0, random_sign: bool = True) -> list[Event]:
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    t0 = rng.uniform(0.0, t_max, size=n_events)
    v = rng.uniform(v_lo, v_hi, size=n_events) if v_hi > v_lo else np.full(n_events, v_lo)
    s = rng.choice([-1, 1], size=n_events) if random_sign else np.ones(n_events, dtype=int)
    return [Event(float(t0[i]), float(v[i]), int(s[i]), amplitude, f0) for i in range(n_events)]


def ricker_events(x: torch.Tensor, fs: float, dx: float, events: list[Event]) -> torch.Tensor:
    """Add Ricker wavelets with linear moveout to ``x`` [n_t, n_ch] in place.

    Wavelet r(tau) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), evaluated
    analytically at each sample's offset from the fractional arrival time
    t_c = t0 + sign * c * dx / v.  Each event is added by a separate indexed
    add with unique indices, so the result does not depend on thread order.
    """
    n_t, n_ch = x.shape
    dev = x.device
    c = torch.arange(n_ch, device=dev, dtype=torch.float64)
    half = int(math.ceil(RICKER_HALF_WINDOW_S * fs))
    offs = torch.arange(-half, half + 1, device=dev, dtype=torch.int64)
    flat = x.view(-1)
    for ev in events:
        tc = ev.t0 + ev.sign * c * dx / ev.velocity                 # [n_ch]
        i0 = torch.floor(tc * fs).to(torch.int64)                    # [n_ch]
        idx = i0[:, None] + offs[None, :]                           # [n_ch, W]
        keep = (idx >= 0) & (idx < n_t)
        if not bool(keep.any()):
            continue
        tau = idx.to(torch.float64) / fs - tc[:, None]
        a = (math.pi * ev.f0) ** 2 * tau * tau
        val = ev.amplitude * (1.0 - 2.0 * a) * torch.exp(-a)
        lin = idx * n_ch + torch.arange(n_ch, device=dev, dtype=torch.int64)[:, None]
        flat.index_add_(0, lin[keep], val[keep].to(torch.float32))
    return x


# ---------------------------------------------------------------------------
# Workload definitions (shapes, filters, STA/LTA windows) and their inputs.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    x: torch.Tensor          # float32 [n_t, n_ch]
    fs: float
    chunk: int               # samples per chunk
    order: int               # total digital filter order
    btype: str               # 'lowpass' | 'highpass' | 'bandpass' | 'bandstop'
    f1: float
    f2: float
    sta_s: float | None      # STA window [s] (None: no STA/LTA stage)
    lta_s: float | None


def make_config1(seed: int = 20133, device="cpu") -> Workload:
    """64 ch x 10,000 samples at 500 Hz; white N(0,1) plus 5 Ricker events
    (f0 = 20 Hz, amplitude 5) with 1500 m/s moveout over 1 m channel spacing;
    4th-order Butterworth 1-50 Hz bandpass, 10 chunks of 1000, STA 0.5 s / LTA 5 s."""
    n_ch, n_t, fs = 64, 10_000, 500.0
    x = white_noise(n_t, n_ch, seed, device)
    moveout = (n_ch - 1) * 1.0 / 1500.0
    ev = draw_events(5, seed + 1, n_t / fs - moveout, 1500.0, 1500.0, random_sign=False)
    ricker_events(x, fs, 1.0, ev)
    return Workload("config1", x, fs, 1000, 4, "bandpass", 1.0, 50.0, 0.5, 5.0)


def make_config2(seed: int = 20134, device="cpu", n_ch: int = 6000, n_t: int = 90_000,
                 n_events: int = 200) -> Workload:
    """6000 ch x 90,000 samples at 1500 Hz (60 s) in 1 s chunks; 1/f noise plus
    200 moveout events with apparent velocity U[300, 5000] m/s; 8th-order
    Butterworth 1-100 Hz bandpass, STA 0.2 s / LTA 2 s."""
    fs = 1500.0
    x = pink_noise(n_t, n_ch, seed, device)
    ev = draw_events(n_events, seed + 1, n_t / fs, 300.0, 5000.0)
    ricker_events(x, fs, 1.0, ev)
    return Workload("config2", x, fs, 1500, 8, "bandpass", 1.0, 100.0, 0.2, 2.0)


def make_config3(seed: int = 20135, device="cpu", n_ch: int = 2000, n_t: int = 100_000) -> Workload:
    """2000 ch x 100,000 samples at 10 kHz (10 s) in 1 s chunks; N(0,1) plus a
    0.1 Hz drift of amplitude 100 with a per-channel phase; 16th-order
    Butterworth highpass at 0.5 Hz (poles within 1e-3 of the unit circle)."""
    fs = 10_000.0
    x = white_noise(n_t, n_ch, seed, device)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    phi = torch.as_tensor(rng.uniform(0.0, 2.0 * math.pi, size=n_ch), device=x.device, dtype=torch.float64)
    t = torch.arange(n_t, device=x.device, dtype=torch.float64) / fs
    drift = 100.0 * torch.sin(2.0 * math.pi * 0.1 * t[:, None] + phi[None, :])
    x.add_(drift.to(torch.float32))
    return Workload("config3", x, fs, 10_000, 16, "highpass", 0.5, 0.0, None, None)


def make_config5(seed: int = 20137, device="cpu", n_ch: int = 6000, n_t: int = 30_000) -> Workload:
    """Differentiation workload: the config-2 generator at 6000 ch x 30,000
    samples, 3000-sample chunks, 8th-order 1-100 Hz bandpass at 1500 Hz,
    STA 0.2 s / LTA 2 s."""
    w = make_config2(seed, device, n_ch=n_ch, n_t=n_t, n_events=max(1, 200 * n_t // 90_000))
    return Workload("config5", w.x, w.fs, 3000, 8, "bandpass", 1.0, 100.0, 0.2, 2.0)


@dataclasses.dataclass
class StreamSpec:
    n_ch: int
    fs: float
    n_t: int        # samples per chunk
    order: int      # total bandpass order (2 K)
    f1: float
    f2: float
    seed: int


def draw_batched_streams(seed: int = 20136, n_streams: int = 12) -> list[StreamSpec]:
    """Draw the uneven multi-stream table: channel counts from
    {500, 1200, 3000, 6000, 12000, 20000}, rates from {100, 500, 1500, 10000} Hz,
    chunk lengths U[0.25, 2] s (n_t = round(fs T)), bandpass orders from
    {2, 4, 6, 8, 10}, f1 = fs 10^U[log10 0.002, log10 0.02], f2 = fs U[0.1, 0.4]."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    out = []
    for i in range(n_streams):
        n_ch = int(rng.choice([500, 1200, 3000, 6000, 12000, 20000]))
        fs = float(rng.choice([100.0, 500.0, 1500.0, 10000.0]))
        T = float(rng.uniform(0.25, 2.0))
        n_t = max(1, int(round(fs * T)))
        order = int(rng.choice([2, 4, 6, 8, 10]))
        f1 = fs * 10.0 ** rng.uniform(math.log10(0.002), math.log10(0.02))
        f2 = fs * rng.uniform(0.1, 0.4)
        out.append(StreamSpec(n_ch, fs, n_t, order, float(f1), float(f2), int(seed) * 100 + i))
    return out


def cf_like(n_t: int, n_ch: int, seed: int = 20138, device="cpu") -> torch.Tensor:
    """A positive FP32 series [n_t, n_ch] shaped like an STA/LTA
    characteristic function: a slow per-channel swing 2 + 1.6 sin(f t + phase)
    (f uniform in [0.005, 0.055] rad/sample, phase uniform) plus N(0, 0.4)
    noise, taken in absolute value, so that thresholds such as 3.0 / 1.5 are
    crossed often, with chattering near them."""
    g = _gen(seed, device)
    t = torch.arange(n_t, device=device, dtype=torch.float32)[:, None]
    f = torch.rand((1, n_ch), generator=g, device=device) * 0.05 + 0.005
    ph = torch.rand((1, n_ch), generator=g, device=device) * 6.283
    noise = torch.randn((n_t, n_ch), generator=g, device=device) * 0.4
    return (2.0 + 1.6 * torch.sin(f * t + ph) + noise).abs().contiguous()
