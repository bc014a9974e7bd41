"""Benchmark of the stateful chunked SOS + STA/LTA hot path on one MI355X.

Workload (the metric's single-GPU configuration): 6000 channels x 90,000
samples at 1500 Hz (60 s), FP32, time-major, processed as 60 chunks of 1500
samples with carried state; 8th-order Butterworth 1-100 Hz bandpass (4
sections) followed by a recursive STA/LTA of 0.2 s / 2 s.  Input: seeded 1/f
noise plus 200 linear-moveout Ricker events, generated on the GPU.

A step is one pass of the whole path over the record: 60 calls of the fused
kernel (filter, STA/LTA, both carried states), writing y and cf.  Inputs are
resident in HBM before timing starts.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-parity]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "channel-samples/s and % HBM peak, plain fwd vs batched vs fwd+adjoint at ≤1e-5 rel err"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "fwd_kernel_6000ch_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Untimed calls before each timed region: after host-side work (parity
# checks, input generation) the GPU comes back at idle clocks and needs
# 10-15 steps (~30 ms) of the plain forward to reach its steady rate
# (2.18 -> 2.00 -> 1.94 -> 1.93 ms per step in blocks of 5 steps after 3 s
# idle).  Under --profile the ramp runs a plain device fill instead, so that
# kernel traces hold exactly the warm-up and timed launches of each leg.
RAMP_S = 0.1
RAMP_WITH_FILL = False
_fill_buf = []


def ramp(torch, fn, *a) -> int:
    """RAMP_S seconds of wall time of calls of fn (of device fills under
    --profile), each synchronised; returns the number of calls of fn."""
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < RAMP_S:
        if RAMP_WITH_FILL:
            if not _fill_buf:
                _fill_buf.append(torch.empty(64 << 20, dtype=torch.float32, device="cuda"))
            _fill_buf[0].fill_(1.0)
        else:
            fn(*a)
            n += 1
        torch.cuda.synchronize()
    return n


def warm(torch, fn, *a) -> int:
    """One warm-up call of fn, then the clock ramp; returns the number of
    calls of fn beyond the first."""
    fn(*a)
    torch.cuda.synchronize()
    return ramp(torch, fn, *a)


def kernel_hash(sources) -> str:
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_2605_20132_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current source of its kernel (else None)."""
    try:
        with open(path) as f:
            t = json.load(f)
        if t.get("kernel_sha256_16") != kernel_hash(t["sources"]):
            return None
    except (OSError, ValueError, KeyError):
        return None
    return t


def copy_bandwidth(torch, dev, mib: int = 512, reps: int = 10) -> float:
    """Bytes read + written per second by torch's device copy over buffers
    rotated so that no copy finds its source in the 256 MB last-level cache."""
    n = (mib << 20) // 4
    bufs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4)]
    for b in bufs:
        b.fill_(1.0)
    bufs[1].copy_(bufs[0])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        bufs[(2 * i + 3) % 4].copy_(bufs[(2 * i + 2) % 4])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del bufs
    return 2.0 * n * 4 / (ms / 1e3) / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_dev, sos, nsta, nlta, chunk, min_seconds=10.0, max_passes=30):
    """Time the FP64 oracle (as it is) on the same record: whole passes over
    all channels in the workload's chunks, state carried, repeated until at
    least `min_seconds` of wall time (bounded by `max_passes`).  Beside it:
    the same on one host thread over a slice of the channels, and the
    oracle's forward + adjoint (the gradient of the differentiation workload's
    loss) over a slice, both scaled to channel-samples/s."""
    import oracle

    cores = len(os.sched_getaffinity(0))
    oracle.set_num_threads(cores)
    xs = x_dev.double().cpu().numpy()
    n_t, n_ch = xs.shape
    s = oracle.Stream(sos, n_ch, nsta, nlta)
    passes = 0
    t0 = time.perf_counter()
    while True:
        for c0 in range(0, n_t, chunk):
            s.process(xs[c0:c0 + chunk])
        passes += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or passes >= max_passes:
            break
    res = {"value": passes * n_ch * n_t / el, "unit": "channel-samples/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{passes} pass(es) over the whole record ({n_ch} channels x {n_t} samples in "
                     f"{(n_t + chunk - 1) // chunk} chunks, state carried), FP64 DF2T cascade + STA/LTA, "
                     f"{el:.1f} s on {cores} host threads"}
    # one thread, the first 1024 channels of the record
    oracle.set_num_threads(1)
    sub = np.ascontiguousarray(xs[:, :1024])
    s1 = oracle.Stream(sos, sub.shape[1], nsta, nlta)
    t0 = time.perf_counter()
    for c0 in range(0, n_t, chunk):
        s1.process(sub[c0:c0 + chunk])
    el1 = time.perf_counter() - t0
    res["single_thread"] = {"value": sub.size / el1, "unit": "channel-samples/s", "cores": 1,
                            "sample": f"{sub.shape[1]} channels x {n_t} samples in chunks of {chunk}, {el1:.1f} s"}
    # forward + adjoint: the oracle's reverse-mode gradient of mean (cf - target)^2
    # over 30,000 samples of 2048 channels, on every host thread
    oracle.set_num_threads(cores)
    n_g = min(n_t, 30_000)
    xg = np.ascontiguousarray(xs[:n_g, :2048])
    tg = np.ascontiguousarray(xg[::-1])
    t0 = time.perf_counter()
    oracle.stalta_grad(sos, xg, tg, nsta, nlta, 1.0 / xg.size)
    elg = time.perf_counter() - t0
    res["fwd_adjoint"] = {"value": xg.size / elg, "unit": "channel-samples/s", "cores": cores,
                          "sample": f"{xg.shape[1]} channels x {n_g} samples, one chunk, gradient wrt x and "
                                    f"all coefficients, {elg:.1f} s"}
    return res


def adj_traffic():
    """adj_kernel's measured HBM bytes per launch against its algorithmic bytes."""
    t = measured_traffic(os.path.join(PROFILES, "adj_kernel_6000ch_traffic.json"))
    if t is None:
        return None
    return {"hbm_bytes_per_launch": t["hbm_bytes_per_launch"],
            "algorithmic_bytes_per_launch": t["algorithmic_bytes_per_launch"],
            "ratio": t["traffic_over_algorithmic"]}


def fwd_adjoint_leg(F, torch, dev, steps: int, parity: bool):
    """Forward + adjoint on the differentiation workload: 6000 ch x 30,000
    samples in 3000-sample chunks, loss = mean (cf - target)^2, target = cf of
    the same input through the band moved to (1.05 f1, 0.95 f2).  A step is
    the chunked forward with per-chunk device checkpoints plus the adjoint
    chain (chunks last to first) giving dL/dx and dL/dtheta."""
    import synth

    w = synth.make_config5(device=dev)
    x = w.x
    n_t, n_ch = x.shape
    chunk = w.chunk
    nsta, nlta = round(w.sta_s * w.fs), round(w.lta_s * w.fs)
    sos = F.sos_design(w.order, w.btype, w.f1, w.f2, w.fs)
    sos_t = F.sos_design(w.order, w.btype, 1.05 * w.f1, 0.95 * w.f2, w.fs)
    K = sos.shape[0]
    splits = [(a, min(n_t, a + chunk)) for a in range(0, n_t, chunk)]
    tgt = torch.empty_like(x)
    st_t, sl_t = F.SOSState(sos_t, n_ch), F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
    for a, b in splits:
        F.sos_stalta_process(st_t, sl_t, x[a:b], cf=tgt[a:b], write_y=False)
    st, sl = F.SOSState(sos, n_ch), F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
    cks = [(st.save(), sl.save()) for _ in splits]
    tapes = [torch.empty(F.adjoint_tape_bytes(st, sl, b - a), dtype=torch.uint8, device=dev) for a, b in splits]
    zero_z, zero_s = st.save(), sl.save()
    cf = torch.empty_like(x)
    gx = torch.empty_like(x)
    adj = torch.zeros((2 * K + 2, n_ch), dtype=torch.float64, device=dev)
    gs = torch.zeros((K, 5), dtype=torch.float64, device=dev)
    scale = 1.0 / x.numel()

    def step(mid=None):
        # the forward records each chunk's tape; the adjoint reads it
        st.load(zero_z)
        sl.load(zero_s)
        for i, (a, b) in enumerate(splits):
            F.sos_stalta_process_tape(st, sl, x[a:b], tape=tapes[i], cf=cf[a:b])
        if mid is not None:
            mid.record()
        adj.zero_()
        gs.zero_()
        for i in reversed(range(len(splits))):
            a, b = splits[i]
            F.sos_stalta_adjoint_tape(st, sl, tapes[i], x[a:b], tgt[a:b], gx[a:b], adj, gs, mode="mse",
                                      scale=scale)

    def step_checkpoints():
        # the same without tapes: state checkpoints per chunk, and the
        # adjoint reruns a states-only forward over each chunk
        st.load(zero_z)
        sl.load(zero_s)
        for i, (a, b) in enumerate(splits):
            st.save(cks[i][0])
            sl.save(cks[i][1])
            F.sos_stalta_process(st, sl, x[a:b], cf=cf[a:b], write_y=False)
        adj.zero_()
        gs.zero_()
        for i in reversed(range(len(splits))):
            a, b = splits[i]
            st.load(cks[i][0])
            sl.load(cks[i][1])
            F.sos_stalta_adjoint(st, sl, x[a:b], tgt[a:b], gx[a:b], adj, gs, mode="mse", scale=scale)

    warm(torch, step)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    mids = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev[0].record()
    for i in range(steps):
        step(mids[i])
        ev[i + 1].record()
    torch.cuda.synchronize()
    st.check()
    ms = ev[0].elapsed_time(ev[steps]) / steps
    ms_f = sum(ev[i].elapsed_time(mids[i]) for i in range(steps)) / steps
    ms_a = sum(mids[i].elapsed_time(ev[i + 1]) for i in range(steps)) / steps
    step_checkpoints()
    torch.cuda.synchronize()
    ev[0].record()
    step_checkpoints()
    ev[1].record()
    torch.cuda.synchronize()
    ms_ck = ev[0].elapsed_time(ev[1])
    # the tape step captured in one HIP graph and replayed (no host launches
    # between its ~80 kernels and copies)
    ms_graph = None
    try:
        graph = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        with torch.cuda.stream(cs):
            step()  # the workspaces exist before the capture
            torch.cuda.synchronize()
            with torch.cuda.graph(graph, stream=cs):
                step()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(steps):
            graph.replay()
        ev[1].record()
        torch.cuda.synchronize()
        ms_graph = ev[0].elapsed_time(ev[1]) / steps
    except Exception as e:  # an optional extra measurement
        log(f"[bench] fwd+adjoint graph capture unavailable: {e}")
    n = n_ch * n_t
    gbs = 20.0 * n / (ms / 1e3) / 1e9
    res = {"workload": f"{n_ch} ch x {n_t} samples @ {w.fs:g} Hz in {len(splits)} chunks of {chunk}; "
                       f"BP order {w.order} ({K} SOS) + STA/LTA {nsta}/{nlta}; loss mean (cf - target)^2; "
                       "grad wrt x and all coefficients",
           "ms_per_step": ms, "value": n / (ms / 1e3), "unit": "channel-samples/s", "algorithmic_gbs": gbs,
           # algorithmic bytes: forward x read + cf written (8 B per channel-sample),
           # adjoint x and target read + dL/dx written (12 B); checkpoints and
           # carried states are under 0.1 % of it
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "whole step: fwd_kernel<K=4, 64-row blocks, stalta> per chunk writing the tape, "
                                  "then per chunk (last first) adj_kernel on its partial last window and "
                                  "adj_kernel on its five full 512-row windows in one launch",
                        "algorithmic_bytes_per_step": 20.0 * n,
                        "forward": {"ms": ms_f, "algorithmic_gbs": 8.0 * n / (ms_f / 1e3) / 1e9,
                                    "frac": 8.0 * n / (ms_f / 1e3) / 1e9 / HBM_PEAK_GBS},
                        "adjoint": {"ms": ms_a, "algorithmic_gbs": 12.0 * n / (ms_a / 1e3) / 1e9,
                                    "frac": 12.0 * n / (ms_a / 1e3) / 1e9 / HBM_PEAK_GBS,
                                    "kernel": "adj_kernel<4, 16, unit, rebuild, full, several windows> (10 launches "
                                              "of 5 windows per step), adj_kernel<4, 16, unit, rebuild> on the "
                                              "partial windows (10) and adj_reduce_kernel (10)",
                                    "adj_kernel_traffic": adj_traffic()}},
           "checkpoint_path_ms_per_step": ms_ck, "graph_replay_ms_per_step": ms_graph}
    if parity:
        # the same path on a 64-channel slice against the oracle's reference gradient
        import numpy as np
        import oracle

        xs = x[:, :64].contiguous()
        ts = tgt[:, :64].contiguous()
        osos = oracle.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
        s2, l2 = F.SOSState(osos, 64), F.StaLtaState(float(nsta), float(nlta), 1.0, 64)
        tp2 = [F.sos_stalta_process_tape(s2, l2, xs[a:b])[2] for a, b in splits]
        g2 = torch.empty_like(xs)
        a2 = torch.zeros((2 * K + 2, 64), dtype=torch.float64, device=dev)
        gs2 = torch.zeros((K, 5), dtype=torch.float64, device=dev)
        sc2 = 1.0 / xs.numel()
        for i in reversed(range(len(splits))):
            a, b = splits[i]
            F.sos_stalta_adjoint_tape(s2, l2, tp2[i], xs[a:b], ts[a:b], g2[a:b], a2, gs2, mode="mse", scale=sc2)
        torch.cuda.synchronize()
        _, ogx, ogs, _ = oracle.stalta_grad(osos, xs.double().cpu().numpy(), ts.double().cpu().numpy(), nsta,
                                            nlta, sc2)
        gxh = g2.double().cpu().numpy()
        num = np.linalg.norm(gxh - ogx, axis=0)
        den = np.linalg.norm(ogx, axis=0)
        res["parity"] = {"channels": 64,
                         "max_rel_rms_gx": float(np.max(num / np.where(den > 0, den, 1.0))),
                         "rel_l2_gtheta": float(np.linalg.norm(gs2.cpu().numpy() - ogs) / np.linalg.norm(ogs)),
                         "tolerance": 1e-5}
    log(f"[bench] fwd+adjoint {ms:.2f} ms/step (forward {ms_f:.2f}, adjoint {ms_a:.2f}; checkpoint path "
        f"{ms_ck:.2f}; graph replay {ms_graph if ms_graph is None else round(ms_graph, 2)}) -> "
        f"{res['value']:.3e} ch-samples/s"
        + (f"; parity gx {res['parity']['max_rel_rms_gx']:.2e} gtheta {res['parity']['rel_l2_gtheta']:.2e}"
           if parity else ""))
    return res


def filtfilt_leg(F, torch, dev, steps: int, parity: bool):
    """Zero-phase filtering of display windows: 6000 ch x 15,000 samples (10 s
    at 1500 Hz) of the plain-forward record through its bandpass (8th order
    1-100 Hz), forward then backward in time, in place.  16 B per
    channel-sample algorithmic (x read, y written, y read, y written).
    Parity: 16 sampled channels against the oracle."""
    import numpy as np

    import synth

    w = synth.make_config2(device=dev, n_t=15_000)
    x = w.x
    n_t, n_ch = x.shape
    sos = F.sos_design(w.order, w.btype, w.f1, w.f2, w.fs)
    st = F.SOSState(sos, n_ch)
    y = torch.empty_like(x)
    warm(torch, st.filtfilt, x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        st.filtfilt(x, y)
    e1.record()
    torch.cuda.synchronize()
    st.check()
    ms = e0.elapsed_time(e1) / steps
    res = {"workload": f"{n_ch} ch x {n_t} samples window, bandpass order {w.order} {w.f1}-{w.f2} Hz @ {w.fs} Hz",
           "ms_per_window": ms, "value": n_ch * n_t / (ms / 1e3), "unit": "channel-samples/s",
           "algorithmic_gbs": n_ch * n_t * 16 / (ms / 1e3) / 1e9}
    log(f"[bench] zero-phase window {ms:.3f} ms -> {res['value']:.3e} ch-samples/s ({res['algorithmic_gbs']:.0f} GB/s)")
    if parity:
        import oracle

        cols = np.random.default_rng(11).choice(n_ch, 16, replace=False)
        tc = torch.as_tensor(cols, device=dev)
        yo = oracle.sos_filtfilt(oracle.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs),
                                 x[:, tc].double().cpu().numpy())
        yg = y[:, tc].double().cpu().numpy()
        err = float(np.max(np.linalg.norm(yg - yo, axis=0) / np.linalg.norm(yo, axis=0)))
        res["parity"] = {"channels": len(cols), "max_rel_rms": err, "tolerance": 1e-5}
        log(f"[bench] zero-phase parity on {len(cols)} channels: {err:.2e}")
    st.close()
    return res


def ema_leg(F, torch, dev, steps: int, parity: bool):
    """Running AGC (2 s exponential power average) over the plain-forward
    record: 6000 ch x 90,000 samples at 1500 Hz in 60 chunks of 1500, state
    carried.  8 B per channel-sample algorithmic.  Parity: 16 sampled
    channels against the oracle."""
    import numpy as np

    import synth

    w = synth.make_config2(device=dev)
    x = w.x
    n_t, n_ch = x.shape
    y = torch.empty_like(x)
    e = F.Ema(n_ch, 2.0, w.fs, "agc")

    def step():
        for a in range(0, n_t, w.chunk):
            e.process(x[a:a + w.chunk], y[a:a + w.chunk])

    warm(torch, step)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res = {"workload": f"running AGC, 2 s average, {n_ch} ch x {n_t} samples in chunks of {w.chunk}",
           "ms_per_step": ms, "value": n_ch * n_t / (ms / 1e3), "unit": "channel-samples/s",
           "algorithmic_gbs": n_ch * n_t * 8 / (ms / 1e3) / 1e9}
    log(f"[bench] running AGC {ms:.3f} ms/step -> {res['value']:.3e} ch-samples/s ({res['algorithmic_gbs']:.0f} GB/s)")
    if parity:
        import oracle

        cols = np.random.default_rng(13).choice(n_ch, 16, replace=False)
        tc = torch.as_tensor(cols, device=dev)
        e2 = F.Ema(n_ch, 2.0, w.fs, "agc")
        for a in range(0, n_t, w.chunk):
            e2.process(x[a:a + w.chunk], y[a:a + w.chunk])
        torch.cuda.synchronize()
        yo = oracle.Ema(len(cols), oracle.window_samples(2.0, w.fs), "agc").process(x[:, tc].double().cpu().numpy())
        yg = y[:, tc].double().cpu().numpy()
        err = float(np.max(np.linalg.norm(yg - yo, axis=0) / np.linalg.norm(yo, axis=0)))
        res["parity"] = {"channels": len(cols), "max_rel_rms": err, "tolerance": 1e-5}
        log(f"[bench] running AGC parity on {len(cols)} channels: {err:.2e}")
        e2.close()
    e.close()
    return res


def fir_taps(M: int = 64):
    """Windowed-sinc (Hamming) lowpass at a quarter of the sample rate."""
    import numpy as np

    n = np.arange(M) - (M - 1) / 2
    return 0.5 * np.sinc(0.5 * n) * np.hamming(M)


# FP32 FMA issue rate without packed FP32 (the library is built without it):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def fir_leg(F, torch, dev, steps: int, parity: bool):
    """Realtime FIR (64-tap lowpass, history carried) over the plain-forward
    record: 6000 ch x 90,000 samples in 60 chunks of 1500, and the same record
    in one call.  8 B and 2 M flops per channel-sample algorithmic.  Parity:
    16 sampled channels against the oracle within the FMA rounding bound."""
    import numpy as np

    import synth

    w = synth.make_config2(device=dev)
    x = w.x
    n_t, n_ch = x.shape
    h = fir_taps(64)
    M = len(h)
    y = torch.empty_like(x)
    f = F.Fir(h, n_ch)

    def chunked():
        for a in range(0, n_t, w.chunk):
            f.process(x[a:a + w.chunk], y[a:a + w.chunk])

    def one_shot():
        f.process(x, y)

    def timed(fn):
        warm(torch, fn)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms = timed(chunked)
    ms1 = timed(one_shot)
    n = n_ch * n_t
    res = {"workload": f"realtime FIR, {M}-tap lowpass, {n_ch} ch x {n_t} samples in chunks of {w.chunk}",
           "ms_per_step": ms, "value": n / (ms / 1e3), "unit": "channel-samples/s",
           "algorithmic_gbs": n * 8 / (ms / 1e3) / 1e9, "tflops": n * 2 * M / (ms / 1e3) / 1e12,
           "one_shot": {"ms_per_step": ms1, "value": n / (ms1 / 1e3), "algorithmic_gbs": n * 8 / (ms1 / 1e3) / 1e9,
                        "tflops": n * 2 * M / (ms1 / 1e3) / 1e12}}
    res["roofline"] = {"bound": "alu", "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "achieved": res["tflops"], "frac": res["tflops"] / FP32_VALU_PEAK_TFLOPS,
                       "one_shot_frac": res["one_shot"]["tflops"] / FP32_VALU_PEAK_TFLOPS,
                       "hbm_frac": res["algorithmic_gbs"] / 8000.0}
    log(f"[bench] FIR {ms:.3f} ms/step chunked ({res['tflops']:.1f} TFLOP/s, {res['algorithmic_gbs']:.0f} GB/s), "
        f"{ms1:.3f} ms one-shot ({res['one_shot']['tflops']:.1f} TFLOP/s)")
    if parity:
        import oracle

        cols = np.random.default_rng(14).choice(n_ch, 16, replace=False)
        tc = torch.as_tensor(cols, device=dev)
        f2 = F.Fir(h, n_ch)
        for a in range(0, n_t, w.chunk):
            f2.process(x[a:a + w.chunk], y[a:a + w.chunk])
        torch.cuda.synchronize()
        xs = x[:, tc].double().cpu().numpy()
        yo = oracle.Fir(h, len(cols)).process(xs)
        bound = (M + 2) * 2.0 ** -24 * oracle.Fir(np.abs(h), len(cols)).process(np.abs(xs)) + 1e-37
        yg = y[:, tc].double().cpu().numpy()
        worst = float(np.max(np.abs(yg - yo) / bound))
        res["parity"] = {"channels": len(cols), "max_err_over_bound": worst, "bound": "(M + 2) 2^-24 sum |h||x|",
                         "ok": worst <= 1.0}
        log(f"[bench] FIR parity on {len(cols)} channels: max error / bound {worst:.3f}")
        f2.close()
    f.close()
    res["long_taps"] = [fir_fft_case(F, torch, dev, x, w.chunk, Ml, steps, parity) for Ml in (256, 1024)]
    return res


def fir_fft_case(F, torch, dev, x, chunk, M, steps, parity):
    """One long lowpass over the same record in chunks: the direct method
    against FFT filtering (2048-row overlap-save windows).  The FFT's
    algorithmic traffic is the direct form's, 8 B per channel-sample (its
    window overlap re-reads (M - 1) / (2049 - M) of the input from L2)."""
    import numpy as np

    n_t, n_ch = x.shape
    h = fir_taps(M)
    y = torch.empty_like(x)
    out = {"taps": M}
    for method in ("direct", "fft"):
        f = F.Fir(h, n_ch)
        f.set_method(method)

        def run():
            for a in range(0, n_t, chunk):
                f.process(x[a:a + chunk], y[a:a + chunk])

        warm(torch, run)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        gbs = n_t * n_ch * 8 / (ms / 1e3) / 1e9
        out[method] = {"ms_per_step": ms, "value": n_t * n_ch / (ms / 1e3), "unit": "channel-samples/s",
                       "algorithmic_gbs": gbs, "hbm_frac": gbs / 8000.0}
        if method == "direct":
            out[method]["tflops"] = n_t * n_ch * 2 * M / (ms / 1e3) / 1e12
        else:
            # algorithmic flops of the FFT method: per channel and 2048-row
            # window, a forward and an inverse 1024-point complex transform
            # (5 N log2 N each) and the spectral pass (~8 per point pair and
            # product); windows per call = ceil(rows / (2049 - M))
            win = -(-chunk // (2049 - M)) * (n_t // chunk) + (-(-(n_t % chunk) // (2049 - M)) if n_t % chunk else 0)
            flops = n_ch * win * (2 * 5 * 1024 * 10 + 16 * 1024)
            tf = flops / (ms / 1e3) / 1e12
            out[method]["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                                       "kernel": "fir_fft_kernel<8, 512>",
                                       "flops": {"achieved_tflops": tf, "peak_tflops": FP32_VALU_PEAK_TFLOPS,
                                                 "frac": tf / FP32_VALU_PEAK_TFLOPS,
                                                 "per_window_per_channel": 2 * 5 * 1024 * 10 + 16 * 1024}}
        if method == "fft" and parity:
            import oracle

            # sampled channels of the whole record in chunks, against the
            # oracle: per block, ||err||_2 <= 156 u max|H| ||window||_2 (the
            # FFT bound the GPU tests check block by block); summed over the
            # blocks, whose windows cover every row 2048 / (2049 - M) times,
            # RMS err <= 156 sqrt(2048 / (2049 - M)) u max|H| RMS x
            f2 = F.Fir(h, n_ch)
            f2.set_method("fft")
            for a in range(0, n_t, chunk):
                f2.process(x[a:a + chunk], y[a:a + chunk])
            torch.cuda.synchronize()
            cols = np.random.default_rng(15).choice(n_ch, 8, replace=False)
            tc = torch.as_tensor(cols, device=dev)
            xs = x[:, tc].double().cpu().numpy()
            h32 = h.astype(np.float32).astype(np.float64)
            yo = oracle.Fir(h32, len(cols)).process(xs)
            yg = y[:, tc].double().cpu().numpy()
            maxH = float(np.max(np.abs(np.fft.fft(h32, 2048))))
            rel = float(np.max(np.sqrt(np.mean((yg - yo) ** 2, axis=0)) /
                               (2.0 ** -24 * maxH * np.sqrt(np.mean(xs * xs, axis=0)))))
            bound = float(156.0 * np.sqrt(2048.0 / (2049 - M)))
            out[method]["parity"] = {"channels": len(cols), "rms_err_over_u_maxH_rms_x": rel, "bound": bound,
                                     "ok": rel <= bound}
            f2.close()
        f.close()
    out["fft_speedup"] = out["direct"]["ms_per_step"] / out["fft"]["ms_per_step"]
    log(f"[bench] FIR {M} taps: direct {out['direct']['ms_per_step']:.3f} ms, fft {out['fft']['ms_per_step']:.3f} ms "
        f"({out['fft']['algorithmic_gbs']:.0f} GB/s), speed-up {out['fft_speedup']:.2f}")
    return out


def config3_leg(F, torch, dev, steps: int, parity: bool):
    """The near-unit-circle configuration: 2000 ch x 100,000 samples at 10 kHz
    in 10 chunks of 10,000 (each chunk 7 launch windows), 16th-order
    Butterworth highpass at 0.5 Hz (8 sections, poles within 1e-3 of the unit
    circle; level matrices from LDS), SOS only, y written.  A step is the
    whole record; algorithmic bytes 8 per channel-sample (x read, y written).
    Parity: y of 2 sampled channels against the oracle (bar 1e-4 for poles
    this close to the unit circle)."""
    import numpy as np

    import synth

    w = synth.make_config3(device=dev)
    x = w.x
    n_t, n_ch = x.shape
    sos = F.sos_design(w.order, w.btype, w.f1, w.f2, w.fs)
    y = torch.empty_like(x)
    st = F.SOSState(sos, n_ch)

    def step():
        for a in range(0, n_t, w.chunk):
            st.process(x[a:a + w.chunk], y[a:a + w.chunk])

    def timed():
        warm(torch, step)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    from paper_2605_20132_amd.autotune import Autotuner

    ms_default = timed()
    tile_default = list(st.tile())
    # 2000 channels in 16-channel groups are 125 workgroups for 256 CUs: the
    # library's tuner searches blocks, waves and groups for this shape
    tile = list(Autotuner(None, block=0, waves=0).tune(st, w.chunk))
    ms = timed()
    n = n_ch * n_t
    gbs = 8.0 * n / (ms / 1e3) / 1e9
    res = {"workload": f"{n_ch} ch x {n_t} samples @ {w.fs:g} Hz in chunks of {w.chunk}; Butterworth HP order "
                       f"{w.order} at {w.f1:g} Hz ({sos.shape[0]} SOS), y written",
           "ms_per_step": ms, "value": n / (ms / 1e3), "unit": "channel-samples/s", "algorithmic_gbs": gbs,
           "frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "tile": tile,
           "default_tile": {"tile": tile_default, "ms_per_step": ms_default}}
    log(f"[bench] config3 {ms:.3f} ms/step with tile {tile} -> {res['value']:.3e} ch-samples/s ({gbs:.0f} GB/s); "
        f"default tile {tile_default}: {ms_default:.3f} ms/step")
    if parity:
        import oracle

        st2 = F.SOSState(sos, n_ch)
        st2.set_tile(*tile)
        for a in range(0, n_t, w.chunk):
            st2.process(x[a:a + w.chunk], y[a:a + w.chunk])
        torch.cuda.synchronize()
        cols = [0, n_ch - 1]
        osos = oracle.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
        yo, _ = oracle.sos_filter(osos, x[:, cols].double().cpu().numpy())
        yg = y[:, cols].double().cpu().numpy()
        err = float(np.max(np.linalg.norm(yg - yo, axis=0) / np.linalg.norm(yo, axis=0)))
        res["parity"] = {"max_rel_rms_y": err, "channels": len(cols), "tolerance": 1e-4}
        log(f"[bench] config3 parity on {len(cols)} channels: y {err:.2e}")
        st2.close()
    st.close()
    return res


def trigger_leg(F, torch, dev, steps: int, parity: bool):
    """Two-threshold trigger (monitor events) on a cf-shaped record of the
    plain-forward shape: 6000 ch x 90,000 samples in 60 chunks of 1500,
    thresholds 3.0 / 1.5, events appended to one device buffer per step.
    Parity: the events of 16 sampled channels against the oracle on the same
    FP32 input (exact)."""
    import numpy as np

    import synth

    n_ch, n_t, chunk, on, off = 6000, 90_000, 1500, 3.0, 1.5
    cf = synth.cf_like(n_t, n_ch, device=dev)
    cap = 8_000_000
    ev = torch.empty((cap, 3), dtype=torch.int64, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    tr = F.Trigger(n_ch, on, off)

    def step(t):
        count.zero_()
        for a in range(0, n_t, chunk):
            t.process(cf[a:a + chunk], ev, count)

    warm(torch, step, tr)  # warm-up (the state carries on, as for a continuing stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step(tr)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    n_ev = int(count.item())
    res = {"workload": f"{n_ch} ch x {n_t} samples in chunks of {chunk}, thresholds {on} / {off}",
           "ms_per_step": ms, "value": n_ch * n_t / (ms / 1e3), "unit": "channel-samples/s", "events_per_step": n_ev,
           "algorithmic_gbs": (n_ch * n_t * 4 + n_ev * 24) / (ms / 1e3) / 1e9}
    log(f"[bench] trigger {ms:.3f} ms/step -> {res['value']:.3e} ch-samples/s ({res['algorithmic_gbs']:.0f} GB/s, "
        f"{n_ev} events)")
    if parity:
        import oracle

        cols = np.random.default_rng(7).choice(n_ch, 16, replace=False)
        t2 = F.Trigger(n_ch, on, off)
        step(t2)
        torch.cuda.synchronize()
        k = int(count.item())
        g = ev[:k].cpu().numpy()
        x = cf[:, torch.as_tensor(cols, device=dev)].cpu().numpy()
        o = oracle.Trigger(len(cols), on, off).process(x)
        o[:, 0] = cols[o[:, 0]]
        key = lambda a: a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))]
        mine = key(g[np.isin(g[:, 0], cols)])
        exact = bool(mine.shape == o.shape and np.array_equal(mine, key(o)))
        res["parity"] = {"channels": len(cols), "events_compared": int(len(o)), "exact": exact}
        log(f"[bench] trigger parity on {len(cols)} channels: {len(o)} events, exact {exact}")
        t2.close()
    tr.close()
    del cf
    res["monitor"] = monitor_chain(F, torch, dev, steps, ev, count)
    return res


def monitor_chain(F, torch, dev, steps: int, ev, count):
    """The monitor chain on the plain-forward record (6000 ch x 90,000 in 60
    chunks of 1500, BP order 8 + STA/LTA 0.2 / 2 s, thresholds 3.0 / 1.5):
    x -> events as two calls per chunk (filark_sos_stalta_process writing cf,
    filark_trigger_process reading it) and as one filark_monitor_process
    launch per chunk (cf kept in registers, not written)."""
    import synth

    w = synth.make_config2(device=dev)
    x = w.x
    n_t, n_ch = x.shape
    chunk, on, off = w.chunk, 3.0, 1.5
    sos = F.sos_design(w.order, w.btype, w.f1, w.f2, w.fs)
    nsta, nlta = round(w.sta_s * w.fs), round(w.lta_s * w.fs)
    cf = torch.empty_like(x)
    objs = [(F.SOSState(sos, n_ch), F.StaLtaState(float(nsta), float(nlta), 1.0, n_ch), F.Trigger(n_ch, on, off))
            for _ in range(2)]

    def two(o):
        count.zero_()
        for a in range(0, n_t, chunk):
            F.sos_stalta_process(o[0], o[1], x[a:a + chunk], cf=cf[a:a + chunk], write_y=False)
            o[2].process(cf[a:a + chunk], ev, count)

    def one(o):
        count.zero_()
        for a in range(0, n_t, chunk):
            F.monitor_process(o[0], o[1], o[2], x[a:a + chunk], ev, count)

    out = {"workload": f"{n_ch} ch x {n_t} samples in chunks of {chunk}: BP order {w.order} + STA/LTA "
                       f"{nsta}/{nlta} + trigger {on} / {off}, x read, events written"}
    for name, fn, o in (("two_calls_ms_per_step", two, objs[0]), ("one_pass_ms_per_step", one, objs[1])):
        warm(torch, fn, o)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn(o)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / steps
        out["events_per_step"] = int(count.item())
    log(f"[bench] monitor chain x -> events: two calls {out['two_calls_ms_per_step']:.3f} ms/step, one pass "
        f"{out['one_pass_ms_per_step']:.3f} ms/step ({out['events_per_step']} events)")
    for o in objs:
        for h in o:
            h.close()
    return out


def batched_leg(F, torch, dev, replays: int, parity: bool, rotate: int = 4):
    """Batched multi-stream launch: 12 seeded streams of uneven shape (channel
    counts, rates, chunk lengths, bandpass orders drawn by
    synth.draw_batched_streams), SOS only, 1/f input; every stream's channel
    group chosen by the library's autotuner at the batch's block (48) and
    waves (8); one persistent kernel per launch, replayed from a graph the
    batch captured.  `rotate` sets of input / output buffers (one batch
    object and graph each) are launched in turn, so the working set (rotate
    x 235 MB) is far larger than the 256 MB MALL and the figure is an HBM
    one.  Reports aggregate channel-samples/s, the roofline of the batched
    kernel and per-stream completion-latency percentiles from the in-kernel
    stamps."""
    import numpy as np

    import synth
    from paper_2605_20132_amd.autotune import Autotuner

    specs = synth.draw_batched_streams()
    tuner = Autotuner(None, block=48, waves=8)
    sts, soss = [], []
    for sp in specs:
        sos = F.sos_design(sp.order, "bandpass", sp.f1, sp.f2, sp.fs)
        st = F.SOSState(sos, sp.n_ch)
        tuner.tune(st, sp.n_t)
        sts.append(st)
        soss.append(sos)
    sets = []
    for r in range(rotate):
        xs = [synth.pink_noise(sp.n_t, sp.n_ch, seed=sp.seed + 1000 * r, device=dev) for sp in specs]
        ys = [torch.empty_like(x) for x in xs]
        b = F.Batch(sts)
        b.bind(xs, ys)
        b.capture()
        sets.append((b, xs, ys))
    res = {"streams": [{"n_ch": sp.n_ch, "fs": sp.fs, "n_t": sp.n_t, "sections": sp.order // 2,
                        "tile": list(st.tile())} for sp, st in zip(specs, sts)],
           "rotating_sets": rotate}
    b0, xs0, ys0 = sets[0]
    if parity:
        # first launch from the zero state vs the oracle on sampled channels of every stream
        import oracle

        b0.launch()
        torch.cuda.synchronize()
        worst = 0.0
        for sp, x, y in zip(specs, xs0, ys0):
            cols = sorted(set([0, sp.n_ch - 1, sp.n_ch // 2]))
            osos = oracle.butter_sos(sp.order, "bandpass", sp.f1, sp.f2, sp.fs)
            yo, _ = oracle.sos_filter(osos, x[:, cols].double().cpu().numpy())
            yg = y[:, cols].double().cpu().numpy()
            den = np.linalg.norm(yo, axis=0)
            worst = max(worst, float(np.max(np.linalg.norm(yg - yo, axis=0) / np.where(den > 0, den, 1.0))))
        res["parity"] = {"max_rel_rms_y": worst, "channels_per_stream": 3, "tolerance": 1e-5}
    for i in range(2 * rotate):
        sets[i % rotate][0].launch()
    torch.cuda.synchronize()
    lat = []
    for i in range(replays):
        b = sets[i % rotate][0]
        b.launch()
        stm = b.stamps()
        lat.append((stm[:-1].astype(np.int64) - int(stm[-1])) / 100.0)  # 100 MHz ticks -> us
    lat = np.array(lat)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(replays):
        sets[i % rotate][0].launch()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / replays
    work = sum(sp.n_ch * sp.n_t for sp in specs)
    bt = measured_traffic(os.path.join(PROFILES, "fwd_batch_kernel_12streams_traffic.json"))
    batch_traffic = bt["hbm_bytes_per_launch"] if bt else None
    # x read and y written (FP32), each stream's state read and written (FP64)
    bytes_launch = 8.0 * work + sum(2 * 2 * (sp.order // 2) * sp.n_ch * 8 for sp in specs)
    achieved = bytes_launch / (ms / 1e3) / 1e9
    res.update({"replays": replays, "ms_per_launch": ms, "value": work / (ms / 1e3), "unit": "channel-samples/s",
                "algorithmic_gbs": achieved,
                "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS, "traffic": batch_traffic,
                             "kernel": "fwd_batch_kernel<KMAX=5> (persistent; the launch's only kernel)",
                             "algorithmic_bytes_per_launch": bytes_launch,
                             "working_set_bytes": rotate * bytes_launch},
                "latency_us": [{"p50": float(np.percentile(lat[:, i], 50)), "p90": float(np.percentile(lat[:, i], 90)),
                                "p99": float(np.percentile(lat[:, i], 99))} for i in range(len(specs))]})
    log(f"[bench] batched {len(specs)} streams ({rotate} rotating sets): {ms:.3f} ms/launch -> "
        f"{res['value']:.3e} ch-samples/s ({achieved:.0f} GB/s, {achieved / HBM_PEAK_GBS:.3f} of HBM peak); "
        f"max p99 latency {max(l['p99'] for l in res['latency_us']):.0f} us"
        + (f"; parity y {res['parity']['max_rel_rms_y']:.2e}" if parity else ""))
    for b, _, _ in sets:
        b.close()
    for st in sts:
        st.close()
    return res


def extras(args, torch, dev, F, st, sl, step, x, y, cf, chunk, n_chunks, n_t, n_ch, stream, e0, e1):
    """Event pair per launch, graph replay of a step and the on-box copy bandwidth."""
    # ---- the same, with an event pair around each launch (adds the event
    # overhead to every launch; reported beside the figure above)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n_chunks)]
    torch.cuda._sleep(200_000_000)  # back the queue up so host launch latency is not timed
    for i in range(n_chunks):
        a, b = i * chunk, min(n_t, (i + 1) * chunk)
        evs[i][0].record(stream)
        F.sos_stalta_process(st, sl, x[a:b], y[a:b], cf[a:b], write_y=True, stream=stream)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    full = [evs[i][0].elapsed_time(evs[i][1]) for i in range(n_chunks) if (i + 1) * chunk <= n_t]
    pair_ms = float(np.mean(full))
    log(f"[bench] kernel avg {pair_ms * 1e3:.1f} us/launch with an event pair per launch")

    # ---- the same 60 launches captured in one graph
    graph = None
    try:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step(st, sl)
        torch.cuda.synchronize()
        for _ in range(2):
            g.replay()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / args.steps
        st.check()
        graph = {"ms_per_step": gms, "value": n_ch * n_t / (gms / 1e3)}
        log(f"[bench] graph replay {gms:.3f} ms/step -> {graph['value']:.3e} ch-samples/s")
    except Exception as e:  # capture is an optional extra measurement
        log(f"[bench] graph capture unavailable: {e}")

    copy_gbs = copy_bandwidth(torch, dev)
    log(f"[bench] on-box device copy {copy_gbs:.0f} GB/s (read + write)")
    return pair_ms, graph, copy_gbs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-trigger", action="store_true")
    ap.add_argument("--no-filtfilt", action="store_true")
    ap.add_argument("--no-ema", action="store_true")
    ap.add_argument("--no-fir", action="store_true")
    ap.add_argument("--no-config3", action="store_true")
    ap.add_argument("--n-ch", type=int, default=6000)
    ap.add_argument("--n-t", type=int, default=90_000)
    ap.add_argument("--profile", action="store_true",
                    help="only the timed launches of each leg run (no parity passes, event pairs, graph replays, "
                         "copy or CPU timing), so a kernel trace averages exactly the launches the bench times")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain device copy of 512 MiB (counter calibration for profiles)")
    args = ap.parse_args()
    if args.profile:
        global RAMP_WITH_FILL
        RAMP_WITH_FILL = True
        args.no_parity = True
        args.no_cpu = True
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(channels would shard across GPUs with no communication in the forward pass; "
                                   "no multi-GPU launch is implemented)"}))
        sys.exit(2)

    import torch

    import paper_2605_20132_amd as F
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    w = synth.make_config2(device=dev, n_ch=args.n_ch, n_t=args.n_t)
    torch.cuda.synchronize()
    log(f"[bench] input {tuple(w.x.shape)} generated in {time.perf_counter() - t_gen:.1f} s")
    x = w.x
    n_t, n_ch = x.shape
    chunk = w.chunk
    n_chunks = (n_t + chunk - 1) // chunk
    sos = F.sos_design(w.order, w.btype, w.f1, w.f2, w.fs)
    K = sos.shape[0]
    y = torch.empty_like(x)
    cf = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    def make_states():
        return F.SOSState(sos, n_ch), F.StaLtaState(w.sta_s, w.lta_s, w.fs, n_ch)

    def step(st, sl, strm=None):
        for i in range(n_chunks):
            a, b = i * chunk, min(n_t, (i + 1) * chunk)
            F.sos_stalta_process(st, sl, x[a:b], y[a:b], cf[a:b], write_y=True, stream=strm)

    # ---- parity of one full pass from the zero state (sampled channels)
    st, sl = make_states()
    if not args.profile:
        step(st, sl)
        torch.cuda.synchronize()
        st.check()
        sl.check()
    parity = None
    if not args.no_parity:
        import oracle

        rng = np.random.default_rng(0)
        cols = sorted(set([0, 63, 64, n_ch // 2, n_ch - 1] + list(rng.integers(0, n_ch, 11))))
        xs = x[:, cols].double().cpu().numpy()
        osos = oracle.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
        nsta, nlta = oracle.window_samples(w.sta_s, w.fs), oracle.window_samples(w.lta_s, w.fs)
        ref = oracle.Stream(osos, len(cols), nsta, nlta)
        yo, cfo = [], []
        for i in range(n_chunks):
            a, b = ref.process(xs[i * chunk:(i + 1) * chunk])
            yo.append(a)
            cfo.append(b)
        yo, cfo = np.concatenate(yo), np.concatenate(cfo)
        yg = y[:, cols].double().cpu().numpy()
        cg = cf[:, cols].double().cpu().numpy()

        def rr(g, o):
            return float(np.max(np.linalg.norm(g - o, axis=0) / np.linalg.norm(o, axis=0)))

        parity = {"channels": len(cols), "max_rel_rms_y": rr(yg, yo), "max_rel_rms_cf": rr(cg, cfo),
                  "tolerance": 1e-5}
        log(f"[bench] parity on {len(cols)} sampled channels: y {parity['max_rel_rms_y']:.2e} "
            f"cf {parity['max_rel_rms_cf']:.2e}")

    # ---- clock ramp (RAMP_S): untimed steps before the warm-up steps proper
    ramp_steps = ramp(torch, step, st, sl)

    # ---- timed steps (states continue across steps: a continuous stream)
    for _ in range(args.warmup):
        step(st, sl)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_host = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step(st, sl, stream)
    e1.record(stream)
    t_host = time.perf_counter() - t_host
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    st.check()
    sl.check()
    value = n_ch * n_t / (ms_step / 1e3)
    log(f"[bench] {ms_step:.3f} ms/step -> {value:.3e} ch-samples/s "
        f"(host enqueue {t_host * 1e3 / args.steps:.3f} ms/step)")

    # ---- average launch duration of the fused kernel: the HIP events around
    # the timed region (on the launch stream) over the launches it holds,
    # which are this kernel's only (one per chunk, each a single window)
    launches = args.steps * n_chunks
    kern_ms = ms_step * args.steps / launches
    # x read, y and cf written (FP32), filter and STA/LTA state read and written (FP64)
    bytes_launch = (n_ch * n_t * 12 + n_chunks * n_ch * (2 * K + 2) * 8 * 2) / n_chunks
    achieved = bytes_launch / (kern_ms / 1e3) / 1e9
    log(f"[bench] kernel avg {kern_ms * 1e3:.1f} us/launch over the timed region -> {achieved:.0f} GB/s algorithmic")

    if args.calib_copy:
        src = torch.empty(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        flush = torch.empty(256 << 20, dtype=torch.float32, device=dev)
        flush.fill_(2.0)  # 1 GiB written after src: src is not cache resident when copied
        del flush
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {src.numel() * 4} bytes done")
        del src, dst

    pair_ms, graph, copy_gbs = None, None, None
    if not args.profile:
        pair_ms, graph, copy_gbs = extras(args, torch, dev, F, st, sl, step, x, y, cf, chunk, n_chunks, n_t, n_ch,
                                          stream, e0, e1)

    batched = None
    if not args.no_batched:
        batched = batched_leg(F, torch, dev, 40 if args.profile else 200, not args.no_parity)

    trig = None
    if not args.no_trigger:
        trig = trigger_leg(F, torch, dev, 5, not args.no_parity)

    ff = None
    if not args.no_filtfilt:
        ff = filtfilt_leg(F, torch, dev, 20, not args.no_parity)

    ema = None
    if not args.no_ema:
        ema = ema_leg(F, torch, dev, 5, not args.no_parity)

    fir = None
    if not args.no_fir:
        fir = fir_leg(F, torch, dev, 5, not args.no_parity)

    fwd_adj = None
    if not args.no_adjoint:
        fwd_adj = fwd_adjoint_leg(F, torch, dev, 3, not args.no_parity)

    cfg3 = None
    if not args.no_config3:
        cfg3 = config3_leg(F, torch, dev, 5, not args.no_parity)

    t = measured_traffic()
    traffic = None
    if t is not None:
        traffic = t["hbm_bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "copy_peak": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "fwd_kernel<K=4,stalta,write_y>", "kernel_us": kern_ms * 1e3,
                "kernel_us_event_pairs": pair_ms * 1e3 if pair_ms is not None else None,
                "algorithmic_bytes_per_launch": bytes_launch}

    cpu = None
    if not args.no_cpu:
        import oracle

        osos = oracle.butter_sos(w.order, w.btype, w.f1, w.f2, w.fs)
        cpu = cpu_baseline(x, osos, oracle.window_samples(w.sta_s, w.fs),
                           oracle.window_samples(w.lta_s, w.fs), chunk)
        log(f"[bench] cpu oracle {cpu['value']:.3e} ch-samples/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC, "value": value, "unit": "channel-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "clock_ramp_steps": ramp_steps, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"plain forward: {n_ch} ch x {n_t} samples FP32 @ {w.fs:g} Hz in "
                               f"{n_chunks} chunks of {chunk}; Butterworth BP order {w.order} "
                               f"{w.f1:g}-{w.f2:g} Hz ({K} SOS) + STA/LTA {w.sta_s:g}/{w.lta_s:g} s; "
                               "y and cf written",
                   "io": "fp32", "filter_arith": "fp64", "stalta_arith": "fp32 block / fp64 carry"},
        "roofline": roofline, "cpu_baseline": cpu, "parity": parity, "graph_replay": graph,
        "fwd_adjoint": fwd_adj, "config3": cfg3, "batched": batched, "trigger": trig, "zero_phase": ff, "running_agc": ema, "fir": fir,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
