"""torch.autograd binding of the fused SOS + STA/LTA path.

``sos_stalta_cf(x, theta, nsta, nlta, chunk)`` runs a record through the
stateful chunked forward kernel (state carried from chunk to chunk, zero
initial state) and returns cf.  The forward records each chunk's adjoint
tape (the forward state at every adjoint window start); the backward pass
runs the adjoint kernel chunk by chunk, last to first, from those tapes and
returns dL/dx and dL/dtheta.  Where the adjoint tile admits no tape, the
forward keeps a device checkpoint of the state per chunk instead and the
adjoint reruns the chunk's forward states.  ``theta`` holds
(b0, b1, b2, a1, a2) of each section (a0 = 1).

Every step runs in libfilark's kernels; this module only marshals tensors.
"""

from __future__ import annotations

import numpy as np
import torch

from . import (FilarkError, SOSState, StaLtaState, adjoint_tape_bytes, sos_stalta_adjoint,
               sos_stalta_adjoint_tape, sos_stalta_process, sos_stalta_process_tape)


def theta_to_sos(theta) -> np.ndarray:
    t = np.asarray(theta.detach().cpu().numpy() if isinstance(theta, torch.Tensor) else theta, dtype=np.float64)
    sos = np.zeros((t.shape[0], 6))
    sos[:, [0, 1, 2, 4, 5]] = t
    sos[:, 3] = 1.0
    return sos


def sos_to_theta(sos) -> np.ndarray:
    s = np.asarray(sos, dtype=np.float64)
    return (s[:, [0, 1, 2, 4, 5]] / s[:, 3:4]).copy()


def _splits(n_t: int, chunk: int):
    return [(a, min(n_t, a + chunk)) for a in range(0, n_t, chunk)]


class SosStaLta(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, theta, nsta: int, nlta: int, chunk: int):
        if not x.is_cuda or x.dtype != torch.float32:
            raise TypeError("x must be a float32 CUDA tensor [n_t, n_ch]")
        x = x.contiguous()
        n_t, n_ch = x.shape
        st = SOSState(theta_to_sos(theta), n_ch)
        sl = StaLtaState(float(nsta), float(nlta), 1.0, n_ch)
        cf = torch.empty_like(x)
        try:
            adjoint_tape_bytes(st, sl, 1)
            use_tape = True
        except FilarkError:
            use_tape = False
        cks = []
        for a, b in _splits(n_t, chunk):
            if use_tape:
                cks.append(sos_stalta_process_tape(st, sl, x[a:b], cf=cf[a:b])[2])
            else:
                cks.append((st.save(), sl.save()))
                sos_stalta_process(st, sl, x[a:b], cf=cf[a:b], write_y=False)
        ctx.save_for_backward(x)
        ctx.state = (st, sl, cks, use_tape, chunk, theta.dtype, theta.device)
        return cf

    @staticmethod
    def backward(ctx, g_cf):
        (x,) = ctx.saved_tensors
        st, sl, cks, use_tape, chunk, th_dtype, th_device = ctx.state
        n_t, n_ch = x.shape
        g_cf = g_cf.to(torch.float32).contiguous()
        gx = torch.empty_like(x)
        adj = torch.zeros((2 * st.n_sec + 2, n_ch), dtype=torch.float64, device=x.device)
        gsos = torch.zeros((st.n_sec, 5), dtype=torch.float64, device=x.device)
        for (a, b), ck in reversed(list(zip(_splits(n_t, chunk), cks))):
            if use_tape:
                sos_stalta_adjoint_tape(st, sl, ck, x[a:b], g_cf[a:b], gx[a:b], adj, gsos, mode="grad")
            else:
                st.load(ck[0])
                sl.load(ck[1])
                sos_stalta_adjoint(st, sl, x[a:b], g_cf[a:b], gx[a:b], adj, gsos, mode="grad")
        return gx, gsos.to(device=th_device, dtype=th_dtype), None, None, None


def sos_stalta_cf(x, theta, nsta: int, nlta: int, chunk: int):
    """cf of the chunked fused path, differentiable in x and theta."""
    return SosStaLta.apply(x, theta, int(nsta), int(nlta), int(chunk))
