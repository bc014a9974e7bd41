"""Tile autotuner for the forward kernels.

For a stream shape (channels, chunk length, sections) it times the candidate
tile shapes on the device with the library's own per-stream entry point and
keeps the fastest; results are cached in memory and, optionally, in a JSON
file keyed by the shape, so a later process reuses them without measuring.
Candidates share the block length and waves per workgroup that a batched
launch requires, and differ in channels per workgroup (group), which sets
both the number of workgroups and the window length.
"""

from __future__ import annotations

import json
import os

import numpy as np

from . import SOSState

GROUPS = (4, 8, 16, 32, 64)


def _key(n_ch: int, n_t: int, n_sec: int, block: int, waves: int) -> str:
    return f"{n_ch}x{n_t}/K{n_sec}/L{block}W{waves}"


class Autotuner:
    def __init__(self, cache_path: str | None = None, block: int = 64, waves: int = 4, reps: int = 5):
        self.cache_path = cache_path
        self.block, self.waves, self.reps = block, waves, reps
        self.table: dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.table = json.load(f)

    def save(self):
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    def _time(self, st: SOSState, x, y) -> float:
        import torch

        st.process(x, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(self.reps):
            st.process(x, y)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / self.reps

    def group_for(self, sos, n_ch: int, n_t: int) -> int:
        """Fastest channel group for this stream shape (measured once, then cached)."""
        import torch

        sos = np.asarray(sos, dtype=np.float64)
        k = _key(n_ch, n_t, sos.shape[0], self.block, self.waves)
        if k in self.table:
            return int(self.table[k]["group"])
        x = torch.randn((max(1, n_t), n_ch), device="cuda", dtype=torch.float32)
        y = torch.empty_like(x)
        times = {}
        for g in GROUPS:
            st = SOSState(sos, n_ch)
            try:
                st.set_tile(self.block, self.waves, g)
                times[g] = self._time(st, x, y)
            finally:
                st.close()
        best = min(times, key=times.get)
        self.table[k] = {"group": best, "us": {str(g): t for g, t in times.items()}}
        self.save()
        return best

    def plan(self, streams) -> list[int]:
        """Groups for a list of (sos, n_ch, n_t)."""
        return [self.group_for(s, c, t) for s, c, t in streams]
