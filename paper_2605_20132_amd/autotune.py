"""Tile autotuning for the forward kernels: a thin caller of the library's
filark_autotune, which times the candidate tiles on the device (HIP events),
applies the fastest and keeps the choices in a JSON cache keyed by the shape
(channels, chunk rows, sections, and the block / waves constraints).

For a batched launch every stream must share the block (48) and the waves
per workgroup; the tuner then picks each stream's channel group.
"""

from __future__ import annotations

from . import SOSState, tune_tile


class Autotuner:
    def __init__(self, cache_path: str | None = None, block: int = 48, waves: int = 8):
        self.cache_path = cache_path
        self.block, self.waves = block, waves

    def tune(self, st: SOSState, n_t: int):
        """Tune st's tile for chunks of n_t rows within the tuner's block and
        waves (0 = searched); returns (block, waves, group), applied to st."""
        return tune_tile(st, n_t, self.block, self.waves, self.cache_path)

    def group_for(self, sos, n_ch: int, n_t: int) -> int:
        """The fastest channel group for this stream shape."""
        st = SOSState(sos, n_ch)
        try:
            return self.tune(st, n_t)[2]
        finally:
            st.close()
