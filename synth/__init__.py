"""Seeded synthetic DAS-shaped inputs.

This package only draws test and benchmark inputs (noise, moveout events,
drift).  It contains none of the filtering or STA/LTA arithmetic, so both the
FP64 oracle and the HIP path can consume its outputs without sharing any of
the method's code.
"""

from .das import (  # noqa: F401
    Event,
    StreamSpec,
    Workload,
    cf_like,
    draw_batched_streams,
    draw_events,
    make_config1,
    make_config2,
    make_config3,
    make_config5,
    pink_noise,
    ricker_events,
    white_noise,
)
