"""Seeded synthetic workloads for the NASGabor / SH-3 appearance path.

This package only draws random numbers and rounds them to a storage dtype.
It contains none of the method's arithmetic, so both the FP64 oracle and the
HIP path can take their inputs from it without sharing any computation.
"""
from .gen import (  # noqa: F401
    Workload,
    Scene,
    draw_workload,
    config0,
    config1,
    config2,
    config3,
    config4,
    f32_to_bf16_bits,
    bf16_bits_to_f32,
    take_primitives,
)
from .raster import SplatScene, draw_splat_scene  # noqa: F401
