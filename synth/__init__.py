"""Seeded synthetic reversed-gradient EPI pairs (stand-ins for the paper's 2D and 3D data).

This package only draws random parameters and applies the continuous physical distortion
model (Section 2, the reversed-gradient identity) to produce image pairs; it contains none
of the discretised method (no interpolation of the discrete images, no residuals, no
solvers). It is shared by the oracle tests, the GPU parity tests and the benchmark.
"""
from .generator import (
    Volume,
    generate,
    to_canonical,
    from_canonical,
    CONFIGS,
    config_volume,
    batch_shapes,
    serving_requests,
    shutdown_pool,
)

__all__ = [
    "Volume",
    "generate",
    "to_canonical",
    "from_canonical",
    "CONFIGS",
    "config_volume",
    "batch_shapes",
    "serving_requests",
    "shutdown_pool",
]
