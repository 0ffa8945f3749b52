"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package generates initial conditions and random test data only.  It holds
none of the compression method's arithmetic (no transform, threshold, encoding
or stencil): everything here is a plain function of a NumPy ``default_rng``
seed, so that both sides of a parity test start from the same bytes.

Array convention: 2-D fields are indexed ``[y, x]`` and 3-D fields ``[z, y, x]``
(x fastest in memory); multi-field states put the field first.
"""
from .fields import (
    fv_gaussians_and_step,
    shear_layer_macroscopic,
    taylor_green_macroscopic,
    worked_example_field,
    random_signal,
    random_coefficient_tiles,
    transport_gaussian,
    riemann_four_quadrants,
    shear_with_vortices,
    taylor_green_jets_3d,
)

__all__ = [
    "fv_gaussians_and_step",
    "shear_layer_macroscopic",
    "taylor_green_macroscopic",
    "worked_example_field",
    "random_signal",
    "random_coefficient_tiles",
    "transport_gaussian",
    "riemann_four_quadrants",
    "shear_with_vortices",
    "taylor_green_jets_3d",
]
