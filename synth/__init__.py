"""Seeded synthetic dexel shapes.

Input generators shared by the tests, the benchmark and the oracle checks.
This package holds no part of the offset method itself: it only ray-casts
analytic solids (spheres, boxes, a gyroid lattice) into canonical CSR dexel
grids (column pointers plus float32 (z_in, z_out) pairs).
"""
from .gen import (  # noqa: F401
    DexelGrid,
    canonical_csr,
    spheres_grid,
    primitives_grid,
    gyroid_grid,
    batch_shapes,
    serving_stream,
    config_grid,
    CONFIGS,
)
