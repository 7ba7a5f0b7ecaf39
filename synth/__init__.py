"""Seeded synthetic inputs shared by the product tests, the oracle tests and
the benchmark.

This package only *builds inputs*: panel geometries (rectangles and right
triangles), lattice/mirror image descriptions, evaluation points and charge
clouds.  It holds none of the boundary-element arithmetic (no Green's-function
integrals, no assembly, no solve); both the CPU oracle and the HIP path consume
what it produces.
"""
from .geometry import (  # noqa: F401
    Geometry,
    Images,
    GeometryBuilder,
    parallel_plates,
    gem_cell,
    strip_cell,
    thgem_double,
)
from .workloads import (  # noqa: F401
    uniform_points,
    gem_eval_points,
    thgem_eval_points,
    charge_cloud,
    serve_requests,
)
