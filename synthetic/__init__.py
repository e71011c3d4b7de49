"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds input matrices, coordinates and right-hand sides.  It
holds none of the factorization's arithmetic, so both the CPU oracle and the
GPU path can draw the very same inputs from it without sharing method code.
"""
from .problems import (  # noqa: F401
    Problem,
    laplacian_2d,
    laplacian_3d,
    fv_diffusion_3d,
    high_contrast_2d,
    rhs,
    workload,
    batch_problems,
    serve_stream,
    poisson_modes,
    poisson_eigvec,
    sketch,
    SKETCH_ROWS,
    WORKLOADS,
)
