"""Seeded synthetic input generators for the n-field block solver.

This package only builds inputs: assembled block matrices, near-nullspace
vectors per field and right-hand sides, on structured Q1 meshes.  It holds
none of the solver's arithmetic (no aggregation, no smoothing, no Krylov
method).  Both the GPU library's tests/benchmarks and the CPU oracle's tests
take their inputs from here, the way they would read a file from disk.
"""
from .systems import (Field, BlockSystem, tsi2d, tsi2d_alpha, ALPHA_SWEEP, fsi3d, lung3d, request_trace,
                      request_rhs, uniform_rhs, permute_fields, one_sided_pattern, SERVE_GRIDS)

__all__ = ["Field", "BlockSystem", "tsi2d", "tsi2d_alpha", "ALPHA_SWEEP", "fsi3d", "lung3d", "request_trace",
           "request_rhs", "uniform_rhs", "permute_fields", "one_sided_pattern", "SERVE_GRIDS"]
