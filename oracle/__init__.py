"""CPU oracle for the Brady dyadic FHT (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does.
"""
from .oracle import (  # noqa: F401
    build,
    lib_path,
    next_pow2,
    threads,
    pattern_offset,
    quadrant,
    full,
    fhtshift_full,
    fhtshift_roll,
    row_quadrant,
    range_transform,
    range_sigma,
    range_params,
    cell,
    full_cell,
    full_cells,
    adjoint_full,
    adjoint_quadrant,
    hough_shape,
    stacked_quadrants,
    quadrant_op,
    full_op,
    range_adjoint,
    range_scaled,
    scaled_sizes,
)
from . import lines  # noqa: F401,E402
