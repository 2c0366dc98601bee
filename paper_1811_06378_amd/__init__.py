"""MI355X-native dyadic Fast Hough Transform (arXiv 1811.06378).

The compute path is libfht.so (hand-written HIP kernels for gfx950) behind the
C ABI in include/fht.h; `fht` is its ctypes binding.  `synth` holds the seeded
input generators.
"""
from . import fht  # noqa: F401  (binding only; the library loads on first call)
from .fht import (  # noqa: F401
    FHTFunction,
    BatchPlan,
    adjoint,
    forward,
    hough_shape,
    range_params,
    range_transform,
    shift,
)
