"""GSta training hot path on MI355X (gfx950).

The compute runs in libgsta.so (hand-written HIP kernels behind the C ABI of
include/gsta.h); this package is its Python binding plus the host-side
training schedule.
"""
from ._lib import GstaError, load  # noqa: F401
from .core import Context, camera_array, camera_struct, n_rows, params_struct  # noqa: F401
