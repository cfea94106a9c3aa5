"""MI355X (gfx950) RASPEN solver for L2/L1-regularised semilinear elliptic optimal control.

The compute path is libraspen.so (hand-written HIP kernels behind the C ABI in
include/raspen.h); ``paper_2411_00546_amd.raspen`` is its Python binding.
"""
from . import raspen  # noqa: F401
