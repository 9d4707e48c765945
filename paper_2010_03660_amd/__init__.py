"""MI355X-native BiCGStab for 7-point variable-coefficient stencil systems.

The solver runs in hand-written HIP kernels for gfx950 behind the C-ABI
library ``libs7.so`` (declared in ``include/s7.h``).  This package is the thin
Python binding: it marshals arguments (device pointers of torch tensors,
streams) and calls the library; every step of the solve runs on the GPU.
"""

# Paper, Table I: 44 floating-point operations per meshpoint per BiCGStab
# iteration (two matrix-vector products 24, four dot products 8, six AXPYs 12).
FLOPS_PER_CELL_ITER = 44

from .binding import *  # noqa: E402,F401,F403
