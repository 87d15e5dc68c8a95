"""MI355X (gfx950) list-mode MLEM reconstruction for the two-strip J-PET detector.

The compute path is libjpet.so (hand-written HIP kernels behind the C-ABI of
include/jpet.h); ``paper_1502_07478_amd.jpet`` is its ctypes binding.
"""

from . import jpet  # noqa: F401
from .jpet import (BatchedMLEM, ChunkedMLEM, Geometry, JPetLogLik, JpetError, Stats, geometry, loglik, loglik_grad, mlem,  # noqa: F401
                   mlem_iterate, prepare, sensitivity, workspace, workspace_size)
