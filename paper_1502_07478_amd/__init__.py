"""MI355X (gfx950) list-mode MLEM reconstruction for the two-strip J-PET detector.

The compute path is libjpet.so (hand-written HIP kernels behind the C-ABI of
include/jpet.h); ``paper_1502_07478_amd.jpet`` is its ctypes binding.
"""

from . import jpet  # noqa: F401
from .jpet import (Geometry, JpetError, Stats, geometry, loglik_grad, mlem, mlem_iterate, prepare,  # noqa: F401
                   sensitivity, workspace, workspace_size)
