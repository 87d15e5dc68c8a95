"""Seeded synthetic inputs for the two-strip J-PET list-mode reconstruction.

This package only *generates data*: phantoms (ellipse tables), simulated
coincidence events and the named workload configurations.  It contains none of
the reconstruction arithmetic (no direct reconstruction, no kernel, no
sensitivity, no MLEM): the oracle under ``oracle/`` and the HIP library under
``paper_1502_07478_amd/`` each implement those independently, and both read
the arrays produced here.

Events follow the detector model of the paper's Setup section: two strips at
y = +R (upper) and y = -R (lower), each of length L along z.  An event is the
triple (z_u, z_d, dl) in millimetres, stored as float32 ``[n, 3]``.
"""

from .phantom import Ellipse, Phantom, table_a_phantom, c1_phantom, c2_phantom, random_phantom, dense_phantom
from .events import simulate_events
from .configs import Workload, get_workload, WORKLOADS

__all__ = [
    "Ellipse", "Phantom", "table_a_phantom", "c1_phantom", "c2_phantom", "random_phantom",
    "dense_phantom", "simulate_events", "Workload", "get_workload", "WORKLOADS",
]
