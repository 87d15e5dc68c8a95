"""Named workloads: detector geometry, resolution, pixel grid, phantom and event count.

The names describe the workloads by what they are:

* ``tiny``      R=450, L=500, 64x64 px of 4 mm, sigma=(10, 63), 20k events, 5 iterations
* ``prod400``   R=450, L=500, 400x400 px of 2 mm, sigma=(10, 63), 10M events, 10 iterations
* ``batch64``   64 independent instances: grids 128/256/512 at 600/N mm, sigma_z in 8..15,
                sigma_dl in 40..90, log-uniform 50k..2M events, 10 iterations
* ``grad200``   R=450, L=500, 200x200 px of 2.5 mm, sigma=(10, 63), 1M events
* ``large1024`` R=450, L=1000, 1024x1024 px of 0.5 mm, sigma=(5, 30), 100M events, 20 iterations
* ``paper130``  the paper's own setting: R=130, L=300, 4 mm pixels (64x76 px covering the strips),
                sigma=(10, 40), the Appendix A phantom, 10M events, 10 iterations
* ``edge400``   prod400 with a position-dependent sigma_z: 10 mm at the strip centre rising by 10%
                towards the ends (sigma_z_edge = 0.1), 10M events, 10 iterations

Seeds are 1502074780 + workload index; instance m of ``batch64`` uses seed + 1000 m.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import phantom as ph
from .events import simulate_events

BASE_SEED = 1502074780


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    R: float
    L: float
    sigma_z: float
    sigma_dl: float
    pixel: float
    n_y: int
    n_z: int
    n_events: int
    n_iter: int
    seed: int
    phantom_kind: str
    sigma_z_edge: float = 0.0  # relative rise of sigma_z from the strip centre to its ends

    def phantom(self) -> ph.Phantom:
        if self.phantom_kind == "c1":
            return ph.c1_phantom()
        if self.phantom_kind == "c2":
            return ph.c2_phantom()
        if self.phantom_kind == "dense":
            return ph.dense_phantom(self.seed)
        if self.phantom_kind == "tablea":
            return ph.table_a_phantom()
        if self.phantom_kind == "random":
            return ph.random_phantom(self.seed)
        raise ValueError(self.phantom_kind)

    def events(self, n: int | None = None, seed_offset: int = 0, workers: int | None = None) -> np.ndarray:
        """The first n events (default: all); workers=1 generates in this process (required inside
        a worker process of a pool)."""
        n = self.n_events if n is None else n
        return simulate_events(self.phantom(), self.R, self.L, self.sigma_z, self.sigma_dl, n,
                               self.seed + seed_offset, workers=workers, sigma_z_edge=self.sigma_z_edge)

    def geometry(self, **over) -> dict:
        g = dict(R=self.R, L=self.L, sigma_z=self.sigma_z, sigma_dl=self.sigma_dl,
                 pixel=self.pixel, n_y=self.n_y, n_z=self.n_z)
        if self.sigma_z_edge:
            g["sigma_z_edge"] = self.sigma_z_edge
        g.update(over)
        return g

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


WORKLOADS = {
    "tiny": Workload("tiny", 450.0, 500.0, 10.0, 63.0, 4.0, 64, 64, 20_000, 5, BASE_SEED + 1, "c1"),
    "prod400": Workload("prod400", 450.0, 500.0, 10.0, 63.0, 2.0, 400, 400, 10_000_000, 10, BASE_SEED + 2, "c2"),
    "grad200": Workload("grad200", 450.0, 500.0, 10.0, 63.0, 2.5, 200, 200, 1_000_000, 5, BASE_SEED + 4, "c2"),
    "large1024": Workload("large1024", 450.0, 1000.0, 5.0, 30.0, 0.5, 1024, 1024, 100_000_000, 20,
                          BASE_SEED + 5, "dense"),
    "paper130": Workload("paper130", 130.0, 300.0, 10.0, 40.0, 4.0, 64, 76, 10_000_000, 10, BASE_SEED + 6, "tablea"),
    "edge400": Workload("edge400", 450.0, 500.0, 10.0, 63.0, 2.0, 400, 400, 10_000_000, 10, BASE_SEED + 7, "c2",
                        sigma_z_edge=0.1),
}


def get_workload(name: str) -> Workload:
    return WORKLOADS[name]


def batch_instances(count: int = 64, base_seed: int = BASE_SEED + 3) -> list:
    """Instances of the batched workload: per-instance grid, resolution and event count."""
    out = []
    for m in range(count):
        seed = base_seed + 1000 * m
        rng = np.random.Generator(np.random.PCG64(seed))
        n = int((128, 256, 512)[int(rng.integers(0, 3))])
        sz = float(rng.uniform(8.0, 15.0))
        sdl = float(rng.uniform(40.0, 90.0))
        ne = int(round(math.exp(rng.uniform(math.log(5e4), math.log(2e6)))))
        out.append(Workload(f"batch64[{m}]", 450.0, 500.0, sz, sdl, 600.0 / n, n, n, ne, 10, seed, "random"))
    return out
