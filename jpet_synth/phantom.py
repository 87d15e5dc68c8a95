"""Ellipse phantoms (activity maps) used to draw emission points.

A phantom is an ordered list of ellipses.  Each ellipse has a centre
(z_c, y_c), semi-axes (a, b), a counter-clockwise rotation phi in degrees and
an activity.  Where ellipses overlap the activity is taken from the *first*
(topmost) matching row, as Appendix A of the paper specifies for its phantom
table.  The paper's table uses (x, y); here x is the coordinate along the
strips (z) and y the coordinate across the gap, and ``a`` is the semi-axis
along the rotated z axis.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Ellipse:
    zc: float
    yc: float
    a: float
    b: float
    phi_deg: float
    activity: float


@dataclasses.dataclass(frozen=True)
class Phantom:
    ellipses: tuple

    def activity(self, z: np.ndarray, y: np.ndarray) -> np.ndarray:
        """Activity at points (z, y); the first matching ellipse wins."""
        z, y = np.broadcast_arrays(np.asarray(z, dtype=np.float64), np.asarray(y, dtype=np.float64))
        shape = z.shape
        z, y = z.ravel(), y.ravel()
        act = np.zeros(z.size, dtype=np.float64)
        todo = np.arange(z.size)
        for e in self.ellipses:
            if todo.size == 0:
                break
            zmin, zmax, ymin, ymax = Phantom((e,)).bounding_box()
            zt, yt = z[todo], y[todo]
            near = (zt >= zmin) & (zt <= zmax) & (yt >= ymin) & (yt <= ymax)
            cand = todo[near]
            phi = math.radians(e.phi_deg)
            cp, sp = math.cos(phi), math.sin(phi)
            dz, dy = z[cand] - e.zc, y[cand] - e.yc
            u = (dz * cp + dy * sp) / e.a
            v = (-dz * sp + dy * cp) / e.b
            inside = u * u + v * v <= 1.0
            act[cand[inside]] = e.activity
            hit = np.zeros(todo.size, dtype=bool)
            hit[np.nonzero(near)[0][inside]] = True
            todo = todo[~hit]
        return act.reshape(shape)

    def bounding_box(self):
        """Axis-aligned (zmin, zmax, ymin, ymax) covering every ellipse."""
        zmin = ymin = math.inf
        zmax = ymax = -math.inf
        for e in self.ellipses:
            phi = math.radians(e.phi_deg)
            hz = math.hypot(e.a * math.cos(phi), e.b * math.sin(phi))
            hy = math.hypot(e.a * math.sin(phi), e.b * math.cos(phi))
            zmin, zmax = min(zmin, e.zc - hz), max(zmax, e.zc + hz)
            ymin, ymax = min(ymin, e.yc - hy), max(ymax, e.yc + hy)
        return zmin, zmax, ymin, ymax

    def max_activity(self) -> float:
        return max(e.activity for e in self.ellipses)


# Appendix A, table "Phantom description": rows (x, y, a, b, phi, rho), topmost wins.
TABLE_A_ROWS = (
    (0.0, 0.0, 30.0, 60.0, 0.0, 0.3),
    (50.0, -62.0, 10.0, 33.0, -40.0, 0.3),
    (-50.0, -63.0, 20.0, 33.0, 45.0, 0.5),
    (60.0, 65.0, 13.0, 14.0, 0.0, 0.5),
    (35.0, 55.0, 12.0, 12.0, 0.0, 0.7),
    (0.0, 0.0, 120.0, 110.0, 0.0, 0.1),
)


def table_a_phantom() -> Phantom:
    """The paper's own phantom (Appendix A), x -> z and y -> y."""
    return Phantom(tuple(Ellipse(*row) for row in TABLE_A_ROWS))


def c1_phantom() -> Phantom:
    """Three nested ellipses with uniform activity ratio 1:2:4 (tiny workload)."""
    return Phantom((
        Ellipse(30.0, -20.0, 12.0, 12.0, 0.0, 4.0),
        Ellipse(-35.0, 25.0, 25.0, 15.0, 30.0, 2.0),
        Ellipse(0.0, 0.0, 100.0, 80.0, 0.0, 1.0),
    ))


def c2_phantom() -> Phantom:
    """Four hot disks (diameters 5, 10, 15, 20 mm) on top of the Appendix A phantom."""
    disks = (
        Ellipse(0.0, -95.0, 2.5, 2.5, 0.0, 1.0),
        Ellipse(-30.0, 80.0, 5.0, 5.0, 0.0, 1.0),
        Ellipse(80.0, -10.0, 7.5, 7.5, 0.0, 1.0),
        Ellipse(-80.0, 20.0, 10.0, 10.0, 0.0, 1.0),
    )
    return Phantom(disks + table_a_phantom().ellipses)


def random_phantom(seed: int) -> Phantom:
    """A background ellipse with 3..8 random inserts (batched-reconstruction instances)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ba = float(rng.uniform(150.0, 250.0))
    bb = float(rng.uniform(100.0, 200.0))
    k = int(rng.integers(3, 9))
    inserts = []
    for _ in range(k):
        a = float(rng.uniform(5.0, 50.0))
        b = float(rng.uniform(5.0, 50.0))
        # keep the insert centre inside the background, away from its rim
        r = float(rng.uniform(0.0, 0.8))
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        zc = r * ba * math.cos(ang)
        yc = r * bb * math.sin(ang)
        inserts.append(Ellipse(zc, yc, a, b, float(rng.uniform(0.0, 180.0)), float(rng.uniform(0.5, 4.0))))
    return Phantom(tuple(inserts) + (Ellipse(0.0, 0.0, ba, bb, 0.0, 1.0),))


def dense_phantom(seed: int, n: int = 200, half_extent: float = 230.0) -> Phantom:
    """n random ellipses with log-normal(0, 0.5) activity (large single-image workload)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        out.append(Ellipse(
            float(rng.uniform(-half_extent, half_extent)),
            float(rng.uniform(-half_extent, half_extent)),
            float(rng.uniform(3.0, 40.0)),
            float(rng.uniform(3.0, 40.0)),
            float(rng.uniform(0.0, 180.0)),
            float(math.exp(rng.normal(0.0, 0.5))),
        ))
    return Phantom(tuple(out))
