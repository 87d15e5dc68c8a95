"""Monte-Carlo simulation of two-strip coincidence events.

The detector is the paper's Setup section: strips at y = +R and y = -R of
length L along z.  For each accepted emission:

1. an emission point (z, y) is drawn with density proportional to the
   phantom's activity (exact rejection sampling from a mixture of the
   ellipses' bounding boxes);
2. an in-plane emission angle theta is drawn uniformly in [-pi/2, pi/2);
3. the true hit positions on the two strips and the path-length difference are
   computed geometrically: z_u = z + (R - y) tan(theta), z_d = z - (R + y) tan(theta)
   and dl = |upper hit - e| - |lower hit - e|;
4. the event is detected only when both hits lie on the strips (|z| <= L/2),
   so detected events are distributed as sensitivity x activity;
5. Gaussian noise N(0, sigma_z^2) is added to z_u and z_d and N(0, sigma_dl^2)
   to dl; events whose measured z_u or z_d leave the strips are rejected.  With
   sigma_z_edge > 0 the z noise of a hit at z has the standard deviation
   sigma_z (1 + sigma_z_edge (2z/L)^2) instead: lowest at the strip centre and
   higher by the fraction sigma_z_edge at its ends.

Events are returned as float32 ``[n, 3]`` rows (z_u, z_d, dl) in mm.
"""

from __future__ import annotations

import multiprocessing
import os

import numpy as np

from .phantom import Phantom

_CHUNK = 1 << 18


def _proposal(phantom: Phantom, R: float):
    """Per-ellipse axis-aligned boxes and mixture weights for the point proposal."""
    boxes, w = [], []
    for e in phantom.ellipses:
        one = Phantom((e,))
        zmin, zmax, ymin, ymax = one.bounding_box()
        ymin, ymax = max(ymin, -R + 1e-6), min(ymax, R - 1e-6)
        boxes.append((zmin, zmax, ymin, ymax))
        w.append((zmax - zmin) * max(ymax - ymin, 0.0) * e.activity)
    w = np.asarray(w, dtype=np.float64)
    return np.asarray(boxes, dtype=np.float64), w / w.sum()


def _draw_points(rng, phantom: Phantom, boxes, weights, act_of, m):
    """m proposals from the box mixture, thinned to density proportional to the activity.

    A proposal picks ellipse e with probability proportional to box area x activity and a
    uniform point in its box, so its density is proportional to the sum of activities of the
    boxes covering the point; keeping it with probability activity(point) / that sum leaves
    points distributed exactly as the (topmost-wins) activity map.
    """
    k = rng.choice(len(weights), size=m, p=weights)
    b = boxes[k]
    z = b[:, 0] + (b[:, 1] - b[:, 0]) * rng.random(m)
    y = b[:, 2] + (b[:, 3] - b[:, 2]) * rng.random(m)
    cover = np.zeros(m)
    for (zmin, zmax, ymin, ymax), a in zip(boxes, act_of):
        cover += np.where((z >= zmin) & (z <= zmax) & (y >= ymin) & (y <= ymax), a, 0.0)
    keep = rng.random(m) * cover < phantom.activity(z, y)
    return z[keep], y[keep]


_BLOCK = 1 << 20


def _simulate_block(args) -> np.ndarray:
    phantom, R, L, sigma_z, sigma_dl, n, seed, block, sigma_z_edge = args
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, block])))
    boxes, weights = _proposal(phantom, R)
    act_of = [e.activity for e in phantom.ellipses]
    half = 0.5 * L
    out = np.empty((n, 3), dtype=np.float32)
    filled = 0
    while filled < n:
        z, y = _draw_points(rng, phantom, boxes, weights, act_of, _CHUNK)
        t = np.tan(rng.uniform(-0.5 * np.pi, 0.5 * np.pi, z.size))
        zu = z + (R - y) * t
        zd = z - (R + y) * t
        hit = (np.abs(zu) <= half) & (np.abs(zd) <= half)
        z, y, zu, zd = z[hit], y[hit], zu[hit], zd[hit]
        dl = np.sqrt((R - y) ** 2 + (zu - z) ** 2) - np.sqrt((R + y) ** 2 + (zd - z) ** 2)
        nz = rng.normal(0.0, 1.0, (z.size, 3))
        if sigma_z_edge:
            mzu = zu + sigma_z * (1.0 + sigma_z_edge * (zu / half) ** 2) * nz[:, 0]
            mzd = zd + sigma_z * (1.0 + sigma_z_edge * (zd / half) ** 2) * nz[:, 1]
        else:
            mzu = zu + sigma_z * nz[:, 0]
            mzd = zd + sigma_z * nz[:, 1]
        mdl = dl + sigma_dl * nz[:, 2]
        ok = (np.abs(mzu) <= half) & (np.abs(mzd) <= half)
        take = min(int(ok.sum()), n - filled)
        if take:
            out[filled:filled + take, 0] = mzu[ok][:take]
            out[filled:filled + take, 1] = mzd[ok][:take]
            out[filled:filled + take, 2] = mdl[ok][:take]
            filled += take
    return out


def simulate_events(phantom: Phantom, R: float, L: float, sigma_z: float, sigma_dl: float,
                    n: int, seed: int, workers: int | None = None, sigma_z_edge: float = 0.0) -> np.ndarray:
    """n events; block b of 2^20 events draws from its own stream seeded by (seed, b).

    The result is a pure function of (phantom, geometry, resolution, seed) and the first m
    events of a request for n >= m events equal a request for m events, whatever the
    number of worker processes.
    """
    nblocks = (n + _BLOCK - 1) // _BLOCK
    jobs = [(phantom, R, L, sigma_z, sigma_dl, min(_BLOCK, n - b * _BLOCK), seed, b, sigma_z_edge)
            for b in range(nblocks)]
    if workers is None:
        workers = min(nblocks, 8, os.cpu_count() or 1)
    if workers <= 1 or nblocks <= 1:
        parts = [_simulate_block(j) for j in jobs]
    else:
        ctx = multiprocessing.get_context("spawn")
        with ctx.Pool(workers) as pool:
            parts = pool.map(_simulate_block, jobs)
    if not parts:
        return np.empty((0, 3), dtype=np.float32)
    return np.concatenate(parts, axis=0)
