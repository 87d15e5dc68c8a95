"""The seeded synthetic inputs (CPU): reproducibility, prefixes, worker independence, and that the
events lie where the detector model puts them.  The generator holds no arithmetic of the method;
these checks only pin the inputs both sides read."""

import numpy as np

from jpet_synth import get_workload
from jpet_synth.configs import batch_instances


def test_prefix_and_worker_independence():
    w = get_workload("prod400")
    a = w.events(1_100_000, workers=1)  # spans two generator blocks of 2^20 events
    b = w.events(1_100_000, workers=2)
    assert np.array_equal(a, b)
    assert np.array_equal(w.events(1000, workers=1), a[:1000])
    assert a.dtype == np.float32 and a.shape == (1_100_000, 3)


def test_events_lie_on_the_strips_and_are_seeded():
    for name in ("tiny", "paper130", "edge400"):
        w = get_workload(name)
        ev = w.events(20_000)
        assert np.all(np.isfinite(ev))
        assert np.all(np.abs(ev[:, :2]) <= 0.5 * w.L)
        # dl of a point between the strips is bounded by the path difference across them
        assert np.all(np.abs(ev[:, 2]) < 2 * w.R / np.cos(np.arctan(w.L / (2 * w.R))) + 10 * w.sigma_dl)
        assert np.array_equal(ev, w.events(20_000))
        assert not np.array_equal(ev, w.events(20_000, seed_offset=1))


def test_batch_instances_follow_the_stated_ranges():
    inst = batch_instances()
    assert len(inst) == 64
    for w in inst:
        assert w.n_y == w.n_z and w.n_y in (128, 256, 512)
        assert w.pixel == 600.0 / w.n_y
        assert 8.0 <= w.sigma_z <= 15.0 and 40.0 <= w.sigma_dl <= 90.0
        assert 50_000 <= w.n_events <= 2_000_000
    assert len({w.seed for w in inst}) == 64
