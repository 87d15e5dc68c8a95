"""The 1024x1024 workload at full size: 100M events (R=450, L=1000, 0.5 mm pixels, sigma=(5, 30))
through ChunkedMLEM in 8M-event chunks, one iteration from rho^0.

Checked against the oracle at sampled pixels (every event whose box reaches a sampled pixel, in
16 worker processes) to relative 1e-5, and by count conservation over the whole image (1e-6).
"""

import time

import numpy as np
import pytest

import oracle
from jpet_synth import get_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1502_07478_amd import jpet  # noqa: E402


def _oracle_backprojection_chunk(args):
    import oracle as orc
    kw, ev_chunk, rho, pix = args
    return orc.backprojection_at(orc.geometry(**kw), ev_chunk, rho, pix)


def test_large1024_chunked_sampled_parity():
    import multiprocessing as mp
    w = get_workload("large1024")
    t0 = time.perf_counter()
    ev_np = w.events(workers=16)
    print(f"large1024: {len(ev_np)} events generated in {time.perf_counter() - t0:.1f}s", flush=True)
    kw = w.geometry()
    g, go = jpet.geometry(**kw), oracle.geometry(**kw)
    s = jpet.sensitivity(g)
    chunk = 8_000_000
    chunks = [torch.from_numpy(ev_np[a:a + chunk]) for a in range(0, len(ev_np), chunk)]
    runner = jpet.ChunkedMLEM(g, chunks, s=s, resident=True)
    rho = (s > 0).to(torch.float32)
    st = runner.iterate(rho, 1, want_stats=True)
    torch.cuda.synchronize()
    print(f"large1024: GPU iteration done, {st}", flush=True)
    assert st["n_unplaced_rows"] == 0
    total = float((s.double() * rho.double()).sum())
    assert total == pytest.approx(st["n_valid"] - st["n_zero_denominator"], rel=1e-6)
    so = oracle.sensitivity(go)
    r0 = oracle.initial_image(so).ravel()
    n = w.n_y
    pix = [512 * n + 512, 300 * n + 700, 700 * n + 300, 450 * n + 610, 620 * n + 420]
    nproc = 16
    jobs = [(kw, c, r0, pix) for c in np.array_split(ev_np, 64)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(nproc) as pool:
        acc = np.sum(pool.map(_oracle_backprojection_chunk, jobs), axis=0)
    got = rho.double().cpu().numpy().ravel()[pix] * so.ravel()[pix]
    print(f"large1024: oracle {time.perf_counter() - t0:.1f}s; GPU {got} oracle {acc}", flush=True)
    np.testing.assert_allclose(got, acc, rtol=1e-5)
