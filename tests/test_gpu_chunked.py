"""Event lists in chunks (jpet_mlem_backproject + jpet_mlem_update, ChunkedMLEM) against the oracle
over the whole list, and against one jpet_mlem_iterate call.

Tolerances: relative L2 1e-4 against the FP64 oracle; 1e-6 against the unchunked GPU path (the
chunks change only which events share a workgroup batch, hence the rounding order of D in FP32).
"""

import numpy as np
import pytest

import oracle
from jpet_synth import get_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1502_07478_amd import jpet  # noqa: E402

DEV = "cuda"


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def case():
    w = get_workload("tiny")
    ev_np = w.events()
    kw = w.geometry()
    return w, ev_np, jpet.geometry(**kw), oracle.geometry(**kw)


@pytest.mark.parametrize("resident", [True, False])
def test_chunked_matches_oracle_and_single_call(case, resident):
    w, ev_np, g, go = case
    so = oracle.sensitivity(go)
    s = jpet.sensitivity(g)
    n_iter = 3
    # ragged chunks, one of them empty
    cuts = [0, 7001, 7001, 13000, len(ev_np)]
    chunks = [torch.from_numpy(ev_np[a:b].copy()) for a, b in zip(cuts[:-1], cuts[1:])]
    if not resident:
        chunks = [c.pin_memory() for c in chunks]
    runner = jpet.ChunkedMLEM(g, chunks, s=s, resident=resident)
    rho = (s > 0).to(torch.float32)
    st = runner.iterate(rho, n_iter, want_stats=True)
    torch.cuda.synchronize()
    rho_o, sto = oracle.mlem(go, ev_np, oracle.initial_image(so), n_iter, s=so)
    assert rel_l2(rho.cpu().numpy(), rho_o) <= 1e-4
    assert st["n_valid"] == sto["n_valid"]
    assert st["n_pairs"] == sto["n_pairs"]
    ev = torch.from_numpy(ev_np).to(DEV)
    rho1 = (s > 0).to(torch.float32)
    jpet.mlem_iterate(g, ev, rho1, n_iter, s=s)
    assert rel_l2(rho.cpu().numpy(), rho1.cpu().numpy()) <= 1e-6


def test_backproject_accumulates_across_calls(case):
    """Two half lists back-projected into one accumulator equal the whole list's accumulator, and
    the update clears it."""
    w, ev_np, g, go = case
    s = jpet.sensitivity(g)
    rho = (s > 0).to(torch.float32)
    ev = torch.from_numpy(ev_np).to(DEV)
    half = len(ev_np) // 2
    acc = jpet.accumulator(g)
    a = jpet.backproject(g, ev[:half].contiguous(), rho, acc, want_stats=True)
    b = jpet.backproject(g, ev[half:].contiguous(), rho, acc, want_stats=True)
    whole = jpet.accumulator(g)
    c = jpet.backproject(g, ev, rho, whole, want_stats=True)
    assert a["n_pairs"] + b["n_pairs"] == c["n_pairs"]
    assert a["n_valid"] + b["n_valid"] == c["n_valid"]
    # each event adds round(2^32 rho P / D) per pixel: sums agree to the per-event rounding
    sa = acc.double() / 2.0**32
    sc = whole.double() / 2.0**32
    assert rel_l2(sa.cpu().numpy(), sc.cpu().numpy()) <= 1e-6
    # total over the image = number of events with D > 0, to the fixed-point rounding
    assert float(sc.sum()) == pytest.approx(c["n_valid"] - c["n_zero_denominator"], rel=1e-7)
    out = torch.empty_like(rho)
    jpet.update(g, acc, out, s)
    assert int(acc.abs().sum()) == 0
    so = oracle.sensitivity(go)
    ref = oracle.mlem(go, ev_np, oracle.initial_image(so), 1, s=so)[0]
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-4
