"""jpet_mlem_iterate_noalloc (the library's per-GPU scratch array as the workspace) against
jpet_mlem_iterate with a caller workspace, through the C-ABI: two calls in a row, the second on a
smaller event list from a different image, each within the parity bar of one MLEM step (relative
L2 <= 1e-4 per iteration; the two runs use the same plan and kernels, so they agree far closer)
with identical counts.  Also the size limit and the argument checks, which return before any
device work."""

import ctypes

import numpy as np
import pytest

from jpet_synth import get_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1502_07478_amd import jpet  # noqa: E402

DEV = "cuda"


def rel_l2(a, b):
    a = a.double().cpu().numpy().ravel()
    b = b.double().cpu().numpy().ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _run_both(g, ev, rho0, s, n_iter):
    r_ref = rho0.clone()
    st_ref = jpet.mlem_iterate(g, ev, r_ref, n_iter, s=s, want_stats=True)
    r_na = rho0.clone()
    st_na = jpet.mlem_iterate_noalloc(g, ev, r_na, n_iter, s=s, want_stats=True)
    torch.cuda.synchronize()
    return r_ref, st_ref, r_na, st_na


def test_noalloc_matches_workspace_entry_point_on_two_calls():
    w = get_workload("tiny")
    g = jpet.geometry(**w.geometry())
    ev_all = torch.from_numpy(w.events()).to(DEV)
    s = jpet.sensitivity(g)
    rho0 = (s > 0).to(torch.float32)
    cases = [(ev_all, rho0, 3, s), (ev_all[:5000].contiguous(), None, 2, None)]
    for k, (ev, r0, n_iter, sk) in enumerate(cases):
        if r0 is None:  # the second call starts from an image the first one did not see
            r0 = rho0.clone()
            jpet.mlem_iterate(g, ev_all, r0, 1, s=s)
        print(f"noalloc call {k}: {ev.shape[0]} events, {n_iter} iterations, s {'set' if sk is not None else 'NULL'}",
              flush=True)
        r_ref, st_ref, r_na, st_na = _run_both(g, ev, r0, sk, n_iter)
        for key in ("n_valid", "n_dropped", "n_pairs", "n_zero_denominator", "n_kappa_nonpositive"):
            assert st_na[key] == st_ref[key], (k, key, st_na[key], st_ref[key])
        assert st_na["n_unplaced_rows"] == 0
        r = rel_l2(r_na, r_ref)
        print(f"noalloc call {k}: rel L2 against jpet_mlem_iterate {r:.3e}", flush=True)
        assert r <= n_iter * 1e-4


def test_noalloc_rejects_oversized_and_flagged_calls():
    w = get_workload("prod400")
    g = jpet.geometry(**w.geometry())
    lib = jpet.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks return first
    b = ctypes.c_size_t(0)
    n_big = 1_000_000
    assert lib.jpet_mlem_workspace_size(ctypes.byref(g), n_big, ctypes.byref(b)) == 0
    assert b.value > jpet.NOALLOC_SCRATCH_BYTES
    assert lib.jpet_mlem_iterate_noalloc(ctypes.byref(g), fake, n_big, None, fake, 1, 0, None,
                                         None) == jpet.JPET_EWORKSPACE
    assert lib.jpet_mlem_iterate_noalloc(ctypes.byref(g), fake, 10, None, fake, 1, jpet.JPET_WS_PREPARED, None,
                                         None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_iterate_noalloc(ctypes.byref(g), fake, 10, None, None, 1, 0, None, None) == jpet.JPET_EINVAL
