"""Parity of the HIP path (through the C-ABI) with the double-precision oracle.

Tolerances (FP32 GPU against FP64 oracle):
  sensitivity: max relative error 1e-6 (evaluated in double precision, rounded to float)
  one MLEM step from the same input image: relative L2 1e-4
  pair / valid / dropped counts: exact
  log-likelihood: relative 1e-6; grad rho: relative L2 1e-4; grad sigma: relative 1e-3
"""

import math

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


def geoms(w, **over):
    kw = w.geometry(**over)
    return jpet.geometry(**kw), oracle.geometry(**kw)


@pytest.fixture(scope="module")
def tiny():
    w = get_workload("tiny")
    ev = w.events()
    return w, ev, torch.from_numpy(ev).to(DEV)


def test_sensitivity_matches_oracle(tiny):
    w, _, _ = tiny
    for over in ({}, dict(n_y=400, n_z=400, pixel=2.0), dict(L=1000.0, n_y=256, n_z=300, pixel=1.7)):
        g, go = geoms(w, **over)
        got = jpet.sensitivity(g).double().cpu().numpy()
        want = oracle.sensitivity(go)
        assert np.array_equal(got == 0, want == 0)
        pos = want > 0
        assert np.max(np.abs(got[pos] / want[pos] - 1)) <= 1e-6


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("with_s", [True, False])
def test_tiny_each_step_from_the_oracle_iterate(tiny, variant, with_s):
    """Every one of 5 iterations, started from the oracle's own iterate, within 1e-4 rel L2."""
    w, ev_np, ev = tiny
    g, go = geoms(w, kernel_variant=variant)
    so = oracle.sensitivity(go)
    s = jpet.sensitivity(g)
    rho_o = oracle.initial_image(so) if with_s else so * oracle.initial_image(so)
    for it in range(w.n_iter):
        nxt, sto = oracle.mlem(go, ev_np, rho_o, 1, s=so if with_s else None)
        rho = torch.from_numpy(rho_o.astype(np.float32)).to(DEV)
        st = jpet.mlem_iterate(g, ev, rho, 1, s=s if with_s else None, want_stats=True)
        got = rho.double().cpu().numpy()
        assert rel_l2(got, nxt) <= 1e-4, (it, rel_l2(got, nxt))
        for key in ("n_valid", "n_dropped", "n_pairs", "n_zero_denominator", "n_kappa_nonpositive"):
            assert st[key] == sto[key], (key, st[key], sto[key])
        assert st["n_unplaced_rows"] == 0
        rho_o = nxt


def test_tiny_trajectory(tiny):
    """Five GPU iterations in one call against five oracle iterations (drift stays small)."""
    w, ev_np, ev = tiny
    g, go = geoms(w)
    so = oracle.sensitivity(go)
    s = jpet.sensitivity(g)
    rho = (s > 0).to(torch.float32)
    jpet.mlem_iterate(g, ev, rho, w.n_iter, s=s)
    want, _ = oracle.mlem(go, ev_np, oracle.initial_image(so), w.n_iter, s=so)
    assert rel_l2(rho.cpu().numpy(), want) <= w.n_iter * 1e-4


def test_prepared_workspace_reuse_gives_same_result(tiny):
    w, _, ev = tiny
    g, _ = geoms(w)
    s = jpet.sensitivity(g)
    ws = jpet.workspace(g, ev.shape[0])
    jpet.prepare(g, ev, ws)
    a = (s > 0).to(torch.float32)
    b = a.clone()
    jpet.mlem_iterate(g, ev, a, 2, s=s, ws=ws, prepared=True)
    jpet.mlem_iterate(g, ev, b, 2, s=s)
    torch.cuda.synchronize()
    assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("name", ["tiny", "prod400"])
def test_direct_image_is_bit_exact(name, tiny, prod):
    """Integer counts per pixel: identical to the oracle's."""
    w, ev_np, ev = tiny if name == "tiny" else prod
    g, go = geoms(w)
    got = jpet.direct_image(g, ev).cpu().numpy()
    want, counted = oracle.direct_image(go, ev_np)
    np.testing.assert_array_equal(got.astype(np.float64), want)
    assert int(got.sum()) == counted


def test_paper_setting_matches_oracle():
    """The paper's own setting (R=130 mm, L=300 mm, 4 mm pixels, sigma=(10, 40), Appendix A
    phantom): the first 30k events, two iterations from rho^0."""
    w = get_workload("paper130")
    g, go = geoms(w)
    ev_np = w.events(30_000)
    so = oracle.sensitivity(go)
    got, want, st, sto = run_both(g, go, ev_np, oracle.initial_image(so), n_iter=2)
    assert st["n_pairs"] == sto["n_pairs"] and st["n_valid"] == sto["n_valid"]
    assert rel_l2(got, want) <= 1e-4


@pytest.mark.parametrize("split", ["wave", "thread"])
def test_comparison_work_splits_match_oracle(tiny, split):
    """The event pass run one wavefront or one thread per event (the paper's GPU granularities,
    kept for comparison) gives the oracle's iterates, on the small grid and the paper's setting."""
    w, ev_np, ev = tiny
    for wl, n in ((w, len(ev_np)), (get_workload("paper130"), 20_000)):
        g, go = geoms(wl)
        e_np = ev_np if wl is w else wl.events(n)
        so = oracle.sensitivity(go)
        rho0 = oracle.initial_image(so)
        s = jpet.sensitivity(g)
        rho = torch.from_numpy(rho0.astype(np.float32)).to(DEV)
        st = jpet.mlem_iterate(g, torch.from_numpy(e_np).to(DEV), rho, 2, s=s, want_stats=True, split=split)
        want, sto = oracle.mlem(go, e_np, rho0, 2, s=so)
        assert st["n_pairs"] == sto["n_pairs"] and st["n_valid"] == sto["n_valid"]
        assert rel_l2(rho.cpu().numpy(), want) <= 1e-4, wl.name


def test_count_conservation_gpu(tiny):
    w, _, ev = tiny
    g, _ = geoms(w)
    s = jpet.sensitivity(g)
    rho = (s > 0).to(torch.float32)
    for _ in range(3):
        st = jpet.mlem_iterate(g, ev, rho, 1, s=s, want_stats=True)
        total = float((s.double() * rho.double()).sum())
        assert total == pytest.approx(st["n_valid"] - st["n_zero_denominator"], rel=1e-5)


# ---------------------------------------------------------------------------------------------
# edge cases


def run_both(g, go, ev_np, rho0, n_iter=1, with_s=True):
    so = oracle.sensitivity(go)
    s = jpet.sensitivity(g)
    ev = torch.from_numpy(np.ascontiguousarray(ev_np, dtype=np.float32).reshape(-1, 3)).to(DEV)
    rho = torch.from_numpy(np.asarray(rho0, dtype=np.float32)).to(DEV).contiguous()
    st = jpet.mlem_iterate(g, ev, rho, n_iter, s=s if with_s else None, want_stats=True)
    assert st["n_unplaced_rows"] == 0
    want, sto = oracle.mlem(go, ev_np, rho0, n_iter, s=so if with_s else None)
    return rho.double().cpu().numpy(), want, st, sto


def test_no_events(tiny):
    w, _, _ = tiny
    g, go = geoms(w)
    got, want, st, sto = run_both(g, go, np.zeros((0, 3), np.float32), np.ones((64, 64)))
    assert np.all(got == 0) and np.all(want == 0)
    assert st["n_events"] == 0 and st["n_valid"] == 0


def test_all_events_invalid(tiny):
    w, _, _ = tiny
    g, go = geoms(w)
    ev = np.array([[300.0, 0.0, 0.0], [np.nan, 1.0, 2.0], [0.0, 0.0, 5000.0], [np.inf, 0, 0]], np.float32)
    got, want, st, sto = run_both(g, go, ev, np.ones((64, 64)))
    assert st["n_dropped"] == 4 == sto["n_dropped"]
    assert np.all(got == 0)


def test_single_event_and_ragged_grid(tiny):
    w, ev_np, _ = tiny
    # non-square grid whose column count is not a multiple of anything convenient
    g, go = geoms(w, n_y=37, n_z=53, pixel=3.3)
    for k in (1, 7, 129, 1000):
        got, want, st, sto = run_both(g, go, ev_np[:k], np.ones((37, 53)))
        assert st["n_pairs"] == sto["n_pairs"] and st["n_valid"] == sto["n_valid"]
        if sto["n_valid"]:
            assert rel_l2(got, want) <= 1e-4


def test_hot_spot_of_identical_events(tiny):
    """60k copies of three events among 5k ordinary ones: one bin holds most of the list (many
    workgroup items on the same region, all adding to the same pixels)."""
    w, ev_np, _ = tiny
    g, go = geoms(w)
    hot = np.repeat(ev_np[:3], 20_000, axis=0)
    ev = np.concatenate([hot, ev_np[3:5003]])
    rng = np.random.default_rng(3)
    ev = np.ascontiguousarray(ev[rng.permutation(len(ev))])
    so = oracle.sensitivity(go)
    got, want, st, sto = run_both(g, go, ev, oracle.initial_image(so), n_iter=2)
    assert st["n_pairs"] == sto["n_pairs"] and st["n_valid"] == sto["n_valid"]
    assert rel_l2(got, want) <= 1e-4


def test_large_grid_with_many_bins():
    """A 2048x2048 grid of 0.2 mm (4M pixels, thousands of bins) with sigma = (1.5, 9) mm: 20k
    events, two iterations from rho^0."""
    from jpet_synth import Workload
    w = Workload("grid2048", 450.0, 500.0, 1.5, 9.0, 0.2, 2048, 2048, 20_000, 2, 13, "c1")
    g, go = geoms(w)
    info = jpet.launch_info(g, w.n_events)
    assert info["binned"] == 1 and info["bins"] > 1000
    ev_np = w.events()
    so = oracle.sensitivity(go)
    got, want, st, sto = run_both(g, go, ev_np, oracle.initial_image(so), n_iter=2)
    assert st["n_pairs"] == sto["n_pairs"] and st["n_valid"] == sto["n_valid"]
    assert rel_l2(got, want) <= 1e-4


@pytest.mark.parametrize("seed", range(8))
def test_random_geometries(seed):
    """Random detector, resolution, grid (some binned, some generic), kernel variant, gamma and
    position-dependent sigma_z; valid events plus non-finite, off-strip, strip-end and off-grid ones.
    Counts exact, images finite and within 1e-4 of the oracle over two iterations."""
    from jpet_synth import Workload
    rng = np.random.default_rng(4100 + seed)
    R = float(rng.uniform(120, 500))
    L = float(rng.uniform(200, 1000))
    sz, sdl = float(rng.uniform(3, 15)), float(rng.uniform(20, 90))
    n_y, n_z = int(rng.integers(16, 160)), int(rng.integers(16, 200))
    pixel = float(rng.uniform(0.05, 0.95)) * 2.0 * R / n_y
    pixel = max(pixel, sz / 30.0) if 0.5 * n_y * max(pixel, sz / 30.0) < R else pixel
    edge = float(rng.choice([0.0, 0.2]))
    szm = sz * (1 + edge)
    gamma = float(rng.choice([0.0, 0.5, -0.6])) * math.sqrt(1 / szm ** 2 / sdl ** 2 / 2)
    variant = int(rng.integers(0, 2))
    pairs_est = math.pi * (1.5 * sdl / pixel) * (2.2 * szm / pixel)
    n = int(max(50, min(2000, 2e7 / max(pairs_est, 1.0))))
    w = Workload(f"fuzz{seed}", R, L, sz, sdl, pixel, n_y, n_z, n, 2, 5000 + seed, "random", sigma_z_edge=edge)
    ev = w.events()
    odd = np.array([[np.nan, 0, 0], [0, np.inf, 0], [0.5 * L + 1, 0, 0], [0, -0.5 * L - 1, 0],
                    [0.5 * L, -0.5 * L, 0], [0.5 * L, 0.5 * L, 10.0], [0, 0, 50 * R], [-0.5 * L, 0.25 * L, -30.0]],
                   np.float32)
    ev = np.ascontiguousarray(np.concatenate([ev, odd]))
    g, go = geoms(w, kernel_variant=variant, gamma=gamma)
    so = oracle.sensitivity(go)
    got, want, st, sto = run_both(g, go, ev, oracle.initial_image(so), n_iter=2)
    assert np.all(np.isfinite(got))
    for k in ("n_valid", "n_dropped", "n_pairs", "n_zero_denominator", "n_kappa_nonpositive"):
        assert st[k] == sto[k], (k, st[k], sto[k])
    if np.linalg.norm(want) > 0:
        assert rel_l2(got, want) <= 1e-4


def test_repeated_runs_agree(tiny):
    """Back-projection sums are integers, so only the order of the double-precision denominator
    sums can differ between runs."""
    w, ev_np, ev = tiny
    g, _ = geoms(w)
    s = jpet.sensitivity(g)
    imgs = []
    for _ in range(3):
        rho = (s > 0).to(torch.float32)
        jpet.mlem_iterate(g, ev, rho, 5, s=s)
        imgs.append(rho.cpu().numpy())
    for a in imgs[1:]:
        assert rel_l2(a, imgs[0]) <= 1e-6


def test_resume_from_a_saved_image(tiny):
    """MLEM keeps no state besides the image: 2 iterations, a round trip of the image through host
    memory, then 3 more equal 5 iterations at once."""
    w, ev_np, ev = tiny
    g, _ = geoms(w)
    s = jpet.sensitivity(g)
    ws = jpet.workspace(g, ev.shape[0])
    jpet.prepare(g, ev, ws)
    a = (s > 0).to(torch.float32)
    jpet.mlem_iterate(g, ev, a, 5, s=s, ws=ws, prepared=True)
    b = (s > 0).to(torch.float32)
    jpet.mlem_iterate(g, ev, b, 2, s=s, ws=ws, prepared=True)
    saved = b.cpu().numpy().copy()
    c = torch.from_numpy(saved).to(DEV)
    jpet.mlem_iterate(g, ev, c, 3, s=s, ws=ws, prepared=True)
    assert rel_l2(c.cpu().numpy(), a.cpu().numpy()) <= 1e-6


def test_zero_denominator_events_are_skipped(tiny):
    w, ev_np, _ = tiny
    g, go = geoms(w)
    rho0 = np.zeros((64, 64))
    rho0[40:48, 10:20] = 1.0
    got, want, st, sto = run_both(g, go, ev_np[:3000], rho0)
    assert st["n_zero_denominator"] == sto["n_zero_denominator"] > 0
    assert rel_l2(got, want) <= 1e-4


def test_events_at_grid_and_strip_edges(tiny):
    w, _, _ = tiny
    g, go = geoms(w)
    rng = np.random.default_rng(3)
    ev = np.stack([rng.uniform(-250, 250, 4000), rng.uniform(-250, 250, 4000), rng.uniform(-700, 700, 4000)], 1)
    ev[:500, 0] = 250.0
    ev[500:1000, 1] = -250.0
    got, want, st, sto = run_both(g, go, ev.astype(np.float32), np.ones((64, 64)))
    assert st["n_valid"] == sto["n_valid"] and st["n_pairs"] == sto["n_pairs"]
    assert rel_l2(got, want) <= 1e-4


def test_long_rows_and_many_rows():
    """sigma large against the pixel: more than 200 rows per event and a region that fits the LDS
    only with 32-bit accumulators."""
    from jpet_synth import Workload
    w = Workload("wide", 450.0, 500.0, 15.0, 90.0, 1.171875, 512, 512, 3000, 1, 7, "c1")
    g, go = geoms(w)
    info = jpet.launch_info(g, w.n_events)
    assert info["binned"] == 1 and info["accumulator_bits"] == 32
    ev_np = w.events()
    got, want, st, sto = run_both(g, go, ev_np, np.ones((512, 512)))
    assert st["n_pairs"] == sto["n_pairs"]
    assert st["n_unplaced_rows"] == 0
    assert rel_l2(got, want) <= 1e-4


@pytest.mark.parametrize("cache_bits", [1, 2])
def test_split_rows_match_oracle(cache_bits):
    """Plans that cut rows longer than a 16- or 32-pixel register cache into two segments, one
    thread each, give the oracle's image and counts: 2 mm pixels with sigma_z = 10 mm (rows up to 21
    pixels, split at 16) and 1 mm pixels (rows up to 43 pixels, split at 32), two steps."""
    from jpet_synth import Workload
    pix, n = (2.0, 96) if cache_bits == 1 else (1.0, 160)
    w = Workload("split", 450.0, 500.0, 10.0, 63.0, pix, n, n, 6000, 2, 91, "random")
    ev = w.events()
    g, go = geoms(w)
    code = next(c for c, _ in jpet.plan_candidates(g, len(ev)) if (c >> 12) & 3 == cache_bits)
    g = jpet.with_plan(g, code)
    info = jpet.launch_info(g, len(ev))
    assert info["row_segments"] == 2 and info["row_cache"] == (16 if cache_bits == 1 else 32)
    so = oracle.sensitivity(go)
    got, want, st, sto = run_both(g, go, ev, oracle.initial_image(so), n_iter=2)
    for k in ("n_valid", "n_pairs", "n_kappa_nonpositive", "n_zero_denominator"):
        assert st[k] == sto[k], (k, st[k], sto[k])
    r = rel_l2(got, want)
    print(f"split rows at {info['row_cache']}: plan {code}, rel L2 {r:.2e}", flush=True)
    assert r <= 2e-4


@pytest.mark.parametrize("edge", [0.0, 0.3])
def test_rows_longer_than_the_register_cache_use_the_generic_pass(edge):
    """Rows of more than 64 pixels (sigma_z = 12 mm on 0.5 mm pixels): the one-wavefront-per-event
    pass with global accumulation (also with sigma_z rising towards the strip ends)."""
    from jpet_synth import Workload
    w = Workload("fine", 450.0, 500.0, 12.0, 40.0, 0.5, 256, 256, 1500, 1, 11, "c1")
    g, go = geoms(w, sigma_z_edge=edge)
    assert jpet.launch_info(g, w.n_events)["binned"] == 0
    ev_np = w.events()
    got, want, st, sto = run_both(g, go, ev_np, np.ones((256, 256)))
    assert st["n_pairs"] == sto["n_pairs"]
    assert rel_l2(got, want) <= 1e-4


# ---------------------------------------------------------------------------------------------
# sigma_z depending on the hit positions (Sec. 3 after Eq. 12): one sigma_z per event


@pytest.mark.parametrize("edge", [0.1, 1.0])
def test_position_dependent_sigma_z_tiny(tiny, edge):
    """Two iterations from rho^0 on the small grid; events near the strip ends get ellipses up to
    (1 + edge) times wider."""
    w, ev_np, ev = tiny
    g, go = geoms(w, sigma_z_edge=edge)
    so = oracle.sensitivity(go)
    got, want, st, sto = run_both(g, go, ev_np, oracle.initial_image(so), n_iter=2)
    assert st["n_pairs"] == sto["n_pairs"] and st["n_valid"] == sto["n_valid"]
    assert rel_l2(got, want) <= 1e-4
    g0, go0 = geoms(w)
    assert st["n_pairs"] > oracle.mlem(go0, ev_np, oracle.initial_image(so), 1, s=so)[1]["n_pairs"]
    # the log-likelihood is defined for one sigma_z shared by all events
    with pytest.raises(jpet.JpetError):
        jpet.loglik_grad(g, ev, torch.from_numpy(want.astype(np.float32)).to(DEV), s=jpet.sensitivity(g))


def test_position_dependent_sigma_z_edge400_first_events():
    """The edge400 workload (400x400 px of 2 mm, sigma_z 10 mm rising 10% to the strip ends):
    the first 30k events, two iterations from rho^0."""
    w = get_workload("edge400")
    g, go = geoms(w)
    ev_np = w.events(30_000)
    so = oracle.sensitivity(go)
    got, want, st, sto = run_both(g, go, ev_np, oracle.initial_image(so), n_iter=2)
    assert st["n_pairs"] == sto["n_pairs"] and st["n_valid"] == sto["n_valid"]
    assert rel_l2(got, want) <= 1e-4


def test_position_dependent_sigma_z_in_a_batch(tiny):
    """An instance with a position-dependent sigma_z inside a batch equals its single call."""
    w, ev_np, ev = tiny
    inst, imgs, singles = [], [], []
    for edge in (0.0, 0.25):
        g = jpet.geometry(**w.geometry(sigma_z_edge=edge))
        s = jpet.sensitivity(g)
        rho = (s > 0).to(torch.float32)
        inst.append((g, ev, s, rho))
        imgs.append(rho)
        r1 = (s > 0).to(torch.float32)
        jpet.mlem_iterate(g, ev, r1, 2, s=s)
        singles.append(r1)
    jpet.BatchedMLEM(inst).iterate(2)
    for a, b in zip(imgs, singles):
        assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-6
    assert rel_l2(imgs[0].cpu().numpy(), imgs[1].cpu().numpy()) > 1e-3


# ---------------------------------------------------------------------------------------------
# production size (10M events, 400x400): sampled outputs and invariants


@pytest.fixture(scope="module")
def prod():
    w = get_workload("prod400")
    ev_np = w.events()
    return w, ev_np, torch.from_numpy(ev_np).to(DEV)


def _oracle_backprojection_chunk(args):
    """Worker (spawned process): the oracle's accumulator at the given pixels from one chunk of
    events.  Each event's denominator involves only that event, so chunks add up exactly."""
    import oracle as orc
    kw, ev_chunk, rho, pix = args
    return orc.backprojection_at(orc.geometry(**kw), ev_chunk, rho, pix)


def test_prod400_sampled_parity(prod):
    import multiprocessing as mp
    w, ev_np, ev = prod
    g, go = geoms(w)
    s = jpet.sensitivity(g)
    so = oracle.sensitivity(go)
    rho0 = (s > 0).to(torch.float32)
    ws = jpet.workspace(g, ev.shape[0])
    jpet.prepare(g, ev, ws)
    rho = rho0.clone()
    st = jpet.mlem_iterate(g, ev, rho, 1, s=s, ws=ws, prepared=True, want_stats=True)
    assert st["n_unplaced_rows"] == 0
    print(f"prod400: GPU iteration done, {st}", flush=True)
    # per-event denominators of 2000 sampled events against the oracle's
    rng = np.random.default_rng(0)
    sel = rng.choice(len(ev_np), 2000, replace=False)
    Do, cnt = oracle.denominators_at(go, ev_np, oracle.initial_image(so).ravel(), sel)
    ll = jpet.loglik_grad(g, ev, rho0, s=s, want_grad_rho=False, want_D=True)
    Dg = ll.D.double().cpu().numpy()[sel]
    ok = Do > 0
    np.testing.assert_allclose(Dg[ok], Do[ok], rtol=2e-5)
    print("prod400: sampled denominators agree", flush=True)
    # count conservation over the whole image
    total = float((s.double() * rho.double()).sum())
    assert total == pytest.approx(st["n_valid"] - st["n_zero_denominator"], rel=1e-6)
    # the new image at sampled pixels: every event touching them, in double precision
    pix = [240 * 400 + 230, 262 * 400 + 236, 180 * 400 + 260, 300 * 400 + 200, 120 * 400 + 160]
    nproc = 16
    r0 = oracle.initial_image(so).ravel()
    jobs = [(w.geometry(), c, r0, pix) for c in np.array_split(ev_np, nproc)]
    with mp.get_context("spawn").Pool(nproc) as pool:
        acc = np.sum(pool.map(_oracle_backprojection_chunk, jobs), axis=0)
    got = rho.double().cpu().numpy().ravel()[pix] * so.ravel()[pix]
    print(f"prod400: sampled pixels GPU {got} oracle {acc}", flush=True)
    np.testing.assert_allclose(got, acc, rtol=1e-5)


def test_edge400_full_size_sampled_parity():
    """All 10M events of edge400, one iteration: count conservation over the image and the new
    image at sampled pixels against the oracle (every event whose box reaches them)."""
    import multiprocessing as mp
    w = get_workload("edge400")
    ev_np = w.events()
    ev = torch.from_numpy(ev_np).to(DEV)
    g, go = geoms(w)
    s = jpet.sensitivity(g)
    so = oracle.sensitivity(go)
    rho = (s > 0).to(torch.float32)
    st = jpet.mlem_iterate(g, ev, rho, 1, s=s, want_stats=True)
    assert st["n_unplaced_rows"] == 0
    print(f"edge400: GPU iteration done, {st}", flush=True)
    total = float((s.double() * rho.double()).sum())
    assert total == pytest.approx(st["n_valid"] - st["n_zero_denominator"], rel=1e-6)
    # the centre and pixels near the phantom's edges
    pix = [200 * 400 + 200, 230 * 400 + 140, 170 * 400 + 260, 260 * 400 + 250, 140 * 400 + 150]
    nproc = 16
    r0 = oracle.initial_image(so).ravel()
    jobs = [(w.geometry(), c, r0, pix) for c in np.array_split(ev_np, nproc)]
    with mp.get_context("spawn").Pool(nproc) as pool:
        acc = np.sum(pool.map(_oracle_backprojection_chunk, jobs), axis=0)
    got = rho.double().cpu().numpy().ravel()[pix] * so.ravel()[pix]
    print(f"edge400: sampled pixels GPU {got} oracle {acc}", flush=True)
    np.testing.assert_allclose(got, acc, rtol=1e-5)


# ---------------------------------------------------------------------------------------------
# log-likelihood and gradient


@pytest.mark.parametrize("variant", [0, 1])
def test_loglik_and_gradients_match_oracle(tiny, variant):
    w, ev_np, ev = tiny
    g, go = geoms(w, kernel_variant=variant)
    so = oracle.sensitivity(go)
    rho_o, _ = oracle.mlem(go, ev_np, oracle.initial_image(so), 2, s=so)
    rho = torch.from_numpy(rho_o.astype(np.float32)).to(DEV)
    s = jpet.sensitivity(g)
    res = jpet.loglik_grad(g, ev, rho, s=s, want_D=True, want_stats=True)
    l, dz, dd, gr, sto, D = oracle.loglik_grad(go, ev_np, rho.double().cpu().numpy(), s=so, return_D=True)
    v = res.value.cpu().numpy()
    assert v[0] == pytest.approx(l, rel=1e-6)
    assert v[1] == pytest.approx(dz, rel=1e-3)
    assert v[2] == pytest.approx(dd, rel=1e-3)
    assert rel_l2(res.grad_rho.cpu().numpy(), gr) <= 1e-4
    np.testing.assert_allclose(res.D.double().cpu().numpy(), D, rtol=2e-5, atol=1e-30)
    assert res.stats["n_pairs"] == sto["n_pairs"]


@pytest.mark.parametrize("seed", range(4))
def test_loglik_random_geometries(seed):
    """The log-likelihood and its gradients on random geometries (binned and generic passes, both
    kernel variants, gamma, a mask at other sigmas) against the oracle, at a textured image."""
    from jpet_synth import Workload
    rng = np.random.default_rng(4200 + seed)
    R = float(rng.uniform(150, 500))
    L = float(rng.uniform(250, 900))
    sz, sdl = float(rng.uniform(4, 14)), float(rng.uniform(25, 85))
    n_y, n_z = int(rng.integers(24, 120)), int(rng.integers(24, 160))
    pixel = min(float(rng.uniform(0.5, 6.0)), 1.9 * R / n_y)
    gamma = float(rng.choice([0.0, 0.4, -0.5])) * math.sqrt(1 / sz ** 2 / sdl ** 2 / 2)
    variant = int(rng.integers(0, 2))
    pairs_est = math.pi * (1.5 * sdl / pixel) * (2.2 * sz / pixel)
    n = int(max(50, min(1500, 1e7 / max(pairs_est, 1.0))))
    w = Workload(f"llfuzz{seed}", R, L, sz, sdl, pixel, n_y, n_z, n, 1, 6000 + seed, "random")
    ev_np = w.events()
    mask = (sz * float(rng.uniform(0.9, 1.1)), sdl * float(rng.uniform(0.9, 1.1))) if seed % 2 else None
    g, go = geoms(w, kernel_variant=variant, gamma=gamma)
    so = oracle.sensitivity(go)
    r_np = ((so > 0) * (0.5 + np.random.default_rng(seed).random(so.shape))).astype(np.float32)
    rho = torch.from_numpy(r_np).to(DEV)
    res = jpet.loglik_grad(g, torch.from_numpy(ev_np).to(DEV), rho, s=jpet.sensitivity(g), sigma_mask=mask,
                           want_stats=True)
    l, dz, dd, gr, sto = oracle.loglik_grad(go, ev_np, r_np.astype(np.float64), s=so, sigma_mask=mask)
    assert res.stats["n_pairs"] == sto["n_pairs"] and res.stats["n_valid"] == sto["n_valid"]
    v = res.value.cpu().numpy()
    if sto["n_zero_denominator"] == 0 and sto["n_valid"] > 0:
        assert v[0] == pytest.approx(l, rel=1e-6)
        assert v[1] == pytest.approx(dz, rel=1e-3, abs=1e-6 * abs(l))
        assert v[2] == pytest.approx(dd, rel=1e-3, abs=1e-6 * abs(l))
        assert rel_l2(res.grad_rho.cpu().numpy(), gr) <= 1e-4


def test_loglik_sigma_gradient_matches_gpu_finite_differences(tiny):
    w, ev_np, ev = tiny
    g, go = geoms(w)
    so = oracle.sensitivity(go)
    rho_o, _ = oracle.mlem(go, ev_np, oracle.initial_image(so), 2, s=so)
    rho = torch.from_numpy(rho_o.astype(np.float32)).to(DEV)
    s = jpet.sensitivity(g)
    base = jpet.loglik_grad(g, ev, rho, s=s, want_grad_rho=False).value.cpu().numpy()
    mask = (w.sigma_z, w.sigma_dl)

    def ll(sz, sd):
        gg = jpet.geometry(**w.geometry(sigma_z=sz, sigma_dl=sd))
        return jpet.loglik_grad(gg, ev, rho, s=s, sigma_mask=mask, want_grad_rho=False).value.cpu().numpy()[0]

    hz, hd = 1e-3 * w.sigma_z, 1e-3 * w.sigma_dl
    fd_z = (ll(w.sigma_z + hz, w.sigma_dl) - ll(w.sigma_z - hz, w.sigma_dl)) / (2 * hz)
    fd_d = (ll(w.sigma_z, w.sigma_dl + hd) - ll(w.sigma_z, w.sigma_dl - hd)) / (2 * hd)
    assert base[1] == pytest.approx(fd_z, rel=1e-3)
    assert base[2] == pytest.approx(fd_d, rel=1e-3)


@pytest.mark.parametrize("gfrac", [0.5, -0.8])
def test_offdiagonal_cinv_mlem_and_loglik(tiny, gfrac):
    """gamma != 0 (Eq. 12): one MLEM step and the log-likelihood with gradients against the oracle."""
    w, ev_np, ev = tiny
    gam = gfrac * math.sqrt(1 / w.sigma_z ** 2 / w.sigma_dl ** 2 / 2)
    g, go = geoms(w, gamma=gam)
    so = oracle.sensitivity(go)
    rho_o, _ = oracle.mlem(go, ev_np, oracle.initial_image(so), 2, s=so)
    s = jpet.sensitivity(g)
    rho = torch.from_numpy(rho_o.astype(np.float32)).to(DEV)
    want, _ = oracle.mlem(go, ev_np, rho.double().cpu().numpy(), 1, s=so)
    jpet.mlem_iterate(g, ev, rho, 1, s=s)
    assert rel_l2(rho.cpu().numpy(), want) <= 1e-4
    r2 = torch.from_numpy(rho_o.astype(np.float32)).to(DEV)
    res = jpet.loglik_grad(g, ev, r2, s=s)
    l, dz, dd, gr, _ = oracle.loglik_grad(go, ev_np, r2.double().cpu().numpy(), s=so)
    v = res.value.cpu().numpy()
    assert v[0] == pytest.approx(l, rel=1e-6)
    assert v[1] == pytest.approx(dz, rel=1e-3)
    assert v[2] == pytest.approx(dd, rel=1e-3)
    assert rel_l2(res.grad_rho.cpu().numpy(), gr) <= 1e-4


def test_loglik_zero_denominator_is_minus_infinity(tiny):
    w, ev_np, ev = tiny
    g, _ = geoms(w)
    rho = torch.zeros(g.shape, device=DEV)
    res = jpet.loglik_grad(g, ev, rho, want_grad_rho=False, want_stats=True)
    assert res.value[0].item() == -math.inf
    assert res.stats["n_zero_denominator"] == res.stats["n_valid"]


# ---------------------------------------------------------------------------------------------
# reading R8: pairs with kappa <= 0 get P := 0 and are counted


def _kappa_events(w, pixel, n_y, n_z):
    """Events of a geometry where kappa changes sign inside ellipses, without the two cases where
    FP32 against FP64 is not a meaningful comparison: a pixel whose kappa lies within 1e-4 of
    zero (relative to the event's largest), where the two precisions may take the sign decision
    differently, and kernel values that spike near kappa = 0+ (more than 30 times the event's
    median: the Laplace form diverges there).  Events whose every pixel has kappa <= 0 stay."""
    import sys
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from laplace import laplace_terms, pixel_centres
    go = oracle.geometry(**w.geometry())
    keep = []
    for e in w.events():
        p_idx, P = oracle.event_pixels(go, e)
        if len(P) == 0 or not np.all(np.isfinite(P)):
            continue
        y, z = pixel_centres(p_idx, n_y, n_z, pixel)
        kappa = -2.0 * laplace_terms(w.R, e, y, z, w.sigma_z, w.sigma_dl)[2]
        if np.any(np.abs(kappa) < 1e-4 * np.abs(kappa).max()):
            continue
        pos = P[P > 0]
        if len(pos) and pos.max() > 30 * np.median(pos):
            continue
        keep.append(e)
    return np.ascontiguousarray(np.array(keep, dtype=np.float32))


@pytest.mark.parametrize("pixel,n_y,n_z,binned", [(3.0, 50, 100, 1), (2.0, 70, 120, 0)])
def test_kappa_nonpositive_pairs_are_zero_and_counted(pixel, n_y, n_z, binned):
    """Strips 80 mm from the axis, sigma_z = 40 mm against sigma_dl = 6 mm: kappa <= 0 over part of
    many ellipses and over the whole of some (those events have D = 0).  The binned pass (3 mm
    pixels) and the generic pass (2 mm: rows too long for the register cache) both count exactly
    the oracle's pairs with kappa <= 0 and zero-denominator events; two steps within 1e-4."""
    from jpet_synth import Workload
    w = Workload("kappa", 80.0, 300.0, 40.0, 6.0, pixel, n_y, n_z, 4000, 2, 77, "random")
    ev = _kappa_events(w, pixel, n_y, n_z)
    g, go = geoms(w)
    assert jpet.launch_info(g, len(ev))["binned"] == binned
    so = oracle.sensitivity(go)
    got, want, st, sto = run_both(g, go, ev, oracle.initial_image(so), n_iter=2)
    print(f"kappa pixel {pixel}: {len(ev)} events, GPU {st}, oracle {sto}", flush=True)
    assert sto["n_kappa_nonpositive"] > 0 and sto["n_zero_denominator"] > 0
    for k in ("n_valid", "n_pairs", "n_kappa_nonpositive", "n_zero_denominator"):
        assert st[k] == sto[k], (k, st[k], sto[k])
    assert rel_l2(got, want) <= 1e-4


def test_loglik_out_of_domain_mask_with_a_caller_workspace_raises(tiny):
    """A sigma mask out of domain is an error even with a caller-supplied workspace (nothing is
    written; only a zero denominator after the pass reads as l = -inf)."""
    w, ev_np, ev = tiny
    g, _ = geoms(w)
    s = jpet.sensitivity(g)
    rho = (s > 0).to(torch.float32)
    ws = jpet.loglik_workspace(g, ev.shape[0])
    with pytest.raises(jpet.JpetError):
        jpet.loglik_grad(g, ev, rho, s=s, ws=ws, sigma_mask=(0.0, 63.0))
    with pytest.raises(jpet.JpetError):
        jpet.loglik_grad(g, ev, rho, s=s, ws=ws, sigma_mask=(0.0, 63.0), want_stats=True)


def test_loglik_value_only_matches_oracle_and_full_call(tiny):
    """JPET_LOGLIK_VALUE_ONLY: the log-likelihood from one forward pass equals the oracle's and the
    full call's; its sigma entries are NaN, its denominators the oracle's."""
    w, ev_np, ev = tiny
    g, go = geoms(w)
    so = oracle.sensitivity(go)
    rho_o, _ = oracle.mlem(go, ev_np, oracle.initial_image(so), 2, s=so)
    rho = torch.from_numpy(rho_o.astype(np.float32)).to(DEV)
    s = jpet.sensitivity(g)
    v = jpet.loglik_grad(g, ev, rho, s=s, want_D=True, value_only=True, want_stats=True)
    full = jpet.loglik_grad(g, ev, rho, s=s, want_grad_rho=False)
    l, dz, dd, gr, sto, D = oracle.loglik_grad(go, ev_np, rho.double().cpu().numpy(), s=so, return_D=True)
    vv = v.value.cpu().numpy()
    assert vv[0] == pytest.approx(l, rel=1e-6)
    assert vv[0] == pytest.approx(float(full.value[0]), rel=1e-6)
    assert np.isnan(vv[1]) and np.isnan(vv[2]) and v.grad_rho is None
    np.testing.assert_allclose(v.D.double().cpu().numpy(), D, rtol=2e-5, atol=1e-30)
    assert v.stats["n_pairs"] == sto["n_pairs"]
    # autograd with nothing to differentiate takes the same path
    lv = jpet.loglik(rho, w.sigma_z, w.sigma_dl, ev, g, s)
    assert float(lv) == pytest.approx(l, rel=1e-6)
