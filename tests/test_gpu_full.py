"""Full-image parity of the configurations the benchmark times, against the double-precision
oracle run over all events (split into chunks across worker processes: one MLEM step is a sum
over events, so the chunks' back-projections add up exactly, Sec. 4 listing).

Bounds, FP32 GPU against the FP64 oracle, for one step from the same input image (Eq. 3):
  relative L2 over the image                    <= 1e-4
  every pixel                                   |d rho| <= 1e-4 max(rho)
  pixels with rho >= 1e-3 max(rho)              |d rho| / rho <= 1e-3
  per-event denominators D_j (all events)       relative <= 1e-4
n-step trajectories: n times the per-step image bounds.  Counts (valid events, pairs) are exact.
"""

import multiprocessing as mp

import numpy as np
import pytest

import oracle
from jpet_synth import get_workload
from jpet_synth.configs import batch_instances

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1502_07478_amd import jpet  # noqa: E402

DEV = "cuda"
PROCS = 16


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def pixel_errors(got, want):
    """(max |d| / max(want), max relative error where want >= 1e-3 max(want))."""
    got = np.asarray(got, dtype=np.float64).ravel()
    want = np.asarray(want, dtype=np.float64).ravel()
    m = float(want.max())
    d = np.abs(got - want)
    big = want >= 1e-3 * m
    return float(d.max() / m), float((d[big] / want[big]).max())


def check_image(got, want, steps=1, label=""):
    r = rel_l2(got, want)
    pa, pr = pixel_errors(got, want)
    print(f"{label}: rel L2 {r:.3e}, max |d|/max {pa:.3e}, max rel (rho >= 1e-3 max) {pr:.3e}", flush=True)
    assert r <= steps * 1e-4, (label, r)
    assert pa <= steps * 1e-4, (label, pa)
    assert pr <= steps * 1e-3, (label, pr)


def _oracle_chunk(args):
    """Worker: one chunk's back-projection rho * sum_j P_j / D_j (the update without the
    sensitivity division) and its denominators."""
    import oracle as orc
    kw, ev, rho = args
    g = orc.geometry(**kw)
    out, st, D = orc.mlem(g, ev, rho, 1, s=None, return_D=True)
    return out, st, D


def map_with_progress(pool, fn, jobs, label):
    """pool.map that reports every tenth of the jobs as they finish (results in job order)."""
    import time
    out = [None] * len(jobs)
    t0 = time.perf_counter()
    step = max(1, len(jobs) // 10)
    for done, (k, r) in enumerate(pool.imap_unordered(_indexed, [(k, fn, j) for k, j in enumerate(jobs)]), 1):
        out[k] = r
        if done % step == 0 or done == len(jobs):
            print(f"{label}: oracle {done}/{len(jobs)} chunks, {time.perf_counter() - t0:.0f} s", flush=True)
    return out


def _indexed(args):
    k, fn, job = args
    return k, fn(job)


def oracle_step(pool, kw, ev_np, rho, so, chunks=64, label="oracle"):
    """One oracle MLEM step over all events: (image, stats, D of every event)."""
    parts = map_with_progress(pool, _oracle_chunk, [(kw, c, rho) for c in np.array_split(ev_np, chunks)], label)
    acc = np.sum([p[0] for p in parts], axis=0)
    img = np.divide(acc, so, out=np.zeros_like(acc), where=so > 0)
    st = {k: sum(p[1][k] for p in parts) for k in parts[0][1]}
    D = np.concatenate([p[2] for p in parts])
    return img, st, D


@pytest.fixture(scope="module")
def pool():
    with mp.get_context("spawn").Pool(PROCS) as p:
        yield p


@pytest.fixture(scope="module")
def prod():
    w = get_workload("prod400")
    ev_np = w.events()
    return w, ev_np, torch.from_numpy(ev_np).to(DEV)


def bench_geometry(w, ev):
    """The geometry with the plan bench.py times: the autotuned one (tune.plan_for)."""
    from paper_1502_07478_amd import tune
    return tune.tuned(jpet.geometry(**w.geometry()), ev)


def test_prod400_full_image_at_the_benchmarked_plan(prod, pool):
    """All 10M events, one step from rho^0: the whole image and every event's denominator as the
    benchmarked pass computes them (the plan bench.py takes), against the oracle."""
    w, ev_np, ev = prod
    kw = w.geometry()
    g, go = bench_geometry(w, ev), oracle.geometry(**kw)
    info = jpet.launch_info(g, len(ev_np))
    print(f"prod400 full: plan {info}", flush=True)
    assert info["binned"] == 1 and info["plan"] == g.plan and info["events_per_workgroup"] >= 256
    s = jpet.sensitivity(g)
    so = oracle.sensitivity(go)
    rho0 = (s > 0).to(torch.float32)
    ws = jpet.workspace(g, ev.shape[0])
    jpet.prepare(g, ev, ws)
    D = jpet.denominators(g, ev, rho0, ws=ws, prepared=True)
    rho = rho0.clone()
    st = jpet.mlem_iterate(g, ev, rho, 1, s=s, ws=ws, prepared=True, want_stats=True)
    assert st["n_unplaced_rows"] == 0
    got = rho.double().cpu().numpy()
    Dg = D.double().cpu().numpy()
    print(f"prod400 full: GPU done {st}", flush=True)
    want, sto, Do = oracle_step(pool, kw, ev_np, oracle.initial_image(so), so, label="prod400 full")
    for k in ("n_valid", "n_dropped", "n_pairs", "n_zero_denominator", "n_kappa_nonpositive"):
        assert st[k] == sto[k], (k, st[k], sto[k])
    check_image(got, want, label="prod400 one step")
    ok = Do > 0
    assert np.array_equal(Dg > 0, ok)
    rel = np.abs(Dg[ok] / Do[ok] - 1.0)
    print(f"prod400 D: {ok.sum()} events, max rel {rel.max():.3e}, p99.9 {np.quantile(rel, 0.999):.3e}", flush=True)
    assert rel.max() <= 1e-4


def test_prod400_ten_step_trajectory_on_a_prefix_with_the_same_plan(prod, pool):
    """The first 600k events take the benchmarked plan (same bins, items, batches and accumulator
    units); ten GPU steps against ten oracle steps, checked after every step."""
    w, ev_np, ev = prod
    n = 600_000
    kw = w.geometry()
    g, go = bench_geometry(w, ev), oracle.geometry(**kw)
    full, pre = jpet.launch_info(g, len(ev_np)), jpet.launch_info(g, n)
    for k in full:
        if k != "max_workgroups":
            assert pre[k] == full[k], (k, pre[k], full[k])
    e_np = ev_np[:n]
    e = ev[:n].contiguous()
    s = jpet.sensitivity(g)
    so = oracle.sensitivity(go)
    ws = jpet.workspace(g, n)
    jpet.prepare(g, e, ws)
    rho = (s > 0).to(torch.float32)
    ro = oracle.initial_image(so)
    for t in range(1, w.n_iter + 1):
        jpet.mlem_iterate(g, e, rho, 1, s=s, ws=ws, prepared=True)
        ro, _, _ = oracle_step(pool, kw, e_np, ro, so, chunks=32, label=f"prod400[:600k] step {t}")
        check_image(rho.double().cpu().numpy(), ro, steps=t, label=f"prod400[:600k] step {t}")


def test_prod400_accumulator_units_32_against_64_bit(prod):
    """The 32-bit accumulator plan (2^-23 units per count, each (event, pixel) term rounded to the
    nearest unit) against the best 64-bit plan (2^-32 units), ten steps over all 10M events: the
    rounding of terms below half a unit does not move low-activity pixels beyond the per-step
    bounds, also where the image is 1e-4 of its maximum and below."""
    w, ev_np, ev = prod
    g = bench_geometry(w, ev)
    n = len(ev_np)
    assert jpet.launch_info(g, n)["accumulator_bits"] == 32
    code64 = next(code for code, _ in jpet.plan_candidates(g, n) if not code & 4)
    g64 = jpet.with_plan(g, code64)
    assert jpet.launch_info(g64, n)["accumulator_bits"] == 64
    s = jpet.sensitivity(g)
    imgs = []
    for gg in (g, g64):
        ws = jpet.workspace(gg, n)
        jpet.prepare(gg, ev, ws)
        rho = (s > 0).to(torch.float32)
        jpet.mlem_iterate(gg, ev, rho, w.n_iter, s=s, ws=ws, prepared=True)
        imgs.append(rho.double().cpu().numpy().ravel())
        del ws
        torch.cuda.empty_cache()
    a, b = imgs
    m = b.max()
    d = np.abs(a - b)
    for lo, hi in ((1e-3, 1.1), (1e-4, 1e-3), (1e-5, 1e-4)):
        sel = (b >= lo * m) & (b < hi * m)
        if sel.any():
            print(f"acc32 vs acc64, rho in [{lo:g}, {hi:g}) max: {sel.sum()} px, max rel {(d[sel] / b[sel]).max():.3e}",
                  flush=True)
    print(f"acc32 vs acc64: rel L2 {rel_l2(a, b):.3e}, max |d|/max {d.max() / m:.3e}", flush=True)
    assert rel_l2(a, b) <= 1e-4
    assert d.max() <= 1e-4 * m
    big = b >= 1e-3 * m
    assert (d[big] / b[big]).max() <= 1e-3
    # pixels the 64-bit plan keeps positive stay positive
    assert not np.any((b > 1e-6 * m) & (a == 0))


def _events_of(args):
    w, n = args
    return w.events(n, workers=1)


def test_batch64_full_size_images(pool):
    """All 64 batched instances at their full event counts, one step from rho^0 in one batched call:
    every instance conserves counts (sum s rho = valid events with a positive denominator, Eq. 3),
    and the largest instance of each grid size (128, 256, 512) matches the oracle over its whole
    image."""
    base = batch_instances()
    evs = pool.map(_events_of, [(w, None) for w in base])
    print(f"batch64: {sum(len(e) for e in evs)} events generated", flush=True)
    inst, images, sens = [], [], []
    for w, ev_np in zip(base, evs):
        g = jpet.geometry(**w.geometry())
        s = jpet.sensitivity(g)
        rho = (s > 0).to(torch.float32)
        inst.append((g, torch.from_numpy(ev_np).to(DEV), s, rho))
        images.append(rho)
        sens.append(s)
    stats = jpet.BatchedMLEM(inst).iterate(1, want_stats=True)
    torch.cuda.synchronize()
    got = [r.double().cpu().numpy() for r in images]
    for k, w in enumerate(base):
        st = stats[k]
        assert st["n_unplaced_rows"] == 0, k
        cons = float((sens[k].double() * images[k].double()).sum())
        want_n = st["n_valid"] - st["n_zero_denominator"]
        assert abs(cons - want_n) <= 1e-4 * max(want_n, 1), (k, cons, want_n)
    del inst, images
    torch.cuda.empty_cache()
    print("batch64: GPU step done, counts conserved in all 64 instances", flush=True)
    largest = {}
    for k, (w, ev_np) in enumerate(zip(base, evs)):
        if w.n_y not in largest or len(ev_np) > len(evs[largest[w.n_y]]):
            largest[w.n_y] = k
    for n_y, k in sorted(largest.items()):
        w, ev_np = base[k], evs[k]
        go = oracle.geometry(**w.geometry())
        so = oracle.sensitivity(go)
        want, sto, _ = oracle_step(pool, w.geometry(), ev_np, oracle.initial_image(so), so, chunks=64,
                                   label=f"{w.name} ({n_y}^2, {len(ev_np)} events)")
        for key in ("n_valid", "n_pairs", "n_zero_denominator"):
            assert stats[k][key] == sto[key], (k, key)
        check_image(got[k], want, label=f"{w.name} n={len(ev_np)} grid={n_y}")
