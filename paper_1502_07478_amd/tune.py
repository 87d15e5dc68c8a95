"""Autotuner of the MLEM event pass's launch plan.

The library's cost model ranks every plan that fits a geometry (jpet_mlem_plan_candidates); this
module times the leading candidates on the caller's own events (jpet_mlem_tune: HIP events around
the event pass, on the device) and keeps the fastest.  Results are cached in JSON, keyed by the
geometry, the resolution and the event count in half-octave buckets:

* ``plans.json`` beside this module holds plans tuned on an MI355X for the standard workloads (see
  ``python -m paper_1502_07478_amd.tune --help``); it is read, never written, at run time;
* ``$JPET_PLAN_CACHE`` (default ``~/.cache/jpet/plans.json``) collects the plans tuned since.

A plan only changes how the work is laid out (tiles, bins, workgroup shape, accumulator width),
never what is computed: any plan gives the same images to FP32 rounding.
"""

from __future__ import annotations

import ctypes
import json
import math
import os
import time

import torch

from . import jpet

_HERE = os.path.dirname(os.path.abspath(__file__))
SHIPPED = os.path.join(_HERE, "plans.json")


def user_cache_path() -> str:
    return os.environ.get("JPET_PLAN_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "jpet", "plans.json"))


def key_of(g: jpet.Geometry, n_events: int, batched: bool = False, loglik: bool = False) -> str:
    """The cache key: pass, geometry, resolution, kernel variant, grid and the event count's
    half-octave."""
    bucket = int(round(2.0 * math.log2(max(int(n_events), 1))))
    kind = "loglik" if loglik else "batched" if batched else "single"
    return (f"{kind}|R={g.R:.6g}|L={g.L:.6g}|sz={g.sigma_z:.6g}|sdl={g.sigma_dl:.6g}|"
            f"gamma={g.gamma:.6g}|edge={g.sigma_z_edge:.6g}|pix={g.pixel:.6g}|{g.n_y}x{g.n_z}|v={g.kernel_variant}|"
            f"n2={bucket}")


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh).get("plans", {})
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    plans = _load(path)
    plans[key] = entry
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump({"plans": plans}, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def batchable(g: jpet.Geometry, code: int, n_events: int) -> bool:
    """Plans the batched pass can run: 32-bit accumulators (and the generic pass)."""
    if code == 3:
        return True
    return jpet.launch_info(jpet.with_plan(g, code), n_events)["accumulator_bits"] == 32


def time_plans(g: jpet.Geometry, events: torch.Tensor, codes, rho: torch.Tensor | None = None, reps: int = 3,
               stream=None) -> list:
    """Milliseconds per event pass of each plan code on these events (-1: does not fit)."""
    n = events.shape[0]
    if rho is None:
        rho = (jpet.sensitivity(g, device=events.device) > 0).to(torch.float32)
    arr = (ctypes.c_int32 * len(codes))(*codes)
    b = ctypes.c_size_t(0)
    jpet._check(jpet.lib().jpet_mlem_tune_workspace_size(ctypes.byref(g), n, arr, len(codes), ctypes.byref(b)),
                "jpet_mlem_tune_workspace_size")
    ws = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=events.device)
    ms = (ctypes.c_double * len(codes))()
    jpet._check(jpet.lib().jpet_mlem_tune(ctypes.byref(g), jpet._ptr(events), n, jpet._ptr(rho), arr, len(codes),
                                          int(reps), jpet._ptr(ws), ws.numel(), ms, jpet._stream(stream)),
                "jpet_mlem_tune")
    return [float(x) for x in ms]


def with_families(g: jpet.Geometry, ranked, n: int, candidates: int, loglik: bool = False) -> list:
    """The first `candidates` codes of a ranked list, plus the best-ranked code of every plan family
    (register cache, row segments, wavefronts per workgroup) that has none among them: the cost
    model's weights for a family (split rows above all) are priors, so each family gets timed."""
    codes = list(ranked[:candidates])
    def family(c):
        li = jpet.launch_info(jpet.with_plan(g, c), n)
        return li["row_cache"], li["row_segments"], li["waves"]
    seen = {family(c) for c in codes}
    for c in ranked[candidates:]:
        f = family(c)
        if f not in seen:
            seen.add(f)
            codes.append(c)
    return codes


def tune(g: jpet.Geometry, events: torch.Tensor, rho: torch.Tensor | None = None, candidates: int = 12,
         reps: int = 3, batched: bool = False) -> dict:
    """Times the cost model's first `candidates` plans and the best of every other plan family (for a
    batch: among the plans the batched pass can run) and returns {"code", "ms", "model_code",
    "model_ms", "timed", "seconds"}."""
    t0 = time.perf_counter()
    n = events.shape[0]
    ranked = [c for c, _ in jpet.plan_candidates(g, n)]
    if batched:
        ranked = [c for c in ranked if batchable(g, c, n)]
    codes = with_families(g, ranked, n, candidates)
    ms = time_plans(g, events, codes, rho, reps)
    timed = [(c, t) for c, t in zip(codes, ms) if t > 0]
    best = min(timed, key=lambda x: x[1]) if timed else (codes[0], -1.0)
    return {"code": int(best[0]), "ms": best[1], "model_code": int(codes[0]), "model_ms": ms[0] if ms else -1.0,
            "timed": [[int(c), round(t, 4)] for c, t in zip(codes, ms)], "seconds": round(time.perf_counter() - t0, 3)}


def time_loglik_plans(g: jpet.Geometry, events: torch.Tensor, codes, rho: torch.Tensor, s: torch.Tensor | None = None,
                      reps: int = 3) -> list:
    """Milliseconds per log-likelihood-and-gradient call (l, dl/dsigma, dl/drho) of each plan code of
    that pass on these events, with the events prepared once per plan; HIP events on the current
    stream."""
    out = []
    n = events.shape[0]
    for c in codes:
        gc = jpet.with_plan(g, c)
        ws = jpet.loglik_workspace(gc, n, device=events.device)
        jpet.loglik_grad(gc, events, rho, s=s, ws=ws)  # prepares, and warms up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            jpet.loglik_grad(gc, events, rho, s=s, ws=ws, prepared=True)
        e1.record()
        e1.synchronize()
        out.append(e0.elapsed_time(e1) / reps)
        del ws
    return out


def tune_loglik(g: jpet.Geometry, events: torch.Tensor, rho: torch.Tensor, s: torch.Tensor | None = None,
                candidates: int = 8, reps: int = 3) -> dict:
    """The log-likelihood pass's counterpart of tune(): times the cost model's first `candidates` plans
    of that pass (64-bit accumulators; whole or split rows), and the best of every other family, on
    these events and this image."""
    t0 = time.perf_counter()
    n = events.shape[0]
    codes = with_families(g, [c for c, _ in jpet.plan_candidates(g, n, loglik=True)], n, candidates)
    ms = time_loglik_plans(g, events, codes, rho, s, reps)
    best = min(zip(codes, ms), key=lambda x: x[1])
    return {"code": int(best[0]), "ms": best[1], "model_code": int(codes[0]), "model_ms": ms[0],
            "timed": [[int(c), round(t, 4)] for c, t in zip(codes, ms)], "seconds": round(time.perf_counter() - t0, 3)}


def loglik_plan_for(g: jpet.Geometry, events: torch.Tensor, rho: torch.Tensor, s: torch.Tensor | None = None,
                    **kw) -> int:
    """The tuned log-likelihood plan code for these events: from a cache, else tuned now (on this
    image) and added to the user cache."""
    code = lookup(g, events.shape[0], loglik=True)
    if code is not None:
        return code
    entry = tune_loglik(g, events, rho, s, **kw)
    _store(user_cache_path(), key_of(g, events.shape[0], loglik=True), entry)
    return entry["code"]


def lookup(g: jpet.Geometry, n_events: int, batched: bool = False, loglik: bool = False):
    """The cached plan code (shipped table first, then the user cache), or None."""
    key = key_of(g, n_events, batched, loglik)
    for path in (SHIPPED, user_cache_path()):
        entry = _load(path).get(key)
        if entry is not None:
            return int(entry["code"])
    return None


def plan_for(g: jpet.Geometry, events: torch.Tensor, rho: torch.Tensor | None = None, batched: bool = False,
             **kw) -> int:
    """The tuned plan code for these events: from a cache, else tuned now and added to the user
    cache."""
    code = lookup(g, events.shape[0], batched)
    if code is not None:
        return code
    entry = tune(g, events, rho, batched=batched, **kw)
    _store(user_cache_path(), key_of(g, events.shape[0], batched), entry)
    return entry["code"]


def tuned(g: jpet.Geometry, events: torch.Tensor, rho: torch.Tensor | None = None, batched: bool = False,
          **kw) -> jpet.Geometry:
    """A copy of g naming its tuned plan."""
    return jpet.with_plan(g, plan_for(g, events, rho, batched=batched, **kw))


def _main():
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="Tune the event pass's plans of named workloads on this GPU and write "
                                             "them to a plan table (JSON).")
    ap.add_argument("--out", default=SHIPPED)
    ap.add_argument("--workloads", default="prod400,grad200,grad200:loglik,large1024,batch64,paper130,edge400")
    ap.add_argument("--candidates", type=int, default=16)
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    root = os.path.dirname(_HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    from jpet_synth import get_workload
    from jpet_synth.configs import batch_instances
    jobs = []
    for name in args.workloads.split(","):
        if name == "batch64":
            jobs += [(w, "batched") for w in batch_instances()]
        elif name == "large1024":
            w = get_workload(name)
            jobs.append((w.replace(n_events=8_000_000), "single"))  # the 8M-event chunks
        elif name.endswith(":loglik"):
            jobs.append((get_workload(name.split(":")[0]), "loglik"))
        else:
            jobs.append((get_workload(name), "single"))
    for w, kind in jobs:
        g = jpet.geometry(**w.geometry())
        ev = torch.from_numpy(w.events(workers=8)).cuda()
        if kind == "loglik":
            # at the image five MLEM iterations reach from rho^0 (where the gradient is evaluated)
            s = jpet.sensitivity(g, device=ev.device)
            rho = (s > 0).to(torch.float32)
            jpet.mlem_iterate(g, ev, rho, 5, s=s)
            entry = tune_loglik(g, ev, rho, s, candidates=args.candidates, reps=args.reps)
        else:
            entry = tune(g, ev, candidates=args.candidates, reps=args.reps, batched=kind == "batched")
        entry["workload"] = w.name
        _store(args.out, key_of(g, ev.shape[0], kind == "batched", kind == "loglik"), entry)
        print(f"{w.name}: plan {entry['code']} {entry['ms']:.3f} ms (model's {entry['model_code']} "
              f"{entry['model_ms']:.3f} ms), {entry['seconds']} s", flush=True)
        del ev
        torch.cuda.empty_cache()


if __name__ == "__main__":
    _main()
