"""Profiling driver for rocprofv3: runs the MLEM event pass on a named synthetic workload.

    python -m paper_1502_07478_amd.profile_pass [workload] [n_events|all] [iterations]

Order of GPU work: a 256 MiB device-to-device copy (a kernel of known traffic, to calibrate the
FETCH_SIZE / WRITE_SIZE counters), the sensitivity image, the one-time event preparation, then
`iterations` MLEM iterations (one event-pass launch each).
"""

from __future__ import annotations

import os
import sys


def main(argv):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    from jpet_synth import get_workload
    from paper_1502_07478_amd import jpet

    w = get_workload(argv[0] if len(argv) > 0 else "prod400")
    n = int(argv[1]) if len(argv) > 1 and argv[1] != "all" else None
    iters = int(argv[2]) if len(argv) > 2 else 2
    ev_np = w.events(n)
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    g = jpet.geometry(**w.geometry())
    ev = torch.from_numpy(ev_np).cuda()
    s = jpet.sensitivity(g)
    rho = (s > 0).float()
    ws = jpet.workspace(g, ev.shape[0])
    jpet.prepare(g, ev, ws)
    st = jpet.mlem_iterate(g, ev, rho, iters, s=s, ws=ws, prepared=True, want_stats=True)
    torch.cuda.synchronize()
    print(f"{w.name}: {iters} iterations, {st}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
