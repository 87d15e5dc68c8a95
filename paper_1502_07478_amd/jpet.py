"""Python binding of libjpet (ctypes).  Argument marshalling only: every step of the
reconstruction runs in the library's HIP kernels; torch provides device memory and streams.

Images are float32 CUDA tensors of shape [n_y, n_z] (row-major), events float32 [n, 3]
(z_u, z_d, dl) in millimetres.  See include/jpet.h for the contract of each call.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjpet.so")

JPET_OK, JPET_EINVAL, JPET_EDOMAIN, JPET_EWORKSPACE, JPET_EHIP, JPET_ENOTSUP = 0, -1, -2, -3, -4, -5
JPET_WS_PREPARED = 1
JPET_PASS_WAVE_PER_EVENT, JPET_PASS_THREAD_PER_EVENT = 2, 4
JPET_LOGLIK_VALUE_ONLY = 8
# bytes of the library's per-GPU scratch array behind jpet_mlem_iterate_noalloc (JPET_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 256 * 1024 * 1024


class JpetError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib().jpet_strerror(code).decode()
        if code == JPET_EHIP:
            msg += f" (hipError {_lib().jpet_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")


class Geometry(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_double), ("L", ctypes.c_double), ("sigma_z", ctypes.c_double),
        ("sigma_dl", ctypes.c_double), ("gamma", ctypes.c_double), ("pixel", ctypes.c_double),
        ("n_y", ctypes.c_int32), ("n_z", ctypes.c_int32), ("kernel_variant", ctypes.c_int32),
        ("plan", ctypes.c_int32), ("sigma_z_edge", ctypes.c_double),
    ]

    @property
    def shape(self):
        return (int(self.n_y), int(self.n_z))


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_events", ctypes.c_int64), ("n_valid", ctypes.c_int64), ("n_dropped", ctypes.c_int64),
        ("n_zero_denominator", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
        ("n_kappa_nonpositive", ctypes.c_int64), ("n_unplaced_rows", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class LaunchInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "binned", "tile_rows", "tile_cols", "halo_rows", "halo_cols", "t_bins", "bins", "waves", "row_cache",
        "events_per_batch", "events_per_workgroup", "accumulator_bits")] + [
        ("t_bin_width", ctypes.c_double), ("lds_bytes", ctypes.c_int64), ("max_workgroups", ctypes.c_int64),
        ("plan", ctypes.c_int32), ("workgroups_per_cu", ctypes.c_int32), ("accumulator_shift", ctypes.c_int32),
        ("row_segments", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Instance(ctypes.Structure):
    """One reconstruction of a batch (jpet_instance)."""
    _fields_ = [("g", Geometry), ("events", ctypes.c_void_p), ("n", ctypes.c_int64), ("s", ctypes.c_void_p),
                ("rho", ctypes.c_void_p)]


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libjpet.so is not built ({LIB_PATH}); run paper_1502_07478_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, gp, sp = ctypes.c_void_p, ctypes.POINTER(Geometry), ctypes.POINTER(Stats)
        i64, sz, u32, i32 = ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_int32
        L.jpet_strerror.argtypes = [ctypes.c_int]
        L.jpet_strerror.restype = ctypes.c_char_p
        L.jpet_last_hip_error.argtypes = []
        L.jpet_abi_version.argtypes = []
        L.jpet_sensitivity.argtypes = [gp, vp, vp]
        L.jpet_direct_image.argtypes = [gp, vp, i64, vp, vp]
        L.jpet_mlem_workspace_size.argtypes = [gp, i64, ctypes.POINTER(sz)]
        L.jpet_mlem_prepare.argtypes = [gp, vp, i64, vp, sz, vp]
        L.jpet_mlem_iterate.argtypes = [gp, vp, i64, vp, vp, i32, vp, sz, u32, sp, vp]
        L.jpet_mlem_iterate_noalloc.argtypes = [gp, vp, i64, vp, vp, i32, u32, sp, vp]
        L.jpet_mlem_backproject.argtypes = [gp, vp, i64, vp, vp, vp, sz, u32, sp, vp]
        L.jpet_mlem_update.argtypes = [gp, vp, vp, vp, vp]
        L.jpet_loglik_workspace_size.argtypes = [gp, ctypes.POINTER(ctypes.c_double), i64, ctypes.POINTER(sz)]
        L.jpet_loglik_grad.argtypes = [gp, ctypes.POINTER(ctypes.c_double), vp, i64, vp, vp, vp, vp, vp, vp, sz,
                                       u32, sp, vp]
        ip = ctypes.POINTER(Instance)
        L.jpet_mlem_batched_workspace_size.argtypes = [ip, i32, ctypes.POINTER(sz)]
        L.jpet_mlem_batched_prepare.argtypes = [ip, i32, vp, sz, vp]
        L.jpet_mlem_batched_iterate.argtypes = [ip, i32, i32, vp, sz, u32, sp, vp]
        L.jpet_mlem_batched_graph_create.argtypes = [ip, i32, i32, vp, sz, u32, vp, ctypes.POINTER(vp)]
        L.jpet_mlem_batched_graph_launch.argtypes = [vp, vp]
        L.jpet_mlem_batched_graph_destroy.argtypes = [vp]
        L.jpet_mlem_launch_info.argtypes = [gp, i64, ctypes.POINTER(LaunchInfo)]
        L.jpet_mlem_plan_candidates.argtypes = [gp, i32, ctypes.POINTER(ctypes.c_double), i64,
                                                ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), i32,
                                                ctypes.POINTER(i32)]
        L.jpet_mlem_denominators.argtypes = [gp, vp, i64, vp, vp, vp, sz, u32, sp, vp]
        L.jpet_mlem_tune_workspace_size.argtypes = [gp, i64, ctypes.POINTER(i32), i32, ctypes.POINTER(sz)]
        L.jpet_mlem_tune.argtypes = [gp, vp, i64, vp, ctypes.POINTER(i32), i32, i32, vp, sz,
                                     ctypes.POINTER(ctypes.c_double), vp]
        L.jpet_profile_enable.argtypes = [ctypes.c_int]
        L.jpet_profile_read.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
        _L = L
    return _L


def lib():
    """The loaded libjpet (raises if it is not built)."""
    return _lib()


def geometry(R, L, sigma_z, sigma_dl, pixel, n_y, n_z, kernel_variant=0, gamma=0.0,
             sigma_z_edge=0.0, plan=0) -> Geometry:
    """sigma_z_edge: relative rise of sigma_z from the strip centre to its ends (0: constant).
    plan: 0 (the library's cost model chooses) or a code from plan_candidates."""
    return Geometry(float(R), float(L), float(sigma_z), float(sigma_dl), float(gamma), float(pixel), int(n_y),
                    int(n_z), int(kernel_variant), int(plan), float(sigma_z_edge))


def with_plan(g: Geometry, plan: int) -> Geometry:
    """A copy of g that names the given plan code."""
    return Geometry(g.R, g.L, g.sigma_z, g.sigma_dl, g.gamma, g.pixel, g.n_y, g.n_z, g.kernel_variant, int(plan),
                    g.sigma_z_edge)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(rc: int, where: str):
    if rc != JPET_OK:
        raise JpetError(rc, where)


def _need(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def profile_enable(on: bool = True):
    """Time every event-pass launch with HIP events on its stream (see jpet_profile_read)."""
    _check(_lib().jpet_profile_enable(1 if on else 0), "jpet_profile_enable")


def profile_read():
    """(timed event-pass launches, their summed duration in ms) since the last read."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(_lib().jpet_profile_read(ctypes.byref(n), ctypes.byref(ms)), "jpet_profile_read")
    return int(n.value), float(ms.value)


def sensitivity(g: Geometry, device=None, stream=None) -> torch.Tensor:
    out = torch.empty(g.shape, dtype=torch.float32, device=device or "cuda")
    _check(_lib().jpet_sensitivity(ctypes.byref(g), _ptr(out), _stream(stream)), "jpet_sensitivity")
    return out


def direct_image(g: Geometry, events: torch.Tensor, stream=None) -> torch.Tensor:
    """Counts of the events' direct-reconstruction points (Eq. 2) per pixel (jpet_direct_image)."""
    _events(events)
    out = torch.empty(g.shape, dtype=torch.float32, device=events.device)
    _check(_lib().jpet_direct_image(ctypes.byref(g), _ptr(events), events.shape[0], _ptr(out), _stream(stream)),
           "jpet_direct_image")
    return out


def workspace_size(g: Geometry, n_events: int) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib().jpet_mlem_workspace_size(ctypes.byref(g), int(n_events), ctypes.byref(b)), "jpet_mlem_workspace_size")
    return int(b.value)


def launch_info(g: Geometry, n_events: int) -> dict:
    """The event pass's launch shape for this geometry and event count."""
    info = LaunchInfo()
    _check(_lib().jpet_mlem_launch_info(ctypes.byref(g), int(n_events), ctypes.byref(info)), "jpet_mlem_launch_info")
    return info.as_dict()


def plan_candidates(g: Geometry, n_events: int, loglik: bool = False, sigma_mask=None, cap: int = 1024):
    """[(plan code, cost-model figure)] of the plans that fit, cheapest first (jpet_mlem_plan_candidates)."""
    codes = (ctypes.c_int32 * cap)()
    cost = (ctypes.c_double * cap)()
    count = ctypes.c_int32(0)
    sm = (ctypes.c_double * 2)(*sigma_mask) if sigma_mask is not None else None
    _check(_lib().jpet_mlem_plan_candidates(ctypes.byref(g), 1 if loglik else 0, sm, int(n_events), codes, cost, cap,
                                            ctypes.byref(count)), "jpet_mlem_plan_candidates")
    return [(int(codes[k]), float(cost[k])) for k in range(min(cap, count.value))]


def workspace(g: Geometry, n_events: int, device=None) -> torch.Tensor:
    return torch.empty(workspace_size(g, n_events), dtype=torch.uint8, device=device or "cuda")


def _events(events):
    _need(events, "events", torch.float32)
    if events.dim() != 2 or events.shape[1] != 3:
        raise ValueError("events must be [n, 3]")
    return events


def prepare(g: Geometry, events: torch.Tensor, ws: torch.Tensor, stream=None):
    """Iteration-invariant per-event work (direct reconstruction, ellipse rows) into ws."""
    _events(events)
    _check(_lib().jpet_mlem_prepare(ctypes.byref(g), _ptr(events), events.shape[0], _ptr(ws), ws.numel(),
                                    _stream(stream)), "jpet_mlem_prepare")


_SPLIT = {None: 0, "wave": JPET_PASS_WAVE_PER_EVENT, "thread": JPET_PASS_THREAD_PER_EVENT}


def mlem_iterate(g: Geometry, events: torch.Tensor, rho: torch.Tensor, n_iter: int, s: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None, prepared: bool = False, want_stats: bool = False, stream=None,
                 split: str | None = None):
    """n_iter MLEM iterations in place on rho; returns the stats dict when want_stats.
    split: None (the planned pass) or, for comparison, "wave" (one wavefront per event) or
    "thread" (one thread per event)."""
    _events(events)
    _need(rho, "rho", torch.float32, g.shape)
    if s is not None:
        _need(s, "s", torch.float32, g.shape)
    if ws is None:
        ws = workspace(g, events.shape[0], rho.device)
        prepared = False
    st = Stats() if want_stats else None
    rc = _lib().jpet_mlem_iterate(ctypes.byref(g), _ptr(events), events.shape[0], _ptr(s), _ptr(rho), int(n_iter),
                                  _ptr(ws), ws.numel(), (JPET_WS_PREPARED if prepared else 0) | _SPLIT[split],
                                  ctypes.byref(st) if st is not None else None, _stream(stream))
    _check(rc, "jpet_mlem_iterate")
    return st.as_dict() if st is not None else None


def mlem_iterate_noalloc(g: Geometry, events: torch.Tensor, rho: torch.Tensor, n_iter: int,
                         s: torch.Tensor | None = None, want_stats: bool = False, stream=None):
    """mlem_iterate with the library's own per-GPU scratch array as the workspace
    (jpet_mlem_iterate_noalloc): no device allocation by the library or by this wrapper.  Calls on
    one GPU share the array: order them on one stream."""
    _events(events)
    _need(rho, "rho", torch.float32, g.shape)
    if s is not None:
        _need(s, "s", torch.float32, g.shape)
    st = Stats() if want_stats else None
    rc = _lib().jpet_mlem_iterate_noalloc(ctypes.byref(g), _ptr(events), events.shape[0], _ptr(s), _ptr(rho),
                                          int(n_iter), 0, ctypes.byref(st) if st is not None else None,
                                          _stream(stream))
    _check(rc, "jpet_mlem_iterate_noalloc")
    return st.as_dict() if st is not None else None


def mlem(events: torch.Tensor, g: Geometry, n_iter: int, sens: torch.Tensor | None = None,
         rho0: torch.Tensor | None = None):
    """Reconstruct from rho0 (default: 1 where sens > 0, or 1 everywhere without sens)."""
    if rho0 is None:
        rho = (sens > 0).to(torch.float32) if sens is not None else torch.ones(g.shape, device=events.device)
    else:
        rho = rho0.clone()
    mlem_iterate(g, events, rho, n_iter, s=sens)
    return rho


def denominators(g: Geometry, events: torch.Tensor, rho: torch.Tensor, ws: torch.Tensor | None = None,
                 prepared: bool = False, want_stats: bool = False, stream=None, split: str | None = None):
    """Per-event forward sums D_j of the MLEM event pass at rho (jpet_mlem_denominators): a float32
    [n] tensor (0 for dropped events), and the stats dict when want_stats."""
    _events(events)
    _need(rho, "rho", torch.float32, g.shape)
    if ws is None:
        ws = workspace(g, events.shape[0], rho.device)
        prepared = False
    D = torch.empty(events.shape[0], dtype=torch.float32, device=rho.device)
    st = Stats() if want_stats else None
    rc = _lib().jpet_mlem_denominators(ctypes.byref(g), _ptr(events), events.shape[0], _ptr(rho), _ptr(D), _ptr(ws),
                                       ws.numel(), (JPET_WS_PREPARED if prepared else 0) | _SPLIT[split],
                                       ctypes.byref(st) if st is not None else None, _stream(stream))
    _check(rc, "jpet_mlem_denominators")
    return (D, st.as_dict()) if want_stats else D


def accumulator(g: Geometry, device=None) -> torch.Tensor:
    """A zeroed back-projection accumulator (int64 [n_y, n_z], 2^-32 units, read as uint64)."""
    return torch.zeros(g.shape, dtype=torch.int64, device=device or "cuda")


def backproject(g: Geometry, events: torch.Tensor, rho: torch.Tensor, acc: torch.Tensor, ws: torch.Tensor | None = None,
                prepared: bool = False, want_stats: bool = False, stream=None, split: str | None = None):
    """One event pass over this event list, added into acc (see jpet_mlem_backproject); split as
    for mlem_iterate."""
    _events(events)
    _need(rho, "rho", torch.float32, g.shape)
    _need(acc, "acc", torch.int64, g.shape)
    if ws is None:
        ws = workspace(g, events.shape[0], rho.device)
        prepared = False
    st = Stats() if want_stats else None
    rc = _lib().jpet_mlem_backproject(ctypes.byref(g), _ptr(events), events.shape[0], _ptr(rho), _ptr(acc), _ptr(ws),
                                      ws.numel(), (JPET_WS_PREPARED if prepared else 0) | _SPLIT[split],
                                      ctypes.byref(st) if st is not None else None, _stream(stream))
    _check(rc, "jpet_mlem_backproject")
    return st.as_dict() if st is not None else None


def update(g: Geometry, acc: torch.Tensor, rho: torch.Tensor, s: torch.Tensor | None = None, stream=None):
    """rho = acc 2^-32 / s (0 where s = 0), acc cleared (see jpet_mlem_update)."""
    _need(rho, "rho", torch.float32, g.shape)
    _need(acc, "acc", torch.int64, g.shape)
    if s is not None:
        _need(s, "s", torch.float32, g.shape)
    _check(_lib().jpet_mlem_update(ctypes.byref(g), _ptr(s), _ptr(acc), _ptr(rho), _stream(stream)),
           "jpet_mlem_update")


class ChunkedMLEM:
    """MLEM over an event list held as chunks (device or pinned-host float32 [n_k, 3] tensors).

    Every chunk is back-projected against the same image into one accumulator, then the image is
    updated once per iteration, so the result equals one jpet_mlem_iterate over the concatenated
    events (exactly: the accumulator is an integer sum).

    resident=True keeps every chunk's events and prepared workspace in device memory, prepared
    once (the fast path when they fit: at 288 GB per GPU they usually do); odd chunks then run on a
    side stream, so one chunk's last workgroups overlap the next chunk's first ones (the
    accumulator's integer atomics make the order irrelevant).  resident=False keeps two device
    slots (events and workspace) and streams the chunks through them every iteration: on a side
    stream, the next chunk is copied from (pinned) host memory and prepared while the current one
    is processed.
    """

    def __init__(self, g: Geometry, chunks, s: torch.Tensor | None = None, resident: bool = True, device=None):
        self.g = g
        self.s = s
        self.device = torch.device(device or "cuda")
        self.resident = resident
        self.chunks = list(chunks)
        for c in self.chunks:
            if c.dim() != 2 or c.shape[1] != 3 or c.dtype != torch.float32:
                raise ValueError("chunks must be float32 [n, 3]")
        self.acc = accumulator(g, self.device)
        self.stats = None
        if resident:
            self.ev = [c.to(self.device, non_blocking=True).contiguous() for c in self.chunks]
            self.ws = [workspace(g, c.shape[0], self.device) for c in self.ev]
            for e, w in zip(self.ev, self.ws):
                prepare(g, e, w)
            self.side = torch.cuda.Stream(device=self.device) if len(self.chunks) > 1 else None
        else:
            cap = max((c.shape[0] for c in self.chunks), default=0)
            self.slots = [torch.empty((cap, 3), dtype=torch.float32, device=self.device) for _ in range(2)]
            # one workspace per slot, prepared again for each chunk: the largest any chunk needs
            wsb = max((workspace_size(g, c.shape[0]) for c in self.chunks), default=workspace_size(g, 0))
            self.ws = [torch.empty(wsb, dtype=torch.uint8, device=self.device) for _ in range(2)]
            self.copy_stream = torch.cuda.Stream(device=self.device)
            self.ready = [torch.cuda.Event() for _ in range(2)]

    def iterate(self, rho: torch.Tensor, n_iter: int, want_stats: bool = False):
        """n_iter iterations in place on rho; the summed stats of the last iteration if asked."""
        tot = None
        side = self.side if self.resident else None
        cur = torch.cuda.current_stream(self.device)
        for it in range(n_iter):
            last = want_stats and it == n_iter - 1
            tot = {} if last else None
            if side is not None:
                side.wait_stream(cur)  # the image and the cleared accumulator are ready
            if not self.resident and self.chunks:
                self.copy_stream.wait_stream(cur)  # slot 0 is free once earlier work is done
                self._stage(0)
            for k in range(len(self.chunks)):
                ev, ws = self._chunk(k, cur)
                st = backproject(self.g, ev, rho, self.acc, ws=ws, prepared=True, want_stats=last,
                                 stream=side if side is not None and k % 2 == 1 else None)
                if last:
                    for key, v in st.items():
                        tot[key] = tot.get(key, 0) + v
            if side is not None:
                cur.wait_stream(side)
            update(self.g, self.acc, rho, self.s)
        return tot

    def _stage(self, k):
        """On the copy stream: chunk k into slot k % 2, then its preparation into that slot's
        workspace; the slot's event marks both done."""
        n = self.chunks[k].shape[0]
        slot = self.slots[k % 2]
        with torch.cuda.stream(self.copy_stream):
            slot[:n].copy_(self.chunks[k], non_blocking=True)
            prepare(self.g, slot[:n], self.ws[k % 2], stream=self.copy_stream)
            self.ready[k % 2].record(self.copy_stream)

    def _chunk(self, k, cur):
        """Events and prepared workspace of chunk k for a pass enqueued next on cur."""
        if self.resident:
            return self.ev[k], self.ws[k]
        if k + 1 < len(self.chunks):
            # slot (k + 1) % 2 held chunk k - 1, whose pass is the last work enqueued on cur
            self.copy_stream.wait_stream(cur)
            self._stage(k + 1)
        cur.wait_event(self.ready[k % 2])
        return self.slots[k % 2][:self.chunks[k].shape[0]], self.ws[k % 2]


class BatchedMLEM:
    """Many independent reconstructions advanced together (jpet_mlem_batched_*): per iteration one
    event-pass launch per class of like instances, one workgroup per workgroup item.

    instances: list of (geometry, events float32 [n, 3], sensitivity or None, rho float32 [n_y, n_z]),
    all CUDA tensors on one device; each rho is updated in place by iterate() and run().  The events
    are prepared once, here.  run(n) launches a HIP graph of n iterations, captured on its first
    use for that n (jpet_mlem_batched_graph_*); iterate(n) enqueues the iterations one by one.
    """

    def __init__(self, instances, stream=None, tuned: bool = False):
        """tuned: each instance takes its autotuned batched plan (paper_1502_07478_amd.tune; from its
        plan cache, else timed now) instead of the cost model's choice."""
        self.keep = []
        arr = (Instance * max(len(instances), 1))()
        if tuned:
            from . import tune
            instances = [(tune.tuned(g, ev, batched=True), ev, s, rho) for g, ev, s, rho in instances]
        self.geometries = [g for g, _, _, _ in instances]
        for k, (g, ev, s, rho) in enumerate(instances):
            _events(ev)
            _need(rho, "rho", torch.float32, g.shape)
            if s is not None:
                _need(s, "s", torch.float32, g.shape)
            arr[k] = Instance(g, ev.data_ptr(), ev.shape[0], s.data_ptr() if s is not None else None, rho.data_ptr())
            self.keep.append((g, ev, s, rho))
        self.count = len(instances)
        self.arr = arr
        b = ctypes.c_size_t(0)
        _check(_lib().jpet_mlem_batched_workspace_size(arr, self.count, ctypes.byref(b)),
               "jpet_mlem_batched_workspace_size")
        dev = instances[0][3].device if instances else torch.device("cuda")
        self.ws = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=dev)
        _check(_lib().jpet_mlem_batched_prepare(arr, self.count, _ptr(self.ws), self.ws.numel(), _stream(stream)),
               "jpet_mlem_batched_prepare")
        self._graphs = {}
        self._table_of = None

    def iterate(self, n_iter: int, want_stats: bool = False, stream=None):
        """n_iter iterations of every instance; per-instance stats dicts when want_stats."""
        st = (Stats * max(self.count, 1))() if want_stats else None
        _check(_lib().jpet_mlem_batched_iterate(self.arr, self.count, int(n_iter), _ptr(self.ws), self.ws.numel(),
                                                JPET_WS_PREPARED, st, _stream(stream)), "jpet_mlem_batched_iterate")
        self._table_of = None  # the eager call rewrote the instance table
        return [st[k].as_dict() for k in range(self.count)] if want_stats else None

    def graph(self, n_iter: int, stream=None):
        """The captured graph of n_iter iterations (created on first use)."""
        if getattr(self, "_table_of", None) != n_iter or n_iter not in self._graphs:
            # a graph relies on the table its creation wrote: recreate after eager calls
            self.close_graphs()
            h = ctypes.c_void_p(None)
            _check(_lib().jpet_mlem_batched_graph_create(self.arr, self.count, int(n_iter), _ptr(self.ws),
                                                         self.ws.numel(), JPET_WS_PREPARED, _stream(stream),
                                                         ctypes.byref(h)), "jpet_mlem_batched_graph_create")
            self._graphs[n_iter] = h
            self._table_of = n_iter
        return self._graphs[n_iter]

    def run(self, n_iter: int = 10, stream=None):
        """The whole reconstruction of every instance: n_iter iterations (the batched workload
        runs 10) as one graph launch; the images are updated in place."""
        h = self.graph(n_iter, stream)
        _check(_lib().jpet_mlem_batched_graph_launch(h, _stream(stream)), "jpet_mlem_batched_graph_launch")

    def close_graphs(self):
        for h in self._graphs.values():
            _lib().jpet_mlem_batched_graph_destroy(h)
        self._graphs = {}

    def __del__(self):
        try:
            if self._graphs:
                torch.cuda.synchronize()
            self.close_graphs()
        except Exception:
            pass


@dataclass
class LogLik:
    value: torch.Tensor        # device double[3]: l, dl/dsigma_z, dl/dsigma_dl
    grad_rho: torch.Tensor | None
    D: torch.Tensor | None
    stats: dict | None


def loglik_workspace(g: Geometry, n_events: int, sigma_mask=None, device=None) -> torch.Tensor:
    """A workspace for jpet_loglik_grad (prepared by its first call, reusable with prepared=True)."""
    b = ctypes.c_size_t(0)
    sm = (ctypes.c_double * 2)(*sigma_mask) if sigma_mask is not None else None
    _check(_lib().jpet_loglik_workspace_size(ctypes.byref(g), sm, int(n_events), ctypes.byref(b)),
           "jpet_loglik_workspace_size")
    return torch.empty(int(b.value), dtype=torch.uint8, device=device or "cuda")


def loglik_grad(g: Geometry, events: torch.Tensor, rho: torch.Tensor, s: torch.Tensor | None = None,
                sigma_mask=None, want_grad_rho: bool = True, want_D: bool = False, ws: torch.Tensor | None = None,
                prepared: bool = False, want_stats: bool = False, stream=None, value_only: bool = False) -> LogLik:
    """l, dl/dsigma and (want_grad_rho) dl/drho (jpet_loglik_grad); value_only: l alone (the
    sigma entries of value are NaN, no grad_rho), one forward pass."""
    _events(events)
    _need(rho, "rho", torch.float32, g.shape)
    if s is not None:
        _need(s, "s", torch.float32, g.shape)
    n = events.shape[0]
    if ws is None:
        ws = loglik_workspace(g, n, sigma_mask, rho.device)
        prepared = False
    out3 = torch.zeros(3, dtype=torch.float64, device=rho.device)
    gr = torch.empty(g.shape, dtype=torch.float32, device=rho.device) if want_grad_rho and not value_only else None
    D = torch.empty(n, dtype=torch.float32, device=rho.device) if want_D else None
    sm = (ctypes.c_double * 2)(*sigma_mask) if sigma_mask is not None else None
    st = Stats() if want_stats else None
    rc = _lib().jpet_loglik_grad(ctypes.byref(g), sm, _ptr(events), n, _ptr(s), _ptr(rho), _ptr(out3), _ptr(gr),
                                 _ptr(D), _ptr(ws), ws.numel(),
                                 (JPET_WS_PREPARED if prepared else 0) | (JPET_LOGLIK_VALUE_ONLY if value_only else 0),
                                 ctypes.byref(st) if st is not None else None, _stream(stream))
    # JPET_EDOMAIN after the pass means a valid event has D = 0 (l = -inf, reported through stats);
    # before it (a geometry or mask out of domain) nothing was written, which is an error
    if not (rc == JPET_EDOMAIN and st is not None and st.n_zero_denominator > 0):
        _check(rc, "jpet_loglik_grad")
    return LogLik(out3, gr, D, st.as_dict() if st is not None else None)


class JPetLogLik(torch.autograd.Function):
    """The list-mode log-likelihood l(rho, sigma_z, sigma_dl) of jpet_loglik_grad as a differentiable
    scalar (float64, on the events' device).

    Forward and backward share one library call: the forward pass evaluates l, dl/drho = B - s and
    the two sigma derivatives together; backward scales them by the incoming gradient.  The sigma
    derivatives hold the 3-sigma ellipse fixed (at sigma_mask, default the sigmas given).

        l = JPetLogLik.apply(rho, sigma_z, sigma_dl, events, g, s, sigma_mask)

    rho: float32 [n_y, n_z] CUDA tensor; sigma_z, sigma_dl: Python floats or 0-dim tensors (they
    override the sigmas of g); s: sensitivity or None; sigma_mask: (sigma_z, sigma_dl) or None.
    """

    @staticmethod
    def forward(ctx, rho, sigma_z, sigma_dl, events, g, s=None, sigma_mask=None):
        sz = float(sigma_z)
        sd = float(sigma_dl)
        gg = Geometry(g.R, g.L, sz, sd, g.gamma, g.pixel, g.n_y, g.n_z, g.kernel_variant, g.plan, g.sigma_z_edge)
        mask = (sz, sd) if sigma_mask is None else tuple(float(x) for x in sigma_mask)
        # with no gradient asked for, the value alone (one forward pass)
        need = any(ctx.needs_input_grad[:3])
        res = loglik_grad(gg, events, rho.detach().contiguous(), s=s, sigma_mask=mask,
                          want_grad_rho=ctx.needs_input_grad[0], value_only=not need)
        ctx.save_for_backward(res.value, res.grad_rho if res.grad_rho is not None else torch.empty(0))
        ctx.sig = [(x.dtype, x.device) if isinstance(x, torch.Tensor) else None for x in (sigma_z, sigma_dl)]
        return res.value[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        value, grad_rho = ctx.saved_tensors
        g_rho = g_sz = g_sd = None
        if ctx.needs_input_grad[0]:
            g_rho = grad_rho * grad_out.to(grad_rho.dtype)
        out = []
        for k, meta in zip((1, 2), ctx.sig):
            if ctx.needs_input_grad[k] and meta is not None:
                out.append((grad_out * value[k]).to(dtype=meta[0], device=meta[1]))
            else:
                out.append(None)
        g_sz, g_sd = out
        return g_rho, g_sz, g_sd, None, None, None, None


def loglik(rho, sigma_z, sigma_dl, events, g, s=None, sigma_mask=None):
    """Differentiable log-likelihood; see JPetLogLik."""
    return JPetLogLik.apply(rho, sigma_z, sigma_dl, events, g, s, sigma_mask)
