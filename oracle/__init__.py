"""ctypes front end of the double-precision CPU oracle (``jpet_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
bench's CPU-baseline leg may use this package; the GPU library never does.
All arrays are numpy; images are ``float64 [n_y, n_z]`` row-major and events
are ``float32 [n, 3]`` rows (z_u, z_d, dl).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jpet_oracle.c")
_LIB = os.path.join(_HERE, "libjpet_oracle.so")

OK, EINVAL, EDOMAIN, ENOMEM = 0, -1, -2, -5


class Geometry(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_double), ("L", ctypes.c_double), ("sigma_z", ctypes.c_double),
        ("sigma_dl", ctypes.c_double), ("gamma", ctypes.c_double), ("pixel", ctypes.c_double),
        ("n_y", ctypes.c_int32), ("n_z", ctypes.c_int32), ("kernel_variant", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("sigma_z_edge", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_events", ctypes.c_int64), ("n_valid", ctypes.c_int64), ("n_dropped", ctypes.c_int64),
        ("n_zero_denominator", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
        ("n_kappa_nonpositive", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE arithmetic)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # JPET_ORACLE_LIB lets the oracle's own mutation checks load a deliberately altered build
        path = os.environ.get("JPET_ORACLE_LIB")
        if not path:
            path = build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        i64p = ctypes.POINTER(ctypes.c_int64)
        gp = ctypes.POINTER(Geometry)
        sp = ctypes.POINTER(Stats)
        L.orc_check_geometry.argtypes = [gp]
        L.orc_sensitivity_point.argtypes = [gp, ctypes.c_double, ctypes.c_double]
        L.orc_sensitivity_point.restype = ctypes.c_double
        L.orc_sensitivity.argtypes = [gp, dp]
        L.orc_direct.argtypes = [gp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_direct.restype = None
        L.orc_direct_image.argtypes = [gp, ctypes.POINTER(ctypes.c_float), ctypes.c_int64, dp]
        L.orc_direct_image.restype = ctypes.c_int64
        L.orc_box_halfsize.argtypes = [ctypes.c_double] * 4 + [dp]
        L.orc_box_halfsize.restype = None
        L.orc_sigma_z_factor.argtypes = [gp, ctypes.c_double, ctypes.c_double]
        L.orc_sigma_z_factor.restype = ctypes.c_double
        L.orc_kernel_points.argtypes = [gp, dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_event_pixels.argtypes = [gp, dp, fp, ctypes.c_int64, i64p, dp]
        L.orc_event_pixels.restype = ctypes.c_int64
        L.orc_mlem.argtypes = [gp, fp, ctypes.c_int64, dp, dp, ctypes.c_int, dp, sp]
        L.orc_loglik_grad.argtypes = [gp, dp, fp, ctypes.c_int64, dp, dp, dp, dp, dp, sp]
        L.orc_backprojection_at.argtypes = [gp, fp, ctypes.c_int64, dp, ctypes.c_int64, i64p, dp]
        L.orc_denominators_at.argtypes = [gp, fp, ctypes.c_int64, i64p, dp, dp, i64p]
        _lib = L
    return _lib


def geometry(R, L, sigma_z, sigma_dl, pixel, n_y, n_z, kernel_variant=0, gamma=0.0,
             sigma_z_edge=0.0) -> Geometry:
    return Geometry(R, L, sigma_z, sigma_dl, gamma, pixel, n_y, n_z, kernel_variant, 0, sigma_z_edge)


def sigma_z_factor(g: Geometry, zu: float, zd: float) -> float:
    """The event's sigma_z over the geometry's (position-dependent resolution)."""
    return lib().orc_sigma_z_factor(ctypes.byref(g), zu, zd)


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _events(ev):
    ev = np.ascontiguousarray(ev, dtype=np.float32)
    if ev.ndim != 2 or ev.shape[1] != 3:
        raise ValueError("events must be [n, 3]")
    return ev


def check_geometry(g: Geometry) -> int:
    return lib().orc_check_geometry(ctypes.byref(g))


def sensitivity(g: Geometry) -> np.ndarray:
    out = np.empty((g.n_y, g.n_z), dtype=np.float64)
    rc = lib().orc_sensitivity(ctypes.byref(g), _ptr(out, ctypes.c_double))
    if rc:
        raise ValueError(f"oracle sensitivity: error {rc}")
    return out


def sensitivity_point(g: Geometry, y: float, z: float) -> float:
    return lib().orc_sensitivity_point(ctypes.byref(g), y, z)


def direct(g: Geometry, zu: float, zd: float, dl: float):
    """(tan theta, 1/cos theta, y~, z~) of one event."""
    out = np.empty(4)
    lib().orc_direct(ctypes.byref(g), zu, zd, dl, _ptr(out, ctypes.c_double))
    return tuple(out)


def direct_image(g: Geometry, events) -> tuple:
    """(counts image [n_y, n_z] of the events' direct-reconstruction points (Eq. 2), events counted)."""
    ev = _events(events)
    out = np.empty((g.n_y, g.n_z), dtype=np.float64)
    n = lib().orc_direct_image(ctypes.byref(g), _ptr(ev, ctypes.c_float), len(ev), _ptr(out, ctypes.c_double))
    return out, int(n)


def box_halfsize(sigma_z, sigma_dl, tan_t, sec_t):
    out = np.empty(2)
    lib().orc_box_halfsize(sigma_z, sigma_dl, tan_t, sec_t, _ptr(out, ctypes.c_double))
    return tuple(out)


def kernel_points(g: Geometry, events: np.ndarray, y: float, z: float):
    """Unmasked kernel P and b C^-1 b for double-precision event triples at one pixel centre."""
    ev = _f64(events).reshape(-1, 3)
    P = np.empty(len(ev))
    q = np.empty(len(ev))
    rc = lib().orc_kernel_points(ctypes.byref(g), _ptr(ev, ctypes.c_double), len(ev), y, z,
                                 _ptr(P, ctypes.c_double), _ptr(q, ctypes.c_double))
    if rc:
        raise ValueError(f"oracle kernel: error {rc}")
    return P, q


def event_pixels(g: Geometry, event, sigma_mask=None):
    """(row-major pixel indices, kernel values) of one event's 3-sigma ellipse."""
    e = np.ascontiguousarray(event, dtype=np.float32).reshape(3)
    sm = None if sigma_mask is None else _f64(sigma_mask)
    n = lib().orc_event_pixels(ctypes.byref(g), _ptr(sm, ctypes.c_double), _ptr(e, ctypes.c_float), 0, None, None)
    if n < 0:
        raise ValueError("oracle event_pixels failed")
    pix = np.empty(n, dtype=np.int64)
    P = np.empty(n, dtype=np.float64)
    lib().orc_event_pixels(ctypes.byref(g), _ptr(sm, ctypes.c_double), _ptr(e, ctypes.c_float), n,
                           _ptr(pix, ctypes.c_int64), _ptr(P, ctypes.c_double))
    return pix, P


def mlem(g: Geometry, events, rho, n_iter: int, s=None, return_D: bool = False):
    """n_iter MLEM iterations from rho (not modified); returns (rho_new, stats[, D of last iteration])."""
    ev = _events(events)
    r = _f64(rho).copy().reshape(g.n_y, g.n_z)
    sv = None if s is None else _f64(s).reshape(g.n_y, g.n_z)
    D = np.zeros(len(ev)) if return_D else None
    st = Stats()
    rc = lib().orc_mlem(ctypes.byref(g), _ptr(ev, ctypes.c_float), len(ev), _ptr(sv, ctypes.c_double),
                        _ptr(r, ctypes.c_double), n_iter, _ptr(D, ctypes.c_double), ctypes.byref(st))
    if rc:
        raise ValueError(f"oracle mlem: error {rc}")
    return (r, st.as_dict(), D) if return_D else (r, st.as_dict())


def loglik_grad(g: Geometry, events, rho, s=None, sigma_mask=None, want_grad_rho=True, return_D=False):
    """(loglik, dl/dsigma_z, dl/dsigma_dl, grad_rho or None, stats[, D])."""
    ev = _events(events)
    r = _f64(rho).reshape(g.n_y, g.n_z)
    sv = None if s is None else _f64(s).reshape(g.n_y, g.n_z)
    sm = None if sigma_mask is None else _f64(sigma_mask)
    out3 = np.zeros(3)
    gr = np.zeros((g.n_y, g.n_z)) if want_grad_rho else None
    D = np.zeros(len(ev)) if return_D else None
    st = Stats()
    rc = lib().orc_loglik_grad(ctypes.byref(g), _ptr(sm, ctypes.c_double), _ptr(ev, ctypes.c_float), len(ev),
                               _ptr(sv, ctypes.c_double), _ptr(r, ctypes.c_double), _ptr(out3, ctypes.c_double),
                               _ptr(gr, ctypes.c_double), _ptr(D, ctypes.c_double), ctypes.byref(st))
    if rc not in (OK, EDOMAIN):
        raise ValueError(f"oracle loglik: error {rc}")
    res = (out3[0], out3[1], out3[2], gr, st.as_dict())
    return res + (D,) if return_D else res


def backprojection_at(g: Geometry, events, rho, pixels):
    """The listing's accumulator sum_j rho_l P_jl / D_j at the given row-major pixel indices."""
    ev = _events(events)
    r = _f64(rho).reshape(-1)
    sel = np.ascontiguousarray(pixels, dtype=np.int64)
    out = np.zeros(len(sel))
    rc = lib().orc_backprojection_at(ctypes.byref(g), _ptr(ev, ctypes.c_float), len(ev), _ptr(r, ctypes.c_double),
                                     len(sel), _ptr(sel, ctypes.c_int64), _ptr(out, ctypes.c_double))
    if rc:
        raise ValueError(f"oracle backprojection_at: error {rc}")
    return out


def denominators_at(g: Geometry, events, rho, event_indices):
    """(D_j, pixel count) of the selected events."""
    ev = _events(events)
    r = _f64(rho).reshape(-1)
    sel = np.ascontiguousarray(event_indices, dtype=np.int64)
    D = np.zeros(len(sel))
    cnt = np.zeros(len(sel), dtype=np.int64)
    rc = lib().orc_denominators_at(ctypes.byref(g), _ptr(ev, ctypes.c_float), len(sel), _ptr(sel, ctypes.c_int64),
                                   _ptr(r, ctypes.c_double), _ptr(D, ctypes.c_double), _ptr(cnt, ctypes.c_int64))
    if rc:
        raise ValueError(f"oracle denominators_at: error {rc}")
    return D, cnt


def initial_image(s: np.ndarray) -> np.ndarray:
    """rho^0 = 1 where the sensitivity is positive, else 0."""
    return (np.asarray(s) > 0).astype(np.float64)
