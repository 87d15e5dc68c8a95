"""Host-side checks of libjpet that need no GPU: the library loads, exports every symbol that
include/jpet.h declares, and validates arguments before touching the device."""

import ctypes
import os
import re

import pytest

from paper_1502_07478_amd import jpet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jpet.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jpet_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(jpet.LIB_PATH):
        from paper_1502_07478_amd import build
        build.build()
    return jpet.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "jpet_mlem_iterate" in names and "jpet_sensitivity" in names and "jpet_loglik_grad" in names
    for name in names:
        assert hasattr(lib, name), name


def test_abi_version_and_strerror(lib):
    assert lib.jpet_abi_version() == 3
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.jpet_strerror(code)
    assert lib.jpet_strerror(-99) == b"unknown status"


def ws_size(g, n):
    b = ctypes.c_size_t(0)
    rc = jpet.lib().jpet_mlem_workspace_size(ctypes.byref(g) if g is not None else None, n, ctypes.byref(b))
    return rc, b.value


GOOD = dict(R=450.0, L=500.0, sigma_z=10.0, sigma_dl=63.0, pixel=2.0, n_y=400, n_z=400)


@pytest.mark.parametrize("over,code", [
    (dict(R=0.0), jpet.JPET_EDOMAIN),
    (dict(R=float("nan")), jpet.JPET_EDOMAIN),
    (dict(L=-1.0), jpet.JPET_EDOMAIN),
    (dict(sigma_z=0.0), jpet.JPET_EDOMAIN),
    (dict(sigma_dl=float("inf")), jpet.JPET_EDOMAIN),
    (dict(pixel=0.0), jpet.JPET_EDOMAIN),
    (dict(n_y=0), jpet.JPET_EDOMAIN),
    (dict(n_z=-5), jpet.JPET_EDOMAIN),
    (dict(n_y=40000), jpet.JPET_EDOMAIN),
    (dict(pixel=2.25), jpet.JPET_EDOMAIN),          # grid reaches |y| >= R
    (dict(kernel_variant=2), jpet.JPET_EDOMAIN),
    (dict(gamma=0.001), jpet.JPET_OK),               # C^-1 positive definite: 2 gamma^2 < u w
    (dict(gamma=-0.001), jpet.JPET_OK),
    (dict(gamma=0.002), jpet.JPET_EDOMAIN),
    (dict(gamma=float("nan")), jpet.JPET_EDOMAIN),
    (dict(sigma_z_edge=0.1), jpet.JPET_OK),          # sigma_z 10% higher at the strip ends
    (dict(sigma_z_edge=1.0), jpet.JPET_OK),
    (dict(sigma_z_edge=-0.1), jpet.JPET_EDOMAIN),
    (dict(sigma_z_edge=1.5), jpet.JPET_EDOMAIN),
    (dict(sigma_z_edge=float("nan")), jpet.JPET_EDOMAIN),
    (dict(gamma=0.00105), jpet.JPET_OK),             # C^-1 positive definite at sigma_z ...
    (dict(gamma=0.00105, sigma_z_edge=0.1), jpet.JPET_EDOMAIN),  # ... but not at 1.1 sigma_z
])
def test_geometry_validation(lib, over, code):
    g = jpet.geometry(**{**GOOD, **over})
    assert ws_size(g, 10)[0] == code


def test_position_dependent_sigma_z(lib):
    """A larger sigma_z at the strip ends widens the plan's ellipse bound; the log-likelihood is
    not defined for it."""
    g0 = jpet.geometry(**GOOD)
    g1 = jpet.geometry(**GOOD, sigma_z_edge=0.4)
    both = {c for c, _ in jpet.plan_candidates(g1, 10**6)}
    code = next(c for c, _ in jpet.plan_candidates(g0, 10**6) if c in both)
    i0 = jpet.launch_info(jpet.with_plan(g0, code), 10**6)
    i1 = jpet.launch_info(jpet.with_plan(g1, code), 10**6)
    assert i1["halo_cols"] > i0["halo_cols"] and i1["lds_bytes"] > i0["lds_bytes"]
    b = ctypes.c_size_t(0)
    assert lib.jpet_loglik_workspace_size(ctypes.byref(g1), None, 10, ctypes.byref(b)) == jpet.JPET_ENOTSUP
    assert lib.jpet_loglik_workspace_size(ctypes.byref(g0), None, 10, ctypes.byref(b)) == jpet.JPET_OK
    assert ctypes.sizeof(jpet.Geometry) == 72


def test_workspace_size_grows_with_events(lib):
    g = jpet.geometry(**GOOD)
    rc0, b0 = ws_size(g, 0)
    rc1, b1 = ws_size(g, 1000)
    assert rc0 == 0 and rc1 == 0 and b1 > b0 > 0
    assert ws_size(g, -1)[0] == jpet.JPET_EINVAL
    assert ws_size(g, 2**31 - 1)[0] == jpet.JPET_OK
    assert ws_size(g, 2**31)[0] == jpet.JPET_EINVAL  # 32-bit event positions on the device
    assert ws_size(None, 10)[0] == jpet.JPET_EINVAL


def test_entry_points_reject_bad_arguments_before_any_device_work(lib):
    g = jpet.geometry(**GOOD)
    gp = ctypes.byref(g)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    aligned_ws = ctypes.c_void_p(0x100000)
    assert lib.jpet_sensitivity(gp, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_sensitivity(None, fake, None) == jpet.JPET_EINVAL
    # negative event count, NULL events with n > 0, NULL rho, negative iterations, unknown flags
    assert lib.jpet_mlem_iterate(gp, fake, -1, None, fake, 1, aligned_ws, 1 << 40, 0, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_iterate(gp, None, 5, None, fake, 1, aligned_ws, 1 << 40, 0, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_iterate(gp, fake, 5, None, None, 1, aligned_ws, 1 << 40, 0, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_iterate(gp, fake, 5, None, fake, -1, aligned_ws, 1 << 40, 0, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_iterate(gp, fake, 5, None, fake, 1, aligned_ws, 1 << 40, 8, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_iterate(gp, fake, 5, None, fake, 1, aligned_ws, 1 << 40, 6, None, None) == jpet.JPET_EINVAL
    # workspace: NULL, misaligned, too small
    assert lib.jpet_mlem_iterate(gp, fake, 5, None, fake, 1, None, 1 << 40, 0, None, None) == jpet.JPET_EWORKSPACE
    assert lib.jpet_mlem_iterate(gp, fake, 5, None, fake, 1, ctypes.c_void_p(0x100004), 1 << 40, 0, None,
                                 None) == jpet.JPET_EWORKSPACE
    assert lib.jpet_mlem_iterate(gp, fake, 5, None, fake, 1, aligned_ws, 16, 0, None, None) == jpet.JPET_EWORKSPACE
    assert lib.jpet_mlem_prepare(gp, fake, 5, aligned_ws, 16, None) == jpet.JPET_EWORKSPACE
    # log-likelihood: NULL out3, bad mask sigma
    assert lib.jpet_loglik_grad(gp, None, fake, 5, None, fake, None, None, None, aligned_ws, 1 << 40, 0, None,
                                None) == jpet.JPET_EINVAL
    bad_mask = (ctypes.c_double * 2)(0.0, 63.0)
    assert lib.jpet_loglik_grad(gp, bad_mask, fake, 5, None, fake, fake, None, None, aligned_ws, 1 << 40, 0, None,
                                None) == jpet.JPET_EDOMAIN
    # direct image: NULL image, negative count, NULL events with n > 0
    assert lib.jpet_direct_image(gp, fake, 5, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_direct_image(gp, fake, -1, fake, None) == jpet.JPET_EINVAL
    assert lib.jpet_direct_image(gp, None, 5, fake, None) == jpet.JPET_EINVAL
    # log-likelihood workspace size: NULL output, negative count, bad mask
    b = ctypes.c_size_t(0)
    assert lib.jpet_loglik_workspace_size(gp, None, 5, None) == jpet.JPET_EINVAL
    assert lib.jpet_loglik_workspace_size(gp, None, -1, ctypes.byref(b)) == jpet.JPET_EINVAL
    assert lib.jpet_loglik_workspace_size(gp, bad_mask, 5, ctypes.byref(b)) == jpet.JPET_EDOMAIN
    assert lib.jpet_loglik_workspace_size(gp, None, 5, ctypes.byref(b)) == jpet.JPET_OK and b.value > 0
    # back-projection into a caller accumulator: NULL accumulator, NULL rho, unknown flags, workspace
    assert lib.jpet_mlem_backproject(gp, fake, 5, fake, None, aligned_ws, 1 << 40, 0, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_backproject(gp, fake, 5, None, fake, aligned_ws, 1 << 40, 0, None, None) == jpet.JPET_EINVAL
    for bad_flags in (8, 6):  # unknown flag; both comparison work splits at once
        assert lib.jpet_mlem_backproject(gp, fake, 5, fake, fake, aligned_ws, 1 << 40, bad_flags, None,
                                         None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_backproject(gp, fake, 5, fake, fake, aligned_ws, 16, 0, None, None) == jpet.JPET_EWORKSPACE
    assert lib.jpet_mlem_update(gp, None, None, fake, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_update(gp, None, fake, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_update(None, None, fake, fake, None) == jpet.JPET_EINVAL


def test_denominators_validation(lib):
    g = jpet.geometry(**GOOD)
    gp = ctypes.byref(g)
    fake = ctypes.c_void_p(0x1000)
    aligned_ws = ctypes.c_void_p(0x100000)
    # NULL D_out with events, NULL rho, unknown flags, small workspace
    assert lib.jpet_mlem_denominators(gp, fake, 5, fake, None, aligned_ws, 1 << 40, 0, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_denominators(gp, fake, 5, None, fake, aligned_ws, 1 << 40, 0, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_denominators(gp, fake, 5, fake, fake, aligned_ws, 1 << 40, 8, None, None) == jpet.JPET_EINVAL
    assert lib.jpet_mlem_denominators(gp, fake, 5, fake, fake, aligned_ws, 16, 0, None, None) == jpet.JPET_EWORKSPACE


def test_plan_candidates_and_named_plans(lib):
    """Plans that fit come back sorted by the cost model; plan 0 is the first; a named plan is used
    as named; malformed codes are EINVAL, plans that do not fit the geometry EDOMAIN."""
    g = jpet.geometry(**GOOD)
    n = 10_000_000
    cands = jpet.plan_candidates(g, n)
    assert len(cands) > 20
    costs = [c for _, c in cands]
    assert costs == sorted(costs)
    assert len({code for code, _ in cands}) == len(cands)
    assert jpet.launch_info(g, n)["plan"] == cands[0][0]
    for code, _ in cands[:: max(1, len(cands) // 7)]:
        info = jpet.launch_info(jpet.with_plan(g, code), n)
        assert info["plan"] == code and info["binned"] == 1
        assert info["waves"] == (16 if code & 3 == 2 else 8)
        assert info["accumulator_bits"] == (32 if code & 4 else 64)
        assert info["workgroups_per_cu"] == (code >> 3) & 7
        assert (info["t_bins"] == 1) == ((code >> 6) & 7 == 0)
        assert info["tile_rows"] == [32, 24, 16, 12, 8][(code >> 9) & 7]
        assert ws_size(jpet.with_plan(g, code), n)[0] == jpet.JPET_OK
    # the generic pass can always be named
    assert jpet.launch_info(jpet.with_plan(g, 3), n)["binned"] == 0
    # malformed codes
    for bad in (-1, 4, 1 | (5 << 3), 1 | (1 << 3) | (6 << 6), 1 | (1 << 3) | (5 << 9), 1 | (1 << 3) | (3 << 12),
                1 | (1 << 3) | (1 << 14), 7):
        assert ws_size(jpet.with_plan(g, bad), n)[0] == jpet.JPET_EINVAL, bad
    # well formed but too large for the LDS: 64-bit accumulators, one 32-row tile, no shear,
    # four workgroups per CU
    big = 1 | (4 << 3) | (0 << 6) | (0 << 9)
    assert big not in {c for c, _ in cands}
    assert ws_size(jpet.with_plan(g, big), n)[0] == jpet.JPET_EDOMAIN
    # log-likelihood plans: 64-bit accumulators only
    ll = jpet.plan_candidates(g, n, loglik=True)
    assert ll and all(code & 4 == 0 for code, _ in ll)
    b = ctypes.c_size_t(0)
    acc32 = next(code for code, _ in cands if code & 4)
    assert lib.jpet_loglik_workspace_size(ctypes.byref(jpet.with_plan(g, acc32)), None, n,
                                          ctypes.byref(b)) == jpet.JPET_EDOMAIN
    # rows of more than 64 pixels (twice the largest cache that is split): only the generic pass
    fine = jpet.geometry(**{**GOOD, "sigma_z": 12.0, "pixel": 0.5})
    assert jpet.plan_candidates(fine, 1000) == [(3, 0.0)]
    # rows of 33..64 pixels: whole rows in a 48/64 cache, or split in two 32-pixel segments
    mid = jpet.geometry(**{**GOOD, "sigma_z": 10.0, "pixel": 0.9})
    mc = jpet.plan_candidates(mid, 10**6)
    caches = {(code >> 12) & 3 for code, _ in mc}
    assert caches == {0, 2}
    split = next(code for code, _ in mc if (code >> 12) & 3 == 2)
    info = jpet.launch_info(jpet.with_plan(mid, split), 10**6)
    assert info["row_cache"] == 32 and info["row_segments"] == 2
    whole = next(code for code, _ in mc if (code >> 12) & 3 == 0)
    info = jpet.launch_info(jpet.with_plan(mid, whole), 10**6)
    assert info["row_cache"] in (48, 64) and info["row_segments"] == 1


def test_binding_requires_built_library(monkeypatch, tmp_path):
    """The binding fails loudly (no fallback) when the library is missing."""
    monkeypatch.setattr(jpet, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(jpet, "_L", None)
    with pytest.raises(RuntimeError, match="not built"):
        jpet.lib()


def test_tuner_times_every_plan_family(lib):
    """The tuner's candidate list: the cost model's leading plans, then the best-ranked plan of each
    family (register cache, row segments, wavefronts) that has none among them, each once."""
    from paper_1502_07478_amd import tune
    from jpet_synth import get_workload
    w = get_workload("large1024")
    g = jpet.geometry(**w.geometry())
    n = 8_000_000
    ranked = [c for c, _ in jpet.plan_candidates(g, n)]

    def family(c):
        li = jpet.launch_info(jpet.with_plan(g, c), n)
        return li["row_cache"], li["row_segments"], li["waves"]

    codes = tune.with_families(g, ranked, n, 4)
    assert codes[:4] == ranked[:4]
    assert len(set(codes)) == len(codes)
    fams = [family(c) for c in codes]
    assert set(fams) == {family(c) for c in ranked}
    # each added code is its family's best-ranked one
    for c, f in zip(codes[4:], fams[4:]):
        assert f not in fams[:4]
        assert ranked.index(c) == min(i for i, r in enumerate(ranked) if family(r) == f)
