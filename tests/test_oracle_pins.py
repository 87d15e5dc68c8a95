"""Pins of the double-precision oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
closed forms, symmetries, brute force, numerical quadrature of the defining
integral, dense-matrix linear algebra, exact invariants of the EM update and
finite differences.  Together they are chosen so that a plausible mistake in
any step of the oracle (a dropped term, a wrong sign or index, a transposed
operand, a wrong prefactor) fails at least one of them.
"""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from jpet_synth import get_workload

R, L = 450.0, 500.0


def geom(sz=10.0, sdl=63.0, pixel=2.0, n=400, variant=0, **kw):
    return oracle.geometry(R, kw.pop("L", L), sz, sdl, pixel, n, kw.pop("n_z", n), kernel_variant=variant, **kw)


# --------------------------------------------------------------------------------------------
# Eq. 1 / Eq. 2: direct reconstruction inverts the measurement model


def forward_eq1(y, z, theta, R=R):
    """Eq. 1 written out for a true emission point: strip hits and path-length difference."""
    t = math.tan(theta)
    zu = z + (R - y) * t
    zd = z - (R + y) * t
    dl = math.sqrt((R - y) ** 2 + (zu - z) ** 2) - math.sqrt((R + y) ** 2 + (zd - z) ** 2)
    return zu, zd, dl


def test_direct_reconstruction_inverts_eq1():
    g = geom()
    rng = np.random.default_rng(1)
    for _ in range(2000):
        y, z = rng.uniform(-400, 400), rng.uniform(-400, 400)
        th = rng.uniform(-1.2, 1.2)
        zu, zd, dl = forward_eq1(y, z, th)
        t, c, yt, zt = oracle.direct(g, zu, zd, dl)
        assert t == pytest.approx(math.tan(th), abs=1e-12)
        assert c == pytest.approx(1.0 / math.cos(th), rel=1e-12)
        assert yt == pytest.approx(y, abs=1e-9)
        assert zt == pytest.approx(z, abs=1e-9)


def test_printed_second_form_of_y_is_not_an_inverse():
    """Documents reading R1: the alternative printed forms of y~ do not invert Eq. 1."""
    zu, zd, dl = forward_eq1(100.0, 40.0, 0.3)
    second = 2 * R * dl / math.sqrt(zu - zd + 4 * R * R)
    t, c, yt, zt = oracle.direct(geom(), zu, zd, dl)
    assert yt == pytest.approx(100.0, abs=1e-9)
    assert abs(second - 100.0) > 50.0


# --------------------------------------------------------------------------------------------
# Eq. 4: sensitivity


def test_sensitivity_centre_closed_form():
    g = geom()
    assert oracle.sensitivity_point(g, 0.0, 0.0) == pytest.approx(2.0 / math.pi * math.atan(L / (2 * R)), rel=1e-14)


def test_sensitivity_symmetry_and_support():
    g = geom()
    rng = np.random.default_rng(2)
    for _ in range(500):
        y, z = rng.uniform(-440, 440), rng.uniform(-300, 300)
        s = oracle.sensitivity_point(g, y, z)
        assert oracle.sensitivity_point(g, -y, z) == pytest.approx(s, abs=1e-15)
        assert oracle.sensitivity_point(g, y, -z) == pytest.approx(s, abs=1e-15)
        if abs(z) >= L / 2:
            assert s == 0.0
        else:
            assert 0.0 < s < 1.0


def test_sensitivity_brute_force_over_angles():
    """Fraction of a dense uniform theta grid whose line hits both strips."""
    g = geom()
    th = (np.arange(4_000_000) + 0.5) / 4_000_000 * math.pi - math.pi / 2
    t = np.tan(th)
    for (y, z) in [(100.0, 37.0), (-150.0, 120.0), (0.0, 0.0), (399.0, -240.0), (-420.0, 10.0)]:
        zu = z + (R - y) * t
        zd = z - (R + y) * t
        frac = np.mean((np.abs(zu) <= L / 2) & (np.abs(zd) <= L / 2))
        assert oracle.sensitivity_point(g, y, z) == pytest.approx(frac, abs=2e-6)


def test_sensitivity_image_is_pointwise():
    g = geom(pixel=4.0, n=64)
    s = oracle.sensitivity(g)
    # pixel (i, k) has its centre at ((i + 1/2 - n/2) p, (k + 1/2 - n/2) p)
    for (i, k) in [(0, 0), (10, 50), (63, 63), (31, 32)]:
        y = (i + 0.5 - 32) * 4.0
        z = (k + 0.5 - 32) * 4.0
        assert s[i, k] == oracle.sensitivity_point(g, y, z)


# --------------------------------------------------------------------------------------------
# Appendix B: bounding box of the 3-sigma ellipse


def bcb(dy, dz, t, c, sz, sdl):
    """b C^-1 b with b of Eq. 10 and the diagonal C^-1 of Eq. 12."""
    b1 = dz - dy * t
    b3 = -2.0 * dy * c
    return (b1 * b1 + b1 * b1) / sz ** 2 + b3 * b3 / sdl ** 2


@pytest.mark.parametrize("sz,sdl", [(10.0, 63.0), (5.0, 30.0), (15.0, 90.0)])
def test_box_closed_forms_and_brute_force(sz, sdl):
    for t in [0.0, 0.15, -0.3, 0.55, 1.1]:
        c = math.sqrt(1 + t * t)
        hy, hz = oracle.box_halfsize(sz, sdl, t, c)
        assert hy == pytest.approx(1.5 * sdl / c, rel=1e-12)
        assert hz == pytest.approx(3.0 * math.sqrt(sz ** 2 / 2 + sdl ** 2 * (t / c) ** 2 / 4), rel=1e-12)
        # brute force: extent of {q <= 9} on a fine grid equals the box to the grid step
        step = min(hy, hz) / 400
        dy = np.arange(-1.2 * hy, 1.2 * hy, step)
        dz = np.arange(-1.2 * hz, 1.2 * hz, step)
        Y, Z = np.meshgrid(dy, dz, indexing="ij")
        inside = bcb(Y, Z, t, c, sz, sdl) <= 9.0
        assert np.abs(Y[inside]).max() == pytest.approx(hy, abs=2 * step)
        assert np.abs(Z[inside]).max() == pytest.approx(hz, abs=2 * step)
        assert np.abs(Y[inside]).max() <= hy and np.abs(Z[inside]).max() <= hz


def test_event_pixels_are_exactly_the_ellipse():
    """Brute force over the whole grid: the oracle's pixel set equals {pixel centres with q <= 9}."""
    g = geom(pixel=2.0, n=400)
    ev = get_workload("prod400").events(200)
    n = 400
    yc = (np.arange(n) + 0.5 - n / 2) * 2.0
    Y, Z = np.meshgrid(yc, yc, indexing="ij")
    for e in ev[:60]:
        t, c, yt, zt = oracle.direct(g, *map(float, e))
        want = np.nonzero((bcb(Y - yt, Z - zt, t, c, 10.0, 63.0) <= 9.0).ravel())[0]
        pix, P = oracle.event_pixels(g, e)
        assert np.array_equal(np.sort(pix), want)
        assert np.all(np.diff(pix) > 0), "pixels are visited in row-major order"
        assert np.all(P > 0)


# --------------------------------------------------------------------------------------------
# Eq. 7: the kernel is the Laplace form of the angular integral of a 3-D Gaussian


def exact_kernel(ev, y, z, sz, sdl):
    """int dtheta N3(e - f(y, z, theta); C) with f the forward model of Eq. 1."""
    u, w = 1 / sz ** 2, 1 / sdl ** 2
    norm = u * math.sqrt(w) / (2 * math.pi) ** 1.5

    def f(th):
        zu, zd, dl = forward_eq1(y, z, th)
        d0, d1, d2 = ev[0] - zu, ev[1] - zd, ev[2] - dl
        return norm * math.exp(-0.5 * (u * d0 * d0 + u * d1 * d1 + w * d2 * d2))

    th0 = math.atan((ev[0] - ev[1]) / (2 * R))
    val, _ = integrate.quad(f, -math.pi / 2 + 1e-9, math.pi / 2 - 1e-9, points=[th0], limit=400,
                            epsabs=0, epsrel=1e-11)
    return val


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("sz,sdl", [(10.0, 63.0), (5.0, 30.0)])
def test_kernel_matches_angular_quadrature(variant, sz, sdl):
    g = geom(sz, sdl, variant=variant)
    rng = np.random.default_rng(5)
    errs = []
    while len(errs) < 200:
        y, z = rng.uniform(-200, 200), rng.uniform(-150, 150)
        th = rng.uniform(-0.45, 0.45)
        zu, zd, dl = forward_eq1(y, z, th)
        ev = np.array([zu + rng.normal() * sz, zd + rng.normal() * sz, dl + rng.normal() * sdl])
        P, q = oracle.kernel_points(g, ev, y, z)
        if q[0] > 9:
            continue
        errs.append(P[0] / exact_kernel(ev, y, z, sz, sdl) - 1)
    errs = np.abs(np.array(errs))
    # Laplace approximation error: measured median ~5e-4, p95 ~7e-3 at these resolutions
    assert np.median(errs) < 2e-3
    assert np.percentile(errs, 95) < 1.5e-2
    assert errs.max() < 4e-2


def taylor(fun, x0, order, radius=2e-3, m=64):
    """Taylor coefficients c_0..c_order of an analytic function at x0 (Cauchy integral, trapezoid rule)."""
    phi = 2 * np.pi * np.arange(m) / m
    vals = np.array([fun(x0 + radius * np.exp(1j * p)) for p in phi])
    out = []
    for k in range(order + 1):
        ck = np.tensordot(np.exp(-1j * k * phi), vals, axes=(0, 0)) / m / radius ** k
        out.append(np.real(ck))
    return out


def forward_vec(y, z, th):
    """f(theta) = (z_u, z_d, dl) of a point (y, z) along direction theta (Eq. 1), analytic in theta."""
    t = np.tan(th)
    zu = z + (R - y) * t
    zd = z - (R + y) * t
    dl = np.sqrt((R - y) ** 2 + (zu - z) ** 2) - np.sqrt((R + y) ** 2 + (zd - z) ** 2)
    return np.array([zu, zd, dl])


@pytest.mark.parametrize("variant", [0, 1])
def test_kernel_is_the_second_order_laplace_form(variant):
    """Eq. 7 is exactly the Gaussian integral over delta of exp(g0 + g1 d + g2 d^2), where g is the
    exponent of N3(e - f(theta~ + d); C) expanded to second order in d, f is the forward model of
    Eq. 1 and theta~ the reconstructed angle.  The Taylor coefficients of f are computed
    numerically here; variant 0 takes the third component of f' at half its value (as printed)."""
    rng = np.random.default_rng(11)
    for sz, sdl in [(10.0, 63.0), (5.0, 30.0), (14.0, 85.0)]:
        g = geom(sz, sdl, variant=variant)
        Cinv = np.diag([1 / sz ** 2, 1 / sz ** 2, 1 / sdl ** 2])
        for _ in range(60):
            y, z = rng.uniform(-300, 300), rng.uniform(-200, 200)
            th = rng.uniform(-0.5, 0.5)
            ev = forward_vec(y, z, th) + rng.normal(size=3) * [sz, sz, sdl]
            th_t = math.atan((ev[0] - ev[1]) / (2 * R))
            f0, f1, f2 = taylor(lambda x: forward_vec(y, z, x), th_t, 2)
            if variant == 0:
                f1 = f1 * np.array([1.0, 1.0, 0.5])
            r0 = f0 - ev
            g0 = -0.5 * r0 @ Cinv @ r0
            g1 = -(f1 @ Cinv @ r0)
            g2 = -0.5 * (f1 @ Cinv @ f1 + 2 * f2 @ Cinv @ r0)
            norm = math.sqrt(np.linalg.det(Cinv)) / (2 * math.pi) ** 1.5
            want = norm * math.exp(g0 - g1 * g1 / (4 * g2)) * math.sqrt(math.pi / -g2)
            P, q = oracle.kernel_points(g, ev, y, z)
            assert q[0] == pytest.approx(-2 * g0, rel=1e-9, abs=1e-9)
            assert P[0] == pytest.approx(want, rel=1e-8)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("gfrac", [0.4, -0.7])
def test_kernel_with_offdiagonal_cinv_is_the_laplace_form(variant, gfrac):
    """The same exact second-order Laplace form with the full C^-1 of Eq. 12,
    [[u, 0, g], [0, u, -g], [g, -g, w]], g = gfrac sqrt(u w / 2) (inside the positive-definite
    range); the oracle's kernel must follow the off-diagonal terms through kappa, b C^-1 a and the
    determinant, and its ellipse test (b C^-1 b) must not change."""
    rng = np.random.default_rng(13)
    for sz, sdl in [(10.0, 63.0), (5.0, 30.0)]:
        u, w = 1 / sz ** 2, 1 / sdl ** 2
        gam = gfrac * math.sqrt(u * w / 2)
        g = geom(sz, sdl, variant=variant, gamma=gam)
        Cinv = np.array([[u, 0.0, gam], [0.0, u, -gam], [gam, -gam, w]])
        for _ in range(40):
            y, z = rng.uniform(-300, 300), rng.uniform(-200, 200)
            th = rng.uniform(-0.5, 0.5)
            ev = forward_vec(y, z, th) + rng.normal(size=3) * [sz, sz, sdl]
            th_t = math.atan((ev[0] - ev[1]) / (2 * R))
            f0, f1, f2 = taylor(lambda x: forward_vec(y, z, x), th_t, 2)
            if variant == 0:
                f1 = f1 * np.array([1.0, 1.0, 0.5])
            r0 = f0 - ev
            g0 = -0.5 * r0 @ Cinv @ r0
            g1 = -(f1 @ Cinv @ r0)
            g2 = -0.5 * (f1 @ Cinv @ f1 + 2 * f2 @ Cinv @ r0)
            norm = math.sqrt(np.linalg.det(Cinv)) / (2 * math.pi) ** 1.5
            want = norm * math.exp(g0 - g1 * g1 / (4 * g2)) * math.sqrt(math.pi / -g2)
            P, q = oracle.kernel_points(g, ev, y, z)
            assert q[0] == pytest.approx(-2 * g0, rel=1e-9, abs=1e-9)
            assert P[0] == pytest.approx(want, rel=1e-8)


@pytest.mark.parametrize("y,z", [(100.0, 37.0), (-150.0, 120.0), (60.0, -200.0)])
def test_kernel_integrates_to_pi_times_sensitivity(y, z):
    """3-D quadrature over measured events on the strips: int P de = pi s(y, z)."""
    sz, sdl = 10.0, 63.0
    g = geom(sz, sdl)
    hz, hd = sz / 4, sdl / 6
    zu = np.arange(-L / 2 + hz / 2, L / 2, hz)
    thmax = math.atan(max((L / 2 + abs(z)) / (R - abs(y)), 1.0))
    dls = np.arange(-2 * abs(y) / math.cos(thmax) - 6 * sdl, 2 * abs(y) / math.cos(thmax) + 6 * sdl, hd)
    U, D = np.meshgrid(zu, zu, indexing="ij")
    total = 0.0
    for d in dls:
        ev = np.stack([U.ravel(), D.ravel(), np.full(U.size, d)], 1)
        P, _ = oracle.kernel_points(g, ev, y, z)
        total += P.sum()
    total *= hz * hz * hd
    assert total / math.pi == pytest.approx(oracle.sensitivity_point(g, y, z), rel=1e-3)


# --------------------------------------------------------------------------------------------
# MLEM: dense-matrix brute force and invariants


def small_problem(n_events=50, seed=7, variant=0):
    g = oracle.geometry(R, L, 10.0, 63.0, 8.0, 10, 12, kernel_variant=variant)
    rng = np.random.default_rng(seed)
    ev = []
    while len(ev) < n_events:
        y, z = rng.uniform(-40, 40), rng.uniform(-48, 48)
        th = rng.uniform(-0.4, 0.4)
        zu, zd, dl = forward_eq1(y, z, th)
        e = [zu + rng.normal() * 10, zd + rng.normal() * 10, dl + rng.normal() * 63]
        if abs(e[0]) <= L / 2 and abs(e[1]) <= L / 2:
            ev.append(e)
    ev.append([260.0, 0.0, 0.0])          # off the strip: dropped
    ev.append([251.0, -240.0, 0.0])       # off the strip although its ellipse covers the grid: dropped
    ev.append([float("nan"), 0.0, 0.0])   # not finite: dropped
    ev.append([0.0, 0.0, 800.0])          # ellipse far outside the grid: dropped
    return g, np.asarray(ev, dtype=np.float32)


def dense_matrix(g, ev):
    P = np.zeros((len(ev), g.n_y * g.n_z))
    for j, e in enumerate(ev):
        pix, val = oracle.event_pixels(g, e)
        P[j, pix] = val
    return P


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("with_s", [True, False])
def test_mlem_matches_dense_matrix_em(variant, with_s):
    g, ev = small_problem(variant=variant)
    P = dense_matrix(g, ev)
    s = oracle.sensitivity(g).ravel()
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, g.n_y * g.n_z)
    want = rho.copy()
    for _ in range(3):
        D = P @ want
        keep = D > 0
        B = P[keep].T @ (1.0 / D[keep])
        want = want * B / (s if with_s else 1.0)
    got, st = oracle.mlem(g, ev, rho, 3, s=s if with_s else None)
    np.testing.assert_allclose(got.ravel(), want, rtol=1e-12, atol=1e-14)
    assert st["n_dropped"] == 4
    assert st["n_valid"] == len(ev) - 4
    assert st["n_pairs"] == int((P > 0).sum())


def test_mlem_zero_denominator_events_are_skipped():
    g, ev = small_problem()
    s = oracle.sensitivity(g)
    rho = np.zeros_like(s)
    rho[0, 0] = 1.0  # most events do not see pixel (0, 0)
    got, st = oracle.mlem(g, ev, rho, 1, s=s)
    assert st["n_zero_denominator"] > 0
    assert np.all(np.isfinite(got))
    assert (s * got).sum() == pytest.approx(st["n_valid"] - st["n_zero_denominator"], rel=1e-12)


@pytest.fixture(scope="module")
def tiny():
    w = get_workload("tiny")
    g = oracle.geometry(**w.geometry())
    ev = w.events(4000)
    s = oracle.sensitivity(g)
    return g, ev, s


def test_count_conservation(tiny):
    g, ev, s = tiny
    rho = oracle.initial_image(s)
    for _ in range(3):
        rho, st = oracle.mlem(g, ev, rho, 1, s=s)
        assert (s * rho).sum() == pytest.approx(st["n_valid"] - st["n_zero_denominator"], rel=1e-12)
    # Eq. 5 form: no sensitivity, sum rho' = number of events
    rp, st = oracle.mlem(g, ev, s * oracle.initial_image(s), 2)
    assert rp.sum() == pytest.approx(st["n_valid"] - st["n_zero_denominator"], rel=1e-12)


def test_loglik_increases_monotonically(tiny):
    g, ev, s = tiny
    rho = oracle.initial_image(s)
    prev = oracle.loglik_grad(g, ev, rho, s=s, want_grad_rho=False)[0]
    for _ in range(5):
        rho, _ = oracle.mlem(g, ev, rho, 1, s=s)
        cur = oracle.loglik_grad(g, ev, rho, s=s, want_grad_rho=False)[0]
        assert cur >= prev - 1e-9 * abs(prev)
        prev = cur


def test_em_step_is_gradient_step(tiny):
    """rho^{t+1} = rho^t + (rho^t / s) dl/drho ties the update to the gradient."""
    g, ev, s = tiny
    rho = oracle.initial_image(s) * np.random.default_rng(4).uniform(0.5, 1.5, s.shape)
    nxt, _ = oracle.mlem(g, ev, rho, 1, s=s)
    _, _, _, grad, _ = oracle.loglik_grad(g, ev, rho, s=s)
    pos = s > 0
    np.testing.assert_allclose(nxt[pos], rho[pos] + rho[pos] / s[pos] * grad[pos], rtol=1e-10, atol=1e-12)


def test_loglik_value_against_dense_matrix():
    g, ev = small_problem()
    P = dense_matrix(g, ev)
    s = oracle.sensitivity(g).ravel()
    rho = np.random.default_rng(8).uniform(0.5, 2.0, g.n_y * g.n_z)
    D = P @ rho
    valid = P.sum(axis=1) > 0
    want = np.sum(np.log(D[valid] / math.pi)) - np.dot(s, rho)
    got = oracle.loglik_grad(g, ev, rho, s=s)
    assert got[0] == pytest.approx(want, rel=1e-13)
    Bwant = P[valid].T @ (1.0 / D[valid])
    np.testing.assert_allclose(got[3].ravel(), Bwant - s, rtol=1e-12, atol=1e-13)


def test_loglik_zero_denominator_is_minus_infinity():
    g, ev = small_problem()
    rho = np.zeros((g.n_y, g.n_z))
    res = oracle.loglik_grad(g, ev, rho, s=oracle.sensitivity(g))
    assert res[0] == -math.inf


# --------------------------------------------------------------------------------------------
# direct-reconstruction image: exact events of known points land in the points' pixels


def test_direct_image_counts_points_of_exact_events():
    """Noise-free events of points placed inside known pixels (Eq. 1 forward model, stored in
    float32) must be counted in exactly those pixels; invalid events and points beyond the grid
    are not counted."""
    g = geom(10.0, 63.0, pixel=4.0, n=64, n_z=80)
    rng = np.random.default_rng(21)
    want = np.zeros((g.n_y, g.n_z))
    rows = []
    while len(rows) < 3000:
        i, k = rng.integers(0, g.n_y), rng.integers(0, g.n_z)
        y = (i + 0.5 - g.n_y / 2 + rng.uniform(-0.4, 0.4)) * g.pixel
        z = (k + 0.5 - g.n_z / 2 + rng.uniform(-0.4, 0.4)) * g.pixel
        th = rng.uniform(-0.6, 0.6)
        zu, zd, dl = forward_eq1(y, z, th)
        if abs(zu) > L / 2 or abs(zd) > L / 2:
            continue
        rows.append((zu, zd, dl))
        want[i, k] += 1
    extra = [(np.nan, 0.0, 0.0), (L, 0.0, 0.0), (0.0, 0.0, 2 * 1e4)]  # non-finite, off strip, y beyond R
    ev = np.array(rows + extra, dtype=np.float32)
    img, counted = oracle.direct_image(g, ev)
    assert counted == len(rows)
    np.testing.assert_array_equal(img, want)


# --------------------------------------------------------------------------------------------
# gradient: central finite differences with the ellipse mask held fixed


@pytest.mark.parametrize("variant,gamma", [(0, 0.0), (1, 0.0), (0, 5e-4)])
def test_sigma_gradient_matches_finite_differences(tiny, variant, gamma):
    g0, ev, s = tiny
    rho = oracle.initial_image(s)
    rho, _ = oracle.mlem(g0, ev, rho, 2, s=s)
    sz, sdl = g0.sigma_z, g0.sigma_dl

    def ll(a, b):
        g = oracle.geometry(g0.R, g0.L, a, b, g0.pixel, g0.n_y, g0.n_z, kernel_variant=variant, gamma=gamma)
        return oracle.loglik_grad(g, ev, rho, s=s, sigma_mask=[sz, sdl], want_grad_rho=False)

    base = ll(sz, sdl)
    hz, hd = 1e-3 * sz, 1e-3 * sdl
    fd_z = (ll(sz + hz, sdl)[0] - ll(sz - hz, sdl)[0]) / (2 * hz)
    fd_d = (ll(sz, sdl + hd)[0] - ll(sz, sdl - hd)[0]) / (2 * hd)
    assert base[1] == pytest.approx(fd_z, rel=1e-5)
    assert base[2] == pytest.approx(fd_d, rel=1e-5)


def test_rho_gradient_matches_finite_differences(tiny):
    g, ev, s = tiny
    rho = oracle.initial_image(s) * np.random.default_rng(9).uniform(0.5, 1.5, s.shape)
    _, _, _, grad, _ = oracle.loglik_grad(g, ev, rho, s=s)
    rng = np.random.default_rng(10)
    flat = rho.ravel()
    for p in rng.choice(np.nonzero(flat > 0)[0], 8, replace=False):
        h = 1e-4 * flat[p]
        up, dn = flat.copy(), flat.copy()
        up[p] += h
        dn[p] -= h
        fd = (oracle.loglik_grad(g, ev, up, s=s, want_grad_rho=False)[0] -
              oracle.loglik_grad(g, ev, dn, s=s, want_grad_rho=False)[0]) / (2 * h)
        assert grad.ravel()[p] == pytest.approx(fd, rel=1e-6, abs=1e-6)


# --------------------------------------------------------------------------------------------
# sampled helpers agree with the full iteration


def test_sampled_helpers_agree_with_full_iteration(tiny):
    g, ev, s = tiny
    rho = oracle.initial_image(s)
    nxt, st, D = oracle.mlem(g, ev, rho, 1, s=s, return_D=True)
    sel = np.array([5, 100, 2047, 3999])
    Ds, cnt = oracle.denominators_at(g, ev, rho, sel)
    np.testing.assert_allclose(Ds, D[sel], rtol=1e-14)
    pix = np.array([32 * 64 + 30, 20 * 64 + 40, 50 * 64 + 10])
    acc = oracle.backprojection_at(g, ev, rho, pix)
    np.testing.assert_allclose(acc / s.ravel()[pix], nxt.ravel()[pix], rtol=1e-12)


# --------------------------------------------------------------------------------------------
# sigma_z depending on the hit positions (Sec. 3 after Eq. 12): one sigma_z per event,
# sigma_z (1 + edge * zeta) with zeta the mean of (z / (L/2))^2 over the two measured hits


def event_sigma_z(sz, edge, zu, zd):
    return sz * (1.0 + edge * 0.5 * ((zu / (L / 2)) ** 2 + (zd / (L / 2)) ** 2))


def test_sigma_z_factor_is_lowest_at_the_centre_and_highest_at_the_ends():
    g = geom(sigma_z_edge=0.1)
    assert oracle.sigma_z_factor(g, 0.0, 0.0) == 1.0
    assert oracle.sigma_z_factor(g, L / 2, -L / 2) == pytest.approx(1.1, rel=1e-15)
    zs = np.linspace(0.0, L / 2, 11)
    f = [oracle.sigma_z_factor(g, z, z) for z in zs]
    assert np.all(np.diff(f) > 0)
    assert oracle.sigma_z_factor(g, 100.0, -30.0) == oracle.sigma_z_factor(g, -30.0, 100.0)
    assert oracle.sigma_z_factor(geom(), 200.0, 100.0) == 1.0
    for bad in (-0.1, 1.5, float("nan")):
        assert oracle.lib().orc_check_geometry(geom(sigma_z_edge=bad)) == oracle.EDOMAIN


@pytest.mark.parametrize("edge", [0.1, 0.4])
def test_position_dependent_kernel_matches_angular_quadrature(edge):
    """The kernel of an event is the angular integral of the 3-D Gaussian at that event's sigma_z."""
    sz, sdl = 10.0, 63.0
    g = geom(sz, sdl, sigma_z_edge=edge)
    rng = np.random.default_rng(17)
    errs = []
    while len(errs) < 120:
        y, z = rng.uniform(-200, 200), rng.uniform(-150, 150)
        th = rng.uniform(-0.5, 0.5)
        zu, zd, dl = forward_eq1(y, z, th)
        ev = np.array([zu + rng.normal() * sz, zd + rng.normal() * sz, dl + rng.normal() * sdl])
        if max(abs(ev[0]), abs(ev[1])) > L / 2:
            continue
        P, q = oracle.kernel_points(g, ev, y, z)
        if q[0] > 9:
            continue
        errs.append(P[0] / exact_kernel(ev, y, z, event_sigma_z(sz, edge, ev[0], ev[1]), sdl) - 1)
    errs = np.abs(np.array(errs))
    assert np.median(errs) < 2e-3
    assert np.percentile(errs, 95) < 1.5e-2


def test_position_dependent_pixels_are_exactly_the_event_ellipse():
    """Brute force: the pixel set is {pixel centres with q <= 9} at the event's own sigma_z, and
    the kernel values equal those of a constant-resolution geometry at that sigma_z."""
    edge = 0.1
    g = geom(pixel=2.0, n=400, sigma_z_edge=edge)
    ev = get_workload("edge400").events(200)
    n = 400
    yc = (np.arange(n) + 0.5 - n / 2) * 2.0
    Y, Z = np.meshgrid(yc, yc, indexing="ij")
    grew = 0
    for e in ev[:60]:
        sz_e = event_sigma_z(10.0, edge, float(e[0]), float(e[1]))
        t, c, yt, zt = oracle.direct(g, *map(float, e))
        want = np.nonzero((bcb(Y - yt, Z - zt, t, c, sz_e, 63.0) <= 9.0).ravel())[0]
        pix, P = oracle.event_pixels(g, e)
        assert np.array_equal(np.sort(pix), want)
        p0, P0 = oracle.event_pixels(geom(sz=sz_e, pixel=2.0, n=400), e)
        assert np.array_equal(pix, p0)
        np.testing.assert_allclose(P, P0, rtol=1e-12)
        grew += len(pix) > len(oracle.event_pixels(geom(pixel=2.0, n=400), e)[0])
    assert grew > 20


def test_position_dependent_mlem_conserves_counts():
    w = get_workload("tiny").replace(sigma_z_edge=0.2)
    g = oracle.geometry(**w.geometry())
    ev = w.events(3000)
    s = oracle.sensitivity(g)
    rho, st = oracle.mlem(g, ev, oracle.initial_image(s), 2, s=s)
    assert (s * rho).sum() == pytest.approx(st["n_valid"] - st["n_zero_denominator"], rel=1e-12)
    rho0, st0 = oracle.mlem(oracle.geometry(**get_workload("tiny").geometry()), ev, oracle.initial_image(s), 2, s=s)
    assert st["n_pairs"] > st0["n_pairs"]
    # the log-likelihood is defined for a constant sigma_z only
    with pytest.raises(ValueError):
        oracle.loglik_grad(g, ev, rho, s=s)


# --------------------------------------------------------------------------------------------
# Reading R8: kappa <= 0 (the angular Gaussian integral behind Eq. 7 diverges)


def test_kappa_nonpositive_pixels_get_zero_and_are_counted():
    """A geometry where kappa changes sign inside the 3-sigma ellipse (strips 80 mm from the axis,
    sigma_z = 40 mm against sigma_dl = 6 mm).  With kappa = -2 g2 computed from the measurement
    model's own Taylor coefficients, the oracle's kernel is 0 at exactly the in-ellipse pixels with
    kappa <= 0, is the Laplace form elsewhere, and the oracle counts exactly those pairs."""
    from jpet_synth import Workload
    from laplace import laplace_terms, pixel_centres
    Rk, Lk, sz, sdl, pix, ny, nz = 80.0, 300.0, 40.0, 6.0, 3.0, 50, 100
    w = Workload("kappa", Rk, Lk, sz, sdl, pix, ny, nz, 200, 1, 77, "random")
    ev = w.events()
    for variant in (0, 1):
        g = oracle.geometry(**w.geometry(kernel_variant=variant))
        count, total, checked = 0, 0, 0
        for e in ev:
            p_idx, P = oracle.event_pixels(g, e)
            if len(p_idx) == 0:
                continue
            y, z = pixel_centres(p_idx, ny, nz, pix)
            g0, g1, g2 = laplace_terms(Rk, e, y, z, sz, sdl, variant)
            kappa = -2.0 * g2
            sure = np.abs(kappa) > 1e-7 * np.abs(kappa).max()
            assert np.array_equal((P == 0)[sure], (kappa <= 0)[sure])
            count += int((kappa <= 0).sum())
            total += len(P)
            # values where the exponent is moderate (near kappa = 0+ it grows without bound and
            # the Taylor coefficients' own rounding is amplified by it)
            ok = sure & (kappa > 0)
            expo = g0[ok] - g1[ok] ** 2 / (4 * g2[ok])
            mod = (np.abs(expo) <= 50.0) & (kappa[ok] > 1e-2 * kappa.max())
            want = np.sqrt(np.pi / -g2[ok][mod]) * np.exp(expo[mod])
            want *= math.sqrt(1 / sz ** 4 / sdl ** 2) / (2 * math.pi) ** 1.5
            np.testing.assert_allclose(P[ok][mod], want, rtol=1e-7)
            checked += int(mod.sum())
        _, st = oracle.mlem(g, ev, np.ones((ny, nz)), 1)
        assert 0 < count < total and checked > 0.5 * total
        assert st["n_kappa_nonpositive"] == count
