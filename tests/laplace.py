"""The Laplace form of the kernel computed from its definition, for tests.

Eq. 7 is the second-order (Laplace) approximation of the angular integral of the 3-D Gaussian
N3(e - f(y, z, theta); C), with f the measurement model of Eq. 1.  Expanding the exponent
g(d) = -(1/2) (f(theta~ + d) - e) C^-1 (f(theta~ + d) - e) to second order in d,
g0 + g1 d + g2 d^2, the integral over d is sqrt(pi / -g2) exp(g0 - g1^2 / (4 g2)) when g2 < 0
and diverges otherwise.  Eq. 7 writes this with kappa = -2 g2.  Here the Taylor coefficients of f
come from Cauchy integrals of the model itself, so nothing is shared with either implementation.
"""

import math

import numpy as np


def forward(R, y, z, th):
    """(z_u, z_d, dl) of points (y, z) along direction th (Eq. 1); analytic in th, vectorised."""
    t = np.tan(th)
    zu = z + (R - y) * t
    zd = z - (R + y) * t
    dl = np.sqrt((R - y) ** 2 + (zu - z) ** 2) - np.sqrt((R + y) ** 2 + (zd - z) ** 2)
    return np.stack([zu, zd, dl], axis=-1)


def laplace_terms(R, event, y, z, sigma_z, sigma_dl, variant=0, radius=2e-3, m=64):
    """(g0, g1, g2) of the exponent at pixel centres (y, z) (arrays of equal shape) for one
    measured event (z_u, z_d, dl); variant 0 takes the third component of f' at half its value,
    as Eq. 9 prints it."""
    e = np.asarray(event, dtype=np.float64)
    th0 = math.atan((e[0] - e[1]) / (2.0 * R))
    y = np.asarray(y, dtype=np.float64)[..., None]
    z = np.asarray(z, dtype=np.float64)[..., None]
    phi = 2.0 * np.pi * np.arange(m) / m
    vals = forward(R, y, z, th0 + radius * np.exp(1j * phi))  # [..., m, 3]
    coef = []
    for k in range(3):
        ck = np.einsum("m,...mc->...c", np.exp(-1j * k * phi), vals) / m / radius ** k
        coef.append(np.real(ck))
    f0, f1, f2 = coef
    if variant == 0:
        f1 = f1 * np.array([1.0, 1.0, 0.5])
    cinv = np.array([1.0 / sigma_z ** 2, 1.0 / sigma_z ** 2, 1.0 / sigma_dl ** 2])
    r0 = f0 - e
    g0 = -0.5 * np.sum(r0 * cinv * r0, axis=-1)
    g1 = -np.sum(f1 * cinv * r0, axis=-1)
    g2 = -0.5 * (np.sum(f1 * cinv * f1, axis=-1) + 2.0 * np.sum(f2 * cinv * r0, axis=-1))
    return g0, g1, g2


def pixel_centres(pix, n_y, n_z, pixel):
    """(y, z) of row-major pixel indices."""
    pix = np.asarray(pix)
    i, k = pix // n_z, pix % n_z
    return (i + 0.5 - 0.5 * n_y) * pixel, (k + 0.5 - 0.5 * n_z) * pixel
