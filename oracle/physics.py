"""Closed forms of the GPAIR derivation and their numerical counterparts.

TEST INFRASTRUCTURE ONLY (see the package docstring).

arXiv 2602.03893, Methods, "Gaussian-kernel-based distribution for the
continuous source discretization":
 - Eq. (pa_wave): the pressure at a point detector is
       p(t) = 1/(4 pi v) d/dt [ 1/(v t) * integral over the sphere S'(t) of
              radius r' = v t around the detector of p0 dS' ]
   (the Poisson / Kirchhoff solution of the wave equation for an initial
   pressure p0 with zero initial velocity);
 - Eq. (sphere_int): for one Gaussian p0 = A exp(-|x - c|^2 / (2 sigma^2)) at
   distance r from the detector that surface integral is
       I = A 2 pi sigma^2 (r'/r) [exp(-(r-r')^2/(2 sigma^2))
                                  - exp(-(r+r')^2/(2 sigma^2))];
 - the equation after it: substituting gives the two-term pressure
       p = A/(2r) [(r - vt) e^{-(r-vt)^2/(2 sigma^2)} + (r + vt) e^{-(r+vt)^2/(2 sigma^2)}];
 - Eq. (single_forward): the far-field pressure keeps the first (outgoing)
   term only.

The numerical functions evaluate the definition (the surface integral of p0
over the sphere, by Gauss-Legendre quadrature on points of the sphere in 3D,
and the time derivative by a fourth-order central difference) without using
any closed form, so they pin the closed forms and the oracle's forward.
"""
import numpy as np


def sphere_integral_closed(amp, sigma, r, rp):
    """Eq. (sphere_int)."""
    s2 = 2.0 * sigma * sigma
    return amp * 2.0 * np.pi * sigma * sigma * (rp / r) * (
        np.exp(-((r - rp) ** 2) / s2) - np.exp(-((r + rp) ** 2) / s2))


def pressure_two_term(amp, sigma, r, t, v):
    """Two-term pressure of one Gaussian (the equation after Eq. (sphere_int))."""
    s2 = 2.0 * sigma * sigma
    a = r - v * t
    b = r + v * t
    return amp / (2.0 * r) * (a * np.exp(-a * a / s2) + b * np.exp(-b * b / s2))


def _gauss_legendre(n, lo, hi):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (hi - lo) * x + 0.5 * (hi + lo), 0.5 * (hi - lo) * w


def sphere_integral_quadrature(amp, sigma, r, rp, nodes=400):
    """Surface integral of p0 over the sphere of radius rp centred at the
    detector (origin), for a Gaussian centred at (0, 0, r), by quadrature on
    sphere points.  The integrand does not depend on the azimuth, so the
    azimuthal integral is 2 pi times one azimuth; the polar angle runs over
    the cap where the Gaussian is above exp(-80) (zero contribution beyond)."""
    r = float(r)
    rp = float(rp)
    centre = np.array([0.0, 0.0, r])
    # |x - c|^2 >= (r - rp)^2 + 4 r rp sin^2(theta/2): cap edge from that bound
    lim = 160.0 * sigma * sigma - (r - rp) ** 2
    if lim <= 0.0:
        return 0.0
    s = min(1.0, np.sqrt(lim / (4.0 * r * rp)))
    theta_max = 2.0 * np.arcsin(s)
    th, w = _gauss_legendre(nodes, 0.0, theta_max)
    pts = rp * np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], axis=1)
    d2 = np.sum((pts - centre) ** 2, axis=1)
    f = amp * np.exp(-d2 / (2.0 * sigma * sigma))
    return 2.0 * np.pi * rp * rp * np.sum(w * f * np.sin(th))


def pressure_poisson(amp, sigma, r, t, v, rel_step=2e-3, nodes=400):
    """Eq. (pa_wave) evaluated numerically for one Gaussian: quadrature of the
    surface integral and a fourth-order central difference in t."""
    h = rel_step * sigma / v

    def g(tt):
        return sphere_integral_quadrature(amp, sigma, r, v * tt, nodes) / (v * tt)

    deriv = (-g(t + 2 * h) + 8 * g(t + h) - 8 * g(t - h) + g(t - 2 * h)) / (12 * h)
    return deriv / (4.0 * np.pi * v)


def pressure_poisson_cloud(amps, centres, sigma, t, v, half_width=0.08,
                           nodes=240, rel_step=2e-3):
    """Eq. (pa_wave) for a superposition of Gaussians (one width) with the
    detector at the origin, by two-dimensional Gauss-Legendre quadrature of
    p0 = sum_k A_k exp(-|x - c_k|^2/(2 sigma^2)) over a patch of the sphere
    |x| = v t that covers every kernel (all kernels must lie within
    `half_width` radians of the +x axis as seen from the origin)."""
    centres = np.asarray(centres, dtype=np.float64)
    amps = np.asarray(amps, dtype=np.float64)
    th, wth = _gauss_legendre(nodes, 0.5 * np.pi - half_width, 0.5 * np.pi + half_width)
    ph, wph = _gauss_legendre(nodes, -half_width, half_width)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(wth, wph) * np.sin(TH)
    unit = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=-1)

    def surface_integral(rp):
        pts = rp * unit
        acc = np.zeros(TH.shape)
        for a, c in zip(amps, centres):
            d2 = np.sum((pts - c) ** 2, axis=-1)
            acc += a * np.exp(-d2 / (2.0 * sigma * sigma))
        return rp * rp * np.sum(W * acc)

    h = rel_step * sigma / v

    def g(tt):
        return surface_integral(v * tt) / (v * tt)

    deriv = (-g(t + 2 * h) + 8 * g(t + h) - 8 * g(t - h) + g(t - 2 * h)) / (12 * h)
    return deriv / (4.0 * np.pi * v)


def pressure_poisson_aniso(amp, centre, cov, t, v, half_width=None, nodes=320,
                           rel_step=2e-3):
    """Eq. (pa_wave) for one anisotropic Gaussian p0 = A exp(-(x-c)^T cov^-1
    (x-c)/2) with the detector at the origin: two-dimensional Gauss-Legendre
    quadrature of p0 over the patch of the sphere |x| = v t around the
    direction of c (polar angle about that direction up to where p0 is below
    exp(-40) on the sphere, full azimuth), and a fourth-order central
    difference in t.  No closed form is used."""
    c = np.asarray(centre, dtype=np.float64)
    cov = np.asarray(cov, dtype=np.float64)
    icov = np.linalg.inv(cov)
    r = float(np.linalg.norm(c))
    e3 = c / r
    # an orthonormal frame (e1, e2, e3) with e3 along c
    a = np.array([1.0, 0.0, 0.0]) if abs(e3[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = a - e3 * np.dot(a, e3)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(e3, e1)
    smax = float(np.sqrt(np.max(np.linalg.eigvalsh(cov))))
    if half_width is None:
        half_width = min(np.pi, 12.0 * smax / r)
    th, wth = _gauss_legendre(nodes, 0.0, half_width)
    ph, wph = _gauss_legendre(nodes, 0.0, 2.0 * np.pi)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(wth, wph) * np.sin(TH)
    unit = (np.sin(TH)[..., None] * (np.cos(PH)[..., None] * e1 + np.sin(PH)[..., None] * e2)
            + np.cos(TH)[..., None] * e3)

    def surface_integral(rp):
        x = rp * unit - c
        q = np.einsum("...i,ij,...j->...", x, icov, x)
        return rp * rp * np.sum(W * amp * np.exp(-0.5 * q))

    h = rel_step * np.sqrt(np.min(np.linalg.eigvalsh(cov))) / v

    def g(tt):
        return surface_integral(v * tt) / (v * tt)

    deriv = (-g(t + 2 * h) + 8 * g(t + h) - 8 * g(t - h) + g(t - 2 * h)) / (12 * h)
    return deriv / (4.0 * np.pi * v)


def pressure_far_aniso(amp, centre, cov, t, v):
    """The far-field closed form of the anisotropic kernel (detector at the
    origin): A sqrt(det cov)/sigma_n^3 d/(2r) exp(-d^2/(2 sigma_n^2)) with
    n = -c/r the direction from the kernel to the detector (sigma_n is even
    in n), sigma_n^2 = n^T cov n, d = r - v t."""
    c = np.asarray(centre, dtype=np.float64)
    cov = np.asarray(cov, dtype=np.float64)
    r = float(np.linalg.norm(c))
    n = c / r
    sn2 = float(n @ cov @ n)
    d = r - v * t
    return amp * np.sqrt(np.linalg.det(cov)) / sn2 ** 1.5 * d / (2.0 * r) * np.exp(-d * d / (2.0 * sn2))
