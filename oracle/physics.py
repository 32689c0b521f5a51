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
