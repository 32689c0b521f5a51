"""Pins of the float64 oracle against the physics it encodes (CPU only).

arXiv 2602.03893, Methods, "Gaussian-kernel-based distribution for the
continuous source discretization": Eq. (pa_wave) (Poisson integral), Eq.
(sphere_int) (its closed form for one Gaussian), the two-term pressure that
follows, Eq. (single_forward) (outgoing term) and the n_sigma window.

The numerical Poisson integral (quadrature of p0 over the sphere plus a
fourth-order time derivative) never uses a closed form, so a dropped factor, a
wrong sign, a wrong sigma power or a wrong distance/time convention in the
oracle makes these tests fail.
"""
import numpy as np
import pytest

from oracle import ops, physics

V = 1500.0
DT = 25e-9


def test_sphere_integral_closed_form_matches_quadrature():
    amp, sigma, r = 1.3, 0.1e-3, 10e-3
    peak = physics.sphere_integral_closed(amp, sigma, r, r)
    for k in (-3.0, -1.0, -0.3, 0.0, 0.5, 1.0, 2.0, 3.0):
        rp = r + k * sigma
        a = physics.sphere_integral_closed(amp, sigma, r, rp)
        b = physics.sphere_integral_quadrature(amp, sigma, r, rp)
        assert abs(a - b) <= 1e-10 * peak, (k, a, b)


def test_two_term_pressure_matches_numerical_poisson():
    amp, sigma, r = 0.7, 0.1e-3, 10e-3
    scale = amp * sigma / (2 * r)
    for k in (-2.5, -1.0, -0.4, 0.0, 0.3, 1.0, 1.7, 2.5):
        t = (r - k * sigma) / V          # d = r - v t = k sigma
        p_num = physics.pressure_poisson(amp, sigma, r, t, V)
        p_cf = physics.pressure_two_term(amp, sigma, r, t, V)
        assert abs(p_num - p_cf) <= 1e-7 * scale, (k, p_num, p_cf)


def _one_pair_geometry(r_target, direction, n_samples, nsig=3.0, dt=DT):
    d = np.asarray(direction, dtype=np.float64)
    d /= np.linalg.norm(d)
    sensor = np.array([[1.0e-3, -2.0e-3, 0.5e-3]], dtype=np.float32)
    centre = (sensor[0].astype(np.float64) + r_target * d).astype(np.float32)[None, :]
    g = ops.Geometry(centre, sensor, n_samples, dt, 0.0, V, nsig)
    r = float(np.linalg.norm(centre[0].astype(np.float64) - sensor[0].astype(np.float64)))
    return g, r


@pytest.mark.parametrize("sigma", [0.05e-3, 0.1e-3])
def test_oracle_forward_matches_numerical_poisson_single_kernel(sigma):
    amp = 0.9
    g, r = _one_pair_geometry(10.3e-3, (0.3, -0.5, 0.8), 512)
    y = ops.forward(g, [amp], [sigma])[0]
    t = np.arange(512) * DT
    d = r - V * t
    win = np.abs(d) <= 3 * sigma
    assert win.sum() >= 2 * int(3 * sigma / (V * DT))
    scale = amp * sigma / (2 * r)
    for n in np.nonzero(win)[0]:
        p = physics.pressure_poisson(amp, sigma, r, t[n], V)
        assert abs(y[n] - p) <= 2e-7 * scale, (n, y[n], p)
    # outside the window the oracle is exactly zero and the true pressure is
    # below the window-edge tail value A/(2r) * 3 sigma * exp(-4.5)
    assert np.all(y[~win] == 0.0)
    tail = amp / (2 * r) * 3 * sigma * np.exp(-4.5)
    for n in np.nonzero(~win)[0][::7]:
        assert abs(physics.pressure_poisson(amp, sigma, r, t[n], V)) <= tail * (1 + 1e-6)


def test_oracle_forward_matches_poisson_for_a_kernel_cloud():
    """Superposition of 27 Gaussians of random amplitude (a 3x3x3 grid around
    the +x axis): oracle forward with a wide window (n_sigma = 8, truncation
    below 1e-12) against a two-dimensional quadrature of the summed p0."""
    rng = np.random.default_rng(5)
    sigma = 0.1e-3
    offs = (np.arange(3) - 1) * 0.2e-3
    Z, Y, X = np.meshgrid(offs, offs, offs, indexing="ij")
    centres = np.stack([10e-3 + X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float32)
    amps = rng.uniform(0.2, 1.0, 27)
    sensor = np.zeros((1, 3), dtype=np.float32)
    nt = 512
    g = ops.Geometry(centres, sensor, nt, DT, 0.0, V, 8.0)
    y = ops.forward(g, amps, np.full(27, sigma))[0]
    scale = amps.sum() * sigma / (2 * 10e-3)
    ns = np.arange(252, 284, 3)  # v t from 9.45 mm to 10.6 mm
    for n in ns:
        p = physics.pressure_poisson_cloud(amps, centres.astype(np.float64), sigma, n * DT, V,
                                           half_width=0.15, nodes=240)
        assert abs(y[n] - p) <= 1e-6 * scale, (n, y[n], p)


def test_special_values_exact_grid():
    """Exactly representable geometry: v dt = 2^-15 m, sigma = 2^-13 m, kernel
    at r = 2^-5 + 2^-13 m from the sensor, so sample n has d = (1028 - n) 2^-15."""
    v, dt, sigma = 1024.0, 2.0 ** -25, 2.0 ** -13
    r = 2.0 ** -5 + 2.0 ** -13
    g = ops.Geometry(np.array([[r, 0.0, 0.0]], np.float32), np.zeros((1, 3), np.float32),
                     2048, dt, 0.0, v, 3.0)
    amp = 1.0
    y = ops.forward(g, [amp], [sigma])[0]
    w = amp / (2 * r)
    assert y[1024] == pytest.approx(w * sigma * np.exp(-0.5), rel=1e-15)  # d = sigma
    assert y[1028] == 0.0                                                  # d = 0
    assert y[1032] == pytest.approx(-w * sigma * np.exp(-0.5), rel=1e-15)  # d = -sigma
    edge = w * 3 * sigma * np.exp(-4.5)
    assert y[1016] == pytest.approx(edge, rel=1e-15)     # d = +3 sigma: inclusive edge
    assert y[1040] == pytest.approx(-edge, rel=1e-15)    # d = -3 sigma
    assert y[1015] == 0.0 and y[1041] == 0.0             # just outside the window
    assert np.count_nonzero(y) == 25 - 1                 # 25 samples, one exact zero
    # the outgoing pulse is positive before arrival (d > 0), negative after
    assert np.all(y[1016:1028] > 0) and np.all(y[1029:1041] < 0)
    # edge / peak ratio 3 e^{-4} of d e^{-d^2/2 sigma^2} (window edge at 3 sigma)
    assert y[1016] / y[1024] == pytest.approx(3 * np.exp(-4.0), rel=1e-14)


def test_window_clipped_at_trace_ends():
    """Pulses straddling sample 0 (negative t0) and sample N_t - 1 lose the
    out-of-range samples only."""
    sigma = 0.1e-3
    g, r = _one_pair_geometry(10e-3, (1.0, 0.2, 0.1), 64)
    n_c = r / (V * DT)
    t0 = (n_c - 2.3) * DT           # pulse centre 2.3 samples after sample 0
    g.t0 = t0
    y = ops.forward(g, [1.0], [sigma])[0]
    t = t0 + np.arange(64) * DT
    d = r - V * t
    ref = np.where(np.abs(d) <= 3 * sigma, d * np.exp(-d * d / (2 * sigma ** 2)) / (2 * r), 0.0)
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    g.n_samples = 3                # pulse centre beyond the end of the trace
    y3 = ops.forward(g, [1.0], [sigma])[0]
    np.testing.assert_allclose(y3, ref[:3], rtol=1e-13, atol=1e-13 * np.abs(ref).max())
