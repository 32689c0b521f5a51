"""Pins of the ASSA oracle (oracle/assa.py): grid parameters for the paper's
settings, the literal three-stage definition against the per-pair form, the
adjoint identity, exact agreement with the direct operator when every time of
flight lies on the fine grid, and the alignment-error bound otherwise."""
import numpy as np
import pytest

from oracle import assa as S
from oracle import ops as O
from paper_2602_03893_amd import inputs as I

DT, V = 25e-9, 1500.0


def test_grid_parameters():
    # sigma = 0.1 mm at 40 MHz: 3 sigma / (v dt) = 8 exactly
    assert S.params(0.1e-3, DT, V) == (8, 2, 16)
    # sigma = 0.05 mm: 4 exactly (evaluates to 4.000000000000001 in float64)
    assert S.params(0.05e-3, DT, V) == (4, 3, 12)
    # sigma = 0.06 mm: 4.8 -> 5, alpha = ceil(12 / 5) = 3
    assert S.params(0.06e-3, DT, V) == (5, 3, 15)
    # wide kernels need no upsampling
    assert S.params(1.0e-3, DT, V)[1] == 1
    h = S.kernel(0.05e-3, DT, V, 3, 12)
    assert h.shape == (25,) and h[12] == 0.0
    assert np.allclose(h, -h[::-1], rtol=0, atol=0)  # odd kernel


def small_geometry(seed, m=300, nd=7, nt=384):
    rng = np.random.default_rng(seed)
    cen = (rng.uniform(-1, 1, (m, 3)) * 1e-3).astype(np.float32)
    sen = I.fibonacci_hemisphere(nd, 6e-3)
    return O.Geometry(cen, sen, nt, DT, 0.0, V, 3.0)


@pytest.mark.parametrize("sigma", [0.05e-3, 0.06e-3, 0.1e-3])
def test_staged_definition_matches_per_pair_form(sigma):
    g = small_geometry(1)
    x = I.standard_normal(g.n_kernels, seed=2).astype(np.float64)
    y1 = S.forward_staged(g, x, sigma)
    y2 = S.forward(g, x, sigma)
    assert np.abs(y1).max() > 0
    assert np.allclose(y1, y2, rtol=0, atol=1e-13 * np.abs(y1).max())
    d = I.standard_normal((g.n_sensors, g.n_samples), seed=3).astype(np.float64)
    g1 = S.adjoint_staged(g, sigma, d)
    g2 = S.adjoint(g, sigma, d)
    assert np.allclose(g1, g2, rtol=0, atol=1e-13 * np.abs(g1).max())


def test_adjoint_identity():
    g = small_geometry(4, m=500, nd=9)
    x = I.standard_normal(g.n_kernels, seed=5).astype(np.float64)
    d = I.standard_normal((g.n_sensors, g.n_samples), seed=6).astype(np.float64)
    lhs = np.sum(S.forward_staged(g, x, 0.05e-3) * d)
    rhs = np.dot(x, S.adjoint_staged(g, 0.05e-3, d))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_equals_direct_operator_when_flights_are_on_the_grid():
    """Kernels on a line through the sensor at distances that are whole
    multiples of the fine-grid step v dt_up: the snapped time of flight is
    exact, and with 3 sigma / (v dt) an integer the two windows coincide, so
    ASSA must give the direct operator's samples.  Units are chosen so that
    every distance is exact in float32: v dt_up = 2^-16 m."""
    v = 1500.0
    alpha, n_half = 3, 4
    step = 2.0 ** -16
    dt = alpha * step / v
    sigma = n_half * v * dt / 3.0
    assert S.params(sigma, dt, v) == (n_half, alpha, alpha * n_half)
    # k not divisible by 3: no sample lands exactly on a window edge
    ks = np.array([1201, 1210, 1228, 1301, 1432])
    assert np.all(ks % 3 != 0)
    cen = np.zeros((ks.size, 3), np.float32)
    cen[:, 0] = (ks * step).astype(np.float32)
    assert np.array_equal(cen[:, 0].astype(np.float64), ks * step)
    sen = np.zeros((1, 3), np.float32)
    g = O.Geometry(cen, sen, 512, dt, 0.0, v, 3.0)
    x = np.array([1.0, -0.5, 2.0, 0.25, 1.5])
    ya = S.forward_staged(g, x, sigma)
    yd = O.forward(g, x, np.full(ks.size, sigma))
    assert np.count_nonzero(yd) == np.count_nonzero(ya) > 20
    assert np.allclose(ya, yd, rtol=0, atol=1e-12 * np.abs(yd).max())


def test_alignment_error_bound():
    """|y_assa - y_direct| per sample <= sum over the pairs that reach the
    sample of |A|/(2r) * max(v dt_up / 2, phi_edge): the kernel
    phi(d) = d exp(-d^2/(2 sigma^2)) is 1-Lipschitz and the snapped distance
    moves d by at most v dt_up / 2; a term inside one window but not the other
    has |d| >= 3 sigma - v dt_up / 2, where |phi| <= phi_edge."""
    sigma = 0.06e-3
    n_half, alpha, K = S.params(sigma, DT, V)
    g = small_geometry(7, m=400, nd=5)
    x = np.abs(I.standard_normal(g.n_kernels, seed=8)).astype(np.float64)
    ya = S.forward(g, x, sigma)
    yd = O.forward(g, x, np.full(g.n_kernels, sigma))
    half = V * DT / alpha / 2.0
    dmin = 3 * sigma - half
    phi_edge = dmin * np.exp(-dmin * dmin / (2 * sigma * sigma))
    # per-sample mass of the pairs whose (widened) window reaches the sample
    r = S._pairs(g)
    t = np.arange(g.n_samples) * DT
    reach = V * (n_half * DT) + 2 * half
    mass = np.zeros_like(ya)
    for j in range(g.n_sensors):
        near = np.abs(r[j][:, None] - V * t[None, :]) <= reach
        mass[j] = (x / (2 * r[j])) @ near
    bound = mass * max(half, phi_edge)
    err = np.abs(ya - yd)
    assert np.all(err <= bound * (1 + 1e-9) + 1e-30)
    assert err.max() > 0  # the approximation is not exact here
