"""Invariants of the float64 oracle operators (CPU only).

 - linearity in A (the forward is a linear map, Methods: superposition);
 - adjointness <A x, y> = <x, A^T y> (the "Adjoint Operator" subsection: the
   adjoint is the transpose), which pins the adjoint to the Poisson-pinned
   forward;
 - gA and gsigma equal central finite differences of the loss <A(x; sigma), y>;
 - invariance under exact rotations of the whole scene and under reordering of
   kernels and sensors;
 - an independent pure-Python brute force on a tiny case.
"""
import math

import numpy as np
import pytest

from oracle import ops
from paper_2602_03893_amd import inputs as I

V, DT = 1500.0, 25e-9


def small_geometry(m=96, nd=7, nt=700, seed=3, nsig=3.0):
    rng = np.random.default_rng(seed)
    centres = (rng.uniform(-1.0e-3, 1.0e-3, (m, 3))).astype(np.float32)
    sensors = I.fibonacci_hemisphere(nd, 12e-3)
    return ops.Geometry(centres, sensors, nt, DT, 0.0, V, nsig)


def test_linearity():
    g = small_geometry()
    rng = np.random.default_rng(0)
    x1, x2 = rng.uniform(-1, 1, g.n_kernels), rng.uniform(0, 1, g.n_kernels)
    s = rng.uniform(0.04e-3, 0.1e-3, g.n_kernels)
    y1, y2 = ops.forward(g, x1, s), ops.forward(g, x2, s)
    y12 = ops.forward(g, 2.5 * x1 - 0.75 * x2, s)
    ref = 2.5 * y1 - 0.75 * y2
    assert np.linalg.norm(y12 - ref) <= 1e-13 * np.linalg.norm(ref)


def test_dot_product_adjointness():
    g = small_geometry()
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, g.n_kernels)
    s = rng.uniform(0.04e-3, 0.1e-3, g.n_kernels)
    yv = rng.standard_normal((g.n_sensors, g.n_samples))
    lhs = float(np.sum(ops.forward(g, x, s) * yv))
    gA, _ = ops.adjoint(g, x, s, yv, want_sigma=False)
    rhs = float(np.dot(x, gA))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(x) * np.linalg.norm(gA))


def test_gradients_match_central_differences():
    g = small_geometry(m=24, nd=5)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.2, 1.0, g.n_kernels)
    s = rng.uniform(0.05e-3, 0.1e-3, g.n_kernels)
    yv = rng.standard_normal((g.n_sensors, g.n_samples))

    def loss(xx, ss):
        return float(np.sum(ops.forward(g, xx, ss) * yv))

    gA, gS = ops.adjoint(g, x, s, yv)
    for k in range(0, g.n_kernels, 3):
        # A: the loss is linear in A_k, the difference quotient is exact
        e = np.zeros_like(x)
        e[k] = 1.0
        fdA = (loss(x + 0.5 * e, s) - loss(x - 0.5 * e, s))
        assert fdA == pytest.approx(gA[k], rel=1e-10, abs=1e-12 * np.abs(gA).max())
        # sigma: central difference, step small enough never to move a window edge
        h = 1e-6 * s[k]
        sp, sm = s.copy(), s.copy()
        sp[k] += h
        sm[k] -= h
        fdS = (loss(x, sp) - loss(x, sm)) / (2 * h)
        assert fdS == pytest.approx(gS[k], rel=1e-6, abs=1e-9 * np.abs(gS).max())


def test_exact_rotation_and_reordering_invariance():
    g = small_geometry(m=40, nd=6)
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, g.n_kernels)
    s = np.full(g.n_kernels, 0.07e-3)
    y = ops.forward(g, x, s)
    # rotate by 90 degrees about z: (x, y, z) -> (-y, x, z), exact in float32
    cen = np.stack([g.cx, g.cy, g.cz], axis=1)
    rot = lambda p: np.stack([-p[:, 1], p[:, 0], p[:, 2]], axis=1)  # noqa: E731
    g2 = ops.Geometry(rot(cen), rot(g.sensors), g.n_samples, DT, 0.0, V, 3.0)
    assert np.array_equal(ops.forward(g2, x, s), y)
    # reorder kernels and sensors
    pk = rng.permutation(g.n_kernels)
    pj = rng.permutation(g.n_sensors)
    g3 = ops.Geometry(cen[pk], g.sensors[pj], g.n_samples, DT, 0.0, V, 3.0)
    y3 = ops.forward(g3, x[pk], s[pk])
    np.testing.assert_allclose(y3, y[pj], rtol=0, atol=1e-14 * np.abs(y).max())


def _brute_force(centres, sensors, amp, sigma, nt, dt, t0, v, nsig):
    y = [[0.0] * nt for _ in sensors]
    for j, sj in enumerate(sensors):
        for c, a, sg in zip(centres, amp, sigma):
            r = math.sqrt(sum((float(sj[i]) - float(c[i])) ** 2 for i in range(3)))
            for n in range(nt):
                d = r - v * (t0 + n * dt)
                if abs(d) <= nsig * sg:
                    y[j][n] += a / (2 * r) * d * math.exp(-d * d / (2 * sg * sg))
    return np.array(y)


def test_oracle_matches_pure_python_brute_force():
    g = small_geometry(m=9, nd=3, nt=560)
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, g.n_kernels)
    s = rng.uniform(0.03e-3, 0.1e-3, g.n_kernels)
    cen = np.stack([g.cx, g.cy, g.cz], axis=1)
    ref = _brute_force(cen, g.sensors, x, s, g.n_samples, DT, 0.0, V, 3.0)
    y = ops.forward(g, x, s)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_tap_count_matches_window_width():
    """Every pair holds floor(2 n_sigma sigma / (v dt)) or one more taps."""
    g = small_geometry(m=50, nd=4)
    sigma = 0.05e-3
    taps, pairs = ops.count_taps(g, np.full(g.n_kernels, sigma))
    w = 2 * 3 * sigma / (V * DT)
    assert pairs == g.n_kernels * g.n_sensors
    assert math.floor(w) * pairs <= taps <= (math.floor(w) + 1) * pairs
