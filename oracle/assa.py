"""Float64 oracle of the paper's ASSA operators (adaptive supersampling alignment).

TEST INFRASTRUCTURE ONLY (see the package docstring).

arXiv 2602.03893, Methods, "Adaptive supersampling alignment for the
differentiable model operator" and its Algorithm (forward and adjoint with
ASSA).  For one kernel width sigma shared by all kernels:

 - grid parameters ("Adaptive Grid Parameters" equation): N_half = the ceiling
   of 3 sigma / (v dt), alpha = max(1, ceil(((N_min - 1)/2) / N_half)) with
   N_min = 25, an alpha-times finer grid with alpha N_t points, K = alpha N_half;
 - projection P_up: the time of flight of each kernel-sensor pair is snapped to
   the nearest point k of the fine grid and x_i / r_ij is added to z_j[k];
 - transposed convolution with h[k] = C d[k] exp(-d[k]^2 / (2 sigma^2)),
   d[k] = -v k dt_up, k = -K..K;
 - decimation S: y_j[n] = z~_j[alpha n];
 - adjoint: zero-filling, correlation with h (convolution with the reversed
   kernel), back-projection g_i = sum_j delta_conv_j[k_ij] / r_ij.

Readings (stated where the paper is silent):
 - C = 1/2, so that an impulse whose time of flight falls on the grid gives
   exactly the direct model A/(2r) d exp(-d^2/(2 sigma^2)) of Eq. (single_forward);
 - the "3" of N_half is the window n_sigma (3 in the paper);
 - the ceiling is taken with a relative tolerance of 1e-9: 3 sigma/(v dt) is an
   exact integer for the paper's sigma = 0.05 mm at 40 MHz but evaluates to
   4.000000000000001 in float64;
 - sample k of the fine grid is at time t0 + k dt_up, so the snapped index is
   floor((r / v - t0) f_up + 0.5);
 - impulses whose index falls outside [0, alpha N_t) are dropped (the impulse
   grid has alpha N_t points).

``forward_staged`` / ``adjoint_staged`` follow the three stages literally
(numpy; small sizes).  ``forward`` / ``adjoint`` evaluate the same sums per
kernel-sensor pair in C (OpenMP) for large sizes; tests/test_oracle_assa.py
pins each against the other, against the direct operator where the two must
agree exactly, and against the alignment-error bound.
"""
import ctypes
import math

import numpy as np

from . import ops as _ops

N_MIN = 25


def params(sigma, dt, c_sound, n_sigma=3.0, n_min=N_MIN):
    """(N_half, alpha, K) of the adaptive grid."""
    x = n_sigma * sigma / (c_sound * dt)
    n_half = max(1, int(math.ceil(x - 1e-9 * max(1.0, x))))
    alpha = max(1, int(math.ceil(((n_min - 1) / 2.0) / n_half)))
    return n_half, alpha, alpha * n_half


def kernel(sigma, dt, c_sound, alpha, K):
    """h[k] for k = -K..K (index k + K)."""
    k = np.arange(-K, K + 1, dtype=np.float64)
    d = -c_sound * k * (dt / alpha)
    return 0.5 * d * np.exp(-(d * d) / (2.0 * sigma * sigma))


def _pairs(g):
    """r_ij (float64, [N_d, M]) from the float32 coordinates, in the same order of
    operations as the C oracle."""
    s = g.sensors.astype(np.float64)
    dx = s[:, 0:1] - g.cx.astype(np.float64)[None, :]
    dy = s[:, 1:2] - g.cy.astype(np.float64)[None, :]
    dz = s[:, 2:3] - g.cz.astype(np.float64)[None, :]
    return np.sqrt(dx * dx + dy * dy + dz * dz)


def snapped_index(r, c_sound, t0, f_up):
    return np.floor((r / c_sound - t0) * f_up + 0.5).astype(np.int64)


def forward_staged(g, x, sigma):
    """y = S(h * P_up(x)), each stage as written in the Methods (float64)."""
    n_half, alpha, K = params(sigma, g.dt, g.c_sound, g.n_sigma)
    ntu = alpha * g.n_samples
    f_up = alpha / g.dt
    r = _pairs(g)
    k = snapped_index(r, g.c_sound, g.t0, f_up)
    x = np.asarray(x, dtype=np.float64)
    # 1. projection onto the fine grid
    z = np.zeros((g.n_sensors, ntu))
    ok = (k >= 0) & (k < ntu)
    jj, ii = np.nonzero(ok)
    np.add.at(z, (jj, k[jj, ii]), x[ii] / r[jj, ii])
    # 2. transposed convolution: z~[k] = sum_m z[m] h[k - m]
    h = kernel(sigma, g.dt, g.c_sound, alpha, K)
    zt = np.stack([np.convolve(z[j], h)[K:K + ntu] for j in range(g.n_sensors)])
    # 3. decimation
    return zt[:, ::alpha][:, :g.n_samples]


def adjoint_staged(g, sigma, delta):
    """g = P_up^T(h_reversed * S^T(delta)), each stage as written (float64)."""
    n_half, alpha, K = params(sigma, g.dt, g.c_sound, g.n_sigma)
    ntu = alpha * g.n_samples
    f_up = alpha / g.dt
    delta = np.asarray(delta, dtype=np.float64)
    # 1. zero filling
    dup = np.zeros((g.n_sensors, ntu))
    dup[:, ::alpha] = delta
    # 2. delta_conv[k] = sum_m h[m - k] dup[m]  (correlation with h)
    h = kernel(sigma, g.dt, g.c_sound, alpha, K)
    dconv = np.stack([np.correlate(np.pad(dup[j], (K, K)), h, mode="valid")
                      for j in range(g.n_sensors)])
    # 3. back-projection at the snapped indices
    r = _pairs(g)
    k = snapped_index(r, g.c_sound, g.t0, f_up)
    ok = (k >= 0) & (k < ntu)
    kc = np.where(ok, k, 0)
    vals = np.take_along_axis(dconv, kc, axis=1) / r
    return np.where(ok, vals, 0.0).sum(axis=0)


_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_dbl = ctypes.c_double


def _lib():
    lib = _ops._load()
    if not getattr(lib, "_assa_ready", False):
        lib.oracle_assa_forward.restype = None
        lib.oracle_assa_forward.argtypes = [_i64, _f32p, _f32p, _f32p, _f64p, _i64, _f32p,
                                            _i64, _dbl, _dbl, _dbl, _dbl, _i64, _i64, _f64p]
        lib.oracle_assa_adjoint.restype = None
        lib.oracle_assa_adjoint.argtypes = [_i64, _f32p, _f32p, _f32p, _i64, _f32p, _i64,
                                            _dbl, _dbl, _dbl, _dbl, _i64, _i64, _f64p, _f64p]
        lib._assa_ready = True
    return lib


def forward(g, x, sigma):
    """The ASSA forward per kernel-sensor pair (C, float64): (N_d, N_t)."""
    n_half, alpha, K = params(sigma, g.dt, g.c_sound, g.n_sigma)
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    y = np.empty((g.n_sensors, g.n_samples))
    _lib().oracle_assa_forward(g.n_kernels, g.cx, g.cy, g.cz, a, g.n_sensors, g.sensors,
                               g.n_samples, g.dt, g.t0, g.c_sound, float(sigma), alpha, K, y)
    return y


def adjoint(g, sigma, delta):
    """The ASSA adjoint per kernel-sensor pair (C, float64): [M]."""
    n_half, alpha, K = params(sigma, g.dt, g.c_sound, g.n_sigma)
    d = np.ascontiguousarray(np.asarray(delta, dtype=np.float64))
    out = np.empty(g.n_kernels)
    _lib().oracle_assa_adjoint(g.n_kernels, g.cx, g.cy, g.cz, g.n_sensors, g.sensors,
                               g.n_samples, g.dt, g.t0, g.c_sound, float(sigma), alpha, K,
                               d, out)
    return out
