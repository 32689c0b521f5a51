"""ctypes front end of the float64 C oracle (``gpair_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

All functions take the geometry as float32 arrays (exactly what the GPU path
receives) and A / sigma / delta as any real arrays, promoted to float64.  They
return float64 arrays.

Definitions (arXiv 2602.03893, Methods):
 - forward: Eq. (single_forward) per kernel-sensor pair, kept inside the
   inclusive window |d| <= n_sigma*sigma_k ("3 sigma principle"), summed over
   kernels, sampled at t0 + n*dt for n in [0, n_samples);
 - adjoint: the transpose of that linear map ("Adjoint Operator" subsection);
 - sigma-gradient: d/dsigma of Eq. (single_forward), A d^3 e / (2 r sigma^3);
 - centre gradient: d/dc_k of Eq. (single_forward) through r = |s - c_k|
   (learnable centres, the paper's stated future work), window held fixed;
 - anisotropic kernels (the other half of that future work): the far-field
   pressure of p0 = A exp(-(x-c)^T Sigma^-1 (x-c)/2), the kernel's marginal
   along the sensor direction n, A sqrt(det Sigma)/sigma_n^3 d/(2r)
   exp(-d^2/(2 sigma_n^2)), sigma_n^2 = n^T Sigma n, inside |d| <= n_sigma
   sigma_n; its transpose, and its gradient with respect to the six
   parameters (xx, yy, zz, xy, xz, yz) of Sigma, window held fixed.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libgpair_oracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_dbl = ctypes.c_double


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.oracle_forward.restype = None
    lib.oracle_forward.argtypes = [_i64, _f32p, _f32p, _f32p, _f64p, _f64p,
                                   _i64, _f32p, _i64, _dbl, _dbl, _dbl, _dbl,
                                   _f64p]
    lib.oracle_adjoint.restype = None
    lib.oracle_adjoint.argtypes = [_i64, _f32p, _f32p, _f32p, _f64p, _f64p,
                                   _i64, _f32p, _i64, _dbl, _dbl, _dbl, _dbl,
                                   _f64p, _f64p, ctypes.c_void_p]
    lib.oracle_adjoint_centres.restype = None
    lib.oracle_adjoint_centres.argtypes = [_i64, _f32p, _f32p, _f32p, _f64p, _f64p,
                                           _i64, _f32p, _i64, _dbl, _dbl, _dbl, _dbl,
                                           _f64p, _f64p]
    lib.oracle_count_taps.restype = None
    lib.oracle_count_taps.argtypes = [_i64, _f32p, _f32p, _f32p, _f64p, _i64,
                                      _f32p, _i64, _dbl, _dbl, _dbl, _dbl,
                                      ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
    lib.oracle_forward_aniso.restype = None
    lib.oracle_forward_aniso.argtypes = [_i64, _f32p, _f32p, _f32p, _f64p, _f64p,
                                         _i64, _f32p, _i64, _dbl, _dbl, _dbl, _dbl, _f64p]
    lib.oracle_adjoint_aniso.restype = None
    lib.oracle_adjoint_aniso.argtypes = [_i64, _f32p, _f32p, _f32p, _f64p, _f64p,
                                         _i64, _f32p, _i64, _dbl, _dbl, _dbl, _dbl,
                                         _f64p, _f64p, ctypes.c_void_p]
    lib.oracle_adjoint_aniso_centres.restype = None
    lib.oracle_adjoint_aniso_centres.argtypes = [_i64, _f32p, _f32p, _f32p, _f64p, _f64p,
                                                 _i64, _f32p, _i64, _dbl, _dbl, _dbl, _dbl,
                                                 _f64p, _f64p]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    _lib = lib
    return lib


def num_threads():
    """OpenMP threads the oracle loops use."""
    return int(_load().oracle_num_threads())


class Geometry:
    """Geometry as the oracle sees it: float32 centres and sensors, float64
    scalars.  ``centres`` is (M, 3), ``sensors`` is (N_d, 3)."""

    def __init__(self, centres, sensors, n_samples, dt, t0, c_sound, n_sigma):
        c = np.asarray(centres, dtype=np.float32)
        self.cx = np.ascontiguousarray(c[:, 0])
        self.cy = np.ascontiguousarray(c[:, 1])
        self.cz = np.ascontiguousarray(c[:, 2])
        self.sensors = np.ascontiguousarray(np.asarray(sensors, np.float32).reshape(-1, 3))
        self.n_kernels = int(c.shape[0])
        self.n_sensors = int(self.sensors.shape[0])
        self.n_samples = int(n_samples)
        self.dt = float(dt)
        self.t0 = float(t0)
        self.c_sound = float(c_sound)
        self.n_sigma = float(n_sigma)

    def subset_sensors(self, idx):
        g = Geometry.__new__(Geometry)
        g.__dict__.update(self.__dict__)
        g.sensors = np.ascontiguousarray(self.sensors[np.asarray(idx)])
        g.n_sensors = int(g.sensors.shape[0])
        return g

    def subset_kernels(self, idx):
        idx = np.asarray(idx)
        g = Geometry.__new__(Geometry)
        g.__dict__.update(self.__dict__)
        g.cx = np.ascontiguousarray(self.cx[idx])
        g.cy = np.ascontiguousarray(self.cy[idx])
        g.cz = np.ascontiguousarray(self.cz[idx])
        g.n_kernels = int(g.cx.shape[0])
        return g


def _vec(a, n, name):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if a.shape[0] != n:
        raise ValueError(f"{name}: expected {n} values, got {a.shape[0]}")
    return a


def forward(g: Geometry, amp, sigma):
    """y[j, n] (float64, shape (N_d, N_t)) of the windowed direct sum."""
    lib = _load()
    a = _vec(amp, g.n_kernels, "amp")
    s = _vec(sigma, g.n_kernels, "sigma")
    y = np.empty((g.n_sensors, g.n_samples), dtype=np.float64)
    lib.oracle_forward(g.n_kernels, g.cx, g.cy, g.cz, a, s, g.n_sensors,
                       g.sensors, g.n_samples, g.dt, g.t0, g.c_sound,
                       g.n_sigma, y)
    return y


def adjoint(g: Geometry, amp, sigma, delta, want_sigma=True):
    """(gA, gsigma) float64 [M]; gsigma is None when want_sigma is False."""
    lib = _load()
    a = _vec(amp, g.n_kernels, "amp")
    s = _vec(sigma, g.n_kernels, "sigma")
    d = np.ascontiguousarray(np.asarray(delta, dtype=np.float64))
    if d.shape != (g.n_sensors, g.n_samples):
        raise ValueError(f"delta: expected {(g.n_sensors, g.n_samples)}, got {d.shape}")
    ga = np.empty(g.n_kernels, dtype=np.float64)
    gs = np.empty(g.n_kernels, dtype=np.float64) if want_sigma else None
    lib.oracle_adjoint(g.n_kernels, g.cx, g.cy, g.cz, a, s, g.n_sensors,
                       g.sensors, g.n_samples, g.dt, g.t0, g.c_sound,
                       g.n_sigma, d, ga,
                       gs.ctypes.data_as(ctypes.c_void_p) if gs is not None else None)
    return ga, gs


def adjoint_centres(g: Geometry, amp, sigma, delta):
    """gc float64 (M, 3): the gradient of <A(x; c), delta> with respect to the
    kernel centres, window membership held fixed."""
    lib = _load()
    a = _vec(amp, g.n_kernels, "amp")
    s = _vec(sigma, g.n_kernels, "sigma")
    d = np.ascontiguousarray(np.asarray(delta, dtype=np.float64))
    if d.shape != (g.n_sensors, g.n_samples):
        raise ValueError(f"delta: expected {(g.n_sensors, g.n_samples)}, got {d.shape}")
    gc = np.empty((g.n_kernels, 3), dtype=np.float64)
    lib.oracle_adjoint_centres(g.n_kernels, g.cx, g.cy, g.cz, a, s, g.n_sensors,
                               g.sensors, g.n_samples, g.dt, g.t0, g.c_sound,
                               g.n_sigma, d, gc)
    return gc


def count_taps(g: Geometry, sigma):
    """(total in-window taps, pairs with >= 1 tap)."""
    lib = _load()
    s = _vec(sigma, g.n_kernels, "sigma")
    taps = _i64(0)
    pairs = _i64(0)
    lib.oracle_count_taps(g.n_kernels, g.cx, g.cy, g.cz, s, g.n_sensors,
                          g.sensors, g.n_samples, g.dt, g.t0, g.c_sound,
                          g.n_sigma, ctypes.byref(taps), ctypes.byref(pairs))
    return int(taps.value), int(pairs.value)


def _sigma6(sigma6, n):
    s = np.ascontiguousarray(np.asarray(sigma6, dtype=np.float64).reshape(-1, 6))
    if s.shape[0] != n:
        raise ValueError(f"sigma6: expected ({n}, 6), got {s.shape}")
    return s


def forward_aniso(g: Geometry, amp, sigma6):
    """y[j, n] (float64, (N_d, N_t)) of anisotropic kernels; sigma6 is (M, 6):
    the covariance entries (xx, yy, zz, xy, xz, yz) in m^2."""
    lib = _load()
    a = _vec(amp, g.n_kernels, "amp")
    s = _sigma6(sigma6, g.n_kernels)
    y = np.empty((g.n_sensors, g.n_samples), dtype=np.float64)
    lib.oracle_forward_aniso(g.n_kernels, g.cx, g.cy, g.cz, a, s, g.n_sensors, g.sensors,
                             g.n_samples, g.dt, g.t0, g.c_sound, g.n_sigma, y)
    return y


def adjoint_aniso(g: Geometry, amp, sigma6, delta, want_sigma=True):
    """(gA [M], gSigma (M, 6) or None) of anisotropic kernels: the transpose
    of forward_aniso, and the gradient of <forward_aniso, delta> with respect
    to the six covariance parameters (an off-diagonal parameter stands for
    both symmetric entries)."""
    lib = _load()
    a = _vec(amp, g.n_kernels, "amp")
    s = _sigma6(sigma6, g.n_kernels)
    d = np.ascontiguousarray(np.asarray(delta, dtype=np.float64))
    if d.shape != (g.n_sensors, g.n_samples):
        raise ValueError(f"delta: expected {(g.n_sensors, g.n_samples)}, got {d.shape}")
    ga = np.empty(g.n_kernels, dtype=np.float64)
    gs = np.empty((g.n_kernels, 6), dtype=np.float64) if want_sigma else None
    lib.oracle_adjoint_aniso(g.n_kernels, g.cx, g.cy, g.cz, a, s, g.n_sensors, g.sensors,
                             g.n_samples, g.dt, g.t0, g.c_sound, g.n_sigma, d, ga,
                             gs.ctypes.data_as(ctypes.c_void_p) if gs is not None else None)
    return ga, gs


def adjoint_aniso_centres(g: Geometry, amp, sigma6, delta):
    """gc float64 (M, 3): the gradient of <forward_aniso, delta> with respect to
    the kernel centres, window membership held fixed."""
    lib = _load()
    a = _vec(amp, g.n_kernels, "amp")
    s = _sigma6(sigma6, g.n_kernels)
    d = np.ascontiguousarray(np.asarray(delta, dtype=np.float64))
    if d.shape != (g.n_sensors, g.n_samples):
        raise ValueError(f"delta: expected {(g.n_sensors, g.n_samples)}, got {d.shape}")
    gc = np.empty((g.n_kernels, 3), dtype=np.float64)
    lib.oracle_adjoint_aniso_centres(g.n_kernels, g.cx, g.cy, g.cz, a, s, g.n_sensors,
                                     g.sensors, g.n_samples, g.dt, g.t0, g.c_sound,
                                     g.n_sigma, d, gc)
    return gc
