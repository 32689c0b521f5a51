"""Host logic of the ASSA entry points (no GPU): the grid parameters of
gpair_assa_grid_params against the oracle's reading of the "Adaptive Grid
Parameters" equation, the sigma checks, and the work-buffer size."""
import ctypes

import numpy as np
import pytest

from oracle import assa as S
from paper_2602_03893_amd import _lib
from paper_2602_03893_amd import inputs as I


def host_plan(cen, sen, nt, smax, t0=0.0, fwd_tile=0, adj_tile=0):
    c = np.ascontiguousarray(np.asarray(cen, np.float32).reshape(-1, 3))
    cols = [np.ascontiguousarray(c[:, i]) for i in range(3)]
    sn = np.ascontiguousarray(np.asarray(sen, np.float32).reshape(-1, 3))
    fp = ctypes.POINTER(ctypes.c_float)
    g = _lib.Geometry()
    g.n_kernels = c.shape[0]
    g.cx, g.cy, g.cz = [a.ctypes.data_as(fp) for a in cols]
    g.n_sensors = sn.shape[0]
    g.sensors = sn.ctypes.data_as(fp)
    g.n_samples = nt
    g.dt, g.t0, g.c_sound, g.n_sigma, g.sigma_max = I.DT, t0, I.C_SOUND, 3.0, smax
    g.fwd_tile, g.adj_tile, g.fwd_waves = fwd_tile, adj_tile, 0
    h = ctypes.c_void_p()
    _lib.check(_lib.gpair_plan_create(ctypes.byref(g), ctypes.byref(h)), "gpair_plan_create")
    return h


def grid(h, sigma):
    g = _lib.AssaGrid()
    st = _lib.gpair_assa_grid_params(h, sigma, ctypes.byref(g))
    return st, g


@pytest.fixture(scope="module")
def toy():
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    h = host_plan(cen, sen, w.n_samples, w.smax)
    yield w, h
    _lib.gpair_plan_destroy(h)


@pytest.mark.parametrize("frac", [1.0, 0.8, 0.5, 0.4, 0.3, 0.2, 0.125, 0.1])
def test_grid_matches_the_oracle(toy, frac):
    w, h = toy
    sigma = frac * w.smax
    st, g = grid(h, sigma)
    assert st == 0
    assert (g.n_half, g.alpha, g.K) == S.params(sigma, I.DT, I.C_SOUND)
    assert g.n_fine == g.alpha * w.n_samples
    # the LDS budget: 63 KiB per workgroup
    assert g.fwd_segment * 64 * 4 <= 63 * 1024 and g.fwd_passes >= 1
    assert g.adj_segment * g.adj_stage_sensors * 4 <= 63 * 1024
    assert 1 <= g.adj_stage_sensors <= 64
    n = ctypes.c_size_t()
    assert _lib.gpair_assa_workspace_size(h, sigma, ctypes.byref(n)) == 0
    assert n.value == w.n_sensors * g.n_fine * 4


def test_paper_sigma_needs_one_pass():
    """sigma = 0.05 mm on the paper's 0.1 mm lattice: N_half = 4 (not 5, the
    float64 ceiling of 4.000000000000001), alpha = 3, one forward pass."""
    w = I.WORKLOADS["mid"]
    cen, sen = I.geometry_arrays(w)
    h = host_plan(cen, sen, w.n_samples, w.smax)
    st, g = grid(h, 0.05e-3)
    _lib.gpair_plan_destroy(h)
    assert st == 0 and (g.n_half, g.alpha, g.K) == (4, 3, 12) and g.fwd_passes == 1


def test_large_tiles_take_several_passes():
    rng = np.random.default_rng(8)
    cen = rng.uniform(-1.5e-3, 1.5e-3, (1000, 3)).astype(np.float32)
    sen = I.fibonacci_hemisphere(70, 12e-3)
    h = host_plan(cen, sen, 53, 0.08e-3, t0=11e-3 / I.C_SOUND, fwd_tile=1024, adj_tile=256)
    st, g = grid(h, 0.05e-3)
    _lib.gpair_plan_destroy(h)
    assert st == 0 and g.fwd_passes > 1


def test_sigma_checks(toy):
    w, h = toy
    for bad in (0.0, -1e-5, float("nan"), float("inf"), 1.0001 * w.smax):
        assert grid(h, bad)[0] == -6  # GPAIR_ERR_SIGMA_RANGE
    n = ctypes.c_size_t()
    assert _lib.gpair_assa_workspace_size(h, 0.0, ctypes.byref(n)) == -6
    # an unbound plan has no workspace: the operators refuse it
    assert _lib.gpair_assa_forward(h, None, w.sigma, None, None) == -1


def test_cawr_rate_matches_the_oracle():
    """gpair_cawr_rate (host code of the library) against the oracle's schedule."""
    from oracle import objective as J
    for T0, Tm in ((10, 1), (7, 2), (3, 3)):
        for t in range(0, 200, 3):
            r = ctypes.c_double()
            assert _lib.gpair_cawr_rate(t, 1e-4, 3e-2, T0, Tm, ctypes.byref(r)) == 0
            assert r.value == pytest.approx(J.cawr(t, 1e-4, 3e-2, T0, Tm), rel=1e-14)
    r = ctypes.c_double()
    assert _lib.gpair_cawr_rate(-1, 0.0, 1.0, 5, 1, ctypes.byref(r)) == -1
    assert _lib.gpair_cawr_rate(0, 0.0, 1.0, 0, 1, ctypes.byref(r)) == -1
    assert _lib.gpair_cawr_rate(0, 0.0, 1.0, 5, 0, ctypes.byref(r)) == -1
