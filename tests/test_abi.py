"""The C-ABI library: exported symbols and host-side validation (CPU only;
no call here launches GPU work)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2602_03893_amd import inputs as I
from tests.conftest import ROOT

HEADERS = [os.path.join(ROOT, "include", h)
           for h in sorted(os.listdir(os.path.join(ROOT, "include"))) if h.endswith(".h")]


def header_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(gpair_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("gpair_plan_create", "gpair_forward", "gpair_adjoint", "gpair_solve",
                     "gpair_residual", "gpair_adam_update", "gpair_pgd_update",
                     "gpair_nn_conv3", "gpair_nn_conv3_wgrad", "gpair_nn_upconv2"):
        assert required in names


def test_library_exports_every_header_function():
    from paper_2602_03893_amd import _lib
    missing = [n for n in header_functions() if not hasattr(_lib.lib, n)]
    assert not missing, missing
    assert _lib.gpair_abi_version() == _lib.ABI_VERSION == 2


def test_status_strings():
    from paper_2602_03893_amd import _lib
    for code, name in _lib.STATUS.items():
        assert _lib.gpair_status_string(code).decode() == name
    assert _lib.gpair_status_string(12345).decode() == "GPAIR_UNKNOWN_STATUS"


def _geometry(centres, sensors, nt=256, dt=25e-9, c=1500.0, nsig=3.0, smax=0.1e-3,
              fwd_tile=0, adj_tile=0, fwd_waves=0):
    from paper_2602_03893_amd import _lib
    fp = ctypes.POINTER(ctypes.c_float)
    keep = [np.ascontiguousarray(np.asarray(centres, np.float32)[:, i]) for i in range(3)]
    sens = np.ascontiguousarray(np.asarray(sensors, np.float32))
    keep.append(sens)
    g = _lib.Geometry()
    g.n_kernels = len(centres)
    g.cx, g.cy, g.cz = (k.ctypes.data_as(fp) for k in keep[:3])
    g.n_sensors = sens.shape[0]
    g.sensors = sens.ctypes.data_as(fp)
    g.n_samples, g.dt, g.t0, g.c_sound = nt, dt, 0.0, c
    g.n_sigma, g.sigma_max, g.fwd_tile, g.adj_tile = nsig, smax, fwd_tile, adj_tile
    g.fwd_waves = fwd_waves
    return g, keep


def _create(g):
    from paper_2602_03893_amd import _lib
    h = ctypes.c_void_p()
    st = _lib.gpair_plan_create(ctypes.byref(g), ctypes.byref(h))
    return st, h


def test_plan_creation_validates_arguments():
    from paper_2602_03893_amd import _lib, inputs as I
    cen = I.grid_centres(8, 8, 8, 0.1e-3)
    sen = I.fibonacci_hemisphere(10, 10e-3)
    g, keep = _geometry(cen, sen)
    st, h = _create(g)
    assert st == 0 and h.value
    info = _lib.PlanInfo()
    assert _lib.gpair_plan_get_info(h, ctypes.byref(info)) == 0
    assert info.n_kernels == 512 and info.fwd_tiles >= 1 and info.max_taps == 17
    assert sum(1 for _ in range(info.fwd_tiles)) == info.fwd_tiles
    _lib.gpair_plan_destroy(h)
    for field, bad, code in (("dt", 0.0, -1), ("c_sound", -1.0, -1), ("n_sigma", 0.0, -1),
                             ("sigma_max", 0.0, -1), ("dt", float("nan"), -3),
                             ("n_samples", 0, -1), ("fwd_tile", 100, -1),
                             ("adj_tile", 32, -1), ("fwd_waves", 3, -1)):
        g, keep = _geometry(cen, sen)
        setattr(g, field, bad)
        st, h = _create(g)
        assert st == code, (field, st)
        assert not h.value
    st = _lib.gpair_plan_create(None, ctypes.byref(ctypes.c_void_p()))
    assert st == -1


def test_plan_rejects_nonfinite_geometry_and_near_field():
    from paper_2602_03893_amd import inputs as I
    cen = I.grid_centres(4, 4, 4, 0.1e-3)
    sen = I.fibonacci_hemisphere(5, 10e-3)
    bad = cen.copy()
    bad[3, 1] = np.nan
    g, keep = _geometry(bad, sen)
    assert _create(g)[0] == -3
    near = sen.copy()
    near[2] = cen[5] + np.array([0.5e-3, 0, 0], np.float32)  # 0.5 mm < 10 sigma_max
    g, keep = _geometry(cen, near)
    assert _create(g)[0] == -2


def test_point_cloud_tiles_cover_every_kernel_once():
    """A random point cloud (not a lattice) is tiled; the tile table covers the
    permuted kernel range exactly."""
    from paper_2602_03893_amd import _lib
    rng = np.random.default_rng(0)
    cen = rng.uniform(-2e-3, 2e-3, (3000, 3)).astype(np.float32)
    g, keep = _geometry(cen, np.array([[0, 0, -15e-3], [3e-3, 0, -14e-3]], np.float32),
                        nt=1024)
    st, h = _create(g)
    assert st == 0
    info = _lib.PlanInfo()
    _lib.gpair_plan_get_info(h, ctypes.byref(info))
    assert info.fwd_tiles >= 3000 // info.fwd_tile
    assert info.adj_tiles >= 3000 // info.adj_tile
    assert info.max_tile_radius < 4e-3
    _lib.gpair_plan_destroy(h)


def _slots(h, which):
    from paper_2602_03893_amd import _lib
    lo, hi = ctypes.c_int64(), ctypes.c_int64()
    assert _lib.gpair_plan_tiling_slots(h, which, ctypes.byref(lo), ctypes.byref(hi)) == 0
    return lo.value, hi.value


@pytest.mark.parametrize("case", ["sparse_cloud", "widest_window", "clipped_ends", "lattice"])
def test_binning_invariant_holds_pair_by_pair(case):
    """Every pair's window (with the padding taps of the unrolled loops) lies
    inside its (tile, sensor) segment, checked pair by pair on the host, for
    geometries that stress the bound: a sparse point cloud whose tiles have
    large bounding spheres, sigma_max of 0.4 mm (33 taps), a time origin that
    cuts windows at both trace ends, and a lattice with the default tiles."""
    from paper_2602_03893_amd import _lib, inputs as I
    rng = np.random.default_rng(21)
    kw = {}
    if case == "sparse_cloud":
        cen = rng.uniform(-6e-3, 6e-3, (1500, 3)).astype(np.float32)
        sen = I.fibonacci_hemisphere(37, 30e-3)
        kw = dict(nt=2048, fwd_tile=512)
    elif case == "widest_window":
        cen = rng.uniform(-1e-3, 1e-3, (900, 3)).astype(np.float32)
        sen = I.fibonacci_hemisphere(29, 15e-3)
        kw = dict(nt=1024, smax=0.4e-3)
    elif case == "clipped_ends":
        cen = rng.uniform(-1.5e-3, 1.5e-3, (800, 3)).astype(np.float32)
        sen = I.fibonacci_hemisphere(70, 12e-3)
        kw = dict(nt=50)
    else:
        cen = I.grid_centres(32, 16, 8, 0.1e-3)
        sen = I.fibonacci_hemisphere(65, 12e-3)
        kw = dict(nt=1024)
    g, keep = _geometry(cen, sen, **kw)
    if case == "clipped_ends":
        g.t0 = 11e-3 / 1500.0
    st, h = _create(g)
    assert st == 0
    info = _lib.PlanInfo()
    _lib.gpair_plan_get_info(h, ctypes.byref(info))
    for which, seg in ((0, info.fwd_segment), (1, info.adj_segment)):
        lo, hi = _slots(h, which)
        assert 0 <= lo and hi <= seg - 1, (case, which, lo, hi, seg)
    assert _lib.gpair_plan_tiling_slots(h, 2, ctypes.byref(ctypes.c_int64()),
                                        ctypes.byref(ctypes.c_int64())) == -1
    _lib.gpair_plan_destroy(h)


def test_filter_routes_close_blocks_to_float64():
    """The planner admits a block to the float32 window filter only when its
    error bound holds for the closest sensor: at the paper-scale shape every
    block (radius 0.52 mm, closest sensor 21-40 mm away) takes the filter
    with three or four steps; a
    cloud whose blocks are a few radii from the sensors is decided in
    float64 throughout."""
    from paper_2602_03893_amd import _lib
    w = I.WORKLOADS["paper"]
    cen, sen = I.geometry_arrays(w)
    g, keep = _geometry(cen, sen, nt=w.n_samples, smax=w.smax)
    st, h = _create(g)
    assert st == 0
    n, k = ctypes.c_int64(), ctypes.c_int32()
    assert _lib.gpair_plan_filter_stats(h, ctypes.byref(n), ctypes.byref(k)) == 0
    assert n.value == 0 and k.value == 4
    _lib.gpair_plan_destroy(h)
    rng = np.random.default_rng(3)
    cen = rng.uniform(-2e-3, 2e-3, (150, 3)).astype(np.float32)
    sen = I.fibonacci_hemisphere(40, 6e-3)
    g, keep = _geometry(cen, sen, nt=512, smax=0.08e-3, fwd_tile=64, adj_tile=64)
    st, h = _create(g)
    assert st == 0
    assert _lib.gpair_plan_filter_stats(h, ctypes.byref(n), ctypes.byref(k)) == 0
    assert n.value == 3 and k.value == 0   # 150 kernels: three tiles, all in float64
    _lib.gpair_plan_destroy(h)
