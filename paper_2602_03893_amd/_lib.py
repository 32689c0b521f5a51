"""ctypes binding of ``libgpair.so`` (the C ABI declared in include/gpair.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Importing this module loads the library and raises ``ImportError``
when it is missing -- there is no fallback implementation.
"""
import ctypes
import os

import torch  # noqa: F401  -- load torch's HIP runtime before libgpair binds to it

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgpair.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
        "(or python paper_2602_03893_amd/build.py) first")

lib = ctypes.CDLL(LIB_PATH)

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_flt = ctypes.c_float
c_vp = ctypes.c_void_p
c_fp = ctypes.POINTER(ctypes.c_float)

STATUS = {
    0: "GPAIR_OK", 1: "GPAIR_NOT_CONVERGED", -1: "GPAIR_ERR_INVALID_ARG",
    -2: "GPAIR_ERR_NEAR_FIELD", -3: "GPAIR_ERR_NONFINITE", -4: "GPAIR_ERR_HIP",
    -5: "GPAIR_ERR_WORKSPACE", -6: "GPAIR_ERR_SIGMA_RANGE",
}
GPAIR_OK = 0
GPAIR_NOT_CONVERGED = 1
TIMER_FORWARD = 0
TIMER_ADJOINT = 1
TIMER_ASSA_FORWARD = 2
TIMER_ASSA_ADJOINT = 3
SOLVE_PGD = 0
SOLVE_ADAM = 1


class GpairError(RuntimeError):
    """A negative status returned by libgpair."""

    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class Geometry(ctypes.Structure):
    _fields_ = [("n_kernels", c_i64), ("cx", c_fp), ("cy", c_fp), ("cz", c_fp),
                ("n_sensors", c_i32), ("sensors", c_fp), ("n_samples", c_i32),
                ("dt", c_dbl), ("t0", c_dbl), ("c_sound", c_dbl), ("n_sigma", c_dbl),
                ("sigma_max", c_dbl), ("fwd_tile", c_i32), ("adj_tile", c_i32),
                ("fwd_waves", c_i32), ("deterministic", c_i32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_kernels", c_i64), ("n_sensors", c_i32), ("n_samples", c_i32),
                ("fwd_tile", c_i32), ("adj_tile", c_i32), ("fwd_waves", c_i32),
                ("fwd_tiles", c_i64),
                ("adj_tiles", c_i64), ("fwd_segment", c_i32), ("adj_segment", c_i32),
                ("max_taps", c_i32), ("max_tile_radius", c_dbl), ("min_distance", c_dbl),
                ("workspace_bytes", ctypes.c_size_t)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("method", c_i32), ("max_iters", c_i32), ("tol", c_dbl), ("step", c_dbl),
                ("lr_A", c_dbl), ("lr_sigma", c_dbl), ("beta1", c_dbl), ("beta2", c_dbl),
                ("eps", c_dbl), ("learn_sigma", c_i32), ("sigma_lo", c_dbl),
                ("sigma_hi", c_dbl), ("a_lo", c_dbl), ("a_hi", c_dbl),
                ("check_every", c_i32), ("npc", c_i32), ("npc_eps", c_dbl),
                ("reg_lambda", c_dbl), ("reg_beta", c_dbl), ("reg_eps", c_dbl),
                ("grid_nx", c_i32), ("grid_ny", c_i32), ("grid_nz", c_i32),
                ("lr_min", c_dbl), ("cawr_T0", c_i32), ("cawr_Tmult", c_i32)]


class SolveReport(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("rel_residual", c_dbl), ("seconds", c_dbl),
                ("converged", c_i32), ("history", ctypes.POINTER(c_dbl))]


def _proto(name, restype, argtypes):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = argtypes
    return f


gpair_status_string = _proto("gpair_status_string", ctypes.c_char_p, [c_i32])
gpair_abi_version = _proto("gpair_abi_version", ctypes.c_int, [])
ABI_VERSION = 2  # GPAIR_ABI_VERSION of include/gpair.h this binding is written for
if gpair_abi_version() != ABI_VERSION:
    raise ImportError(f"{LIB_PATH} has ABI version {gpair_abi_version()}, this binding "
                      f"expects {ABI_VERSION}: rebuild the library")
gpair_plan_create = _proto("gpair_plan_create", c_i32,
                           [ctypes.POINTER(Geometry), ctypes.POINTER(c_vp)])
gpair_plan_workspace_size = _proto("gpair_plan_workspace_size", c_i32,
                                   [c_vp, ctypes.POINTER(ctypes.c_size_t)])
gpair_plan_bind_workspace = _proto("gpair_plan_bind_workspace", c_i32,
                                   [c_vp, c_vp, ctypes.c_size_t, c_vp])
gpair_plan_destroy = _proto("gpair_plan_destroy", None, [c_vp])
gpair_plan_get_info = _proto("gpair_plan_get_info", c_i32, [c_vp, ctypes.POINTER(PlanInfo)])
gpair_plan_tiling_slots = _proto("gpair_plan_tiling_slots", c_i32,
                                 [c_vp, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)])
gpair_plan_filter_stats = _proto("gpair_plan_filter_stats", c_i32,
                                 [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i32)])
gpair_forward = _proto("gpair_forward", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp])
gpair_prepare = _proto("gpair_prepare", c_i32, [c_vp, c_vp, c_vp, c_vp])
gpair_forward_prepared = _proto("gpair_forward_prepared", c_i32, [c_vp, c_vp, c_vp])
gpair_adjoint_prepared = _proto("gpair_adjoint_prepared", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp])
gpair_adjoint = _proto("gpair_adjoint", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp])
gpair_forward_aniso = _proto("gpair_forward_aniso", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp])
gpair_adjoint_aniso = _proto("gpair_adjoint_aniso", c_i32,
                             [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp])
gpair_adjoint_aniso_centres = _proto("gpair_adjoint_aniso_centres", c_i32,
                                     [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp])
gpair_adjoint_centres = _proto("gpair_adjoint_centres", c_i32,
                               [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp])
gpair_sigma_violations = _proto("gpair_sigma_violations", c_i32,
                                [c_vp, ctypes.POINTER(c_i64), c_vp])
gpair_residual = _proto("gpair_residual", c_i32, [c_vp, c_vp, c_vp, c_flt, c_vp, c_vp, c_vp])
gpair_pgd_update = _proto("gpair_pgd_update", c_i32,
                          [c_i64, c_vp, c_vp, c_flt, c_flt, c_flt, c_vp])
gpair_adam_update = _proto("gpair_adam_update", c_i32,
                           [c_i64, c_vp, c_vp, c_vp, c_vp, c_flt, c_flt, c_flt, c_flt,
                            c_flt, c_i32, c_flt, c_flt, c_vp])
gpair_solve_workspace_size = _proto("gpair_solve_workspace_size", c_i32,
                                    [c_vp, ctypes.POINTER(SolveOpts),
                                     ctypes.POINTER(ctypes.c_size_t)])
gpair_solve = _proto("gpair_solve", c_i32,
                     [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(SolveOpts), c_vp,
                      ctypes.c_size_t, ctypes.POINTER(SolveReport), c_vp])
class WarmReport(ctypes.Structure):
    _fields_ = [("c_star", c_dbl), ("rho", c_dbl), ("fell_back", c_i32), ("pad", c_i32)]


gpair_warm_rescale = _proto("gpair_warm_rescale", c_i32,
                            [c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(WarmReport), c_vp])
class AssaGrid(ctypes.Structure):
    _fields_ = [("n_half", c_i32), ("alpha", c_i32), ("K", c_i32), ("n_fine", c_i32),
                ("fwd_segment", c_i32), ("fwd_passes", c_i32), ("adj_segment", c_i32),
                ("adj_stage_sensors", c_i32)]


gpair_assa_grid_params = _proto("gpair_assa_grid_params", c_i32,
                                [c_vp, c_dbl, ctypes.POINTER(AssaGrid)])
gpair_assa_workspace_size = _proto("gpair_assa_workspace_size", c_i32,
                                   [c_vp, c_dbl, ctypes.POINTER(ctypes.c_size_t)])
gpair_assa_forward = _proto("gpair_assa_forward", c_i32, [c_vp, c_vp, c_dbl, c_vp, c_vp])
gpair_assa_adjoint = _proto("gpair_assa_adjoint", c_i32,
                            [c_vp, c_dbl, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp])
gpair_assa_adjoint_static = _proto("gpair_assa_adjoint_static", c_i32,
                                   [c_vp, c_dbl, c_vp, c_vp, c_vp])
gpair_assa_static_scratch_bytes = _proto("gpair_assa_static_scratch_bytes", ctypes.c_size_t, [])
gpair_peak_probe = _proto("gpair_peak_probe", c_i32,
                          [c_i32, c_i32, c_i32, c_vp, ctypes.POINTER(c_i64), c_vp])
gpair_npc_map = _proto("gpair_npc_map", c_i32, [c_i64, c_vp, c_dbl, c_vp, c_vp])
gpair_npc_grad = _proto("gpair_npc_grad", c_i32, [c_i64, c_vp, c_vp, c_dbl, c_vp, c_vp])
gpair_vcr_workspace_size = _proto("gpair_vcr_workspace_size", c_i32,
                                  [c_i32, c_i32, c_i32, ctypes.POINTER(ctypes.c_size_t)])
gpair_vcr = _proto("gpair_vcr", c_i32, [c_i32, c_i32, c_i32, c_vp, c_dbl, c_dbl, c_dbl, c_vp,
                                        c_vp, c_vp, ctypes.c_size_t, c_vp])
gpair_cawr_rate = _proto("gpair_cawr_rate", c_i32,
                         [c_i64, c_dbl, c_dbl, c_i64, c_i32, ctypes.POINTER(c_dbl)])
gpair_plan_set_timing = _proto("gpair_plan_set_timing", c_i32, [c_vp, ctypes.c_int])
gpair_plan_kernel_times = _proto("gpair_plan_kernel_times", c_i32,
                                 [c_vp, ctypes.c_int, c_fp, c_i32, ctypes.POINTER(c_i32)])
TIMER_SLOTS = 64


def check(status, where):
    """Raise GpairError on a negative status; return the status otherwise."""
    if status < 0:
        raise GpairError(status, where)
    return status
