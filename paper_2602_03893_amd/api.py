"""Python front end of libgpair: plans, operators, residual, updates, solver.

Thin marshalling over the C ABI (include/gpair.h): torch supplies device
memory and the current HIP stream, and every step runs in the library's HIP
kernels.  Shapes and dtypes are checked here because the C ABI receives bare
pointers.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import GpairError, check


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, name, numel=None, dtype=torch.float32, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: on {t.device}, plan is on {device}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A bound plan: geometry + spatial tiling + device workspace.

    centres  (M, 3) kernel centres in metres (host array-like, taken as float32)
    sensors  (N_d, 3) sensor positions in metres
    n_samples, dt, t0, c_sound, n_sigma, sigma_max: see gpair_geometry.
    deterministic: bitwise reproducible forward (int64 flush; gpair_forward).
    """

    def __init__(self, centres, sensors, n_samples, dt, c_sound, n_sigma=3.0,
                 sigma_max=None, t0=0.0, fwd_tile=0, adj_tile=0, fwd_waves=0,
                 device=None, deterministic=False):
        if sigma_max is None:
            raise ValueError("sigma_max is required")
        c = np.ascontiguousarray(np.asarray(centres, dtype=np.float32).reshape(-1, 3))
        self._cx = np.ascontiguousarray(c[:, 0])
        self._cy = np.ascontiguousarray(c[:, 1])
        self._cz = np.ascontiguousarray(c[:, 2])
        self._sens = np.ascontiguousarray(np.asarray(sensors, dtype=np.float32).reshape(-1, 3))
        fp = ctypes.POINTER(ctypes.c_float)
        g = _lib.Geometry()
        g.n_kernels = c.shape[0]
        g.cx = self._cx.ctypes.data_as(fp)
        g.cy = self._cy.ctypes.data_as(fp)
        g.cz = self._cz.ctypes.data_as(fp)
        g.n_sensors = self._sens.shape[0]
        g.sensors = self._sens.ctypes.data_as(fp)
        g.n_samples = int(n_samples)
        g.dt = float(dt)
        g.t0 = float(t0)
        g.c_sound = float(c_sound)
        g.n_sigma = float(n_sigma)
        g.sigma_max = float(sigma_max)
        g.fwd_tile = int(fwd_tile)
        g.adj_tile = int(adj_tile)
        g.fwd_waves = int(fwd_waves)
        g.deterministic = 1 if deterministic else 0
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self._h = ctypes.c_void_p()
        check(_lib.gpair_plan_create(ctypes.byref(g), ctypes.byref(self._h)), "gpair_plan_create")
        nbytes = ctypes.c_size_t()
        check(_lib.gpair_plan_workspace_size(self._h, ctypes.byref(nbytes)),
              "gpair_plan_workspace_size")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            check(_lib.gpair_plan_bind_workspace(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                                 nbytes.value, _stream()),
                  "gpair_plan_bind_workspace")
        self.n_kernels = int(c.shape[0])
        self.n_sensors = int(self._sens.shape[0])
        self.n_samples = int(n_samples)
        self.dt, self.t0, self.c_sound = float(dt), float(t0), float(c_sound)
        self.n_sigma, self.sigma_max = float(n_sigma), float(sigma_max)

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.gpair_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- information ------------------------------------------------------
    def info(self):
        i = _lib.PlanInfo()
        check(_lib.gpair_plan_get_info(self._h, ctypes.byref(i)), "gpair_plan_get_info")
        return {f: getattr(i, f) for f, _ in i._fields_}

    def filter_stats(self):
        """(adjoint tiles decided in float64 throughout, most filter steps)."""
        n, k = ctypes.c_int64(), ctypes.c_int32()
        check(_lib.gpair_plan_filter_stats(self._h, ctypes.byref(n), ctypes.byref(k)),
              "gpair_plan_filter_stats")
        return int(n.value), int(k.value)

    # -- operators --------------------------------------------------------
    def forward(self, A, sigma, out=None):
        """y (N_d, N_t) float32 = A(x; sigma)."""
        M = self.n_kernels
        pa = _dev(A, "A", M, device=self.device)
        ps = _dev(sigma, "sigma", M, device=self.device)
        if out is None:
            out = torch.empty((self.n_sensors, self.n_samples), dtype=torch.float32,
                              device=self.device)
        py = _dev(out, "y", self.n_sensors * self.n_samples, device=self.device)
        check(_lib.gpair_forward(self._h, pa, ps, py, _stream()), "gpair_forward")
        return out

    def adjoint(self, A, sigma, delta, want_sigma=True, out_A=None, out_sigma=None):
        """(gA, gsigma) float32 [M]; gsigma is None unless want_sigma."""
        M = self.n_kernels
        ps = _dev(sigma, "sigma", M, device=self.device)
        pd = _dev(delta, "delta", self.n_sensors * self.n_samples, device=self.device)
        pa = _dev(A, "A", M, device=self.device) if (want_sigma or A is not None) else None
        gA = out_A if out_A is not None else torch.empty(M, dtype=torch.float32, device=self.device)
        pga = _dev(gA, "gA", M, device=self.device)
        gS = None
        pgs = None
        if want_sigma:
            gS = out_sigma if out_sigma is not None else torch.empty(M, dtype=torch.float32,
                                                                     device=self.device)
            pgs = _dev(gS, "gsigma", M, device=self.device)
        check(_lib.gpair_adjoint(self._h, pa, ps, pd, pga, pgs, _stream()), "gpair_adjoint")
        return gA, gS

    def prepare(self, A, sigma):
        """Build the coefficient records from (A, sigma) for the _prepared
        calls (gpair_prepare); A may be None (zero amplitudes)."""
        M = self.n_kernels
        pa = _dev(A, "A", M, device=self.device) if A is not None else None
        check(_lib.gpair_prepare(self._h, pa, _dev(sigma, "sigma", M, device=self.device),
                                 _stream()), "gpair_prepare")

    def forward_prepared(self, out=None):
        """y = A(x; sigma) with the records of the last build."""
        if out is None:
            out = torch.empty((self.n_sensors, self.n_samples), dtype=torch.float32,
                              device=self.device)
        py = _dev(out, "y", self.n_sensors * self.n_samples, device=self.device)
        check(_lib.gpair_forward_prepared(self._h, py, _stream()), "gpair_forward_prepared")
        return out

    def adjoint_prepared(self, delta, want_sigma=True, out_A=None, out_sigma=None):
        """(gA, gsigma or None) with the records of the last build."""
        M = self.n_kernels
        pd = _dev(delta, "delta", self.n_sensors * self.n_samples, device=self.device)
        gA = out_A if out_A is not None else torch.empty(M, dtype=torch.float32, device=self.device)
        gS = None
        if want_sigma:
            gS = out_sigma if out_sigma is not None else torch.empty(M, dtype=torch.float32,
                                                                     device=self.device)
        check(_lib.gpair_adjoint_prepared(self._h, pd, _dev(gA, "gA", M, device=self.device),
                                          _dev(gS, "gsigma", M, device=self.device)
                                          if want_sigma else None, _stream()),
              "gpair_adjoint_prepared")
        return gA, gS

    def adjoint_centres(self, A, sigma, delta, want_sigma=True):
        """(gA, gsigma or None, gcentres (M, 3)) float32: the adjoint with the
        gradient with respect to the kernel centres (gpair_adjoint_centres)."""
        M = self.n_kernels
        pa = _dev(A, "A", M, device=self.device)
        ps = _dev(sigma, "sigma", M, device=self.device)
        pd = _dev(delta, "delta", self.n_sensors * self.n_samples, device=self.device)
        gA = torch.empty(M, dtype=torch.float32, device=self.device)
        gS = torch.empty(M, dtype=torch.float32, device=self.device) if want_sigma else None
        gC = torch.empty((M, 3), dtype=torch.float32, device=self.device)
        check(_lib.gpair_adjoint_centres(self._h, pa, ps, pd, _dev(gA, "gA", M),
                                         _dev(gS, "gsigma", M) if want_sigma else None,
                                         _dev(gC, "gcentres", 3 * M), _stream()),
              "gpair_adjoint_centres")
        return gA, gS, gC

    def forward_aniso(self, A, sigma6, out=None):
        """y (N_d, N_t) float32 of anisotropic kernels (gpair_forward_aniso);
        sigma6 is (6, M): the covariance entries xx, yy, zz, xy, xz, yz (m^2)."""
        M = self.n_kernels
        pa = _dev(A, "A", M, device=self.device)
        ps = _dev(sigma6, "sigma6", 6 * M, device=self.device)
        if out is None:
            out = torch.empty((self.n_sensors, self.n_samples), dtype=torch.float32,
                              device=self.device)
        py = _dev(out, "y", self.n_sensors * self.n_samples, device=self.device)
        check(_lib.gpair_forward_aniso(self._h, pa, ps, py, _stream()), "gpair_forward_aniso")
        return out

    def adjoint_aniso(self, A, sigma6, delta, want_sigma=True):
        """(gA [M], gsigma6 (6, M) or None) float32 of anisotropic kernels
        (gpair_adjoint_aniso)."""
        M = self.n_kernels
        ps = _dev(sigma6, "sigma6", 6 * M, device=self.device)
        pd = _dev(delta, "delta", self.n_sensors * self.n_samples, device=self.device)
        pa = _dev(A, "A", M, device=self.device) if (want_sigma or A is not None) else None
        gA = torch.empty(M, dtype=torch.float32, device=self.device)
        gS = torch.empty((6, M), dtype=torch.float32, device=self.device) if want_sigma else None
        check(_lib.gpair_adjoint_aniso(self._h, pa, ps, pd, _dev(gA, "gA", M),
                                       _dev(gS, "gsigma6", 6 * M) if want_sigma else None,
                                       _stream()),
              "gpair_adjoint_aniso")
        return gA, gS

    def adjoint_aniso_centres(self, A, sigma6, delta, want_sigma=True):
        """(gA [M], gsigma6 (6, M) or None, gcentres (M, 3)) float32 of
        anisotropic kernels (gpair_adjoint_aniso_centres)."""
        M = self.n_kernels
        pa = _dev(A, "A", M, device=self.device)
        ps = _dev(sigma6, "sigma6", 6 * M, device=self.device)
        pd = _dev(delta, "delta", self.n_sensors * self.n_samples, device=self.device)
        gA = torch.empty(M, dtype=torch.float32, device=self.device)
        gS = torch.empty((6, M), dtype=torch.float32, device=self.device) if want_sigma else None
        gC = torch.empty((M, 3), dtype=torch.float32, device=self.device)
        check(_lib.gpair_adjoint_aniso_centres(self._h, pa, ps, pd, _dev(gA, "gA", M),
                                               _dev(gS, "gsigma6", 6 * M) if want_sigma else None,
                                               _dev(gC, "gcentres", 3 * M), _stream()),
              "gpair_adjoint_aniso_centres")
        return gA, gS, gC

    def residual(self, y, b, scale=1.0, delta=None):
        """norms (2,) float64 on device = (sum (y-b)^2, sum b^2); writes
        delta = scale (y - b) when `delta` is given (may be y itself)."""
        n = self.n_sensors * self.n_samples
        py = _dev(y, "y", n, device=self.device)
        pb = _dev(b, "b", n, device=self.device)
        pdl = _dev(delta, "delta", n, device=self.device) if delta is not None else None
        norms = torch.empty(2, dtype=torch.float64, device=self.device)
        pn = _dev(norms, "norms", 2, dtype=torch.float64, device=self.device)
        check(_lib.gpair_residual(self._h, py, pb, float(scale), pdl, pn, _stream()),
              "gpair_residual")
        return norms

    def warm_rescale(self, A, sigma, b, y_scratch=None):
        """Rescale the start A in place by c* = max(0, <A x, b>/||A x||^2), or
        zero it when that does not beat the zero start; returns the report."""
        n = self.n_sensors * self.n_samples
        if y_scratch is None:
            y_scratch = torch.empty(n, dtype=torch.float32, device=self.device)
        rep = _lib.WarmReport()
        check(_lib.gpair_warm_rescale(
            self._h, _dev(A, "A", self.n_kernels, device=self.device),
            _dev(sigma, "sigma", self.n_kernels, device=self.device),
            _dev(b, "b", n, device=self.device), _dev(y_scratch, "y_scratch", n, device=self.device),
            ctypes.byref(rep), _stream()), "gpair_warm_rescale")
        return {"c_star": rep.c_star, "rho": rep.rho, "fell_back": bool(rep.fell_back)}

    # -- ASSA operators (shared sigma) -----------------------------------
    def assa_grid(self, sigma):
        """Grid of the ASSA operators for the shared width sigma: dict with
        n_half, alpha, K, n_fine and the LDS segment lengths."""
        g = _lib.AssaGrid()
        check(_lib.gpair_assa_grid_params(self._h, float(sigma), ctypes.byref(g)),
              "gpair_assa_grid_params")
        return {f: getattr(g, f) for f, _ in g._fields_}

    def assa_workspace_bytes(self, sigma):
        n = ctypes.c_size_t()
        check(_lib.gpair_assa_workspace_size(self._h, float(sigma), ctypes.byref(n)),
              "gpair_assa_workspace_size")
        return int(n.value)

    def assa_forward(self, x, sigma, out=None):
        """y (N_d, N_t) float32 = S(h * P_up(x)) with one shared sigma."""
        px = _dev(x, "x", self.n_kernels, device=self.device)
        if out is None:
            out = torch.empty((self.n_sensors, self.n_samples), dtype=torch.float32,
                              device=self.device)
        py = _dev(out, "y", self.n_sensors * self.n_samples, device=self.device)
        check(_lib.gpair_assa_forward(self._h, px, float(sigma), py, _stream()),
              "gpair_assa_forward")
        return out

    def assa_adjoint(self, sigma, delta, out=None, work=None):
        """g [M] float32 = the transpose of assa_forward applied to delta.
        `work` (uint8 device tensor of assa_workspace_bytes(sigma) bytes) is
        allocated here when not given."""
        pd = _dev(delta, "delta", self.n_sensors * self.n_samples, device=self.device)
        g = out if out is not None else torch.empty(self.n_kernels, dtype=torch.float32,
                                                    device=self.device)
        pg = _dev(g, "g", self.n_kernels, device=self.device)
        nbytes = self.assa_workspace_bytes(sigma)
        if work is None:
            work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        pw = _dev(work, "work", dtype=torch.uint8, device=self.device)
        check(_lib.gpair_assa_adjoint(self._h, float(sigma), pd, pg, pw, work.numel(),
                                      _stream()), "gpair_assa_adjoint")
        return g

    def assa_adjoint_static(self, sigma, delta, out=None):
        """assa_adjoint with the library's fixed device buffer as its work
        space (gpair_assa_adjoint_static: the call allocates nothing; `out`
        must be given for that)."""
        pd = _dev(delta, "delta", self.n_sensors * self.n_samples, device=self.device)
        g = out if out is not None else torch.empty(self.n_kernels, dtype=torch.float32,
                                                    device=self.device)
        pg = _dev(g, "g", self.n_kernels, device=self.device)
        check(_lib.gpair_assa_adjoint_static(self._h, float(sigma), pd, pg, _stream()),
              "gpair_assa_adjoint_static")
        return g

    def sigma_violations(self):
        n = ctypes.c_int64()
        check(_lib.gpair_sigma_violations(self._h, ctypes.byref(n), _stream()),
              "gpair_sigma_violations")
        return int(n.value)

    # -- timing -----------------------------------------------------------
    def set_timing(self, enable=True):
        check(_lib.gpair_plan_set_timing(self._h, 1 if enable else 0), "gpair_plan_set_timing")

    def kernel_times(self, which):
        """Durations (ms) of the main kernel of the recorded calls of kind
        'forward', 'adjoint', 'assa_forward' or 'assa_adjoint' since the last
        read (at most 64, oldest first)."""
        w = {"forward": _lib.TIMER_FORWARD, "adjoint": _lib.TIMER_ADJOINT,
             "assa_forward": _lib.TIMER_ASSA_FORWARD,
             "assa_adjoint": _lib.TIMER_ASSA_ADJOINT}[which]
        buf = (ctypes.c_float * _lib.TIMER_SLOTS)()
        n = ctypes.c_int32()
        check(_lib.gpair_plan_kernel_times(self._h, w, buf, _lib.TIMER_SLOTS, ctypes.byref(n)),
              "gpair_plan_kernel_times")
        return [float(buf[i]) for i in range(min(n.value, _lib.TIMER_SLOTS))]

    # -- solver -----------------------------------------------------------
    def solve(self, b, A, sigma, method="adam", max_iters=100, tol=0.0, step=0.0,
              lr_A=1e-2, lr_sigma=0.0, beta1=0.9, beta2=0.999, eps=1e-8,
              learn_sigma=False, sigma_lo=None, sigma_hi=None, a_lo=0.0,
              a_hi=float("inf"), check_every=1, npc=False, npc_eps=1e-8, reg_lambda=0.0,
              reg_beta=1.0, reg_eps=1e-8, grid=None, lr_min=0.0, cawr_T0=0, cawr_Tmult=1):
        """Run gpair_solve in place on A (and sigma).  Returns a dict report.
        npc: A holds the latent z on entry and x = (z + npc_eps)^2 on return.
        reg_lambda != 0 needs grid = (nx, ny, nz) of the kernel lattice.
        cawr_T0 > 0: learning rate of A (or z) by the warm-restart schedule."""
        o = _lib.SolveOpts()
        o.method = {"pgd": _lib.SOLVE_PGD, "adam": _lib.SOLVE_ADAM}[method]
        o.max_iters = int(max_iters)
        o.tol = float(tol)
        o.step = float(step)
        o.lr_A = float(lr_A)
        o.lr_sigma = float(lr_sigma)
        o.beta1, o.beta2, o.eps = float(beta1), float(beta2), float(eps)
        o.learn_sigma = 1 if learn_sigma else 0
        o.sigma_lo = float(sigma_lo if sigma_lo is not None else 0.5 * self.sigma_max)
        o.sigma_hi = float(sigma_hi if sigma_hi is not None else self.sigma_max)
        o.a_lo, o.a_hi = float(a_lo), float(a_hi)
        o.check_every = int(check_every)
        o.npc = 1 if npc else 0
        o.npc_eps = float(npc_eps)
        o.reg_lambda, o.reg_beta, o.reg_eps = float(reg_lambda), float(reg_beta), float(reg_eps)
        o.grid_nx, o.grid_ny, o.grid_nz = (int(v) for v in (grid or (0, 0, 0)))
        o.lr_min, o.cawr_T0, o.cawr_Tmult = float(lr_min), int(cawr_T0), int(cawr_Tmult)
        nbytes = ctypes.c_size_t()
        check(_lib.gpair_solve_workspace_size(self._h, ctypes.byref(o), ctypes.byref(nbytes)),
              "gpair_solve_workspace_size")
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        M = self.n_kernels
        pb = _dev(b, "b", self.n_sensors * self.n_samples, device=self.device)
        pa = _dev(A, "A", M, device=self.device)
        ps = _dev(sigma, "sigma", M, device=self.device)
        hist = (ctypes.c_double * (max_iters + 1))()
        rep = _lib.SolveReport()
        rep.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        st = check(_lib.gpair_solve(self._h, pb, pa, ps, ctypes.byref(o),
                                    ctypes.c_void_p(ws.data_ptr()), nbytes.value,
                                    ctypes.byref(rep), _stream()), "gpair_solve")
        return {"status": _lib.STATUS[st], "iters": rep.iters, "rel_residual": rep.rel_residual,
                "seconds": rep.seconds, "converged": bool(rep.converged),
                "history": [h for h in hist[: max_iters + 1]]}


def pgd_update(x, g, step, lo=0.0, hi=float("inf")):
    n = x.numel()
    check(_lib.gpair_pgd_update(n, _dev(x, "x", n), _dev(g, "g", n), float(step), float(lo),
                                float(hi), _stream()), "gpair_pgd_update")
    return x


def adam_update(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0,
                lo=float("-inf"), hi=float("inf")):
    n = x.numel()
    check(_lib.gpair_adam_update(n, _dev(x, "x", n), _dev(g, "g", n), _dev(m, "m", n),
                                 _dev(v, "v", n), float(grad_scale), float(lr), float(beta1),
                                 float(beta2), float(eps), int(t), float(lo), float(hi),
                                 _stream()), "gpair_adam_update")
    return x


def npc_map(z, eps=1e-8, out=None):
    """x = (z + eps)^2 (float32 device tensors; out may be z)."""
    n = z.numel()
    out = torch.empty_like(z) if out is None else out
    check(_lib.gpair_npc_map(n, _dev(z, "z", n), float(eps), _dev(out, "x", n), _stream()),
          "gpair_npc_map")
    return out


def npc_grad(z, gx, eps=1e-8, out=None):
    """gz = gx * 2 (z + eps) (out may be gx)."""
    n = z.numel()
    out = torch.empty_like(gx) if out is None else out
    check(_lib.gpair_npc_grad(n, _dev(z, "z", n), _dev(gx, "gx", n), float(eps),
                              _dev(out, "gz", n), _stream()), "gpair_npc_grad")
    return out


def vcr(x, beta, eps=1e-8, lam=1.0, grad=None, want_value=True, work=None):
    """The vessel continuity regulariser of a float32 volume x of shape
    (nz, ny, nx): returns (value as a float64 device tensor or None, grad), with
    grad += lam * dR/dx when `grad` is given (a zero tensor is made when
    grad is None and lam != 0)."""
    if x.dim() != 3:
        raise ValueError("x: expected a (nz, ny, nx) volume")
    nz, ny, nx = x.shape
    nbytes = ctypes.c_size_t()
    check(_lib.gpair_vcr_workspace_size(nx, ny, nz, ctypes.byref(nbytes)),
          "gpair_vcr_workspace_size")
    if work is None:
        work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=x.device)
    if grad is None and lam != 0.0:
        grad = torch.zeros_like(x)
    value = torch.empty(1, dtype=torch.float64, device=x.device) if want_value else None
    check(_lib.gpair_vcr(nx, ny, nz, _dev(x, "x", x.numel()), float(beta), float(eps),
                         float(lam), _dev(grad, "grad", x.numel()) if grad is not None else None,
                         _dev(value, "value", 1, dtype=torch.float64) if value is not None
                         else None, _dev(work, "work", dtype=torch.uint8), work.numel(),
                         _stream()), "gpair_vcr")
    return value, grad


def cawr_rate(t, eta_min, eta_max, T0, Tmult=1):
    r = ctypes.c_double()
    check(_lib.gpair_cawr_rate(int(t), float(eta_min), float(eta_max), int(T0), int(Tmult),
                               ctypes.byref(r)), "gpair_cawr_rate")
    return r.value


__all__ = ["Plan", "pgd_update", "adam_update", "npc_map", "npc_grad", "vcr", "cawr_rate",
           "GpairError"]


PEAK_PROBES = {0: "v_fma_f32", 1: "v_fma_f64", 2: "v_exp_f32", 3: "v_rsq_f32", 4: "v_rsq_f64"}


def peak_probe(kind, blocks=8192, iters=256, repeats=5):
    """Issue rate of one vector instruction (gpair_peak_probe): returns
    (wave64 instructions per second, kernel ms), the best of `repeats` timed
    launches after one warm-up, timed with events on the current stream."""
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    per_wave = ctypes.c_int64()

    def launch():
        check(_lib.gpair_peak_probe(int(kind), int(blocks), int(iters), _dev(out, "out"),
                                    ctypes.byref(per_wave), _stream()), "gpair_peak_probe")

    launch()
    best = None
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        launch()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    waves = blocks * 256 // 64
    return waves * per_wave.value / (best * 1e-3), best
