"""gpair_assa_adjoint_static, the entry point that allocates nothing, called
through the C ABI and checked against gpair_assa_adjoint (the same operator
with a caller work buffer) on the same inputs: two calls in a row, the second
with a smaller input than the first, then an input too large for the fixed
device buffer, which is refused before anything is launched.

Bar: relative L2 <= 1e-5 against the work-buffer entry point (both run the
same kernels, so the results are expected to be identical)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2602_03893_amd import inputs as I
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _plan(w, n_samples=None):
    from paper_2602_03893_amd import Plan
    cen, sen = I.geometry_arrays(w)
    return Plan(cen, sen, n_samples or w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma,
                sigma_max=w.smax, device="cuda:0")


def test_static_adjoint_matches_the_work_buffer_entry_point():
    from paper_2602_03893_amd import _lib
    torch.cuda.set_device(0)
    cap = int(_lib.gpair_assa_static_scratch_bytes())
    _say(f"fixed buffer: {cap} bytes")
    for name, seed in (("mid", 81), ("toy", 82)):   # the second input is smaller
        w = I.WORKLOADS[name]
        plan = _plan(w)
        grid = plan.assa_grid(w.sigma)
        used = w.n_sensors * grid["n_fine"] * 4
        _say(f"case: {name}: {w.n_kernels} kernels, {w.n_sensors} sensors, sigma {w.sigma}, "
             f"alpha {grid['alpha']}, residual buffer {used} bytes")
        assert used <= cap
        delta = torch.as_tensor(I.standard_normal((w.n_sensors, w.n_samples), seed=seed),
                                device="cuda:0")
        out = torch.full((w.n_kernels,), float("nan"), dtype=torch.float32, device="cuda:0")
        st = _lib.gpair_assa_adjoint_static(plan._h, float(w.sigma), _ptr(delta), _ptr(out),
                                            _stream())
        assert st == 0, _lib.gpair_status_string(st)
        ref = plan.assa_adjoint(w.sigma, delta)
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        err = rel_l2(got, want)
        _say(f"  rel L2 against gpair_assa_adjoint {err:.3e}, identical: "
             f"{bool(np.array_equal(got, want))}")
        assert np.all(np.isfinite(got)) and np.abs(want).max() > 0
        assert err <= 1e-5
        del plan
    # 64 sensors x 3 x 100,000 fine samples x 4 B = 76.8 MB > 64 MiB: refused.
    w = I.WORKLOADS["toy"]
    plan = _plan(w, n_samples=100_000)
    sigma = 0.05e-3
    assert w.n_sensors * plan.assa_grid(sigma)["n_fine"] * 4 > cap
    delta = torch.zeros((w.n_sensors, 100_000), dtype=torch.float32, device="cuda:0")
    out = torch.full((w.n_kernels,), float("nan"), dtype=torch.float32, device="cuda:0")
    st = _lib.gpair_assa_adjoint_static(plan._h, sigma, _ptr(delta), _ptr(out), _stream())
    _say(f"case: oversized residual buffer: status {_lib.gpair_status_string(st)}")
    assert _lib.gpair_status_string(st) == b"GPAIR_ERR_WORKSPACE"
    torch.cuda.synchronize()
    assert torch.isnan(out).all()
