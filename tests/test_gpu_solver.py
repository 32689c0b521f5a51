"""GPU parity of the reconstruction rows: residual and norms, PGD and Adam
updates, the gpair_solve driver and the autograd Function, against the float64
oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from oracle import ops as O, solvers as S
from paper_2602_03893_amd import inputs as I
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def toy():
    from paper_2602_03893_amd import Plan
    _say("case: toy workload for the solver rows")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan = Plan(cen, sen, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma, sigma_max=w.smax)
    g = O.Geometry(cen, sen, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    x_true = I.phantom(w)
    sigma = np.full(w.n_kernels, w.sigma, np.float32)
    b = O.forward(g, x_true, sigma.astype(np.float64)).astype(np.float32)
    return w, plan, g, x_true, sigma, b


def test_residual_and_norms(toy):
    w, plan, g, _, _, b = toy
    y = I.standard_normal((w.n_sensors, w.n_samples), seed=40) * 1e-3 + b
    yt, bt = dev(y), dev(b)
    delta = torch.empty_like(yt)
    norms = host(plan.residual(yt, bt, scale=0.37, delta=delta))
    r64 = y.astype(np.float64) - b.astype(np.float64)
    assert norms[0] == pytest.approx(np.sum(r64 * r64), rel=1e-12)
    assert norms[1] == pytest.approx(np.sum(b.astype(np.float64) ** 2), rel=1e-12)
    ref = np.float32(0.37) * (y - b)
    assert np.array_equal(host(delta).astype(np.float32), ref)
    again = host(plan.residual(yt, bt))
    assert np.array_equal(again, norms)   # fixed summation order: bitwise stable
    # in place (delta aliases y)
    plan.residual(yt, bt, scale=2.0, delta=yt)
    assert np.array_equal(host(yt).astype(np.float32), np.float32(2.0) * (y - b))


def test_pgd_and_adam_updates():
    from paper_2602_03893_amd import adam_update, pgd_update
    n = 10007
    x0 = I.uniform(n, seed=50, lo=-0.2, hi=1.0)
    gvec = I.standard_normal(n, seed=51)
    x = dev(x0)
    pgd_update(x, dev(gvec), 0.05, lo=0.0, hi=0.8)
    ref = np.clip(x0.astype(np.float64) - 0.05 * gvec.astype(np.float64), 0.0, 0.8)
    assert np.max(np.abs(host(x) - ref)) <= 1e-6
    # Adam: ten steps against the float64 oracle step
    x = dev(x0)
    m = torch.zeros_like(x)
    v = torch.zeros_like(x)
    xr = x0.astype(np.float64)
    mr = np.zeros(n)
    vr = np.zeros(n)
    for t in range(1, 11):
        gt = I.standard_normal(n, seed=60 + t) * (1.0 + 0.1 * t)
        adam_update(x, dev(gt), m, v, t, 1e-2, 0.9, 0.999, 1e-8, lo=0.0, hi=1.0)
        xr = S.adam_step(xr, gt.astype(np.float64), mr, vr, t, 1e-2, 0.9, 0.999, 1e-8, 0.0, 1.0)
    assert rel_l2(host(x), xr) <= 1e-5


def test_solve_pgd_matches_oracle(toy):
    """20 projected-gradient iterations from zero with step 1/||A^T A||."""
    w, plan, g, _, sigma, b = toy
    lam = S.power_iteration(g, sigma.astype(np.float64), iters=100, seed=0)
    step = 1.0 / lam
    A = torch.zeros(w.n_kernels, dtype=torch.float32, device="cuda")
    rep = plan.solve(dev(b), A, dev(sigma), method="pgd", max_iters=20, step=step)
    x_ref, hist_ref = S.pgd(g, sigma.astype(np.float64), b.astype(np.float64),
                            np.zeros(w.n_kernels), step, 20)
    hist = np.array(rep["history"])
    _say(f"  PGD rho: gpu {hist[-1]:.6f} oracle {hist_ref[-1]:.6f}")
    assert rep["iters"] == 20 and rep["status"] == "GPAIR_NOT_CONVERGED"
    assert np.max(np.abs(hist - hist_ref) / np.array(hist_ref)) <= 1e-5
    assert rel_l2(host(A), x_ref) <= 1e-4
    assert hist[-1] < hist[0]


def test_solve_adam_matches_oracle(toy):
    """20 Adam iterations on A and sigma (sigma clamped) from zero."""
    w, plan, g, _, sigma, b = toy
    A = torch.zeros(w.n_kernels, dtype=torch.float32, device="cuda")
    sg = dev(sigma)
    lr_s = 1e-3 * w.sigma
    rep = plan.solve(dev(b), A, sg, method="adam", max_iters=20, lr_A=0.05, lr_sigma=lr_s,
                     learn_sigma=True, sigma_lo=0.5 * w.sigma, sigma_hi=w.smax)
    a_ref, s_ref, hist_ref = S.adam(g, np.zeros(w.n_kernels), sigma.astype(np.float64),
                                    b.astype(np.float64), 20, lr_a=0.05, lr_s=lr_s,
                                    learn_sigma=True, s_lo=0.5 * w.sigma, s_hi=w.smax)
    hist = np.array(rep["history"])
    _say(f"  Adam rho: gpu {hist[-1]:.6f} oracle {hist_ref[-1]:.6f}")
    assert np.max(np.abs(hist - hist_ref) / np.array(hist_ref)) <= 1e-3
    assert rel_l2(host(A), a_ref) <= 1e-3
    assert rel_l2(host(sg), s_ref) <= 1e-6


def test_solve_stops_at_tolerance_and_rejects_nonfinite(toy):
    from paper_2602_03893_amd import GpairError
    w, plan, g, x_true, sigma, b = toy
    A = torch.zeros(w.n_kernels, dtype=torch.float32, device="cuda")
    rep = plan.solve(dev(b), A, dev(sigma), method="adam", max_iters=400, tol=0.2,
                     lr_A=0.05)
    assert rep["converged"] and rep["status"] == "GPAIR_OK"
    assert rep["rel_residual"] <= 0.2 and rep["iters"] < 400
    assert rep["history"][rep["iters"]] == pytest.approx(rep["rel_residual"])
    bad = b.copy()
    bad[3, 100] = np.nan
    with pytest.raises(GpairError, match="NONFINITE"):
        plan.solve(dev(bad), A, dev(sigma), method="adam", max_iters=2)


def test_autograd_matches_oracle_and_differences(toy):
    """loss = 0.5 ||y(A, sigma) - b||^2 through GpairForward; the gradients
    against the oracle adjoint of the oracle residual, and the sigma-gradient
    against central differences of the oracle loss at 16 kernels."""
    from paper_2602_03893_amd import GpairForward
    w, plan, g, x_true, sigma, b = toy
    A0 = (0.8 * x_true).astype(np.float32)
    s0 = I.uniform(w.n_kernels, seed=70, lo=0.6 * w.sigma, hi=w.sigma)
    A = dev(A0).requires_grad_(True)
    sg = dev(s0).requires_grad_(True)
    y = GpairForward.apply(A, sg, plan)
    loss = 0.5 * torch.sum((y.double() - dev(b).double()) ** 2)
    loss.backward()
    s64 = s0.astype(np.float64)
    r = O.forward(g, A0, s64) - b.astype(np.float64)
    gA, gS = O.adjoint(g, A0, s64, r)
    eA, eS = rel_l2(host(A.grad), gA), rel_l2(host(sg.grad), gS)
    _say(f"  autograd: gA {eA:.2e} gsigma {eS:.2e}")
    assert eA <= 1e-5 and eS <= 1e-5
    pick = np.random.default_rng(71).choice(w.n_kernels, 16, replace=False)
    gs = host(sg.grad)
    for k in pick:
        h = 1e-6 * s64[k]
        sp, sm = s64.copy(), s64.copy()
        sp[k] += h
        sm[k] -= h
        lp = 0.5 * np.sum((O.forward(g, A0, sp) - b) ** 2)
        lm = 0.5 * np.sum((O.forward(g, A0, sm) - b) ** 2)
        fd = (lp - lm) / (2 * h)
        assert abs(gs[k] - fd) <= 1e-3 * max(abs(fd), 1e-3 * np.abs(gs).max()), (k, gs[k], fd)


def test_autograd_rejects_widths_the_operator_would_clamp(toy):
    """A sigma_k outside (0, sigma_max] makes the autograd forward raise
    (the operator would clamp it and differentiate another function);
    check=False accepts the clamped operator, whose output equals the one at
    the clamped widths."""
    from paper_2602_03893_amd import gpair_forward
    w, plan, g, x_true, sigma, b = toy
    _say("case: autograd forward with out-of-range widths")
    A = dev(x_true)
    s_bad = sigma.copy()
    s_bad[5] = 1.5 * w.smax
    s_bad[9] = -1.0
    y_ok = host(gpair_forward(A, dev(sigma), plan))
    assert np.isfinite(y_ok).all()
    with pytest.raises(ValueError, match="2 kernel"):
        gpair_forward(A, dev(s_bad), plan)
    y_clamped = host(gpair_forward(A, dev(s_bad), plan, check=False))
    s_clamp = sigma.copy()
    s_clamp[5] = w.smax
    s_clamp[9] = w.smax
    y_ref = host(gpair_forward(A, dev(s_clamp), plan))
    assert rel_l2(y_clamped, y_ref) <= 1e-6
