"""GPU parity of the anisotropic operators (gpair_forward_aniso,
gpair_adjoint_aniso: learnable anisotropic Gaussians) against the float64
oracle: relative L2 <= 1e-5 for the traces, gA and the six covariance
gradients."""
import numpy as np
import pytest
import torch

from oracle import ops as O
from paper_2602_03893_amd import inputs as I
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def plan_of(cen, sen, nt, smax, **kw):
    from paper_2602_03893_amd import Plan
    plan = Plan(cen, sen, nt, I.DT, I.C_SOUND, n_sigma=3.0, sigma_max=smax, **kw)
    return plan, O.Geometry(cen, sen, nt, I.DT, kw.get("t0", 0.0), I.C_SOUND, 3.0)


def check(plan, g, A, S6, delta, label, rows=None, ks=None):
    """S6 is (6, M) float32; the oracle takes (M, 6) float64 of the same values."""
    s_or = S6.astype(np.float64).T
    a64 = A.astype(np.float32).astype(np.float64)
    y = host(plan.forward_aniso(dev(A), dev(S6)))
    if rows is None:
        rows = np.arange(g.n_sensors)
    y_ref = O.forward_aniso(g.subset_sensors(rows), a64, s_or)
    ef = rel_l2(y[rows], y_ref)
    gA, gS = plan.adjoint_aniso(dev(A), dev(S6), dev(delta))
    gA, gS = host(gA), host(gS)
    if ks is None:
        ks = np.arange(len(A))
    rA, rS = O.adjoint_aniso(g.subset_kernels(ks), a64[ks], s_or[ks],
                             delta.astype(np.float32).astype(np.float64))
    eA, eS = rel_l2(gA[ks], rA), rel_l2(gS[:, ks].T, rS)
    _say(f"  {label}: forward {ef:.3e} gA {eA:.3e} gSigma {eS:.3e}")
    assert np.abs(y_ref).max() > 0 and np.abs(rS).max() > 0
    assert ef <= TOL and eA <= TOL and eS <= TOL


def test_toy_anisotropic():
    _say("case: toy workload, anisotropic covariances, signed amplitudes")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = I.uniform(w.n_kernels, seed=201, lo=-1.0, hi=1.0)
    S6 = I.covariances(w.n_kernels, seed=202, lo=0.3 * w.smax, hi=w.smax)
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=203)
    check(plan, g, A, S6, delta, "toy")


def test_point_cloud_clipped_windows():
    """A random cloud whose windows are clipped at both trace ends, with tiles
    of 64 kernels."""
    _say("case: point cloud, clipped windows, anisotropic")
    rng = np.random.default_rng(204)
    cen = rng.uniform(-1.5e-3, 1.5e-3, (1100, 3)).astype(np.float32)
    sen = I.fibonacci_hemisphere(70, 14e-3)
    t0 = 11e-3 / I.C_SOUND
    nt = int((8e-3 / I.C_SOUND) / I.DT)
    smax = 0.08e-3
    plan, g = plan_of(cen, sen, nt, smax, t0=t0, fwd_tile=64, adj_tile=64)
    A = I.uniform(len(cen), seed=205, lo=-0.5, hi=1.0)
    S6 = I.covariances(len(cen), seed=206, lo=0.2 * smax, hi=smax)
    delta = I.standard_normal((len(sen), nt), seed=207)
    check(plan, g, A, S6, delta, "point cloud")


def test_isotropic_covariance_matches_the_isotropic_operators():
    """Sigma = sigma^2 I through the anisotropic path against the oracle's
    isotropic operators (Eq. (single_forward))."""
    _say("case: toy workload, isotropic covariances through the anisotropic path")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = I.uniform(w.n_kernels, seed=208, lo=-1.0, hi=1.0)
    sig = I.uniform(w.n_kernels, seed=209, lo=0.4 * w.smax, hi=w.smax)
    S6 = np.zeros((6, w.n_kernels), np.float32)
    S6[0] = S6[1] = S6[2] = sig * sig
    y = host(plan.forward_aniso(dev(A), dev(S6)))
    s64 = np.sqrt(S6[0].astype(np.float64))
    y_ref = O.forward(g, A.astype(np.float64), s64)
    assert rel_l2(y, y_ref) <= TOL


def test_out_of_range_covariances_are_counted_and_replaced():
    """A covariance that is not positive definite and one whose largest
    eigenvalue exceeds sigma_max^2 are counted and evaluated as sigma_max^2 I."""
    _say("case: invalid covariances counted and replaced")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = I.uniform(w.n_kernels, seed=210, lo=0.2, hi=1.0)
    S6 = I.covariances(w.n_kernels, seed=211, lo=0.3 * w.smax, hi=0.9 * w.smax)
    bad = [7, 1234]
    S6[:, 7] = [1e-9, 1e-9, 1e-9, 2e-9, 0.0, 0.0]             # not positive definite
    S6[:, 1234] = [(1.5 * w.smax) ** 2, 1e-9, 1e-9, 0.0, 0.0, 0.0]  # too wide
    n0 = plan.sigma_violations()
    y = host(plan.forward_aniso(dev(A), dev(S6)))
    assert plan.sigma_violations() - n0 == 2
    ref6 = S6.astype(np.float64).T.copy()
    smax2 = (w.smax * (1.0 + 1e-6)) ** 2
    for k in bad:
        ref6[k] = [smax2, smax2, smax2, 0.0, 0.0, 0.0]
    y_ref = O.forward_aniso(g, A.astype(np.float64), ref6)
    assert rel_l2(y, y_ref) <= TOL


def test_paper_scale_anisotropic_sampled():
    """8,388,608 kernels x 1024 sensors x 4096 samples with axes in
    [0.035, 0.05] mm: the forward on 4 sensors, the gradients on 65,536
    kernels (every 128th)."""
    _say("case: paper workload, anisotropic covariances, sampled")
    w = I.WORKLOADS["paper"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = I.phantom(w) + 0.05
    S6 = I.covariances(w.n_kernels, seed=212, lo=0.35 * w.smax, hi=0.5 * w.smax)
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=213)
    check(plan, g, A.astype(np.float32), S6, delta, "paper scale",
          rows=np.array([0, 341, 682, 1023]), ks=np.arange(5, w.n_kernels, 128))


def test_admission_matches_the_eigenvalue_rule():
    """Covariances drawn across the boundary (axes up to 1.2 sigma_max): the
    operators count exactly those whose largest eigenvalue (numpy eigvalsh of
    the float32 entries) exceeds sigma_max^2 (1 + 1e-6)^2."""
    _say("case: admission of covariances across the sigma_max boundary")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    S6 = I.covariances(w.n_kernels, seed=214, lo=0.3 * w.smax, hi=1.2 * w.smax)
    xx, yy, zz, xy, xz, yz = S6.astype(np.float64)
    M = np.stack([np.stack([xx, xy, xz], -1), np.stack([xy, yy, yz], -1),
                  np.stack([xz, yz, zz], -1)], -2)
    expected = int(np.sum(np.linalg.eigvalsh(M)[:, -1] > (w.smax * (1.0 + 1e-6)) ** 2))
    assert 0 < expected < w.n_kernels
    A = I.uniform(w.n_kernels, seed=215, lo=0.2, hi=1.0)
    n0 = plan.sigma_violations()
    plan.forward_aniso(dev(A), dev(S6))
    assert plan.sigma_violations() - n0 == expected


def test_needle_and_pancake_covariances():
    """Strongly anisotropic kernels (axes from 0.01 to 1 of sigma_max): from
    some directions the window holds no sample or one, and the amplitude factor
    sqrt(det)/sigma_n^3 varies by orders of magnitude across sensors."""
    _say("case: toy workload, axes 0.01 .. 1 of sigma_max")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = I.uniform(w.n_kernels, seed=216, lo=-1.0, hi=1.0)
    S6 = I.covariances(w.n_kernels, seed=217, lo=0.01 * w.smax, hi=w.smax)
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=218)
    check(plan, g, A, S6, delta, "needles and pancakes")


def test_autograd_function_and_a_descent():
    """The autograd Function: loss = 0.5 ||y(A, Sigma) - b||^2; its gradients
    equal the oracle's adjoint of the residual for A and the six covariance
    parameters, and Adam on A and Sigma lowers the loss."""
    _say("case: toy workload, autograd through the anisotropic operators")
    from paper_2602_03893_amd import aniso_forward
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    S_true = I.covariances(w.n_kernels, seed=219, lo=0.4 * w.smax, hi=0.8 * w.smax)
    b = O.forward_aniso(g, I.phantom(w).astype(np.float64), S_true.astype(np.float64).T)
    A = torch.tensor(I.uniform(w.n_kernels, seed=220, lo=0.0, hi=0.5), device="cuda",
                     requires_grad=True)
    S6 = torch.tensor(I.covariances(w.n_kernels, seed=221, lo=0.4 * w.smax, hi=0.8 * w.smax),
                      device="cuda", requires_grad=True)
    bt = dev(b)
    y = aniso_forward(A, S6, plan)
    loss = 0.5 * torch.sum((y - bt) ** 2)
    loss.backward()
    resid = host(y - bt)
    rA, rS = O.adjoint_aniso(g, host(A), host(S6).T, resid)
    eA, eS = rel_l2(host(A.grad), rA), rel_l2(host(S6.grad).T, rS)
    _say(f"  autograd gA {eA:.3e} gSigma {eS:.3e}")
    assert eA <= TOL and eS <= TOL
    opt = torch.optim.Adam([{"params": [A], "lr": 1e-2},
                            {"params": [S6], "lr": 1e-3 * (0.6 * w.smax) ** 2}])
    losses = []
    for _ in range(8):
        opt.zero_grad()
        l = 0.5 * torch.sum((aniso_forward(A, S6, plan) - bt) ** 2)
        l.backward()
        opt.step()
        losses.append(float(l))
    assert losses[-1] < 0.9 * losses[0]


def test_centre_gradient_of_anisotropic_kernels():
    """gpair_adjoint_aniso_centres against the oracle: the centre gradient (all
    three components as one vector), with gA and gSigma from the same call, on
    the toy workload and on strongly anisotropic covariances (float64 window
    and direction terms); isotropic covariances give the isotropic centre
    gradient."""
    _say("case: centre gradient of anisotropic kernels")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = I.uniform(w.n_kernels, seed=222, lo=-1.0, hi=1.0)
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=223)
    a64 = A.astype(np.float64)
    for label, S6 in (("axes 0.3 .. 1", I.covariances(w.n_kernels, seed=224, lo=0.3 * w.smax,
                                                      hi=w.smax)),
                      ("axes 0.01 .. 1", I.covariances(w.n_kernels, seed=225, lo=0.01 * w.smax,
                                                       hi=w.smax))):
        gA, gS, gC = plan.adjoint_aniso_centres(dev(A), dev(S6), dev(delta))
        s_or = S6.astype(np.float64).T
        rC = O.adjoint_aniso_centres(g, a64, s_or, delta.astype(np.float64))
        rA, rS = O.adjoint_aniso(g, a64, s_or, delta.astype(np.float64))
        eC, eA, eS = rel_l2(host(gC), rC), rel_l2(host(gA), rA), rel_l2(host(gS).T, rS)
        _say(f"  {label}: gcentres {eC:.3e} gA {eA:.3e} gSigma {eS:.3e}")
        assert eC <= TOL and eA <= TOL and eS <= TOL
    sig = I.uniform(w.n_kernels, seed=226, lo=0.4 * w.smax, hi=w.smax)
    S6 = np.zeros((6, w.n_kernels), np.float32)
    S6[0] = S6[1] = S6[2] = sig * sig
    _, _, gC = plan.adjoint_aniso_centres(dev(A), dev(S6), dev(delta), want_sigma=False)
    rC = O.adjoint_centres(g, a64, np.sqrt(S6[0].astype(np.float64)), delta.astype(np.float64))
    e = rel_l2(host(gC), rC)
    _say(f"  isotropic covariances: gcentres {e:.3e}")
    assert e <= TOL


def test_deterministic_anisotropic_forward():
    """With the plan's deterministic option the anisotropic forward is
    bitwise equal over two calls and still within 1e-5 of the oracle."""
    _say("case: point cloud, deterministic anisotropic forward")
    rng = np.random.default_rng(227)
    cen = rng.uniform(-1.5e-3, 1.5e-3, (900, 3)).astype(np.float32)
    sen = I.fibonacci_hemisphere(70, 14e-3)
    nt = 512
    smax = 0.08e-3
    plan, g = plan_of(cen, sen, nt, smax, deterministic=True, fwd_tile=64, adj_tile=64)
    A = I.uniform(len(cen), seed=228, lo=-0.5, hi=1.0)
    S6 = I.covariances(len(cen), seed=229, lo=0.2 * smax, hi=smax)
    y1 = host(plan.forward_aniso(dev(A), dev(S6)))
    y2 = host(plan.forward_aniso(dev(A), dev(S6)))
    assert np.array_equal(y1, y2)
    y_ref = O.forward_aniso(g, A.astype(np.float64), S6.astype(np.float64).T)
    e = rel_l2(y1, y_ref)
    _say(f"  deterministic forward {e:.3e}")
    assert e <= TOL


def test_autograd_rejects_covariances_the_operator_would_replace():
    """A covariance outside the admitted set (not positive definite, or an
    eigenvalue above sigma_max^2) makes the autograd forward raise; with
    check=False the output equals the forward at sigma_max^2 I for those
    kernels."""
    from paper_2602_03893_amd import aniso_forward
    _say("case: toy workload, autograd with inadmissible covariances")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = dev(I.phantom(w))
    S6 = I.covariances(w.n_kernels, seed=231, lo=0.4 * w.smax, hi=0.8 * w.smax)
    y_ok = host(aniso_forward(A, dev(S6), plan))
    assert np.isfinite(y_ok).all()
    bad = S6.copy()
    bad[:, 7] = [2.0 * w.smax ** 2, 0.5 * w.smax ** 2, 0.5 * w.smax ** 2, 0.0, 0.0, 0.0]
    bad[:, 11] = [0.5 * w.smax ** 2, 0.5 * w.smax ** 2, -0.1 * w.smax ** 2, 0.0, 0.0, 0.0]
    with pytest.raises(ValueError, match="2 kernel"):
        aniso_forward(A, dev(bad), plan)
    y_rep = host(aniso_forward(A, dev(bad), plan, check=False))
    fixed = bad.copy()
    fixed[:, 7] = fixed[:, 11] = [w.smax ** 2, w.smax ** 2, w.smax ** 2, 0.0, 0.0, 0.0]
    y_ref = host(aniso_forward(A, dev(fixed), plan))
    assert rel_l2(y_rep, y_ref) <= 1e-6
