"""GPU parity of the centre gradient (gpair_adjoint_centres, learnable kernel
centres) against the float64 oracle: relative L2 <= 1e-5 for the centre
gradient (all three components as one vector), and for the amplitude and
sigma gradients the same call returns."""
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


def check(plan, g, A, sigma, delta, label, ks=None):
    gA, gS, gC = plan.adjoint_centres(dev(A), dev(sigma), dev(delta))
    gA, gS, gC = host(gA), host(gS), host(gC)
    s64 = sigma.astype(np.float32).astype(np.float64)
    d64 = delta.astype(np.float32).astype(np.float64)
    a64 = A.astype(np.float32).astype(np.float64)
    if ks is None:
        ks = np.arange(len(A))
    gk = g.subset_kernels(ks)
    rC = O.adjoint_centres(gk, a64[ks], s64[ks], d64)
    rA, rS = O.adjoint(gk, a64[ks], s64[ks], d64)
    eC, eA, eS = rel_l2(gC[ks], rC), rel_l2(gA[ks], rA), rel_l2(gS[ks], rS)
    _say(f"  {label}: gcentres {eC:.3e} gA {eA:.3e} gsigma {eS:.3e}")
    assert np.abs(rC).max() > 0
    assert eC <= TOL and eA <= TOL and eS <= TOL


def plan_of(cen, sen, nt, smax, **kw):
    from paper_2602_03893_amd import Plan
    plan = Plan(cen, sen, nt, I.DT, I.C_SOUND, n_sigma=3.0, sigma_max=smax, **kw)
    return plan, O.Geometry(cen, sen, nt, I.DT, kw.get("t0", 0.0), I.C_SOUND, 3.0)


def test_toy_centre_gradient():
    _say("case: toy workload, per-kernel sigma, signed amplitudes")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = I.uniform(w.n_kernels, seed=101, lo=-1.0, hi=1.0)
    sigma = I.uniform(w.n_kernels, seed=102, lo=0.4 * w.smax, hi=w.smax)
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=103)
    check(plan, g, A, sigma, delta, "toy")


def test_point_cloud_clipped_windows_and_float64_blocks():
    """A random point cloud whose windows are clipped at both trace ends,
    plus a sparse cluster decided in float64 throughout."""
    _say("case: point cloud with clipped windows and float64 blocks")
    rng = np.random.default_rng(104)
    dense = rng.uniform(-1.5e-3, 1.5e-3, (900, 3))
    sparse = rng.uniform(-2e-3, 2e-3, (120, 3)) + np.array([0.0, 6e-3, 0.0])
    cen = np.concatenate([dense, sparse]).astype(np.float32)
    sen = I.fibonacci_hemisphere(70, 14e-3)
    t0 = 11e-3 / I.C_SOUND
    nt = int((8e-3 / I.C_SOUND) / I.DT)
    smax = 0.08e-3
    plan, g = plan_of(cen, sen, nt, smax, t0=t0, fwd_tile=64, adj_tile=64)
    nf64, _ = plan.filter_stats()
    _say(f"  blocks in float64: {nf64} of {plan.info()['adj_tiles']}")
    A = I.uniform(len(cen), seed=105, lo=-0.5, hi=1.0)
    sigma = I.uniform(len(cen), seed=106, lo=0.3 * smax, hi=smax)
    delta = I.standard_normal((len(sen), nt), seed=107)
    check(plan, g, A, sigma, delta, "point cloud")


def test_paper_scale_centre_gradient_sampled():
    """8,388,608 kernels x 1024 sensors x 4096 samples at the benchmark's
    sigma spread: the centre gradient on 131,072 kernels (every 64th)."""
    _say("case: paper workload, sigma 0.05 mm +-5 %, centre gradient sampled")
    w = I.WORKLOADS["paper"]
    cen, sen = I.geometry_arrays(w)
    plan, g = plan_of(cen, sen, w.n_samples, w.smax)
    A = I.phantom(w) + 0.05
    sigma = (w.sigma * I.uniform(w.n_kernels, seed=108, lo=0.95, hi=1.05)).astype(np.float32)
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=109)
    check(plan, g, A, sigma, delta, "paper scale", ks=np.arange(11, w.n_kernels, 64))
