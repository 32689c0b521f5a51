"""GPU parity of the full objective (through the C ABI): the non-negativity
parameterisation, the vessel continuity regulariser (value and gradient) and
gpair_solve with NPC, VCR and the warm-restart schedule (Algorithm 2), against
the float64 oracle (oracle/objective.py).

Bars: NPC elementwise relative 1e-6 (float32); VCR value relative 1e-11 (float64
differences and sums on both sides), gradient relative L2 1e-6 and max error
1e-5 of its largest entry (normalised terms stored in float32); solver replays
rho per iteration 1e-3 relative, as the Adam replay of the data term.
"""
import numpy as np
import pytest
import torch

from oracle import objective as J
from oracle import ops as O
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


def test_npc_map_and_chain_rule():
    from paper_2602_03893_amd import npc_grad, npc_map
    rng = np.random.default_rng(0)
    z = rng.normal(size=100_003).astype(np.float32)
    gx = rng.normal(size=z.size).astype(np.float32)
    x = host(npc_map(dev(z)))
    ref = J.npc_map(z.astype(np.float64))
    assert np.all(np.abs(x - ref) <= 1e-6 * ref + 1e-30)
    gz = host(npc_grad(dev(z), dev(gx)))
    refg = J.npc_grad(z.astype(np.float64), gx.astype(np.float64))
    assert np.all(np.abs(gz - refg) <= 1e-6 * np.abs(refg) + 1e-30)
    # in place on the gradient
    g = dev(gx)
    npc_grad(dev(z), g, out=g)
    assert np.array_equal(host(g), gz)


def check_vcr(x, beta, lam, label):
    from paper_2602_03893_amd import vcr
    _say(f"VCR parity: {label}, shape {x.shape}, beta {beta}, lambda {lam}")
    x32 = x.astype(np.float32)
    x64 = x32.astype(np.float64)
    # an existing gradient of the same size as lambda * grad R: grad += lambda dR/dx
    # (a much larger one would only measure the float32 rounding of the sum)
    g0 = (lam * np.random.default_rng(9).normal(size=x.shape)).astype(np.float32)
    val, grad = vcr(dev(x32), beta, lam=lam, grad=dev(g0))
    val = float(host(val)[0])
    ref_v = J.vcr_value(x64, beta)
    ref_g = g0.astype(np.float64) + lam * J.vcr_grad(x64, beta)
    gg = host(grad)
    dv = abs(val - ref_v) / abs(ref_v)
    eg = rel_l2(gg - g0, ref_g - g0)
    scale = np.abs(ref_g - g0).max()
    # a volume with no interior stencil has a zero gradient: then exactly g0
    em = np.abs(gg - ref_g).max() / scale if scale > 0 else np.abs(gg - g0).max()
    _say(f"  value rel {dv:.2e}, gradient rel L2 {eg:.2e}, max {em:.2e}")
    assert dv <= 1e-11
    assert eg <= 1e-6 and em <= 1e-5


@pytest.mark.parametrize("shape", [(5, 6, 7), (1, 2, 7), (2, 1, 1), (33, 17, 9), (7, 1, 300)])
def test_vcr_small_and_degenerate_volumes(shape):
    x = np.random.default_rng(1).uniform(size=shape)
    check_vcr(x, 0.5, 1.0, "uniform random")
    check_vcr(x, 0.0, 2.5, "Hessian only")


def test_vcr_mid_phantom_and_value_only():
    from paper_2602_03893_amd import vcr
    w = I.WORKLOADS["mid"]
    x = I.phantom(w).reshape(w.grid[2], w.grid[1], w.grid[0])
    check_vcr(x, 0.3, 1e-3, "mid vessel phantom")
    val, grad = vcr(dev(x), 0.3, lam=0.0, want_value=True)
    assert grad is None
    assert float(host(val)[0]) == pytest.approx(J.vcr_value(x.astype(np.float64), 0.3),
                                                 rel=1e-11)


def test_vcr_paper_volume():
    w = I.WORKLOADS["paper"]
    x = I.phantom(w).reshape(w.grid[2], w.grid[1], w.grid[0])
    check_vcr(x, 1.0, 1e-4, "paper-scale vessel phantom (256x256x128)")


@pytest.fixture(scope="module")
def toy():
    from paper_2602_03893_amd import Plan
    _say("case: toy workload for Algorithm 2 with NPC, VCR and CAWR")
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan = Plan(cen, sen, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma, sigma_max=w.smax)
    g = O.Geometry(cen, sen, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    x_true = I.phantom(w)
    sigma = np.full(w.n_kernels, w.sigma, np.float32)
    b = O.forward(g, x_true, sigma.astype(np.float64)).astype(np.float32)
    return w, plan, g, sigma, b


@pytest.mark.parametrize("lam", [0.0, 1e-4])
def test_solve_full_objective_matches_oracle(toy, lam):
    w, plan, g, sigma, b = toy
    grid = w.grid
    z0 = 0.3 * I.uniform(w.n_kernels, seed=5)
    kw = dict(lam=lam, beta=0.5, eta_min=1e-3, eta_max=0.05, T0=8, Tmult=2)
    z = dev(z0)
    rep = plan.solve(dev(b), z, dev(sigma), method="adam", max_iters=30, lr_A=kw["eta_max"],
                     npc=True, reg_lambda=lam, reg_beta=kw["beta"], grid=grid,
                     lr_min=kw["eta_min"], cawr_T0=kw["T0"], cawr_Tmult=kw["Tmult"])
    x_ref, z_ref, hist_ref = J.gpair(g, sigma.astype(np.float64), b.astype(np.float64), grid,
                                     30, kw["lam"], kw["beta"], kw["eta_min"], kw["eta_max"],
                                     kw["T0"], kw["Tmult"], z0=z0.astype(np.float64))
    hist = np.array(rep["history"])
    _say(f"  lambda {lam}: rho gpu {hist[0]:.4f} -> {hist[-1]:.6f}, oracle -> {hist_ref[-1]:.6f}")
    assert np.max(np.abs(hist - hist_ref) / np.array(hist_ref)) <= 1e-3
    x = host(z)  # on return the array holds x = (z + eps)^2
    assert np.all(x >= 0)
    assert rel_l2(x, x_ref) <= 1e-3
    assert hist[-1] < 0.5 * hist[0]


def test_solve_from_zero_latent_as_in_the_algorithm(toy):
    """z^(0) = 0 as in the algorithm: x = eps^2 and the first gradients are
    2 eps times the adjoint, so the first Adam steps are far below lr_0 (the
    gradient is comparable to Adam's eps); the replay still has to follow the
    oracle and descend."""
    w, plan, g, sigma, b = toy
    z = dev(np.zeros(w.n_kernels, np.float32))
    rep = plan.solve(dev(b), z, dev(sigma), method="adam", max_iters=40, lr_A=0.02, npc=True,
                     reg_lambda=1e-5, reg_beta=0.5, grid=w.grid, lr_min=1e-3, cawr_T0=20,
                     cawr_Tmult=1)
    _, _, hist_ref = J.gpair(g, sigma.astype(np.float64), b.astype(np.float64), w.grid, 40,
                             1e-5, 0.5, 1e-3, 0.02, 20, 1)
    hist = np.array(rep["history"])
    _say(f"  z0 = 0: rho {hist[0]:.4f} -> {hist[-1]:.4f} (oracle {hist_ref[-1]:.4f})")
    assert hist[0] == pytest.approx(1.0, rel=1e-6)
    assert np.max(np.abs(hist - hist_ref) / np.array(hist_ref)) <= 1e-3
    assert hist[-1] < 0.9


def test_solve_rejects_a_grid_that_does_not_match(toy):
    from paper_2602_03893_amd import GpairError
    w, plan, g, sigma, b = toy
    with pytest.raises(GpairError, match="INVALID_ARG"):
        plan.solve(dev(b), dev(np.zeros(w.n_kernels)), dev(sigma), method="adam", max_iters=1,
                   reg_lambda=1e-4, grid=(16, 16, 15))
    with pytest.raises(GpairError, match="INVALID_ARG"):
        plan.solve(dev(b), dev(np.zeros(w.n_kernels)), dev(sigma), method="pgd", max_iters=1,
                   npc=True)
