"""GPU parity of the learned warm start (row a8): the least-squares rescale
with fallback, and the whole chain half-resolution adjoint -> U-Net ->
trilinear x2 -> rescale, against the float64 oracles (through the C ABI)."""
import os

import numpy as np
import pytest
import torch

from oracle import nn as N
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


@pytest.fixture(scope="module")
def toy():
    from paper_2602_03893_amd import Plan
    w = I.WORKLOADS["toy"]
    cen, sen = I.geometry_arrays(w)
    plan = Plan(cen, sen, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma, sigma_max=w.smax)
    g = O.Geometry(cen, sen, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    x_true = I.phantom(w)
    sigma = np.full(w.n_kernels, w.sigma, np.float32)
    b = O.forward(g, x_true, sigma.astype(np.float64)).astype(np.float32)
    return w, plan, g, x_true, sigma, b


def test_warm_rescale_matches_least_squares(toy):
    w, plan, g, x_true, sigma, b = toy
    _say("case: warm rescale, toy workload")
    x0 = np.maximum(0.6 * x_true + 0.05 * I.standard_normal(w.n_kernels, seed=90), 0).astype(np.float32)
    A = dev(x0)
    rep = plan.warm_rescale(A, dev(sigma), dev(b))
    y = O.forward(g, x0, sigma.astype(np.float64))
    b64 = b.astype(np.float64)
    c = max(0.0, float(y @ b64.ravel() if y.ndim == 1 else np.sum(y * b64)) / float(np.sum(y * y)))
    rho = np.linalg.norm(c * y - b64) / np.linalg.norm(b64)
    _say(f"  c* gpu {rep['c_star']:.8f} oracle {c:.8f}; rho gpu {rep['rho']:.6f} oracle {rho:.6f}")
    assert not rep["fell_back"]
    assert rep["c_star"] == pytest.approx(c, rel=1e-5)
    assert rep["rho"] == pytest.approx(rho, rel=1e-4, abs=1e-6)
    assert rep["rho"] < 1.0
    assert rel_l2(host(A), c * x0.astype(np.float64)) <= 1e-6
    # an anti-correlated start falls back to zero
    A = dev(-x0)
    rep = plan.warm_rescale(A, dev(sigma), dev(b))
    assert rep["fell_back"] and rep["c_star"] == 0.0 and rep["rho"] == 1.0
    assert not host(A).any()
    # b = 0 is rejected, the start untouched
    from paper_2602_03893_amd import GpairError
    A = dev(x0)
    with pytest.raises(GpairError, match="INVALID_ARG"):
        plan.warm_rescale(A, dev(sigma), torch.zeros_like(dev(b)))
    assert np.array_equal(host(A), x0.astype(np.float64))


def test_warm_start_chain_matches_oracle():
    """Full grid 32 x 32 x 16 (0.2 mm), half grid 16 x 16 x 8 (0.4 mm), 64
    sensors; a 4-level U-Net with seeded weights."""
    from paper_2602_03893_amd import Plan
    from paper_2602_03893_amd import nn as m
    _say("case: warm start chain, full 32x32x16 / half 16x16x8, 4 levels")
    nx, ny, nz = 32, 32, 16
    sp, sp2 = 0.2e-3, 0.4e-3
    s_full, s_half = 0.1e-3, 0.2e-3
    nt, dt, c = 512, I.DT, I.C_SOUND
    cen = I.grid_centres(nx, ny, nz, sp)
    cen2 = I.grid_centres(nx // 2, ny // 2, nz // 2, sp2)
    sen = I.fibonacci_hemisphere(64, 10e-3)
    full = Plan(cen, sen, nt, dt, c, n_sigma=3.0, sigma_max=s_full)
    half = Plan(cen2, sen, nt, dt, c, n_sigma=3.0, sigma_max=s_half)
    gf = O.Geometry(cen, sen, nt, dt, 0.0, c, 3.0)
    gh = O.Geometry(cen2, sen, nt, dt, 0.0, c, 3.0)
    x_true = I.vessel_phantom((nx, ny, nz), sp, seed=91)
    sf = np.full(cen.shape[0], s_full, np.float32)
    sh = np.full(cen2.shape[0], s_half, np.float32)
    b = O.forward(gf, x_true, sf.astype(np.float64)).astype(np.float32)
    levels = 4
    params = m.unet_init_params(levels, 2024).numpy()
    inv_kappa = 1.0 / 37.0
    ws = m.WarmStart(full, half, levels, params, (nz // 2, ny // 2, nx // 2), inv_kappa)
    A, rep = ws(dev(b), dev(sf), dev(sh))
    # oracle chain
    gA, _ = O.adjoint(gh, np.zeros(cen2.shape[0]), sh.astype(np.float64), b.astype(np.float64),
                      want_sigma=False)
    vol = (np.float32(inv_kappa) * gA.astype(np.float32)).reshape(1, nz // 2, ny // 2, nx // 2)
    xh, _ = N.unet_forward(levels, params, vol)
    xf = N.upsample2(xh).reshape(-1)
    y = O.forward(gf, xf, sf.astype(np.float64))
    yb, yy, bb = np.sum(y * b), np.sum(y * y), np.sum(b.astype(np.float64) ** 2)
    cs = max(0.0, yb / yy) if yy > 0 else 0.0
    rho = np.sqrt(max(0.0, 1 - (yb / yy) * (yb / bb))) if cs > 0 else 1.0
    fall = cs == 0.0 or rho >= 1.0
    _say(f"  gpu: c* {rep['c_star']:.6e} rho {rep['rho']:.6f} fell_back {rep['fell_back']}; "
         f"oracle: c* {cs:.6e} rho {rho:.6f} fell_back {fall}; |x_half| {np.abs(xh).max():.3e}")
    assert rep["fell_back"] == fall
    if not fall:
        assert rep["c_star"] == pytest.approx(cs, rel=2e-2)
        assert rep["rho"] == pytest.approx(rho, abs=1e-2)
        assert rel_l2(host(A), cs * xf) <= 2e-2
    else:
        assert not host(A).any()


WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2602_03893_amd", "weights",
                       "unet4_c4.npy")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights")
def test_trained_warm_start_beats_scaled_adjoint_at_paper_scale():
    """Paper-scale acquisition, a held-out phantom (seed 100010): the trained
    network's rescaled start has a lower relative residual than the rescaled
    back-projection (the control), and neither is worse than the zero start."""
    from paper_2602_03893_amd import nn as m, pgd_update
    from paper_2602_03893_amd import warmstart as W
    _say("case: trained warm start vs scaled adjoint, paper scale, seed 100010")
    prob = W.Problem()
    prob.kappa = W.TRAINED_KAPPA  # the value the weights were trained with
    _, x, _ = W.phantom_sample(100010)
    b = prob.traces(x, 100010)
    params = np.load(WEIGHTS, allow_pickle=False)
    ws = m.WarmStart(prob.full, prob.half, W.LEVELS, params, prob.vol_half, 1.0 / prob.kappa)
    A, rep = ws(b, prob.sig_full, prob.sig_half)
    Ac = prob.full.adjoint(None, prob.sig_full, b, want_sigma=False)[0]
    pgd_update(Ac, Ac, 0.0, lo=0.0)
    rc = prob.full.warm_rescale(Ac, prob.sig_full, b)
    # relative error of the upsampled start against the truth
    xt = torch.as_tensor(x).cuda()
    e_l = float(torch.linalg.vector_norm(A - xt) / torch.linalg.vector_norm(xt))
    e_c = float(torch.linalg.vector_norm(Ac - xt) / torch.linalg.vector_norm(xt))
    _say(f"  learned: rho {rep['rho']:.4f} c* {rep['c_star']:.3f} rel err {e_l:.3f}; "
         f"scaled adjoint: rho {rc['rho']:.4f} rel err {e_c:.3f}")
    assert not rep["fell_back"] and rep["rho"] < rc["rho"] <= 1.0
    assert e_l < e_c
