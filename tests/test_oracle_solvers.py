"""Pins of the oracle's reconstruction loops (CPU only).

 - projected gradient descent converges to the non-negative least-squares
   solution that scipy.optimize.nnls (an active-set method) finds;
 - the Adam step equals torch.optim.Adam's on the same gradient sequence;
 - power iteration returns the largest eigenvalue numpy finds for A^T A.
The explicit matrix A is built column by column with the oracle forward.
"""
import numpy as np
import pytest
import scipy.optimize
import torch

from oracle import ops, solvers
from paper_2602_03893_amd import inputs as I

V, DT = 1500.0, 25e-9


def tiny_problem(m=27, nd=12, nt=420, seed=7):
    offs = (np.arange(3) - 1) * 0.3e-3
    Z, Y, X = np.meshgrid(offs, offs, offs, indexing="ij")
    cen = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float32)[:m]
    g = ops.Geometry(cen, I.fibonacci_hemisphere(nd, 8e-3), nt, DT, 0.0, V, 3.0)
    sigma = np.full(m, 0.15e-3)
    rng = np.random.default_rng(seed)
    x_true = np.where(rng.uniform(size=m) < 0.5, rng.uniform(0.2, 1.0, m), 0.0)
    b = ops.forward(g, x_true, sigma) + 1e-3 * rng.standard_normal((nd, nt))
    return g, sigma, x_true, b


def explicit_matrix(g, sigma):
    cols = []
    for k in range(g.n_kernels):
        e = np.zeros(g.n_kernels)
        e[k] = 1.0
        cols.append(ops.forward(g, e, sigma).ravel())
    return np.stack(cols, axis=1)


def test_power_iteration_matches_eigvalsh():
    g, sigma, _, _ = tiny_problem()
    Amat = explicit_matrix(g, sigma)
    lam_ref = np.linalg.eigvalsh(Amat.T @ Amat).max()
    lam = solvers.power_iteration(g, sigma, iters=300, seed=0)
    assert lam == pytest.approx(lam_ref, rel=1e-6)


def test_pgd_converges_to_nnls():
    g, sigma, _, b = tiny_problem()
    Amat = explicit_matrix(g, sigma)
    x_ref, _ = scipy.optimize.nnls(Amat, b.ravel(), maxiter=10000)
    L = np.linalg.eigvalsh(Amat.T @ Amat).max()
    x, hist = solvers.pgd(g, sigma, b, np.zeros(g.n_kernels), 1.0 / L, 6000)
    assert np.all(x >= 0)
    assert np.all(np.diff(hist) <= 1e-12)            # monotone with step 1/L
    assert np.linalg.norm(x - x_ref) <= 1e-5 * np.linalg.norm(x_ref)


def test_adam_step_matches_torch():
    rng = np.random.default_rng(11)
    n = 50
    x0 = rng.uniform(0, 1, n)
    lr, b1, b2, eps = 3e-2, 0.9, 0.999, 1e-8
    xt = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([xt], lr=lr, betas=(b1, b2), eps=eps)
    x = x0.copy()
    m = np.zeros(n)
    v = np.zeros(n)
    for t in range(1, 31):
        grad = rng.standard_normal(n) * (1.0 + t)
        opt.zero_grad()
        xt.grad = torch.tensor(grad, dtype=torch.float64)
        opt.step()
        with torch.no_grad():
            xt.clamp_(0.0, 0.8)
        x = solvers.adam_step(x, grad, m, v, t, lr, b1, b2, eps, 0.0, 0.8)
        np.testing.assert_allclose(x, xt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_solver_decreases_residual():
    g, sigma, _, b = tiny_problem()
    a, s, hist = solvers.adam(g, np.zeros(g.n_kernels), sigma, b, 60, lr_a=0.05)
    assert hist[0] == pytest.approx(1.0)
    assert hist[-1] < 0.5 and np.all(a >= 0)
