"""Float64 reconstruction loops on top of the oracle operators.

TEST INFRASTRUCTURE ONLY (see the package docstring).

arXiv 2602.03893, Methods, "Optimization formulation and algorithm" and
Algorithm 2: iterate forward -> data residual -> adjoint -> parameter update.
This build's loops keep the data term only (no regulariser, no non-negativity
reparameterisation, no learning-rate schedule) and enforce A >= 0 by
projection:
 - relative residual rho(x) = ||A(x) - b|| / ||b||;
 - projected gradient descent on 0.5 ||A x - b||^2:  x <- max(0, x - eta A^T(Ax - b));
 - Adam (Kingma and Ba, with bias correction) on 0.5 ||A x - b||^2 / ||b||^2 for
   A (and sigma), followed by the clamps;
 - power iteration for ||A^T A||, used to pick eta = 1 / ||A^T A||.
"""
import numpy as np

from . import ops


def rel_residual(g, amp, sigma, b):
    y = ops.forward(g, amp, sigma)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(y - b) / np.linalg.norm(b))


def power_iteration(g, sigma, iters=100, seed=0):
    """Largest eigenvalue of A^T A by power iteration from a seeded start."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(g.n_kernels)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        z, _ = ops.adjoint(g, np.ones(g.n_kernels), sigma, ops.forward(g, x, sigma),
                           want_sigma=False)
        lam = float(np.dot(x, z))
        x = z / np.linalg.norm(z)
    return lam


def pgd(g, sigma, b, x0, step, iters, lo=0.0, hi=np.inf):
    """Projected gradient descent; returns (x, rho history of length iters+1)."""
    x = np.array(x0, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    hist = []
    for _ in range(iters):
        r = ops.forward(g, x, sigma) - b
        hist.append(float(np.linalg.norm(r) / nb))
        gA, _ = ops.adjoint(g, x, sigma, r, want_sigma=False)
        x = np.clip(x - step * gA, lo, hi)
    hist.append(rel_residual(g, x, sigma, b))
    return x, hist


def adam_step(x, grad, m, v, t, lr, beta1, beta2, eps, lo, hi):
    """One Adam step with bias correction, then the clamp; t is 1-based.
    Updates m, v in place and returns the new x."""
    m *= beta1
    m += (1.0 - beta1) * grad
    v *= beta2
    v += (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    x = x - lr * mhat / (np.sqrt(vhat) + eps)
    return np.clip(x, lo, hi)


def adam(g, amp0, sigma0, b, iters, lr_a, lr_s=0.0, beta1=0.9, beta2=0.999,
         eps=1e-8, learn_sigma=False, a_lo=0.0, a_hi=np.inf,
         s_lo=0.0, s_hi=np.inf):
    """Adam on L = 0.5 ||A(x;sigma) - b||^2 / ||b||^2.  Returns
    (A, sigma, rho history of length iters+1)."""
    a = np.array(amp0, dtype=np.float64)
    s = np.array(sigma0, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb2 = float(np.dot(b.ravel(), b.ravel()))
    ma = np.zeros_like(a)
    va = np.zeros_like(a)
    ms = np.zeros_like(s)
    vs = np.zeros_like(s)
    hist = []
    for t in range(1, iters + 1):
        r = ops.forward(g, a, s) - b
        hist.append(float(np.sqrt(np.dot(r.ravel(), r.ravel()) / nb2)))
        gA, gS = ops.adjoint(g, a, s, r / nb2, want_sigma=learn_sigma)
        a = adam_step(a, gA, ma, va, t, lr_a, beta1, beta2, eps, a_lo, a_hi)
        if learn_sigma:
            s = adam_step(s, gS, ms, vs, t, lr_s, beta1, beta2, eps, s_lo, s_hi)
    hist.append(rel_residual(g, a, s, b))
    return a, s, hist
