"""Pins of the oracle's centre gradient (learnable kernel centres): central
differences of the float64 forward, and torch autograd of an independent
torch formulation of Eq. (single_forward) over the same windows."""
import numpy as np
import pytest

from oracle import ops as O
from paper_2602_03893_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore")


def cloud(m, nd, nt=512, seed=0):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-1e-3, 1e-3, (m, 3)).astype(np.float32)
    sen = I.fibonacci_hemisphere(nd, 10e-3)
    g = O.Geometry(cen, sen, nt, I.DT, 0.0, I.C_SOUND, 3.0)
    A = rng.uniform(-1.0, 1.0, m)
    sigma = rng.uniform(0.05e-3, 0.1e-3, m).astype(np.float32).astype(np.float64)
    delta = rng.standard_normal((nd, nt))
    return cen, sen, g, A, sigma, delta


def test_centre_gradient_against_central_differences():
    """dL/dc_k of L = <A(x; c), delta>, one kernel at a time, each axis:
    steps of ~4 nm in float32 centres (the exact float32 difference is the
    denominator); a step that moves a window edge across a sample is
    detected from the trace supports and skipped."""
    cen, sen, g, A, sigma, delta = cloud(200, 16)
    gc = O.adjoint_centres(g, A, sigma, delta)
    rng = np.random.default_rng(1)
    checked = 0
    for k in rng.choice(200, 12, replace=False):
        for a in range(3):
            cp, cm = cen[k].copy(), cen[k].copy()
            cp[a] = np.float32(cen[k, a] + np.float32(4e-9))
            cm[a] = np.float32(cen[k, a] - np.float32(4e-9))
            gp = O.Geometry(cp[None], sen, g.n_samples, g.dt, g.t0, g.c_sound, g.n_sigma)
            gm = O.Geometry(cm[None], sen, g.n_samples, g.dt, g.t0, g.c_sound, g.n_sigma)
            yp = O.forward(gp, [A[k]], [sigma[k]])
            ym = O.forward(gm, [A[k]], [sigma[k]])
            if not np.array_equal(yp != 0, ym != 0):
                continue
            fd = (np.sum(yp * delta) - np.sum(ym * delta)) / (float(cp[a]) - float(cm[a]))
            assert abs(gc[k, a] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gc).max()), (k, a)
            checked += 1
    assert checked >= 30


def test_centre_gradient_against_torch_autograd():
    """The same gradient from torch autograd of an independent float64 torch
    formulation (p = A/(2r) d exp(-d^2/(2 sigma^2)), d = r - v t, summed over
    the in-window samples, the window decided without gradient)."""
    import torch
    cen, sen, g, A, sigma, delta = cloud(12, 5, nt=512, seed=3)
    gc = O.adjoint_centres(g, A, sigma, delta)
    c = torch.tensor(cen.astype(np.float64), requires_grad=True)
    s = torch.tensor(sen.astype(np.float64))
    t = torch.arange(g.n_samples, dtype=torch.float64) * g.dt + g.t0
    r = torch.linalg.vector_norm(s[None, :, :] - c[:, None, :], dim=2)          # (M, Nd)
    d = r[:, :, None] - g.c_sound * t[None, None, :]                            # (M, Nd, Nt)
    sg = torch.tensor(sigma)[:, None, None]
    mask = (d.detach().abs() <= g.n_sigma * sg).double()
    p = torch.tensor(A)[:, None, None] / (2 * r[:, :, None]) * d * torch.exp(-d * d / (2 * sg * sg))
    L = torch.sum(mask * p * torch.tensor(delta)[None, :, :])
    L.backward()
    ref = c.grad.numpy()
    assert np.max(np.abs(gc - ref)) <= 1e-12 * np.abs(ref).max()


def test_centre_gradient_vanishes_for_zero_amplitude_and_is_linear():
    cen, sen, g, A, sigma, delta = cloud(50, 8, seed=5)
    assert np.all(O.adjoint_centres(g, np.zeros(50), sigma, delta) == 0.0)
    g1 = O.adjoint_centres(g, A, sigma, delta)
    g2 = O.adjoint_centres(g, A, sigma, 2.5 * delta)
    assert np.max(np.abs(g2 - 2.5 * g1)) <= 1e-13 * np.abs(g1).max()
