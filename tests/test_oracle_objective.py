"""Pins of the objective oracle (oracle/objective.py): NPC chain rule, the VCR
value against brute-force loops and closed forms, its gradient against torch
autograd and central differences, CAWR against torch's scheduler, and the
Algorithm-2 loop against a hand-unrolled first iteration."""
import math

import numpy as np
import pytest
import torch

from oracle import objective as J

EPS = 1e-8


def test_npc_chain_rule_by_central_differences():
    rng = np.random.default_rng(0)
    z = rng.normal(size=50)
    gx = rng.normal(size=50)
    # L(z) = <gx, phi(z)> has dL/dz_i = gx_i phi'(z_i); phi is quadratic, so the
    # central difference is exact up to rounding
    h = 1e-3
    fd = gx * (J.npc_map(z + h) - J.npc_map(z - h)) / (2 * h)
    assert np.allclose(J.npc_grad(z, gx), fd, rtol=1e-11, atol=1e-13)
    assert np.all(J.npc_map(rng.normal(size=1000)) >= 0)
    assert J.npc_map(np.array([-1e-8]))[0] == 0.0


def brute_force_vcr(x, beta, eps):
    """Each difference by explicit index arithmetic, one voxel at a time."""
    nz, ny, nx = x.shape

    def at(iz, iy, ix):
        if 0 <= iz < nz and 0 <= iy < ny and 0 <= ix < nx:
            return x[iz, iy, ix]
        return None

    total = 0.0
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                c = x[iz, iy, ix]
                step = {"x": (0, 0, 1), "y": (0, 1, 0), "z": (1, 0, 0)}
                s_t = 0.0
                for d in "xyz":
                    o = step[d]
                    f = at(iz + o[0], iy + o[1], ix + o[2])
                    s_t += 0.0 if f is None else (f - c) ** 2
                s_h = 0.0
                for d in "xyz":
                    o = step[d]
                    f = at(iz + o[0], iy + o[1], ix + o[2])
                    bk = at(iz - o[0], iy - o[1], ix - o[2])
                    if f is not None and bk is not None:
                        s_h += (f - 2 * c + bk) ** 2
                for p, q in (("x", "y"), ("y", "x"), ("x", "z"), ("z", "x"), ("y", "z"),
                             ("z", "y")):
                    op, oq = step[p], step[q]
                    fpq = at(iz + op[0] + oq[0], iy + op[1] + oq[1], ix + op[2] + oq[2])
                    if fpq is not None:
                        fp = at(iz + op[0], iy + op[1], ix + op[2])
                        fq = at(iz + oq[0], iy + oq[1], ix + oq[2])
                        s_h += (fpq - fp - fq + c) ** 2
                total += math.sqrt(s_h + eps) + beta * math.sqrt(s_t + eps)
    return total


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 2, 7), (2, 1, 1), (4, 3, 2)])
def test_vcr_value_against_brute_force(shape):
    x = np.random.default_rng(1).uniform(size=shape)
    for beta in (0.0, 0.3, 2.0):
        assert J.vcr_value(x, beta) == pytest.approx(brute_force_vcr(x, beta, EPS), rel=1e-13)


def test_vcr_closed_forms():
    nz, ny, nx = 4, 5, 6
    M = nz * ny * nx
    # constant volume: every difference vanishes
    x = np.full((nz, ny, nx), 0.7)
    assert J.vcr_value(x, 0.5) == pytest.approx(M * math.sqrt(EPS) * 1.5, rel=1e-12)
    assert np.abs(J.vcr_grad(x, 0.5)).max() == 0.0
    # linear ramp along x: no second differences; D_x = a except on the last x-plane
    a = 0.25
    ix = np.arange(nx, dtype=float)
    x = np.broadcast_to(a * ix, (nz, ny, nx)).copy()
    tv = nz * ny * ((nx - 1) * math.sqrt(a * a + EPS) + math.sqrt(EPS))
    assert J.vcr_value(x, 1.0) == pytest.approx(M * math.sqrt(EPS) + tv, rel=1e-12)
    # quadratic along y: D_yy = 2 c on the interior planes, mixed terms vanish
    c = 0.1
    iy = np.arange(ny, dtype=float)
    x = np.broadcast_to((c * iy * iy)[None, :, None], (nz, ny, nx)).copy()
    h = nz * nx * ((ny - 2) * math.sqrt(4 * c * c + EPS) + 2 * math.sqrt(EPS))
    assert J.vcr_value(x, 0.0) == pytest.approx(h, rel=1e-12)


def torch_vcr(x, beta, eps):
    """The same definition written with torch slicing (zero-padded stencils)."""
    nz, ny, nx = x.shape
    P = torch.nn.functional.pad(x, (1, 1, 1, 1, 1, 1))  # pads x, y, z by 1
    ones = torch.nn.functional.pad(torch.ones_like(x), (1, 1, 1, 1, 1, 1))

    def sh(t, dz, dy, dx):
        return t[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]

    c = x
    s_t = 0
    s_h = 0
    for o in ((0, 0, 1), (0, 1, 0), (1, 0, 0)):
        m = sh(ones, *o)
        s_t = s_t + ((sh(P, *o) - c) * m) ** 2
        mb = sh(ones, *[-k for k in o]) * m
        s_h = s_h + ((sh(P, *o) - 2 * c + sh(P, *[-k for k in o])) * mb) ** 2
    for op, oq in (((0, 0, 1), (0, 1, 0)), ((0, 0, 1), (1, 0, 0)), ((0, 1, 0), (1, 0, 0))):
        opq = tuple(a + b for a, b in zip(op, oq))
        m = sh(ones, *opq)
        s_h = s_h + 2 * ((sh(P, *opq) - sh(P, *op) - sh(P, *oq) + c) * m) ** 2
    return torch.sqrt(s_h + eps).sum() + beta * torch.sqrt(s_t + eps).sum()


@pytest.mark.parametrize("shape", [(5, 6, 7), (3, 8, 2)])
def test_vcr_gradient_against_autograd_and_differences(shape):
    x = np.random.default_rng(2).uniform(size=shape)
    beta = 0.4
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    val = torch_vcr(xt, beta, EPS)
    val.backward()
    assert val.item() == pytest.approx(J.vcr_value(x, beta), rel=1e-13)
    g = J.vcr_grad(x, beta)
    assert np.allclose(g, xt.grad.numpy(), rtol=1e-11, atol=1e-12)
    # central differences at a few voxels
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(8):
        idx = tuple(rng.integers(0, s) for s in shape)
        e = np.zeros(shape)
        e[idx] = h
        fd = (J.vcr_value(x + e, beta) - J.vcr_value(x - e, beta)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("T0,Tmult", [(10, 1), (7, 2), (5, 3)])
def test_cawr_against_torch_scheduler(T0, Tmult):
    p = torch.nn.Parameter(torch.zeros(1))
    opt = torch.optim.SGD([p], lr=0.1)
    sch = torch.optim.lr_scheduler.CosineAnnealingWarmRestarts(opt, T_0=T0, T_mult=Tmult,
                                                               eta_min=0.001)
    for t in range(120):
        assert J.cawr(t, 0.001, 0.1, T0, Tmult) == pytest.approx(opt.param_groups[0]["lr"],
                                                                  rel=1e-12)
        opt.step()
        sch.step()


def test_cawr_printed_formula_for_unit_multiplier():
    for t in range(50):
        printed = 0.01 + 0.5 * (1.0 - 0.01) * (1 + math.cos(math.pi * (t % 8) / 8))
        assert J.cawr(t, 0.01, 1.0, 8, 1) == pytest.approx(printed, rel=1e-15)


def test_gpair_loop_first_iteration_by_hand():
    """One iteration from z = 0 equals the hand-unrolled chain: x = eps^2,
    forward, residual, adjoint + lambda grad R, chain rule, Adam's first step
    (lr_0 * sign of the gradient)."""
    from oracle import ops as O
    from paper_2602_03893_amd import inputs as I
    grid = (4, 3, 2)
    cen = I.grid_centres(*grid, 0.2e-3)
    sen = I.fibonacci_hemisphere(6, 5e-3)
    g = O.Geometry(cen, sen, 256, I.DT, 0.0, I.C_SOUND, 3.0)
    sigma = np.full(24, 0.1e-3)
    b = O.forward(g, np.random.default_rng(4).uniform(size=24), sigma)
    lam, beta = 1e-3, 0.5
    x, z, hist = J.gpair(g, sigma, b, grid, 1, lam, beta, 1e-4, 1e-2, 5, 1)
    x0 = np.full(24, EPS * EPS)
    r = O.forward(g, x0, sigma) - b
    nb2 = float(np.sum(b * b))
    gx = O.adjoint(g, x0, sigma, r / nb2, want_sigma=False)[0]
    gx = gx + lam * J.vcr_grad(x0.reshape(2, 3, 4), beta).ravel()
    gz = gx * 2 * EPS
    z_hand = -1e-2 * gz / (np.abs(gz) + 1e-8)  # Adam's first step: m/sqrt(v) = sign
    assert np.allclose(z, z_hand, rtol=1e-12, atol=0)
    assert hist[0] == pytest.approx(1.0, rel=1e-12)  # rho(x = eps^2) = 1 up to 1e-16
