"""Pins of the network oracle (oracle/nn.py) against brute force, adjoint
identities, finite differences and library routines.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import nn as N
from paper_2602_03893_amd import inputs as I


def rnd(shape, seed):
    return I.standard_normal(shape, seed=seed).astype(np.float64)


def brute_conv3(x, w, b):
    n, d, h, wd, ci = x.shape
    co = w.shape[2]
    out = np.zeros((n, d, h, wd, co))
    for bi in range(n):
        for z in range(d):
            for y in range(h):
                for xx in range(wd):
                    acc = np.array(b, dtype=np.float64).copy()
                    for t, (dz, dy, dx) in enumerate(N.TAPS3):
                        zz, yy, x2 = z + dz, y + dy, xx + dx
                        if 0 <= zz < d and 0 <= yy < h and 0 <= x2 < wd:
                            for c in range(ci):
                                acc += x[bi, zz, yy, x2, c] * w[t, c, :]
                    out[bi, z, y, xx] = acc
    return out


def test_conv3_matches_brute_force():
    x = rnd((2, 4, 2, 4, 3), 1)
    w = rnd((27, 3, 5), 2)
    b = rnd(5, 3)
    assert np.allclose(N.conv3(x, w, b), brute_conv3(x, w, b), rtol=0, atol=1e-12)
    r = N.conv3(x, w, b, relu=True)
    assert np.array_equal(r, np.maximum(N.conv3(x, w, b), 0))


def test_conv3_tap_convention_single_tap():
    """A weight on tap (dz,dy,dx) = (1,0,-1) reads in[z+1][y][x-1]."""
    x = rnd((1, 4, 4, 4, 1), 4)
    w = np.zeros((27, 1, 1))
    t = (1 + 1) * 9 + (0 + 1) * 3 + (-1 + 1)
    w[t, 0, 0] = 1.0
    out = N.conv3(x, w)[0, :, :, :, 0]
    ref = np.zeros((4, 4, 4))
    ref[:3, :, 1:] = x[0, 1:, :, :3, 0]
    assert np.array_equal(out, ref)


def test_conv3_gradients_are_adjoints():
    """<conv3(x), g> = <x, dgrad(g)> and = sum(w * wgrad(x, g))."""
    x = rnd((2, 4, 4, 8, 3), 5)
    w = rnd((27, 3, 4), 6)
    g = rnd((2, 4, 4, 8, 4), 7)
    lhs = np.sum(N.conv3(x, w) * g)
    assert np.sum(x * N.conv3_dgrad(g, w)) == pytest.approx(lhs, rel=1e-12)
    dw, db = N.conv3_wgrad(x, g)
    assert np.sum(w * dw) == pytest.approx(lhs, rel=1e-12)
    assert np.allclose(db, g.reshape(-1, 4).sum(0), rtol=1e-13)
    act = rnd(x.shape, 8)
    assert np.array_equal(N.conv3_dgrad(g, w, mask_act=act), N.conv3_dgrad(g, w) * (act > 0))


def test_maxpool_brute_force_and_ties():
    x = rnd((1, 4, 4, 2, 3), 9)
    x[0, 0, 0, 0, 0] = x[0, 1, 1, 1, 0] = 10.0  # tie in window (0,0,0), channel 0
    out, arg = N.maxpool2(x)
    for z in range(2):
        for y in range(2):
            for xx in range(1):
                for c in range(3):
                    vals = [x[0, 2 * z + tz, 2 * y + ty, 2 * xx + tx, c] for tz, ty, tx in N.TAPS2]
                    assert out[0, z, y, xx, c] == max(vals)
                    assert arg[0, z, y, xx, c] == int(np.argmax(vals))
    assert arg[0, 0, 0, 0, 0] == 0  # the first child wins a tie
    # backward: routed gradient lands on the argmax child only
    g = rnd(out.shape, 10)
    act = np.abs(rnd(x.shape, 11)) + 0.1
    gin = N.maxpool2_backward(g, arg, act)
    assert gin.sum() == pytest.approx(g.sum(), rel=1e-12)
    assert gin[0, 0, 0, 0, 0] == g[0, 0, 0, 0, 0] and gin[0, 1, 1, 1, 0] == 0.0
    skip = rnd(x.shape, 12)
    act[0, 0, 0, 0, 1] = -1.0
    gin2 = N.maxpool2_backward(g, arg, act, gskip=skip)
    ref = (N.maxpool2_backward(g, arg, np.ones_like(act)) + skip) * (act > 0)
    assert np.array_equal(gin2, ref)
    assert gin2[0, 0, 0, 0, 1] == 0.0


def test_maxpool_matches_torch():
    x = rnd((2, 4, 8, 4, 5), 13)
    out, _ = N.maxpool2(x)
    ref = torch.nn.functional.max_pool3d(torch.as_tensor(np.moveaxis(x, -1, 1)), 2)
    assert np.array_equal(out, np.moveaxis(ref.numpy(), 1, -1))


def test_upconv_brute_force_and_adjoints():
    x = rnd((1, 2, 2, 2, 3), 14)
    w = rnd((8, 3, 4), 15)
    b = rnd(4, 16)
    out = N.upconv2(x, w, b)
    for z in range(4):
        for y in range(4):
            for xx in range(4):
                t = (z % 2) * 4 + (y % 2) * 2 + (xx % 2)
                ref = x[0, z // 2, y // 2, xx // 2] @ w[t] + b
                assert np.allclose(out[0, z, y, xx], ref, rtol=0, atol=1e-13)
    # against torch's transposed convolution (weight [ci][co][kz][ky][kx])
    wt = torch.as_tensor(w.reshape(2, 2, 2, 3, 4).transpose(3, 4, 0, 1, 2).copy())
    ref = torch.nn.functional.conv_transpose3d(torch.as_tensor(np.moveaxis(x, -1, 1)), wt,
                                               torch.as_tensor(b), stride=2)
    assert np.allclose(out, np.moveaxis(ref.numpy(), 1, -1), rtol=0, atol=1e-13)
    g = rnd(out.shape, 17)
    lhs = np.sum(N.upconv2(x, w, np.zeros(4)) * g)
    assert np.sum(x * N.upconv2_dgrad(g, w)) == pytest.approx(lhs, rel=1e-12)
    dw, db = N.upconv2_wgrad(x, g)
    assert np.sum(w * dw) == pytest.approx(lhs, rel=1e-12)
    assert np.allclose(db, g.reshape(-1, 4).sum(0), rtol=1e-13)


def test_head_and_mse():
    x = rnd((1, 2, 2, 2, 4), 18)
    w = rnd(4, 19)
    y = N.head(x, w, 0.1)
    for idx in np.ndindex(1, 2, 2, 2):
        assert y[idx] == pytest.approx(max(0.0, float(x[idx] @ w) + 0.1), abs=1e-15)
    g = rnd(y.shape, 20)
    gin, dw, db = N.head_backward(x, w, y, g)
    gp = g * (y > 0)
    assert db == pytest.approx(gp.sum())
    assert np.allclose(dw, np.einsum("ndhw,ndhwc->c", gp, x))
    assert np.allclose(gin, gp[..., None] * w * (x > 0))
    p, t = rnd(10, 21), rnd(10, 22)
    L, gl = N.mse(p, t)
    assert L == pytest.approx(np.sum((p - t) ** 2) / 10)
    assert np.allclose(gl, 0.2 * (p - t))


def test_upsample_matches_torch_and_reproduces_linear():
    x = rnd((2, 3, 4, 5), 23)
    ref = torch.nn.functional.interpolate(torch.as_tensor(x)[:, None], scale_factor=2,
                                          mode="trilinear", align_corners=False)[:, 0]
    assert np.allclose(N.upsample2(x), ref.numpy(), rtol=0, atol=1e-13)
    # a linear ramp is reproduced exactly away from the clamped edges
    z = np.arange(6, dtype=np.float64)
    lin = np.broadcast_to(z[None, :, None, None], (1, 6, 2, 2))
    up = N.upsample2(lin)[0, 1:-1, 0, 0]
    fine = (np.arange(1, 11) + 0.5) / 2 - 0.5
    assert np.allclose(up, fine, atol=1e-14)


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -3.14159], np.float32)
    r = N.bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0  # tie -> even (mantissa 0)
    assert r[2] == 1.0 + 4 * 2 ** -8    # tie -> even (rounds up)
    assert r[3] == 1.0
    assert abs(r[4] + 3.14159) <= 2 ** -7 * 4


def test_unet_gradient_matches_finite_differences():
    """Levels 2 on 4x4x4 (float64, no rounding): autograd gradient against
    central differences of the loss at 12 parameters; the plain numpy forward
    (round_bf16=False) agrees with the torch formulation."""
    levels = 2
    layers = N.unet_layers(levels)
    n_par = sum(t * ci * co + co for _, _, t, ci, co in layers)
    rng = np.random.default_rng(24)
    params = rng.standard_normal(n_par) * 0.3
    x = np.abs(rnd((1, 4, 4, 4), 25))
    target = np.abs(rnd((1, 4, 4, 4), 26))
    L, grad, y = N.unet_loss_and_grad(levels, params, x, target)
    y_np, _ = N.unet_forward(levels, params, x, round_bf16=False)
    assert np.allclose(y_np, y, rtol=1e-12, atol=1e-12)
    assert y.max() > 0
    pick = rng.choice(n_par, 12, replace=False)
    for k in pick:
        h = 1e-6
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        lp = np.mean((N.unet_forward(levels, pp, x, round_bf16=False)[0] - target) ** 2)
        lm = np.mean((N.unet_forward(levels, pm, x, round_bf16=False)[0] - target) ** 2)
        fd = (lp - lm) / (2 * h)
        assert abs(grad[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, grad[k], fd)


def test_unet_chain_rule_backward_matches_autograd():
    """The layer-by-layer backward (no rounding) equals torch autograd."""
    for levels in (1, 2, 3):
        layers = N.unet_layers(levels)
        n_par = sum(t * ci * co + co for _, _, t, ci, co in layers)
        rng = np.random.default_rng(30 + levels)
        params = rng.standard_normal(n_par) * 0.3
        x = np.abs(rnd((2, 4, 4, 8), 31))
        target = np.abs(rnd((2, 4, 4, 8), 32))
        L, grad, y = N.unet_loss_and_grad(levels, params, x, target)
        gy = 2.0 * (y - target) / y.size
        g2 = N.unet_backward(levels, params, x, gy, round_bf16=False)
        assert np.allclose(g2, grad, rtol=1e-10, atol=1e-12 * np.abs(grad).max()), levels
