"""Python front end of the warm-start network kernels (include/gpair_nn.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every layer runs in libgpair's HIP kernels.  Activations are bfloat16
tensors shaped (N, D, H, W, C) whose last dimension is contiguous; a channel
slice ``t[..., c0:c1]`` of a wider tensor is a valid view (its voxel stride is
the wider tensor's channel count).
"""
import ctypes

import torch

from . import _lib
from ._lib import c_flt, c_i32, c_i64, c_vp, check

EPI_BIAS_RELU = 0
EPI_BIAS = 1
EPI_MASK = 2
EPI_NONE = 3
MSE_PARTIALS = 1024


class Tensor(ctypes.Structure):
    _fields_ = [("data", c_vp), ("n", c_i32), ("d", c_i32), ("h", c_i32), ("w", c_i32),
                ("c", c_i32), ("cs", c_i32)]


_P = ctypes.POINTER(Tensor)
_sz = ctypes.c_size_t
_proto = _lib._proto
_conv3 = _proto("gpair_nn_conv3", c_i32, [_P, c_vp, c_vp, _P, ctypes.c_int, _P, c_vp])
_wsize = _proto("gpair_nn_wgrad_partial_size", _sz, [_P, _P, ctypes.c_int])
_conv3_wgrad = _proto("gpair_nn_conv3_wgrad", c_i32, [_P, _P, c_vp, c_vp, c_vp, c_vp])
_maxpool = _proto("gpair_nn_maxpool2", c_i32, [_P, _P, c_vp, c_vp])
_maxpool_bwd = _proto("gpair_nn_maxpool2_backward", c_i32, [_P, c_vp, _P, _P, _P, c_vp])
_upconv = _proto("gpair_nn_upconv2", c_i32, [_P, c_vp, c_vp, _P, c_vp])
_upconv_dgrad = _proto("gpair_nn_upconv2_dgrad", c_i32, [_P, c_vp, _P, _P, c_vp])
_upconv_wgrad = _proto("gpair_nn_upconv2_wgrad", c_i32, [_P, _P, c_vp, c_vp, c_vp, c_vp])
_head = _proto("gpair_nn_head", c_i32, [_P, c_vp, c_vp, c_vp, c_vp])
_head_psize = _proto("gpair_nn_head_partial_size", _sz, [_P])
_head_bwd = _proto("gpair_nn_head_backward", c_i32,
                   [_P, c_vp, c_vp, c_vp, _P, c_vp, c_vp, c_vp, c_vp])
_mse = _proto("gpair_nn_mse", c_i32, [c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp])
_pack = _proto("gpair_nn_pack_weights", c_i32,
               [c_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, c_vp, c_vp, c_vp])
_from_float = _proto("gpair_nn_from_float", c_i32, [c_vp, c_flt, _P, c_vp])
_upsample2 = _proto("gpair_nn_upsample2", c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp])


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, dtype=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def view(t, name="tensor"):
    """ctypes view of a (N, D, H, W, C) bfloat16 device tensor (or channel slice)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.bfloat16:
        raise ValueError(f"{name}: expected a bfloat16 device tensor")
    if t.dim() != 5 or t.stride(4) != 1:
        raise ValueError(f"{name}: expected (N, D, H, W, C) with contiguous channels")
    n, d, h, w, c = t.shape
    cs = t.stride(3)
    if (t.stride(2) != w * cs or t.stride(1) != h * w * cs or
            (n > 1 and t.stride(0) != d * h * w * cs)):
        raise ValueError(f"{name}: voxels must be evenly strided")
    return Tensor(ctypes.c_void_p(t.data_ptr()), n, d, h, w, c, cs)


def _ref(v):
    return ctypes.byref(v) if v is not None else None


def conv3(x, w, bias, out, epilogue=EPI_BIAS_RELU, aux=None):
    """3x3x3 convolution (implicit GEMM on the matrix cores) into ``out``."""
    check(_conv3(_ref(view(x, "x")), _ptr(w, "w", torch.bfloat16), _ptr(bias, "bias", torch.float32),
                 _ref(view(out, "out")), epilogue, _ref(view(aux, "aux")), _stream()),
          "gpair_nn_conv3")
    return out


def _scratch(nbytes, device):
    return torch.empty(max(1, (nbytes + 3) // 4), dtype=torch.float32, device=device)


def conv3_wgrad(x, gout, dw, db=None, partial=None):
    vx, vg = view(x, "x"), view(gout, "gout")
    if partial is None:
        partial = _scratch(_wsize(ctypes.byref(vx), ctypes.byref(vg), 27), x.device)
    check(_conv3_wgrad(ctypes.byref(vx), ctypes.byref(vg), _ptr(partial, "partial"),
                       _ptr(dw, "dw", torch.float32), _ptr(db, "db", torch.float32), _stream()),
          "gpair_nn_conv3_wgrad")
    return dw, db


def maxpool2(x, out, argmax):
    check(_maxpool(_ref(view(x, "x")), _ref(view(out, "out")), _ptr(argmax, "argmax", torch.uint8),
                   _stream()), "gpair_nn_maxpool2")
    return out, argmax


def maxpool2_backward(gout, argmax, act, gin, gskip=None):
    check(_maxpool_bwd(_ref(view(gout, "gout")), _ptr(argmax, "argmax", torch.uint8),
                       _ref(view(gskip, "gskip")), _ref(view(act, "act")), _ref(view(gin, "gin")),
                       _stream()), "gpair_nn_maxpool2_backward")
    return gin


def upconv2(x, w, bias, out):
    check(_upconv(_ref(view(x, "x")), _ptr(w, "w", torch.bfloat16), _ptr(bias, "bias", torch.float32),
                  _ref(view(out, "out")), _stream()), "gpair_nn_upconv2")
    return out


def upconv2_dgrad(gout, wt, gin, aux=None):
    check(_upconv_dgrad(_ref(view(gout, "gout")), _ptr(wt, "wt", torch.bfloat16),
                        _ref(view(gin, "gin")), _ref(view(aux, "aux")), _stream()),
          "gpair_nn_upconv2_dgrad")
    return gin


def upconv2_wgrad(x, gout, dw, db=None, partial=None):
    vx, vg = view(x, "x"), view(gout, "gout")
    if partial is None:
        partial = _scratch(_wsize(ctypes.byref(vx), ctypes.byref(vg), 8), x.device)
    check(_upconv_wgrad(ctypes.byref(vx), ctypes.byref(vg), _ptr(partial, "partial"),
                        _ptr(dw, "dw", torch.float32), _ptr(db, "db", torch.float32), _stream()),
          "gpair_nn_upconv2_wgrad")
    return dw, db


def head(x, w, b, out):
    check(_head(_ref(view(x, "x")), _ptr(w, "w", torch.float32), _ptr(b, "b", torch.float32),
                _ptr(out, "out", torch.float32), _stream()), "gpair_nn_head")
    return out


def head_backward(x, w, out, gout, gin, dw, db, partial=None):
    vx = view(x, "x")
    if partial is None:
        partial = _scratch(_head_psize(ctypes.byref(vx)), x.device)
    check(_head_bwd(ctypes.byref(vx), _ptr(w, "w", torch.float32), _ptr(out, "out", torch.float32),
                    _ptr(gout, "gout", torch.float32), _ref(view(gin, "gin")), _ptr(partial, "partial"),
                    _ptr(dw, "dw", torch.float32), _ptr(db, "db", torch.float32), _stream()),
          "gpair_nn_head_backward")
    return gin, dw, db


def mse(pred, target, gpred=None, loss=None, partial=None):
    """Mean squared error (float64 device scalar) and optionally its gradient."""
    dev = pred.device
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=dev)
    if partial is None:
        partial = torch.empty(MSE_PARTIALS, dtype=torch.float64, device=dev)
    check(_mse(pred.numel(), _ptr(pred, "pred", torch.float32), _ptr(target, "target", torch.float32),
               _ptr(gpred, "gpred", torch.float32), _ptr(loss, "loss", torch.float64),
               _ptr(partial, "partial", torch.float64), _stream()), "gpair_nn_mse")
    return loss


def pack_weights(master, taps, c_in, c_out, fwd, dgrad=None):
    check(_pack(_ptr(master, "master", torch.float32), taps, c_in, c_out,
                _ptr(fwd, "fwd", torch.bfloat16), _ptr(dgrad, "dgrad", torch.bfloat16), _stream()),
          "gpair_nn_pack_weights")
    return fwd, dgrad


def from_float(x, scale, out):
    check(_from_float(_ptr(x, "x", torch.float32), float(scale), _ref(view(out, "out")), _stream()),
          "gpair_nn_from_float")
    return out


def upsample2(x, out):
    n, d, h, w = x.shape
    check(_upsample2(_ptr(x, "x", torch.float32), n, d, h, w, _ptr(out, "out", torch.float32),
                     _stream()), "gpair_nn_upsample2")
    return out


# ---------------------------------------------------------------------------
# The U-Net executor
# ---------------------------------------------------------------------------
_u64 = ctypes.c_uint64
_unet_count = _proto("gpair_unet_param_count", c_i64, [ctypes.c_int])
_unet_init = _proto("gpair_unet_init_params", c_i32, [ctypes.c_int, _u64, c_vp])
_unet_wsize = _proto("gpair_unet_workspace_size", _sz,
                     [ctypes.c_int, c_i32, c_i32, c_i32, c_i32])
_unet_fwd = _proto("gpair_unet_forward", c_i32,
                   [ctypes.c_int, c_vp, c_i32, c_i32, c_i32, c_i32, c_vp, c_flt, c_vp, c_vp,
                    _sz, c_vp])
_unet_bwd = _proto("gpair_unet_backward", c_i32,
                   [ctypes.c_int, c_vp, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, _sz, c_vp])
_unet_step = _proto("gpair_unet_train_step", c_i32,
                    [ctypes.c_int, c_vp, c_vp, c_vp, c_vp, c_i32, c_flt, c_flt, c_flt, c_flt,
                     c_i32, c_i32, c_i32, c_i32, c_vp, c_flt, c_vp, c_vp, c_vp, _sz, c_vp])


def unet_param_count(levels):
    n = int(_unet_count(levels))
    if n <= 0:
        raise ValueError(f"unsupported levels {levels}")
    return n


def unet_init_params(levels, seed):
    """Seeded initial parameters (host float32 tensor)."""
    p = torch.empty(unet_param_count(levels), dtype=torch.float32)
    check(_unet_init(levels, seed, ctypes.c_void_p(p.data_ptr())), "gpair_unet_init_params")
    return p


class UNet:
    """Parameters, Adam moments and workspace of the warm-start network for
    one batch shape (n, d, h, w)."""

    def __init__(self, levels, shape, params=None, seed=0, device="cuda"):
        self.levels = levels
        self.shape = tuple(int(s) for s in shape)
        n, d, h, w = self.shape
        self.device = torch.device(device)
        nbytes = int(_unet_wsize(levels, n, d, h, w))
        if nbytes == 0:
            raise ValueError(f"unsupported U-Net shape {self.shape} at {levels} levels")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if params is None:
            params = unet_init_params(levels, seed)
        self.params = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        if self.params.numel() != unet_param_count(levels):
            raise ValueError("parameter vector has the wrong length")
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)

    def _vol(self, x, name):
        if tuple(x.shape) != self.shape:
            raise ValueError(f"{name}: expected shape {self.shape}, got {tuple(x.shape)}")
        if not x.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
        return _ptr(x, name, torch.float32)

    def forward(self, x, scale=1.0, out=None):
        n, d, h, w = self.shape
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        check(_unet_fwd(self.levels, _ptr(self.params, "params"), n, d, h, w, self._vol(x, "x"),
                        float(scale), self._vol(out, "out"), _ptr(self.ws, "ws"), self.ws.numel(),
                        _stream()), "gpair_unet_forward")
        return out

    def backward(self, gy):
        n, d, h, w = self.shape
        check(_unet_bwd(self.levels, _ptr(self.params, "params"), n, d, h, w, self._vol(gy, "gy"),
                        _ptr(self.grad, "grad"), _ptr(self.ws, "ws"), self.ws.numel(), _stream()),
              "gpair_unet_backward")
        return self.grad

    def train_step(self, x, target, lr, scale=1.0, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step on the MSE loss; returns the loss (device float64 [1])."""
        n, d, h, w = self.shape
        self.t += 1
        check(_unet_step(self.levels, _ptr(self.params, "params"), _ptr(self.grad, "grad"),
                         _ptr(self.m, "m"), _ptr(self.v, "v"), self.t, float(lr), float(beta1),
                         float(beta2), float(eps), n, d, h, w, self._vol(x, "x"), float(scale),
                         self._vol(target, "target"), _ptr(self.loss, "loss"), _ptr(self.ws, "ws"),
                         self.ws.numel(), _stream()), "gpair_unet_train_step")
        return self.loss


_ws_size = _proto("gpair_warm_start_workspace_size", _sz, [ctypes.c_int, c_i32, c_i32, c_i32, c_i64])
_warm_start = _proto("gpair_warm_start", c_i32,
                     [c_vp, c_vp, c_vp, c_vp, ctypes.c_int, c_vp, c_i32, c_i32, c_i32, c_flt,
                      c_vp, c_vp, c_vp, _sz, ctypes.POINTER(_lib.WarmReport), c_vp])


class WarmStart:
    """The learned warm start: half-resolution adjoint, U-Net, trilinear x2
    upsampling and least-squares rescale with fallback (gpair_warm_start).

    full / half: bound ``Plan`` objects on (2d, 2h, 2w) and (d, h, w) kernel
    grids in grid order; params: U-Net parameters; inv_kappa: the input
    normalisation (1 / the half operator's squared norm)."""

    def __init__(self, full, half, levels, params, dims, inv_kappa):
        self.full, self.half, self.levels = full, half, levels
        self.dims = tuple(int(v) for v in dims)
        self.inv_kappa = float(inv_kappa)
        self.params = torch.as_tensor(params, dtype=torch.float32).to(full.device).contiguous()
        d, h, w = self.dims
        nbytes = int(_ws_size(levels, d, h, w, full.n_sensors * full.n_samples))
        if nbytes == 0:
            raise ValueError("unsupported warm-start shape")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=full.device)

    def __call__(self, b, sigma_full, sigma_half, out=None):
        d, h, w = self.dims
        if out is None:
            out = torch.empty(8 * d * h * w, dtype=torch.float32, device=self.full.device)
        rep = _lib.WarmReport()
        check(_warm_start(self.full._h, _ptr(sigma_full, "sigma_full", torch.float32), self.half._h,
                          _ptr(sigma_half, "sigma_half", torch.float32), self.levels,
                          _ptr(self.params, "params"), d, h, w, self.inv_kappa,
                          _ptr(b, "b", torch.float32), _ptr(out, "out", torch.float32),
                          _ptr(self.ws, "ws"), self.ws.numel(), ctypes.byref(rep), _stream()),
              "gpair_warm_start")
        return out, {"c_star": rep.c_star, "rho": rep.rho, "fell_back": bool(rep.fell_back)}
