"""Python binding of the surrogate kernels (include/lbm_nn.h).

Argument marshalling only: torch tensors provide device memory and the
stream; every operation runs in liblbm.so.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import lbm

BF16, FP32 = 0, 1
EXPORTS = ["lbm_nn_packed_words", "lbm_nn_pack", "lbm_nn_conv_work_bytes", "lbm_nn_conv", "lbm_nn_conv_x",
           "lbm_nn_pool_x", "lbm_nn_up_x",
           "lbm_nn_wgrad_partial_words", "lbm_nn_wgrad",
           "lbm_nn_bias_grad", "lbm_nn_relu_bwd", "lbm_nn_add", "lbm_nn_pool", "lbm_nn_pool_bwd", "lbm_nn_up",
           "lbm_nn_up_bwd", "lbm_nn_mse", "lbm_nn_adam", "lbm_nn_augment", "lbm_nn_warm_fields",
           "lbm_nn_bias_grad_noalloc"]

_lib = None


def load():
    global _lib
    if _lib is None:
        lib = lbm.load()
        vp, i, i64, f = C.c_void_p, C.c_int, C.c_int64, C.c_float
        lib.lbm_nn_packed_words.argtypes = [i, i]
        lib.lbm_nn_packed_words.restype = C.c_size_t
        lib.lbm_nn_pack.argtypes = [vp, i, i, i, i, vp, vp]
        lib.lbm_nn_conv_work_bytes.argtypes = [i, i, i, i, i]
        lib.lbm_nn_conv_work_bytes.restype = C.c_size_t
        lib.lbm_nn_conv.argtypes = [vp, i, vp, vp, vp, vp, i, i, i, i, i, i, vp, vp]
        lib.lbm_nn_conv_x.argtypes = [vp, vp, i, vp, vp, vp, vp, vp, i, i, i, i, i, vp, vp]
        lib.lbm_nn_pool_x.argtypes = [vp, i, i, i, i, vp, vp]
        lib.lbm_nn_up_x.argtypes = [vp, i, i, i, i, vp, vp]
        lib.lbm_nn_wgrad_partial_words.argtypes = [i, i, i, i, i]
        lib.lbm_nn_wgrad_partial_words.restype = C.c_size_t
        lib.lbm_nn_wgrad.argtypes = [vp, i, vp, i, i, i, i, vp, vp, i, vp]
        lib.lbm_nn_bias_grad.argtypes = [vp, i, i64, vp, vp, vp]
        lib.lbm_nn_bias_grad_noalloc.argtypes = [vp, i, i64, vp, vp]
        lib.lbm_nn_relu_bwd.argtypes = [vp, vp, i64, vp]
        lib.lbm_nn_add.argtypes = [vp, vp, i64, vp]
        lib.lbm_nn_pool.argtypes = [vp, i, i, i, i, vp, vp]
        lib.lbm_nn_pool_bwd.argtypes = [vp, i, i, i, i, vp, i, vp]
        lib.lbm_nn_up.argtypes = [vp, i, i, i, i, vp, vp]
        lib.lbm_nn_up_bwd.argtypes = [vp, i, i, i, i, vp, vp]
        lib.lbm_nn_mse.argtypes = [vp, vp, vp, i, i64, vp, vp, vp]
        lib.lbm_nn_adam.argtypes = [vp, vp, vp, vp, i64, f, f, f, f, i, vp]
        lib.lbm_nn_augment.argtypes = [vp, vp, i, i, i, i, vp, vp, i, vp, vp, vp]
        lib.lbm_nn_warm_fields.argtypes = [vp, vp, i64, vp, C.c_double, i, vp, vp, vp, vp]
        for n in EXPORTS:
            if n not in ("lbm_nn_packed_words", "lbm_nn_wgrad_partial_words", "lbm_nn_conv_work_bytes"):
                getattr(lib, n).restype = C.c_int
        _lib = lib
    return _lib


def _s():
    return torch.cuda.current_stream().cuda_stream


def _p(t):
    if t is None:
        return None
    assert t.is_contiguous()
    return t.data_ptr()


def _chk(name, rc):
    if rc != 0:
        raise lbm.LbmError(name, rc)


def pack(W: torch.Tensor, transpose: bool, prec: int) -> torch.Tensor:
    lib = load()
    co, ci = W.shape[0], W.shape[1]
    out = torch.empty(lib.lbm_nn_packed_words(co, ci), dtype=torch.int32, device=W.device)
    _chk("lbm_nn_pack", lib.lbm_nn_pack(_p(W), co, ci, int(transpose), prec, _p(out), _s()))
    return out


def conv(X: torch.Tensor, packed: torch.Tensor, c_out: int, bias=None, skip=None, relu=False, prec=BF16,
         out=None) -> torch.Tensor:
    c_in, D, H, W = X.shape
    lib = load()
    Y = torch.empty((c_out, D, H, W), dtype=torch.float32, device=X.device) if out is None else out
    wb = lib.lbm_nn_conv_work_bytes(c_in, D, H, W, prec)
    work = torch.empty(wb, dtype=torch.uint8, device=X.device) if wb else None
    _chk("lbm_nn_conv", lib.lbm_nn_conv(_p(X), c_in, _p(packed), _p(bias), _p(skip), _p(Y), c_out, D, H, W,
                                        int(relu), prec, _p(work), _s()))
    return Y


def conv_x(packed: torch.Tensor, c_out: int, c_in: int, dhw, X=None, xb=None, bias=None, skip=None, relu=False,
           want_y=True, want_yb=False):
    """BF16 convolution of a chain (lbm_nn_conv_x): input X (FP32) or xb (the
    BF16 channels-innermost copy a previous call returned); returns (Y or
    None, yb or None)."""
    D, H, W = dhw
    lib = load()
    dev = (X if X is not None else xb).device
    Y = torch.empty((c_out, D, H, W), dtype=torch.float32, device=dev) if want_y else None
    yb = torch.empty(lib.lbm_nn_conv_work_bytes(c_out, D, H, W, BF16), dtype=torch.uint8, device=dev) \
        if want_yb else None
    work = None
    if xb is None:
        work = torch.empty(lib.lbm_nn_conv_work_bytes(c_in, D, H, W, BF16), dtype=torch.uint8, device=dev)
    _chk("lbm_nn_conv_x", lib.lbm_nn_conv_x(_p(X), _p(xb), c_in, _p(packed), _p(bias), _p(skip), _p(Y), _p(yb),
                                            c_out, D, H, W, int(relu), _p(work), _s()))
    return Y, yb


def pool_x(X: torch.Tensor) -> torch.Tensor:
    """2x2x2 average pooling into the BF16 input layout of a convolution (lbm_nn_pool_x)."""
    c, D, H, W = X.shape
    lib = load()
    xb = torch.empty(lib.lbm_nn_conv_work_bytes(c, D // 2, H // 2, W // 2, BF16), dtype=torch.uint8, device=X.device)
    _chk("lbm_nn_pool_x", lib.lbm_nn_pool_x(_p(X), c, D, H, W, _p(xb), _s()))
    return xb


def up_x(X: torch.Tensor) -> torch.Tensor:
    """Nearest 2x upsampling into the BF16 input layout of a convolution (lbm_nn_up_x)."""
    c, D, H, W = X.shape
    lib = load()
    xb = torch.empty(lib.lbm_nn_conv_work_bytes(c, 2 * D, 2 * H, 2 * W, BF16), dtype=torch.uint8, device=X.device)
    _chk("lbm_nn_up_x", lib.lbm_nn_up_x(_p(X), c, D, H, W, _p(xb), _s()))
    return xb


def wgrad(X: torch.Tensor, dY: torch.Tensor, prec=BF16) -> torch.Tensor:
    lib = load()
    c_in, D, H, W = X.shape
    c_out = dY.shape[0]
    part = torch.empty(lib.lbm_nn_wgrad_partial_words(c_out, c_in, D, H, W), dtype=torch.float32, device=X.device)
    dW = torch.empty((c_out, c_in, 27), dtype=torch.float32, device=X.device)
    _chk("lbm_nn_wgrad", lib.lbm_nn_wgrad(_p(X), c_in, _p(dY), c_out, D, H, W, _p(dW), _p(part), prec, _s()))
    return dW


def bias_grad(dY: torch.Tensor) -> torch.Tensor:
    c = dY.shape[0]
    db = torch.empty(c, dtype=torch.float32, device=dY.device)
    scratch = torch.empty(64 * c, dtype=torch.float64, device=dY.device)
    _chk("lbm_nn_bias_grad", load().lbm_nn_bias_grad(_p(dY), c, dY[0].numel(), _p(db), _p(scratch), _s()))
    return db


def relu_bwd(Y: torch.Tensor, dY: torch.Tensor) -> None:
    _chk("lbm_nn_relu_bwd", load().lbm_nn_relu_bwd(_p(Y), _p(dY), dY.numel(), _s()))


def augment(X: torch.Tensor, shift, flip, swap: bool, src, sign) -> torch.Tensor:
    """Y[k](r) = sign[k] X[src[k]](g^-1 r) for g = shift o flips o (D, H) exchange
    (lbm_nn_augment); X float32 [c, D, H, W] on the device."""
    c, D, H, W = X.shape
    Y = torch.empty_like(X)
    sh = (C.c_int * 3)(*[int(v) for v in shift])
    fl = (C.c_int * 3)(*[int(bool(v)) for v in flip])
    sr = (C.c_int * c)(*[int(v) for v in src])
    sg = (C.c_float * c)(*[float(v) for v in sign])
    _chk("lbm_nn_augment", load().lbm_nn_augment(_p(X), _p(Y), c, D, H, W, sh, fl, int(bool(swap)), sr, sg, _s()))
    return Y


def warm_fields(Y: torch.Tensor, mask: torch.Tensor, c, shift_x: float, dtype=torch.float64):
    """Solver start (rho0 [1, P], u0 [3, P]) of the given dtype from the
    network output Y float32 [4, ...] (lbm_nn_warm_fields)."""
    P = Y[0].numel()
    rho0 = torch.empty((1, P), dtype=dtype, device=Y.device)
    u0 = torch.empty((3, P), dtype=dtype, device=Y.device)
    scratch = torch.empty(2 + 512, dtype=torch.float64, device=Y.device)
    cc = (C.c_double * 4)(*[float(v) for v in c])
    _chk("lbm_nn_warm_fields", load().lbm_nn_warm_fields(_p(Y), _p(mask), P, cc, float(shift_x),
                                                         8 if dtype == torch.float64 else 4, _p(rho0), _p(u0),
                                                         _p(scratch), _s()))
    return rho0, u0


def add_(y: torch.Tensor, x: torch.Tensor) -> None:
    _chk("lbm_nn_add", load().lbm_nn_add(_p(y), _p(x), y.numel(), _s()))


def pool(X: torch.Tensor) -> torch.Tensor:
    c, D, H, W = X.shape
    Y = torch.empty((c, D // 2, H // 2, W // 2), dtype=torch.float32, device=X.device)
    _chk("lbm_nn_pool", load().lbm_nn_pool(_p(X), c, D, H, W, _p(Y), _s()))
    return Y


def pool_bwd(dY: torch.Tensor, dX: torch.Tensor, accumulate: bool) -> None:
    c, D, H, W = dX.shape
    _chk("lbm_nn_pool_bwd", load().lbm_nn_pool_bwd(_p(dY), c, D, H, W, _p(dX), int(accumulate), _s()))


def up(X: torch.Tensor) -> torch.Tensor:
    c, D, H, W = X.shape
    Y = torch.empty((c, 2 * D, 2 * H, 2 * W), dtype=torch.float32, device=X.device)
    _chk("lbm_nn_up", load().lbm_nn_up(_p(X), c, D, H, W, _p(Y), _s()))
    return Y


def up_bwd(dY: torch.Tensor) -> torch.Tensor:
    c, D, H, W = dY.shape
    dX = torch.empty((c, D // 2, H // 2, W // 2), dtype=torch.float32, device=dY.device)
    _chk("lbm_nn_up_bwd", load().lbm_nn_up_bwd(_p(dY), c, D // 2, H // 2, W // 2, _p(dX), _s()))
    return dX


def mse(Y: torch.Tensor, T: torch.Tensor, mask: torch.Tensor, want_grad=True):
    c = Y.shape[0]
    P = Y[0].numel()
    loss = torch.empty(2 + 512, dtype=torch.float64, device=Y.device)
    dY = torch.empty_like(Y) if want_grad else None
    _chk("lbm_nn_mse", load().lbm_nn_mse(_p(Y), _p(T), _p(mask), c, P, _p(loss), _p(dY), _s()))
    return loss[0], dY


def adam_(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, t: int, lr: float,
          b1=0.9, b2=0.999, eps=1e-8) -> None:
    _chk("lbm_nn_adam", load().lbm_nn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, b1, b2, eps, t, _s()))
