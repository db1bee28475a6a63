"""Python binding of the warm-start network kernels (include/lddmm_cnn.h).

Argument marshalling only: every operation runs in liblddmm.so.  Tensors are
torch device tensors, channels-last [n, d, h, w, c]; bf16 tensors are
torch.bfloat16 (the same 16-bit pattern the library uses).
"""

from __future__ import annotations

import ctypes

import torch

from .lddmm import _check, _ptr, _stream, load

BF16, F32 = 0, 1


class _Shape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("d", ctypes.c_int32), ("h", ctypes.c_int32),
                ("w", ctypes.c_int32), ("c", ctypes.c_int32)]


EXPORTED = ["lddmm_conv3d_forward", "lddmm_conv3d_backward_data", "lddmm_conv3d_wgrad_workspace",
            "lddmm_conv3d_backward_weight", "lddmm_cnn_transpose_weight", "lddmm_cnn_to_bf16",
            "lddmm_cnn_upcat", "lddmm_cnn_upcat_backward", "lddmm_cnn_mse",
            "lddmm_cnn_mse_workspace", "lddmm_cnn_adam", "lddmm_cnn_pack_masks",
            "lddmm_cnn_pool_velocity", "lddmm_cnn_expand_velocity"]

_bound = False


def _lib():
    global _bound
    lib = load()
    if _bound:
        return lib
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    sz = ctypes.c_size_t
    sig = {
        "lddmm_conv3d_forward": [vp, _Shape, vp, vp, i32, i32, i32, vp, i32, vp],
        "lddmm_conv3d_backward_data": [vp, _Shape, i32, i32, vp, vp, vp, i32, i32, vp, i32, vp],
        "lddmm_conv3d_backward_weight": [vp, vp, _Shape, i32, i32, vp, vp, vp, sz, vp],
        "lddmm_cnn_transpose_weight": [vp, i32, i32, vp, vp],
        "lddmm_cnn_to_bf16": [vp, i64, vp, vp],
        "lddmm_cnn_upcat": [vp, _Shape, vp, i32, vp, vp],
        "lddmm_cnn_upcat_backward": [vp, _Shape, i32, vp, vp],
        "lddmm_cnn_mse": [vp, vp, i64, vp, vp, vp, sz, vp],
        "lddmm_cnn_adam": [vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp, vp],
        "lddmm_cnn_pack_masks": [vp, vp, i64, vp, vp],
        "lddmm_cnn_pool_velocity": [vp, i32, i32, i32, i32, f32, vp, vp],
        "lddmm_cnn_expand_velocity": [vp, i32, i32, i32, i32, f32, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lddmm_conv3d_wgrad_workspace.argtypes = [_Shape, i32, i32]
    lib.lddmm_conv3d_wgrad_workspace.restype = sz
    lib.lddmm_cnn_mse_workspace.argtypes = [i64]
    lib.lddmm_cnn_mse_workspace.restype = sz
    _bound = True
    return lib


def _shape(t):
    n, d, h, w, c = t.shape
    return _Shape(n, d, h, w, c)


def _dt(t):
    if t.dtype == torch.bfloat16:
        return BF16
    if t.dtype == torch.float32:
        return F32
    raise ValueError(f"unsupported dtype {t.dtype}")


def out_extent(n, stride):
    return (n - 1) // stride + 1


def conv3d_forward(x, w, bias, stride, relu, out_dtype=torch.bfloat16, out=None, stream=None):
    """y = act(conv(x, w) + bias); x [n,d,h,w,ci] bf16, w [co,3,3,3,ci] bf16."""
    n, d, h, wd, ci = x.shape
    co = w.shape[0]
    if tuple(w.shape) != (co, 3, 3, 3, ci) or x.dtype != torch.bfloat16 or w.dtype != torch.bfloat16:
        raise ValueError("conv3d_forward: bad operand shapes or dtypes")
    if bias is not None and (bias.dtype != torch.float32 or bias.numel() != co):
        raise ValueError("conv3d_forward: bias must be float32 [co]")
    shp = (n, out_extent(d, stride), out_extent(h, stride), out_extent(wd, stride), co)
    if out is None:
        out = torch.empty(shp, dtype=out_dtype, device=x.device)
    elif tuple(out.shape) != shp:
        raise ValueError("conv3d_forward: bad output shape")
    _check(_lib().lddmm_conv3d_forward(_ptr(x), _shape(x), _ptr(w), _ptr(bias), co, stride,
                                       int(bool(relu)), _ptr(out), _dt(out), _stream(stream)),
           "lddmm_conv3d_forward")
    return out


def conv3d_backward_data(dy, in_shape, wt, stride, mask=None, add=None, add_off=0,
                         out_dtype=torch.bfloat16, out=None, stream=None):
    """dx = conv^T(dy) [* 1[mask > 0]] [+ add[..., add_off:add_off+ci]];
    wt [ci, 27 co] bf16 (transpose_weight)."""
    n, d, h, wd, ci = in_shape
    co = dy.shape[-1]
    if wt.numel() != ci * 27 * co or dy.dtype != torch.bfloat16 or wt.dtype != torch.bfloat16:
        raise ValueError("conv3d_backward_data: bad operand shapes or dtypes")
    exp = (n, out_extent(d, stride), out_extent(h, stride), out_extent(wd, stride), co)
    if tuple(dy.shape) != exp:
        raise ValueError("conv3d_backward_data: dy shape does not match")
    if mask is not None and (tuple(mask.shape) != tuple(in_shape) or mask.dtype != torch.bfloat16):
        raise ValueError("conv3d_backward_data: bad mask")
    add_stride = 0
    if add is not None:
        if tuple(add.shape[:4]) != tuple(in_shape[:4]) or add.dtype != torch.bfloat16:
            raise ValueError("conv3d_backward_data: bad addend")
        add_stride = add.shape[-1]
    if out is None:
        out = torch.empty(tuple(in_shape), dtype=out_dtype, device=dy.device)
    s = _Shape(*in_shape)
    _check(_lib().lddmm_conv3d_backward_data(_ptr(dy), s, co, stride, _ptr(wt), _ptr(mask),
                                             _ptr(add), add_stride, add_off, _ptr(out), _dt(out),
                                             _stream(stream)),
           "lddmm_conv3d_backward_data")
    return out


def wgrad_workspace_bytes(in_shape, co, stride):
    return int(_lib().lddmm_conv3d_wgrad_workspace(_Shape(*in_shape), co, stride))


def conv3d_backward_weight(dy, x, stride, ws=None, dw=None, db=None, stream=None):
    """dw [co,3,3,3,ci] and db [co] (float32) of the convolution."""
    co = dy.shape[-1]
    ci = x.shape[-1]
    need = wgrad_workspace_bytes(tuple(x.shape), co, stride)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    if dw is None:
        dw = torch.empty((co, 3, 3, 3, ci), dtype=torch.float32, device=x.device)
    if db is None:
        db = torch.empty(co, dtype=torch.float32, device=x.device)
    _check(_lib().lddmm_conv3d_backward_weight(_ptr(dy), _ptr(x), _shape(x), co, stride, _ptr(dw),
                                               _ptr(db), _ptr(ws), ws.numel(), _stream(stream)),
           "lddmm_conv3d_backward_weight")
    return dw, db


def transpose_weight(w, out=None, stream=None):
    co, ci = w.shape[0], w.shape[-1]
    if out is None:
        out = torch.empty((ci, 27 * co), dtype=torch.bfloat16, device=w.device)
    _check(_lib().lddmm_cnn_transpose_weight(_ptr(w), co, ci, _ptr(out), _stream(stream)),
           "lddmm_cnn_transpose_weight")
    return out


def to_bf16(src, out=None, stream=None):
    if out is None:
        out = torch.empty(src.shape, dtype=torch.bfloat16, device=src.device)
    _check(_lib().lddmm_cnn_to_bf16(_ptr(src), src.numel(), _ptr(out), _stream(stream)),
           "lddmm_cnn_to_bf16")
    return out


def upcat(coarse, skip, out=None, stream=None):
    n, d, h, w, cc = coarse.shape
    cs = skip.shape[-1]
    if tuple(skip.shape[:4]) != (n, 2 * d, 2 * h, 2 * w):
        raise ValueError("upcat: skip must be twice the coarse extent")
    if out is None:
        out = torch.empty((n, 2 * d, 2 * h, 2 * w, cc + cs), dtype=torch.bfloat16,
                          device=coarse.device)
    _check(_lib().lddmm_cnn_upcat(_ptr(coarse), _shape(coarse), _ptr(skip), cs, _ptr(out),
                                  _stream(stream)), "lddmm_cnn_upcat")
    return out


def upcat_backward(dcat, coarse_shape, out=None, stream=None):
    cs = dcat.shape[-1] - coarse_shape[-1]
    if out is None:
        out = torch.empty(tuple(coarse_shape), dtype=torch.bfloat16, device=dcat.device)
    _check(_lib().lddmm_cnn_upcat_backward(_ptr(dcat), _Shape(*coarse_shape), cs, _ptr(out),
                                           _stream(stream)), "lddmm_cnn_upcat_backward")
    return out


def mse(out, target, dout=None, loss=None, ws=None, stream=None):
    """loss (device float64 scalar tensor) and dout (bf16) of mean squared error."""
    n = out.numel()
    if target.numel() != n:
        raise ValueError("mse: size mismatch")
    need = int(_lib().lddmm_cnn_mse_workspace(n))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=out.device)
    if dout is None:
        dout = torch.empty(out.shape, dtype=torch.bfloat16, device=out.device)
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=out.device)
    _check(_lib().lddmm_cnn_mse(_ptr(out), _ptr(target), n, _ptr(dout), _ptr(loss), _ptr(ws),
                                ws.numel(), _stream(stream)), "lddmm_cnn_mse")
    return loss, dout


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, p_bf16=None, stream=None):
    _check(_lib().lddmm_cnn_adam(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), step, lr, beta1,
                                 beta2, eps, _ptr(p_bf16), _stream(stream)), "lddmm_cnn_adam")


def pack_masks(M0, M1, out=None, stream=None):
    """[d, h, w] float32 masks -> [d, h, w, 2] bf16 network input."""
    if out is None:
        out = torch.empty(tuple(M0.shape) + (2,), dtype=torch.bfloat16, device=M0.device)
    _check(_lib().lddmm_cnn_pack_masks(_ptr(M0), _ptr(M1), M0.numel(), _ptr(out),
                                       _stream(stream)), "lddmm_cnn_pack_masks")
    return out


def pool_velocity(v, scale, out=None, stream=None):
    """v [T, 3, d, h, w] -> label [d/4, h/4, w/4, 3T] (times scale)."""
    T, _, d, h, w = v.shape
    if out is None:
        out = torch.empty((d // 4, h // 4, w // 4, 3 * T), dtype=torch.float32, device=v.device)
    _check(_lib().lddmm_cnn_pool_velocity(_ptr(v), T, d, h, w, scale, _ptr(out), _stream(stream)),
           "lddmm_cnn_pool_velocity")
    return out


def expand_velocity(out, T, scale, v=None, scratch=None, stream=None):
    """Network output [d, h, w, 3T] -> v [T, 3, 4d, 4h, 4w] (times scale, two cell-centred
    trilinear 2x upsamplings)."""
    d, h, w, C = out.shape
    if C != 3 * T:
        raise ValueError("expand_velocity: channel count is not 3T")
    if v is None:
        v = torch.empty((T, 3, 4 * d, 4 * h, 4 * w), dtype=torch.float32, device=out.device)
    need = 3 * T * (8 * d * h * w + d * h * w)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.float32, device=out.device)
    _check(_lib().lddmm_cnn_expand_velocity(_ptr(out), T, d, h, w, scale, _ptr(v), _ptr(scratch),
                                            _stream(stream)), "lddmm_cnn_expand_velocity")
    return v
