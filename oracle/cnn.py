"""FP64 CPU oracle of the warm-start network -- TEST INFRASTRUCTURE ONLY.

The paper registers every brain from v = 0; it has no network.  The warm start
is an addition of this library: a small 3-D convolutional encoder-decoder maps
the mask pair (M0, M1) to an initial velocity, which the paper's gradient
descent (Methods, Registration) then refines.  This module is the plain
definition of every operation the GPU trains and runs it with, written out in
FP64 NumPy so the GPU kernels can be compared element by element:

* 3x3x3 cross-correlation with zero padding 1 and stride s in {1, 2}, on
  channels-last tensors x[b, z, y, x, c], weights w[co, kz, ky, kx, ci], plus
  its input gradient (the adjoint map) and weight / bias gradients;
* ReLU, nearest 2x upsampling concatenated with a skip tensor, mean squared
  error, 4x4x4 block averaging of the label velocity, and one Adam step
  (Kingma and Ba's update with bias correction);
* the whole network and its reverse pass.

Storage precision is mirrored, arithmetic is not: the GPU stores weights and
activations as bfloat16 (round to nearest even) and accumulates in FP32; the
oracle rounds the same tensors to bfloat16 at the same points and sums in
FP64.  Only tests/ may import this module.

Pins (tests/test_oracle_cnn.py): torch.nn.functional.conv3d in float64 and its
autograd (library routines), brute-force finite differences on tiny inputs,
the adjoint identity, torch's bfloat16 cast, torch.optim.Adam and
torch's avg_pool3d.
"""

from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ bf16 ----

def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    bfloat16 keeps the top 16 bits of the IEEE binary32 pattern."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------------ conv ----

def out_size(n, stride):
    """Output extent of a 3-tap window with zero padding 1."""
    return (n - 1) // stride + 1


def conv3d(x, w, bias, stride):
    """y[b, o, co] = bias[co] + sum_{k, ci} w[co, k, ci] x[b, s*o + k - 1, ci]
    (o and k are 3-D; samples outside x are zero)."""
    B, D, H, W, Ci = x.shape
    Co = w.shape[0]
    Do, Ho, Wo = out_size(D, stride), out_size(H, stride), out_size(W, stride)
    xp = np.zeros((B, D + 2, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    y = np.zeros((B, Do, Ho, Wo, Co))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                patch = xp[:, kz:kz + stride * (Do - 1) + 1:stride,
                           ky:ky + stride * (Ho - 1) + 1:stride,
                           kx:kx + stride * (Wo - 1) + 1:stride]
                y += patch @ w[:, kz, ky, kx, :].T
    return y + bias


def conv3d_dgrad(dy, w, in_shape, stride):
    """Input gradient: dx[b, i, ci] = sum over (o, k) with s*o + k - 1 = i of
    w[co, k, ci] dy[b, o, co] -- the adjoint of conv3d in x."""
    B, D, H, W, Ci = in_shape
    _, Do, Ho, Wo, Co = dy.shape
    dxp = np.zeros((B, D + 2, H + 2, W + 2, Ci))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                dxp[:, kz:kz + stride * (Do - 1) + 1:stride,
                    ky:ky + stride * (Ho - 1) + 1:stride,
                    kx:kx + stride * (Wo - 1) + 1:stride] += dy @ w[:, kz, ky, kx, :]
    return dxp[:, 1:-1, 1:-1, 1:-1]


def conv3d_wgrad(dy, x, stride):
    """Weight and bias gradients: dw[co, k, ci] = sum_{b, o} dy[b, o, co] x[b, s*o + k - 1, ci],
    db[co] = sum_{b, o} dy[b, o, co]."""
    B, D, H, W, Ci = x.shape
    _, Do, Ho, Wo, Co = dy.shape
    xp = np.zeros((B, D + 2, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    dw = np.zeros((Co, 3, 3, 3, Ci))
    g = dy.reshape(-1, Co)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                patch = xp[:, kz:kz + stride * (Do - 1) + 1:stride,
                           ky:ky + stride * (Ho - 1) + 1:stride,
                           kx:kx + stride * (Wo - 1) + 1:stride]
                dw[:, kz, ky, kx, :] = g.T @ patch.reshape(-1, Ci)
    return dw, g.sum(axis=0)


# ------------------------------------------------------ other layers ----

def relu(a):
    return np.maximum(a, 0.0)


def upcat(coarse, skip):
    """Nearest 2x upsampling of `coarse`, then channels [coarse, skip]."""
    up = coarse.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    return np.concatenate([up, skip], axis=-1)


def upcat_bwd(dcat, c_coarse):
    """Gradients of upcat: the coarse part sums its 2x2x2 children."""
    d_up = dcat[..., :c_coarse]
    B, D, H, W, C = d_up.shape
    d_coarse = d_up.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4, 6))
    return d_coarse, dcat[..., c_coarse:]


def mse(out, target):
    """Mean squared error and its gradient in `out`."""
    diff = out - target
    return float((diff * diff).mean()), 2.0 * diff / diff.size


def pool4(v, T):
    """Label of one registration: v[T][3][Z][Y][X] averaged over 4x4x4 blocks and laid
    out channels-last as [Z/4][Y/4][X/4][3T] with channel 3j + d."""
    _, _, Z, Y, X = v.shape
    p = v.reshape(T, 3, Z // 4, 4, Y // 4, 4, X // 4, 4).mean(axis=(3, 5, 7))
    return p.reshape(3 * T, Z // 4, Y // 4, X // 4).transpose(1, 2, 3, 0)


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step count t >= 1): returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------- network ----

# (name, stride): encoder 2 -> 16 -> 32 -> 64 -> 128 over four
# resolutions (levels 1, 1/2, 1/4, 1/8), decoder back to 1/4, head to 3T channels.
LAYERS = (("enc0", 1), ("enc1", 2), ("enc2", 2), ("enc3", 2), ("dec", 1), ("head", 1))


def layer_channels(T, width=(16, 32, 64, 128)):
    c0, c1, c2, c3 = width
    return {"enc0": (2, c0), "enc1": (c0, c1), "enc2": (c1, c2), "enc3": (c2, c3),
            "dec": (c3 + c2, c2), "head": (c2, 3 * T)}


def _identity(a):
    return np.asarray(a, dtype=np.float64)


def net_forward(params, x, quant=True):
    """Forward pass with bfloat16 storage of weights and activations (quant=False:
    no rounding anywhere, for structural checks).  params[name] = (w [co,3,3,3,ci],
    b [co]) in FP64 (master copies); x [B,Z,Y,X,2] masks.  Returns (out [B, Z/4,
    Y/4, X/4, 3T] in FP64, cache for the reverse)."""
    bf16_round = globals()["bf16_round"] if quant else _identity
    wq = {k: bf16_round(w) for k, (w, b) in params.items()}
    bias = {k: b for k, (w, b) in params.items()}
    a = {"in": bf16_round(x)}
    a["enc0"] = bf16_round(relu(conv3d(a["in"], wq["enc0"], bias["enc0"], 1)))
    a["enc1"] = bf16_round(relu(conv3d(a["enc0"], wq["enc1"], bias["enc1"], 2)))
    a["enc2"] = bf16_round(relu(conv3d(a["enc1"], wq["enc2"], bias["enc2"], 2)))
    a["enc3"] = bf16_round(relu(conv3d(a["enc2"], wq["enc3"], bias["enc3"], 2)))
    a["cat"] = upcat(a["enc3"], a["enc2"])
    a["dec"] = bf16_round(relu(conv3d(a["cat"], wq["dec"], bias["dec"], 1)))
    out = conv3d(a["dec"], wq["head"], bias["head"], 1)
    return out, (wq, a, quant)


def net_backward(cache, dout):
    """Reverse pass of net_forward for the output gradient dout.  Gradients of
    activations are stored as bfloat16 where the GPU stores them (after the
    ReLU mask); weight gradients are exact sums.  Returns {name: (dw, db)}."""
    wq, a, quant = cache
    bf16_round = globals()["bf16_round"] if quant else _identity
    grads = {}
    d = bf16_round(dout)
    grads["head"] = conv3d_wgrad(d, a["dec"], 1)
    d = bf16_round(conv3d_dgrad(d, wq["head"], a["dec"].shape, 1) * (a["dec"] > 0))
    grads["dec"] = conv3d_wgrad(d, a["cat"], 1)
    dcat = bf16_round(conv3d_dgrad(d, wq["dec"], a["cat"].shape, 1) * (a["cat"] > 0))
    d3, dskip = upcat_bwd(dcat, a["enc3"].shape[-1])
    d = bf16_round(d3)
    grads["enc3"] = conv3d_wgrad(d, a["enc2"], 2)
    d = bf16_round(conv3d_dgrad(d, wq["enc3"], a["enc2"].shape, 2) * (a["enc2"] > 0) + dskip)
    grads["enc2"] = conv3d_wgrad(d, a["enc1"], 2)
    d = bf16_round(conv3d_dgrad(d, wq["enc2"], a["enc1"].shape, 2) * (a["enc1"] > 0))
    grads["enc1"] = conv3d_wgrad(d, a["enc0"], 2)
    d = bf16_round(conv3d_dgrad(d, wq["enc1"], a["enc0"].shape, 2) * (a["enc0"] > 0))
    grads["enc0"] = conv3d_wgrad(d, a["in"], 1)
    return grads
