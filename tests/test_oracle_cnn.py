"""Pins of the warm-start network oracle (oracle/cnn.py) against library
routines (torch CPU float64 conv3d and autograd, bfloat16 cast, avg_pool3d,
nearest interpolation, torch.optim.Adam), adjoint identities and finite
differences."""

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import cnn as C


def _t(a):
    return torch.as_tensor(a, dtype=torch.float64)


def _ncdhw(x):          # channels-last -> torch layout
    return _t(x).permute(0, 4, 1, 2, 3)


def _w_torch(w):        # [co, kz, ky, kx, ci] -> [co, ci, kz, ky, kx]
    return _t(w).permute(0, 4, 1, 2, 3)


def test_bf16_round_matches_torch_cast():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, -3.5e-3])])
    # exact ties between two bf16 values: mantissa ends in 0x8000
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32).astype(np.float64)
    for x in (a, ties, -ties):
        ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
        np.testing.assert_array_equal(C.bf16_round(x), ref)


@pytest.mark.parametrize("shape,ci,co,stride", [((5, 6, 7), 3, 4, 1), ((5, 6, 7), 3, 4, 2),
                                                 ((8, 8, 8), 2, 16, 2), ((4, 5, 3), 5, 2, 1)])
def test_conv3d_matches_torch(shape, ci, co, stride):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2,) + shape + (ci,))
    w = rng.normal(size=(co, 3, 3, 3, ci))
    b = rng.normal(size=co)
    y = C.conv3d(x, w, b, stride)
    ref = F.conv3d(_ncdhw(x), _w_torch(w), _t(b), stride=stride, padding=1)
    np.testing.assert_allclose(y, ref.permute(0, 2, 3, 4, 1).numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("shape,ci,co,stride", [((5, 6, 7), 3, 4, 1), ((5, 6, 7), 3, 4, 2),
                                                 ((6, 4, 8), 2, 3, 2)])
def test_conv_gradients_match_torch_autograd(shape, ci, co, stride):
    rng = np.random.default_rng(2)
    x = _t(rng.normal(size=(2,) + shape + (ci,))).requires_grad_(True)
    w = _t(rng.normal(size=(co, 3, 3, 3, ci))).requires_grad_(True)
    b = _t(rng.normal(size=co)).requires_grad_(True)
    y = F.conv3d(x.permute(0, 4, 1, 2, 3), w.permute(0, 4, 1, 2, 3), b, stride=stride,
                 padding=1).permute(0, 2, 3, 4, 1)
    dy = rng.normal(size=tuple(y.shape))
    gx, gw, gb = torch.autograd.grad(y, (x, w, b), _t(dy))
    dx = C.conv3d_dgrad(dy, w.detach().numpy(), tuple(x.shape), stride)
    dw, db = C.conv3d_wgrad(dy, x.detach().numpy(), stride)
    np.testing.assert_allclose(dx, gx.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dw, gw.numpy(), rtol=1e-11, atol=1e-10)
    np.testing.assert_allclose(db, gb.numpy(), rtol=1e-11, atol=1e-11)


def test_conv_gradients_brute_force_tiny():
    # finite differences of L = <conv(x, w, b), dy> in single entries of x and w
    rng = np.random.default_rng(3)
    x = rng.normal(size=(1, 3, 4, 5, 2))
    w = rng.normal(size=(2, 3, 3, 3, 2))
    b = rng.normal(size=2)
    for stride in (1, 2):
        dy = rng.normal(size=C.conv3d(x, w, b, stride).shape)
        L = lambda xx, ww: float((C.conv3d(xx, ww, b, stride) * dy).sum())
        dx = C.conv3d_dgrad(dy, w, x.shape, stride)
        dw, db = C.conv3d_wgrad(dy, x, stride)
        for idx in [(0, 0, 0, 0, 0), (0, 1, 2, 3, 1), (0, 2, 3, 4, 0), (0, 2, 0, 4, 1)]:
            e = np.zeros_like(x)
            e[idx] = 1.0
            assert abs((L(x + e, w) - L(x - e, w)) / 2.0 - dx[idx]) < 1e-9
        for idx in [(0, 0, 0, 0, 0), (1, 1, 2, 0, 1), (0, 2, 2, 2, 1)]:
            e = np.zeros_like(w)
            e[idx] = 1.0
            assert abs((L(x, w + e) - L(x, w - e)) / 2.0 - dw[idx]) < 1e-9
        assert np.allclose(db, dy.reshape(-1, 2).sum(0))


def test_upcat_matches_interpolate_and_is_adjoint():
    rng = np.random.default_rng(4)
    c = rng.normal(size=(2, 3, 2, 4, 5))
    s = rng.normal(size=(2, 6, 4, 8, 3))
    cat = C.upcat(c, s)
    up = F.interpolate(_ncdhw(c), scale_factor=2, mode="nearest").permute(0, 2, 3, 4, 1).numpy()
    np.testing.assert_array_equal(cat[..., :5], up)
    np.testing.assert_array_equal(cat[..., 5:], s)
    d = rng.normal(size=cat.shape)
    dc, ds = C.upcat_bwd(d, 5)
    assert abs((cat * d).sum() - (c * dc).sum() - (s * ds).sum()) < 1e-10


def test_pool4_matches_avg_pool3d():
    rng = np.random.default_rng(5)
    T = 3
    v = rng.normal(size=(T, 3, 8, 12, 16))
    p = C.pool4(v, T)
    ref = F.avg_pool3d(_t(v).reshape(1, 3 * T, 8, 12, 16), 4)[0]     # channel 3j + d
    np.testing.assert_allclose(p, ref.permute(1, 2, 3, 0).numpy(), rtol=1e-13, atol=1e-14)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    tp = _t(p0.copy()).requires_grad_(True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = _t(g)
        opt.step()
        p, m, v = C.adam(p, g, m, v, t, 1e-2)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_mse_gradient_finite_difference():
    rng = np.random.default_rng(7)
    o, t = rng.normal(size=(2, 3, 4)), rng.normal(size=(2, 3, 4))
    L, g = C.mse(o, t)
    e = np.zeros_like(o)
    e[1, 2, 3] = 1e-6
    assert abs((C.mse(o + e, t)[0] - C.mse(o - e, t)[0]) / 2e-6 - g[1, 2, 3]) < 1e-8
    assert abs(L - ((o - t) ** 2).mean()) < 1e-15


def _torch_net(params, x):
    """The same network written with torch ops (float64, no rounding)."""
    def conv(a, name, stride):
        w, b = params[name]
        return F.conv3d(a, w.permute(0, 4, 1, 2, 3), b, stride=stride, padding=1)
    a = x.permute(0, 4, 1, 2, 3)
    e0 = torch.relu(conv(a, "enc0", 1))
    e1 = torch.relu(conv(e0, "enc1", 2))
    e2 = torch.relu(conv(e1, "enc2", 2))
    e3 = torch.relu(conv(e2, "enc3", 2))
    cat = torch.cat([F.interpolate(e3, scale_factor=2, mode="nearest"), e2], dim=1)
    d = torch.relu(conv(cat, "dec", 1))
    return conv(d, "head", 1).permute(0, 2, 3, 4, 1)


def _params(T, rng, width=(4, 6, 8, 10)):
    ch = C.layer_channels(T, width)
    return {k: (rng.normal(size=(co, 3, 3, 3, ci)) / np.sqrt(27 * ci), 0.1 * rng.normal(size=co))
            for k, (ci, co) in ch.items()}


def test_network_matches_torch_autograd_without_rounding():
    rng = np.random.default_rng(8)
    T = 2
    params = _params(T, rng)
    x = (rng.random(size=(2, 16, 16, 16, 2)) > 0.5).astype(np.float64)
    out, cache = C.net_forward(params, x, quant=False)
    tgt = rng.normal(size=out.shape)
    L, dout = C.mse(out, tgt)
    grads = C.net_backward(cache, dout)
    tp = {k: (_t(w).requires_grad_(True), _t(b).requires_grad_(True)) for k, (w, b) in params.items()}
    o = _torch_net(tp, _t(x))
    np.testing.assert_allclose(out, o.detach().numpy(), rtol=1e-11, atol=1e-12)
    Lt = ((o - _t(tgt)) ** 2).mean()
    Lt.backward()
    assert abs(L - float(Lt)) < 1e-12
    for k, (w, b) in tp.items():
        np.testing.assert_allclose(grads[k][0], w.grad.numpy(), rtol=1e-9, atol=1e-12, err_msg=k)
        np.testing.assert_allclose(grads[k][1], b.grad.numpy(), rtol=1e-9, atol=1e-12, err_msg=k)


def test_network_rounding_is_storage_only():
    # with bf16 storage the result stays within bf16 resolution of the exact one
    rng = np.random.default_rng(9)
    params = _params(2, rng)
    x = (rng.random(size=(1, 16, 16, 16, 2)) > 0.5).astype(np.float64)
    out_q, _ = C.net_forward(params, x)
    out, _ = C.net_forward(params, x, quant=False)
    rel = np.abs(out_q - out).max() / np.abs(out).max()
    assert 1e-5 < rel < 5e-2
