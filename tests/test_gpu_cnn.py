"""GPU parity of the warm-start network kernels against the FP64 oracle
(oracle/cnn.py), through the C ABI.

Operands are drawn on the CPU, rounded to bf16 once, and handed to both
sides, so the only differences are the GPU's FP32 accumulation order and, for
bf16 outputs, the final rounding.  For an FP32 output of a K-term sum the
MFMA path adds 32-term blocks and then ~K/32 partial sums in sequence, so the
error is below (K/32 + 32) * 2^-24 * sum |terms|; the tests check
|gpu - oracle| <= 4 * that bound + 1e-6 with sum |terms| from the oracle's
convolution of |x| with |w|.
"""

import sys

import numpy as np
import pytest
import torch

from oracle import cnn as C
from oracle import lddmm as O
from paper_1605_02060_amd import cnn as G

pytestmark = pytest.mark.gpu
DEV = "cuda"
U = 2.0 ** -24


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def bf(a):
    """CPU array -> (bf16-rounded float64 array, bf16 device tensor)."""
    q = C.bf16_round(a)
    return q, torch.as_tensor(q, dtype=torch.float32).to(torch.bfloat16).to(DEV).contiguous()


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def bound(K, absconv):
    return 4.0 * (K / 32.0 + 32.0) * U * absconv + 1e-6


CONV_CASES = [
    # (n, (d, h, w), ci, co, stride)
    (2, (9, 10, 11), 16, 32, 1),
    (2, (9, 10, 11), 16, 32, 2),
    (1, (12, 7, 9), 2, 16, 1),        # first layer: 2 input channels (unvectorised loads)
    (2, (8, 8, 8), 32, 64, 2),
    (1, (6, 5, 7), 192, 64, 1),       # decoder: 3 column tiles
    (2, (6, 6, 6), 64, 30, 1),        # head: 30 outputs
    (1, (5, 9, 6), 64, 128, 2),
]


@pytest.mark.parametrize("n,dims,ci,co,stride", CONV_CASES)
def test_conv_forward_matches_oracle(n, dims, ci, co, stride):
    say(f"conv fwd n={n} {dims} {ci}->{co} s={stride}")
    rng = np.random.default_rng(11)
    xq, xg = bf(rng.normal(size=(n,) + dims + (ci,)))
    wq, wg = bf(rng.normal(size=(co, 3, 3, 3, ci)) / np.sqrt(27 * ci))
    b = rng.normal(size=co).astype(np.float32).astype(np.float64)
    bg = torch.as_tensor(b, dtype=torch.float32, device=DEV)
    ref = C.conv3d(xq, wq, b, stride)
    absref = C.conv3d(np.abs(xq), np.abs(wq), np.abs(b), stride)
    y = G.conv3d_forward(xg, wg, bg, stride, relu=False, out_dtype=torch.float32)
    torch.cuda.synchronize()
    err = np.abs(host(y) - ref)
    assert np.all(err <= bound(27 * ci, absref)), err.max()
    # bf16 output with ReLU: within one bf16 step of the rounded exact value
    yb = host(G.conv3d_forward(xg, wg, bg, stride, relu=True))
    rb = C.bf16_round(C.relu(ref))
    assert np.all(np.abs(yb - rb) <= 2.0 ** -7 * np.abs(rb) + 1e-6)


@pytest.mark.parametrize("n,dims,ci,co,stride", CONV_CASES)
def test_conv_backward_data_matches_oracle(n, dims, ci, co, stride):
    say(f"conv dgrad n={n} {dims} {ci}->{co} s={stride}")
    rng = np.random.default_rng(12)
    xshape = (n,) + dims + (ci,)
    oshape = (n,) + tuple(C.out_size(k, stride) for k in dims) + (co,)
    dyq, dyg = bf(rng.normal(size=oshape))
    wq, wg = bf(rng.normal(size=(co, 3, 3, 3, ci)) / np.sqrt(27 * co))
    wt = G.transpose_weight(wg)
    np.testing.assert_array_equal(host(wt).reshape(ci, 3, 3, 3, co), wq.transpose(4, 1, 2, 3, 0))
    ref = C.conv3d_dgrad(dyq, wq, xshape, stride)
    absref = C.conv3d_dgrad(np.abs(dyq), np.abs(wq), xshape, stride)
    dx = G.conv3d_backward_data(dyg, xshape, wt, stride, out_dtype=torch.float32)
    torch.cuda.synchronize()
    err = np.abs(host(dx) - ref)
    assert np.all(err <= bound(27 * co, absref)), err.max()
    # with a ReLU mask and an addend taken from a wider tensor
    maskq, maskg = bf(rng.normal(size=xshape))
    addq, addg = bf(rng.normal(size=xshape[:4] + (ci + 5,)))
    dx2 = G.conv3d_backward_data(dyg, xshape, wt, stride, mask=maskg, add=addg, add_off=3,
                                 out_dtype=torch.float32)
    ref2 = ref * (maskq > 0) + addq[..., 3:3 + ci]
    err2 = np.abs(host(dx2) - ref2)
    assert np.all(err2 <= bound(27 * co, absref) + 1e-6 * np.abs(addq[..., 3:3 + ci])), err2.max()


@pytest.mark.parametrize("n,dims,ci,co,stride", CONV_CASES)
def test_conv_backward_weight_matches_oracle(n, dims, ci, co, stride):
    say(f"conv wgrad n={n} {dims} {ci}->{co} s={stride}")
    rng = np.random.default_rng(13)
    xshape = (n,) + dims + (ci,)
    oshape = (n,) + tuple(C.out_size(k, stride) for k in dims) + (co,)
    xq, xg = bf(rng.normal(size=xshape))
    dyq, dyg = bf(rng.normal(size=oshape))
    ref_w, ref_b = C.conv3d_wgrad(dyq, xq, stride)
    abs_w, abs_b = C.conv3d_wgrad(np.abs(dyq), np.abs(xq), stride)
    dw, db = G.conv3d_backward_weight(dyg, xg, stride)
    torch.cuda.synchronize()
    K = int(np.prod(oshape[:4]))
    # split-K partial tiles are summed in FP32 as well: allow the K-term sequential bound
    tol_w = 4.0 * (K / 32.0 + 64.0) * U * abs_w + 1e-6
    assert np.all(np.abs(host(dw) - ref_w) <= tol_w), np.abs(host(dw) - ref_w).max()
    tol_b = 4.0 * (K / 8.0 + 64.0) * U * abs_b + 1e-6
    assert np.all(np.abs(host(db) - ref_b) <= tol_b)
    # deterministic: a second call gives the same bits
    dw2, db2 = G.conv3d_backward_weight(dyg, xg, stride)
    assert torch.equal(dw, dw2) and torch.equal(db, db2)


def test_upcat_and_backward():
    say("upcat")
    rng = np.random.default_rng(14)
    cq, cg = bf(rng.normal(size=(2, 3, 4, 5, 6)))
    sq, sg = bf(rng.normal(size=(2, 6, 8, 10, 4)))
    out = G.upcat(cg, sg)
    np.testing.assert_array_equal(host(out), C.upcat(cq, sq))
    dq, dg = bf(rng.normal(size=(2, 6, 8, 10, 10)))
    dc = G.upcat_backward(dg, (2, 3, 4, 5, 6))
    ref, _ = C.upcat_bwd(dq, 6)
    assert np.all(np.abs(host(dc) - C.bf16_round(ref)) <= 2.0 ** -7 * np.abs(ref) + 1e-30)


def test_mse_adam_and_bf16():
    say("mse / adam / to_bf16")
    rng = np.random.default_rng(15)
    o = rng.normal(size=(3, 4, 5, 6)).astype(np.float32)
    t = rng.normal(size=(3, 4, 5, 6)).astype(np.float32)
    loss, dout = G.mse(torch.as_tensor(o, device=DEV), torch.as_tensor(t, device=DEV))
    L, g = C.mse(o.astype(np.float64), t.astype(np.float64))
    assert abs(float(loss) - L) <= 1e-12 * L
    assert np.all(np.abs(host(dout) - C.bf16_round(g)) <= 2.0 ** -7 * np.abs(g))
    x = rng.normal(size=1000).astype(np.float32)
    np.testing.assert_array_equal(host(G.to_bf16(torch.as_tensor(x, device=DEV))),
                                  C.bf16_round(x))
    p = rng.normal(size=777).astype(np.float32)
    pg = torch.as_tensor(p, device=DEV)
    mg, vg = torch.zeros_like(pg), torch.zeros_like(pg)
    pb = torch.empty(777, dtype=torch.bfloat16, device=DEV)
    pr, mr, vr = p.astype(np.float64), np.zeros(777), np.zeros(777)
    for step in range(1, 5):
        gr = rng.normal(size=777).astype(np.float32)
        G.adam(pg, torch.as_tensor(gr, device=DEV), mg, vg, step, 1e-2, p_bf16=pb)
        pr, mr, vr = C.adam(pr, gr.astype(np.float64), mr, vr, step, 1e-2)
    np.testing.assert_allclose(host(pg), pr, rtol=1e-5, atol=1e-6)
    np.testing.assert_array_equal(host(pb), C.bf16_round(host(pg)))


def test_pool_and_expand_velocity():
    say("pool / expand velocity")
    rng = np.random.default_rng(16)
    T = 3
    v = rng.normal(size=(T, 3, 8, 12, 16)).astype(np.float32)
    lab = G.pool_velocity(torch.as_tensor(v, device=DEV), 0.5)
    np.testing.assert_allclose(host(lab), 0.5 * C.pool4(v.astype(np.float64), T), rtol=1e-5,
                               atol=1e-6)
    out = rng.normal(size=(3, 4, 5, 3 * T)).astype(np.float32)
    ve = G.expand_velocity(torch.as_tensor(out, device=DEV), T, 2.0)
    planar = 2.0 * out.astype(np.float64).transpose(3, 0, 1, 2)          # [3T][d][h][w]
    ref = np.stack([O.upsample2_clamp(O.upsample2_clamp(f, (6, 8, 10)), (12, 16, 20))
                    for f in planar])
    np.testing.assert_allclose(host(ve).reshape(3 * T, 12, 16, 20), ref, rtol=1e-5, atol=1e-5)


def test_pack_masks():
    say("pack masks")
    rng = np.random.default_rng(17)
    M0 = (rng.random((5, 6, 7)) > 0.5).astype(np.float32)
    M1 = (rng.random((5, 6, 7)) > 0.5).astype(np.float32)
    x = G.pack_masks(torch.as_tensor(M0, device=DEV), torch.as_tensor(M1, device=DEV))
    np.testing.assert_array_equal(host(x), np.stack([M0, M1], axis=-1))
