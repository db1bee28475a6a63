"""The paper's flow integrator on the GPU (LDDMM_FLAG_RK4): fourth-order
Runge-Kutta departure points against the FP64 oracle, and the order of
convergence against the exact flow of an affine field."""

import sys

import numpy as np
import pytest
import torch
from scipy.linalg import expm

from oracle import lddmm as O
from paper_1605_02060_amd import lddmm as L
from paper_1605_02060_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def host(x):
    return x.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _lp(prm, **kw):
    return L.Params(alpha=prm.alpha, gamma=prm.gamma, sigma=prm.sigma, T=prm.T,
                    n_levels=prm.n_levels, iters=prm.iters, step=prm.step, guard=prm.guard,
                    weight=prm.weight, flags=L.FLAG_RK4, **kw)


@pytest.mark.parametrize("shape,h", [((32, 32, 32), 0.05), ((20, 27, 33), 0.1)])
def test_rk4_energy_and_gradient_match_oracle(shape, h):
    say(f"rk4 energy/gradient {shape} h={h}")
    p = synth.blob_pair(shape, 6, max_disp=2.0, sigma=(2.0, 4.0))
    P = tuple(O.smooth7(n) for n in shape)
    T = 4
    v = (h * synth.random_velocity(P, T, 120, vmax=2.0, sigma_s=3.0)).astype(np.float32)
    prm = O.Params(T=T, spacing=h, integrator="rk4", weight=(1.0, 0.3))
    prob = O.Problem(p.M0, p.M1, p.MI0, p.MI1)
    ref = O.energy(prob, prm, v.astype(np.float64))
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    out = host(L.lddmm_energy(*args, t(v), _lp(prm), spacing=h))
    assert rel(out[0], ref["E"]) < 1e-5 and rel(out[2], ref["D"]) < 1e-5
    # the integrator matters at this displacement: the first-order energy differs
    ref1 = O.energy(prob, O.Params(T=T, spacing=h, weight=(1.0, 0.3)), v.astype(np.float64))
    assert rel(ref1["D"], ref["D"]) > 1e-4
    g_ref, st, _ = O.gradient(prob, prm, v.astype(np.float64), kind="V")
    g, _ = L.lddmm_gradient(*args, t(v), _lp(prm), kind=L.GRAD_V, spacing=h)
    err = np.abs(host(g) - g_ref).max() / np.abs(g_ref).max()
    assert err < 2e-5, err


def test_rk4_register_matches_oracle():
    say("rk4 register blobs32 T=4")
    p = synth.config_pair("blobs32")
    h = 0.05
    prm = O.Params(T=4, iters=(8,), step=0.05, spacing=h, integrator="rk4")
    ref = O.register(O.Problem(p.M0, p.M1, p.MI0, p.MI1), prm)
    res = L.lddmm_register(t(p.M0), t(p.M1), t(p.MI0), t(p.MI1), params=_lp(prm), spacing=h)
    torch.cuda.synchronize()
    tr = host(res["trace"])
    rt = np.array(ref.trace)
    np.testing.assert_array_equal(tr[:, 6], rt[:, 6])
    fin = np.isfinite(rt[:, 0])
    assert np.all(np.abs(tr[fin, 0] - rt[fin, 0]) <= 1e-5 * np.abs(rt[fin, 0]))
    assert np.abs(host(res["phi10"]) - ref.phi10).max() / h < 1e-4
    assert np.abs(host(res["phi01"]) - ref.phi01).max() / h < 1e-4
    assert res["status"] == ref.status


def _affine_error(T):
    shape = (24, 28, 30)                      # 7-smooth: the computational grid is the image grid
    P = L.lddmm_comp_grid(shape, L.Params(T=T), 0, 1.0)
    A = np.array([[0.05, -0.9, 0.1], [0.9, 0.0, -0.2], [0.0, 0.3, -0.05]])
    c = np.array([shape[2] / 2 - 0.3, shape[1] / 2 + 0.2, shape[0] / 2 - 0.1]).reshape(3, 1, 1, 1)
    vP = np.einsum("ab,b...->a...", A, O.index_positions(P) - c)
    v = np.broadcast_to(vP, (T, 3) + P).astype(np.float32)
    zeros = np.zeros(shape, np.float32)
    prm = L.Params(T=T, iters=(0,), step=0.01, guard=False, flags=L.FLAG_RK4)
    res = L.lddmm_register(t(zeros), t(zeros), params=prm, spacing=1.0, v=t(v))
    torch.cuda.synchronize()
    d = O.index_positions(shape) - c
    exact10 = np.einsum("ab,b...->a...", expm(-A), d) - d      # phi_10 - id
    exact01 = np.einsum("ab,b...->a...", expm(A), d) - d       # phi_01 - id
    m = np.linalg.norm(d, axis=0) < 5.0
    return (np.abs(host(res["phi10"]) - exact10)[:, m].max(),
            np.abs(host(res["phi01"]) - exact01)[:, m].max())


def test_rk4_fourth_order_on_the_gpu():
    # trilinear sampling of an affine field is exact, so only the time integration errs:
    # halving the step divides the error by about 2^4 (FP32 keeps it well above rounding)
    say("rk4 order, affine field")
    e2, e4, e8 = _affine_error(2), _affine_error(4), _affine_error(8)
    print("rk4 errors", e2, e4, e8)
    for k in (0, 1):
        assert e2[k] < 3e-3 and 12.0 < e2[k] / e4[k] < 20.0
        # at T = 8 the error nears FP32 rounding of 4-voxel displacements, which
        # bounds the ratio from below less tightly
        assert np.isfinite(e8[k]) and 6.0 < e4[k] / e8[k] < 20.0


def test_rk4_rejected_where_not_defined():
    say("rk4 rejected: batched, exact gradient")
    p = synth.blob_pair((16, 16, 16), 7, max_disp=1.0)
    prm = L.Params(T=2, iters=(1,), flags=L.FLAG_RK4)
    d = {"M0": t(p.M0), "M1": t(p.M1)}
    with pytest.raises(L.LddmmError):
        L.lddmm_register_batched([d, d], prm)
    v = torch.zeros((2, 3, 16, 16, 16), device=DEV)
    with pytest.raises(L.LddmmError):
        L.lddmm_gradient(d["M0"], d["M1"], None, None, v, prm, kind=L.GRAD_L2)


def test_rk4_staged_backward_is_bitwise_the_grid_stride_one():
    # the LDS-staged body-force sweep and the grid-stride one take the same RK4
    # departure points; forcing each in turn must give the same bits everywhere,
    # including the min-det trace column, whose reduction is sized by the
    # staged/grid-stride choice, and the oracle's trajectory
    say("rk4 staged vs grid-stride backward, ragged 20x27x33")
    p = synth.blob_pair((20, 27, 33), 9, max_disp=2.0, sigma=(2.0, 4.0))
    h = 0.1
    prm = O.Params(T=4, iters=(6,), step=0.02, spacing=h, integrator="rk4", weight=(1.0, 0.5))
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    out = {}
    try:
        for name, thr in (("staged", 1), ("grid", 1 << 30)):
            L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, thr)
            res = L.lddmm_register(*args, params=_lp(prm), spacing=h)
            torch.cuda.synchronize()
            out[name] = {k: host(res[k]) for k in ("v", "phi10", "phi01", "trace")}
    finally:
        L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, 2048)
    for k in ("v", "phi10", "phi01", "trace"):
        np.testing.assert_array_equal(out["staged"][k], out["grid"][k], err_msg=k)
    ref = O.register(O.Problem(p.M0, p.M1, p.MI0, p.MI1), prm)
    tr, rt = out["staged"]["trace"], np.array(ref.trace)
    np.testing.assert_array_equal(tr[:, 6], rt[:, 6])
    fin = np.isfinite(rt[:, 0])
    assert np.all(np.abs(tr[fin, 0] - rt[fin, 0]) <= 1e-5 * np.abs(rt[fin, 0]))
    assert np.abs(out["staged"]["phi10"] - ref.phi10).max() / h < 1e-4
