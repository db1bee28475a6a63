"""Pins of the oracle's method-level functions: K, the energy, the flow, the
gradients and the registration loop (CPU only).

Each pin is independent of the formula it checks: K is checked by applying
the stencil operator L twice to K b, the flow by closed-form invariants
(zero / constant / integer-shift fields), the exact gradient by brute-force
finite differences, the plain gradient by its relation to the exact one."""

import math

import numpy as np
import pytest

from oracle import lddmm as O
from paper_1605_02060_amd import synth


def _smooth_v(T, shape, seed, vmax):
    return synth.random_velocity(shape, T, seed, vmax=vmax, sigma_s=1.5).astype(np.float64)


# --------------------------------------------------------------------- K ----

@pytest.mark.parametrize("h,alpha,gamma", [(1.0, 0.02, 1.0), (0.05, 0.02, 1.0), (2.0, 0.7, 0.5)])
def test_K_inverts_LdaggerL_stencil(h, alpha, gamma):
    P = (6, 10, 9)
    b = np.random.default_rng(0).normal(size=(3,) + P)
    Kb = O.apply_K(b, alpha, gamma, h)
    back = O.L_op(O.L_op(Kb, alpha, gamma, h), alpha, gamma, h)
    np.testing.assert_allclose(back, b, atol=1e-10)


def test_K_single_mode_and_constant():
    P = (8, 10, 12)
    h, alpha, gamma = 1.0, 0.02, 1.0
    X = O.index_positions(P)
    k = (2, 3, 1)
    mode = np.cos(2 * math.pi * (k[0] * X[0] / P[2] + k[1] * X[1] / P[1] + k[2] * X[2] / P[0]))
    b = np.stack([mode, 2 * mode, -mode])
    Kb = O.apply_K(b, alpha, gamma, h)
    # L mode = (gamma + alpha lam) mode with lam from the stencil applied to the mode
    lam = -(O.lap_periodic(mode, h) / mode)[np.abs(mode) > 0.5].mean()
    np.testing.assert_allclose(Kb, b / (gamma + alpha * lam) ** 2, atol=1e-13)
    c = np.ones((3,) + P)
    np.testing.assert_allclose(O.apply_K(c, alpha, 0.5, h), c / 0.25, atol=1e-12)


def test_K_symmetric():
    P = (5, 6, 7)
    rng = np.random.default_rng(1)
    x, y = rng.normal(size=(2, 3) + P)
    a = (O.apply_K(x, 0.3, 1.0, 1.0) * y).sum()
    b = (x * O.apply_K(y, 0.3, 1.0, 1.0)).sum()
    assert abs(a - b) < 1e-12 * abs(a)


# ---------------------------------------------------------------- energy ----

def test_reg_energy_parseval():
    T, P, h, alpha, gamma = 3, (6, 8, 10), 0.5, 0.1, 1.3
    v = np.random.default_rng(2).normal(size=(T, 3) + P)
    R = O.reg_energy(v, alpha, gamma, h)
    Lam = gamma + alpha * O.laplacian_symbol(P, h)
    n = np.prod(P)
    spec = 0.0
    for j in range(T):
        for c in range(3):
            spec += (Lam ** 2 * np.abs(np.fft.fftn(v[j, c])) ** 2).sum()
    spec *= (1.0 / T) * h ** 3 / n
    assert abs(R - spec) < 1e-10 * R


def test_reg_energy_constant_field_closed_form():
    T, P, h, gamma = 4, (5, 6, 7), 0.3, 1.7
    c = np.array([0.2, -0.4, 0.9])
    v = np.broadcast_to(c[None, :, None, None, None], (T, 3) + P).copy()
    R = O.reg_energy(v, 0.5, gamma, h)
    assert abs(R - gamma ** 2 * (c ** 2).sum() * np.prod(P) * h ** 3) < 1e-10


# ------------------------------------------------------------------ flow ----

def test_zero_velocity_gives_identity():
    p = synth.blob_pair((8, 9, 10), 3, max_disp=1.0, center_frac=(0.3, 0.7))
    prob = O.Problem(p.M0, p.M1, p.MI0, p.MI1)
    prm = O.Params(T=4)
    J0, J1, P = O._single_level(prob)
    v = np.zeros((4, 3) + P)
    st = O.energy_terms(v, J0, J1, prm, 1.0)
    assert all(np.all(u == 0) for u in st["u0"])
    assert all(np.all(u == 0) for u in O.backward_maps(v, 1.0))
    assert st["R"] == 0.0
    np.testing.assert_allclose(st["D"], ((J0[0] - J1[0]) ** 2).sum(), rtol=1e-14)
    np.testing.assert_allclose(st["img_ssd"], ((J0[1] - J1[1]) ** 2).sum(), rtol=1e-14)


@pytest.mark.parametrize("h", [1.0, 0.05])
def test_constant_velocity_is_exact_translation(h):
    T, P = 5, (6, 7, 8)
    c = np.array([0.37, -0.81, 0.55]) * h
    v = np.broadcast_to(c[None, :, None, None, None], (T, 3) + P).copy()
    J0 = [np.random.default_rng(4).normal(size=P)]
    u0, _ = O.forward_sweep(v, J0, h, [0])
    u1 = O.backward_maps(v, h)
    np.testing.assert_allclose(u0[T], -np.broadcast_to(c[:, None, None, None], (3,) + P),
                               atol=1e-12)
    np.testing.assert_allclose(u1[0], np.broadcast_to(c[:, None, None, None], (3,) + P),
                               atol=1e-12)


def test_integer_translation_shifts_template_and_zeroes_data_term():
    T, P = 4, (10, 11, 12)
    rng = np.random.default_rng(5)
    J0 = np.zeros(P)
    J0[3:7, 3:8, 3:9] = rng.uniform(0.2, 1.0, size=(4, 5, 6))
    s = np.array([2, -1, 1])                     # (x, y, z) voxels
    v = np.broadcast_to(s[None, :, None, None, None].astype(float), (T, 3) + P).copy()
    u0, J0t = O.forward_sweep(v, [J0], 1.0, [0])
    shifted = np.zeros(P)
    # J0 o phi_10 (x) = J0(x - s)
    shifted[3 + s[2]:7 + s[2], 3 + s[1]:8 + s[1], 3 + s[0]:9 + s[0]] = J0[3:7, 3:8, 3:9]
    np.testing.assert_allclose(J0t[0][T], shifted, atol=1e-12)
    st = O.energy_terms(v, [J0], [shifted], O.Params(T=T), 1.0)
    assert st["D"] < 1e-20


def test_forward_and_backward_maps_become_inverse_as_T_grows():
    # phi_10 o phi_01 = id in the continuum; the discrete error must shrink with T
    n = 20
    P = (n, n, n)
    v1 = synth.random_velocity(P, 1, 6, vmax=2.0, sigma_s=4.0).astype(np.float64)[0]
    X = O.index_positions(P)
    errs = []
    for T in (2, 4, 8, 16):
        v = np.broadcast_to(v1, (T, 3) + P).copy()
        u0, _ = O.forward_sweep(v, [np.zeros(P)], 1.0, [])
        u1 = O.backward_maps(v, 1.0)
        # phi_10(phi_01(x)) - x = u1_0(x) + u0_T(x + u1_0(x))
        comp = u1[0] + O.sample_clamp_vec(u0[T], X + u1[0])
        inner = (slice(4, n - 4),) * 3
        errs.append(np.abs(comp[(slice(None),) + inner]).max())
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.3 * errs[0], errs


# ------------------------------------------------------------- gradients ----

def _tiny_problem(seed=7, n=8):
    p = synth.blob_pair((n, n, n), seed, max_disp=1.0, sigma=(1.2, 2.0), center_frac=(0.35, 0.65))
    return O.Problem(p.M0 * 0.8 + 0.1 * p.I0, p.M1 * 0.8 + 0.1 * p.I1, p.MI0, p.MI1)


def test_exact_gradient_matches_bruteforce_fd_on_8cubed():
    prob = _tiny_problem()
    T = 2
    prm = O.Params(T=T, alpha=0.05, weight=(1.0, 0.5))
    J0, J1, P = O._single_level(prob)
    v = _smooth_v(T, P, 8, 0.9) + 0.05 * np.random.default_rng(9).normal(size=(T, 3) + P)
    g, _, _ = O.gradient(prob, prm, v, kind="L2")
    eps = 1e-6
    fd = np.zeros_like(v)
    flat = v.reshape(-1)
    for i in range(flat.size):
        old = flat[i]
        flat[i] = old + eps
        ep = O.energy_terms(v, J0, J1, prm, 1.0)["E"]
        flat[i] = old - eps
        em = O.energy_terms(v, J0, J1, prm, 1.0)["E"]
        flat[i] = old
        fd.reshape(-1)[i] = (ep - em) / (2 * eps)
    scale = np.abs(g).max()
    assert np.abs(g - fd).max() < 2e-6 * scale


def test_exact_gradient_matches_bruteforce_fd_on_non_cubic_grid():
    p = synth.blob_pair((6, 7, 9), 7, max_disp=1.0, sigma=(1.2, 2.0), center_frac=(0.35, 0.65))
    prob = O.Problem(p.M0 * 0.8 + 0.1 * p.I0, p.M1 * 0.8 + 0.1 * p.I1)
    T = 2
    prm = O.Params(T=T, alpha=0.05)
    J0, J1, P = O._single_level(prob)
    v = synth.random_velocity(P, T, 8, vmax=0.9, sigma_s=1.5).astype(np.float64)
    v += 0.05 * np.random.default_rng(9).normal(size=(T, 3) + P)
    g, _, _ = O.gradient(prob, prm, v, kind="L2")
    eps = 1e-6
    fd = np.zeros_like(v)
    flat = v.reshape(-1)
    for i in range(flat.size):
        old = flat[i]
        flat[i] = old + eps
        ep = O.energy_terms(v, J0, J1, prm, 1.0)["E"]
        flat[i] = old - eps
        em = O.energy_terms(v, J0, J1, prm, 1.0)["E"]
        flat[i] = old
        fd.reshape(-1)[i] = (ep - em) / (2 * eps)
    assert np.abs(g - fd).max() < 2e-6 * np.abs(g).max()


@pytest.mark.parametrize("sigma", [1.0, 0.5])
def test_exact_gradient_directional_fd_physical_spacing(sigma):
    prob = _tiny_problem(11, 10)
    T = 3
    h = 0.05
    prm = O.Params(T=T, spacing=h, sigma=sigma, weight=(1.0, 0.5))
    J0, J1, P = O._single_level(prob)
    v = h * _smooth_v(T, P, 12, 1.0)
    d = h * _smooth_v(T, P, 13, 1.0)
    g, _, _ = O.gradient(prob, prm, v, kind="L2")
    eps = 1e-5
    ep = O.energy_terms(v + eps * d, J0, J1, prm, h)["E"]
    em = O.energy_terms(v - eps * d, J0, J1, prm, h)["E"]
    fd = (ep - em) / (2 * eps)
    assert abs(fd - (g * d).sum()) < 1e-5 * abs(fd)


@pytest.mark.parametrize("sigma", [1.0, 0.5])
def test_plain_gradient_is_K_of_exact_gradient_to_discretisation_error(sigma):
    # Beg's V-gradient g satisfies K^-1 g ~ dE/dv / (dt h^3) up to O(dt, h) terms:
    # compare the two as directional derivatives along smooth directions.
    p = synth.blob_pair((16, 16, 16), 14, max_disp=1.5, sigma=(2.5, 4.0), center_frac=(0.3, 0.7))
    prob = O.Problem(p.I0, p.I1)
    T = 8
    prm = O.Params(T=T, alpha=0.5, sigma=sigma, weight=(1.0, 0.0))
    J0, J1, P = O._single_level(prob)
    v = _smooth_v(T, P, 15, 0.6) * 3.0
    gV, _, _ = O.gradient(prob, prm, v, kind="V")
    gL, _, _ = O.gradient(prob, prm, v, kind="L2")
    Lam2 = (prm.gamma + prm.alpha * O.laplacian_symbol(P, 1.0)) ** 2
    KinvgV = np.stack([np.stack([np.real(np.fft.ifftn(Lam2 * np.fft.fftn(gV[j, c])))
                                 for c in range(3)]) for j in range(T)])
    dt = 1.0 / T
    ratios = []
    for s in range(3):
        d = _smooth_v(T, P, 100 + s, 1.0)
        ratios.append((dt * KinvgV * d).sum() / (gL * d).sum())
    assert all(abs(r - 1.0) < 0.15 for r in ratios), ratios


def test_plain_gradient_descends_monotonically_without_guard():
    p = synth.config_pair("blobs32")
    prob = O.Problem(p.M0, p.M1)
    prm = O.Params(T=4, iters=(6,), step=0.05, guard=False)
    res = O.register(prob, prm)
    E = np.array([r[0] for r in res.trace])
    assert np.all(np.diff(E) < 0), E


# ---------------------------------------------------------- registration ----

def test_guard_halves_and_keeps_energy_monotone():
    p = synth.config_pair("blobs32")
    prob = O.Problem(p.M0, p.M1)
    prm = O.Params(T=3, iters=(8,), step=50.0, guard=True)
    res = O.register(prob, prm)
    tr = np.array(res.trace)
    assert (tr[1:, 6] == 0).any()                      # some trial rejected
    assert np.all(np.diff(tr[:, 7]) <= 0)              # best energy never rises
    steps = tr[1:, 3]
    rej = np.where(tr[1:, 6] == 0)[0]
    for k in rej:                                      # step halves after a rejection
        if k + 1 < len(steps):
            assert steps[k + 1] == 0.5 * steps[k]


def test_resume_equals_straight_run():
    p = synth.config_pair("blobs32")
    prob = O.Problem(p.M0, p.M1, p.MI0, p.MI1)
    prm = O.Params(T=3, iters=(4,), step=0.02, spacing=0.05)
    a = O.register(prob, prm)
    b = O.register(prob, prm, v_init=a.v)
    prm8 = O.Params(T=3, iters=(8,), step=0.02, spacing=0.05)
    c = O.register(prob, prm8)
    assert np.all(np.array(c.trace)[1:, 6] == 1)
    np.testing.assert_allclose(b.v, c.v, atol=1e-12)
    np.testing.assert_allclose(b.phi10, c.phi10, atol=1e-12)


def test_nonfinite_velocity_reports_status():
    p = synth.blob_pair((8, 8, 8), 1, max_disp=1.0, center_frac=(0.3, 0.7))
    prob = O.Problem(p.M0, p.M1)
    prm = O.Params(T=2, iters=(2,))
    v = np.zeros((2, 3, 8, 8, 8))
    v[1, 0, 3, 3, 3] = np.nan
    res = O.register(prob, prm, v_init=v)
    assert res.status == O.STATUS_ENONFINITE


def test_pyramid_transfer_exact_on_linear_fields():
    Pc = (6, 8, 10)
    Pf = (12, 16, 20)
    Xf = O.index_positions(Pf)
    a = np.array([0.2, -0.3, 0.5])
    f = 1.0 + a @ Xf.reshape(3, -1)
    f = f.reshape(Pf)
    down = O.downsample2(f)
    Xc = O.index_positions(Pc)
    # block average of a linear field = its value at the block centre 2i + 1/2
    exact_c = 1.0 + a @ (2.0 * Xc + 0.5).reshape(3, -1)
    np.testing.assert_allclose(down, exact_c.reshape(Pc), atol=1e-12)
    up = O.upsample2_clamp(down, Pf)
    inner = (slice(1, Pf[0] - 1), slice(1, Pf[1] - 1), slice(1, Pf[2] - 1))
    np.testing.assert_allclose(up[inner], f[inner], atol=1e-12)


def test_apply_linear_and_nearest():
    P = (6, 7, 8)
    rng = np.random.default_rng(16)
    src = rng.normal(size=P)
    lab = rng.integers(0, 9, size=P).astype(np.int32)
    u = np.zeros((3,) + P)
    u[0] += 1.0                       # shift by one voxel along x
    out = O.apply_warp(u, src, 1.0, "linear")
    np.testing.assert_allclose(out[:, :, :-1], src[:, :, 1:], atol=1e-14)
    assert np.all(out[:, :, -1] == 0)
    out = O.apply_warp(u * 0.4, lab, 1.0, "nearest")
    np.testing.assert_array_equal(out, lab)
    out = O.apply_warp(u * 0.6, lab, 1.0, "nearest")
    np.testing.assert_array_equal(out[:, :, :-1], lab[:, :, 1:])


def test_nearest_f32_decides_ties_in_float32_and_agrees_away_from_them():
    # away from ties the FP32 decision equals the FP64 sampler; at an exact
    # half-integer both round up (floor(y + 1/2)); a displacement whose FP32
    # product lands on the half-integer rounds as float32 says
    P = (5, 6, 7)
    rng = np.random.default_rng(21)
    lab = rng.integers(1, 50, size=P).astype(np.int32)
    h = 0.3
    u = (h * rng.uniform(-2.2, 2.2, size=(3,) + P)).astype(np.float32)
    f32 = O.apply_nearest_f32(u, lab, h)
    f64 = O.apply_warp(u.astype(np.float64), lab, h, "nearest")
    frac = np.abs((u.astype(np.float64) / h + 0.5) % 1.0)
    safe = np.all((frac > 1e-5) & (frac < 1 - 1e-5), axis=0)
    assert safe.mean() > 0.99
    np.testing.assert_array_equal(f32[safe], f64[safe])
    half = np.zeros((3,) + P, np.float32)
    half[0] = 0.5                                   # h = 1: exactly half a voxel in x
    out = O.apply_nearest_f32(half, lab, 1.0)
    np.testing.assert_array_equal(out[:, :, :-1], lab[:, :, 1:])
    assert np.all(out[:, :, -1] == 0)
    # 0.15 / 0.3 in float32 is 0.49999997..., so the FP32 decision keeps the voxel
    tie = np.zeros((3,) + P, np.float32)
    tie[1] = np.float32(0.15)
    d = np.float32(0.15) * np.float32(1.0 / 0.3) + np.float32(0.5)
    out = O.apply_nearest_f32(tie, lab, 0.3)
    if np.floor(d) == 0:
        np.testing.assert_array_equal(out, lab)
    else:
        np.testing.assert_array_equal(out[:, :-1], lab[:, 1:])
