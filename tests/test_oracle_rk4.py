"""Pins of the fourth-order Runge-Kutta departure points (the paper's flow
integrator, Methods, Registration) in the oracle: exact translation for a
constant field, and the order of convergence against the exact flow of an
affine velocity field -- for which trilinear sampling and the semi-Lagrangian
composition are exact, so only the time integration errs."""

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import lddmm as O


def _affine_v(shape, A, c, T):
    X = O.index_positions(shape)
    v = np.einsum("ab,b...->a...", A, X - c.reshape(3, 1, 1, 1))
    return np.broadcast_to(v, (T,) + v.shape).copy(), X


def _interior(X, c, R):
    return np.linalg.norm(X - c.reshape(3, 1, 1, 1), axis=0) < R


A = np.array([[0.05, -0.9, 0.1], [0.9, 0.0, -0.2], [0.0, 0.3, -0.05]])


def _errors(T, integrator, shape=(26, 28, 30)):
    c = np.array([shape[2] / 2 - 0.3, shape[1] / 2 + 0.2, shape[0] / 2 - 0.1])
    v, X = _affine_v(shape, A, c, T)
    u0, _ = O.forward_sweep(v, [np.zeros(shape)], 1.0, [], integrator)
    u1 = O.backward_maps(v, 1.0, integrator)
    d = X - c.reshape(3, 1, 1, 1)
    exact10 = np.einsum("ab,b...->a...", expm(-A), d) - d      # phi_10 - id
    exact01 = np.einsum("ab,b...->a...", expm(A), d) - d       # phi_01 - id
    m = _interior(X, c, 5.0)
    return np.abs(u0[T] - exact10)[:, m].max(), np.abs(u1[0] - exact01)[:, m].max()


def test_constant_field_is_an_exact_translation():
    shape = (12, 13, 14)
    T = 4
    vc = np.array([0.7, -0.4, 0.25])
    v = np.broadcast_to(vc.reshape(1, 3, 1, 1, 1), (T, 3) + shape).copy()
    X = O.index_positions(shape)
    m = np.all((X > 2) & (X < np.array(shape[::-1]).reshape(3, 1, 1, 1) - 3), axis=0)
    for integ in ("euler", "rk4"):
        u0, _ = O.forward_sweep(v, [np.zeros(shape)], 1.0, [], integ)
        u1 = O.backward_maps(v, 1.0, integ)
        assert np.abs(u0[T] + vc.reshape(3, 1, 1, 1))[:, m].max() < 1e-12
        assert np.abs(u1[0] - vc.reshape(3, 1, 1, 1))[:, m].max() < 1e-12


def test_rk4_converges_fourth_order_and_euler_first():
    e4 = {T: _errors(T, "rk4") for T in (4, 8)}
    e1 = {T: _errors(T, "euler") for T in (4, 8)}
    for k in (0, 1):                                   # phi_10 and phi_01
        assert 12.0 < e4[4][k] / e4[8][k] < 20.0       # 2^4
        assert 1.6 < e1[4][k] / e1[8][k] < 2.6         # 2^1
        assert e4[4][k] < 1e-2 * e1[4][k]


def test_rk4_maps_are_near_inverse():
    # phi_01(phi_10(x)) = x up to the integration error, for a smooth nonlinear field
    shape = (20, 22, 24)
    rng = np.random.default_rng(3)
    T = 4
    X = O.index_positions(shape)
    c = np.array([12.0, 11.0, 10.0]).reshape(3, 1, 1, 1)
    g = np.exp(-((X - c) ** 2).sum(0) / (2 * 5.0 ** 2))
    v = np.stack([np.stack([a * g for a in rng.normal(size=3)]) for _ in range(T)]) * 2.0
    m = np.linalg.norm(X - c, axis=0) < 4.0
    err = {}
    for integ in ("euler", "rk4"):
        u0, _ = O.forward_sweep(v, [np.zeros(shape)], 1.0, [], integ)
        u1 = O.backward_maps(v, 1.0, integ)
        comp = O.sample_clamp_vec(u1[0], X + u0[T]) + u0[T]      # phi_01 o phi_10 - id
        err[integ] = np.abs(comp)[:, m].max()
    assert err["rk4"] < err["euler"]


def test_exact_gradient_rejects_rk4():
    shape = (6, 6, 6)
    prm = O.Params(T=2, integrator="rk4")
    prob = O.Problem(np.zeros(shape), np.zeros(shape))
    with pytest.raises(ValueError):
        O.gradient(prob, prm, np.zeros((2, 3) + shape), kind="L2")
    g, st, md = O.gradient(prob, prm, np.zeros((2, 3) + shape), kind="V")
    assert np.all(np.isfinite(g))
