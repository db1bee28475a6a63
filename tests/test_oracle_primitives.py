"""Pins of the oracle's primitives against library routines, closed forms and
brute force (CPU only).  These are what make the oracle trustworthy: each
check would fail under a plausible slip (a swapped axis, a dropped term, a
wrong sign or boundary rule)."""

import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import lddmm as O


def _rand_field(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def _positions(shape, seed, lo=-2.0, hi_pad=2.0):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    n = 500
    pos = np.stack([rng.uniform(lo, nx - 1 + hi_pad, n), rng.uniform(lo, ny - 1 + hi_pad, n),
                    rng.uniform(lo, nz - 1 + hi_pad, n)])
    return pos


def _scipy_coords(pos):
    # map_coordinates wants (axis0, axis1, axis2) = (z, y, x)
    return np.stack([pos[2], pos[1], pos[0]])


@pytest.mark.parametrize("shape", [(5, 6, 7), (4, 9, 3)])
def test_sample_zero_matches_map_coordinates(shape):
    f = _rand_field(shape, 1)
    pos = _positions(shape, 2)
    ref = ndimage.map_coordinates(f, _scipy_coords(pos), order=1, mode="grid-constant", cval=0.0)
    np.testing.assert_allclose(O.sample_zero(f, pos), ref, atol=1e-12)


@pytest.mark.parametrize("shape", [(5, 6, 7), (4, 9, 3)])
def test_sample_clamp_matches_map_coordinates(shape):
    f = _rand_field(shape, 3)
    pos = _positions(shape, 4)
    ref = ndimage.map_coordinates(f, _scipy_coords(pos), order=1, mode="nearest")
    np.testing.assert_allclose(O.sample_clamp(f, pos), ref, atol=1e-12)


def test_sample_zero_half_cell_outside():
    # zero outside: half a cell beyond the first/last sample gives half the edge value
    f = np.zeros((3, 3, 4))
    f[1, 1, 0] = 2.0
    f[1, 1, 3] = 4.0
    pos = np.array([[-0.5, 3.5], [1.0, 1.0], [1.0, 1.0]])
    np.testing.assert_allclose(O.sample_zero(f, pos), [1.0, 2.0], atol=1e-15)


def test_samplers_reproduce_linear_field_in_interior():
    shape = (6, 7, 8)
    X = O.index_positions(shape)
    a = np.array([0.3, -1.2, 0.7])
    f = 2.0 + a[0] * X[0] + a[1] * X[1] + a[2] * X[2]
    rng = np.random.default_rng(5)
    pos = np.stack([rng.uniform(0, 7, 300), rng.uniform(0, 6, 300), rng.uniform(0, 5, 300)])
    exact = 2.0 + a @ pos
    np.testing.assert_allclose(O.sample_zero(f, pos), exact, atol=1e-12)
    np.testing.assert_allclose(O.sample_clamp(f, pos), exact, atol=1e-12)


def test_sample_nearest_matches_map_coordinates_off_ties():
    shape = (5, 6, 7)
    f = np.random.default_rng(6).integers(0, 50, size=shape).astype(np.int32)
    pos = _positions(shape, 7, lo=-1.3, hi_pad=1.3)
    # keep away from exact .5 ties, where rounding conventions may differ
    frac = pos - np.floor(pos)
    keep = np.all(np.abs(frac - 0.5) > 1e-3, axis=0)
    pos = pos[:, keep]
    ref = ndimage.map_coordinates(f.astype(np.float64), _scipy_coords(pos), order=0,
                                  mode="grid-constant", cval=0.0)
    np.testing.assert_array_equal(O.sample_nearest(f, pos), ref.astype(np.int32))


def test_sample_nearest_ties_round_up():
    f = np.arange(4 * 4 * 4, dtype=np.int32).reshape(4, 4, 4)
    pos = np.array([[0.5, 1.5, -0.5], [0.0, 2.0, 0.0], [1.0, 1.0, 1.0]])
    out = O.sample_nearest(f, pos)
    assert out[0] == f[1, 0, 1] and out[1] == f[1, 2, 2] and out[2] == f[1, 0, 0]


@pytest.mark.parametrize("which", ["zero", "clamp"])
def test_sampler_derivatives_match_central_differences(which):
    shape = (5, 6, 7)
    f = _rand_field(shape, 8)
    pos = _positions(shape, 9, lo=-0.9 if which == "zero" else 0.05, hi_pad=0.9 if which == "zero" else -0.05)
    # avoid cell boundaries where the interpolant has kinks
    frac = pos - np.floor(pos)
    keep = np.all((frac > 1e-3) & (frac < 1 - 1e-3), axis=0)
    pos = pos[:, keep]
    S = O.sample_zero if which == "zero" else O.sample_clamp
    dS = O.dsample_zero if which == "zero" else O.dsample_clamp
    got = dS(f, pos)
    eps = 1e-6
    for b in range(3):
        e = np.zeros((3, 1))
        e[b] = eps
        fd = (S(f, pos + e) - S(f, pos - e)) / (2 * eps)
        np.testing.assert_allclose(got[b], fd, atol=1e-7)


def test_dsample_clamp_zero_where_clamped():
    f = _rand_field((4, 4, 4), 10)
    pos = np.array([[-0.7, 1.2], [1.3, 5.0], [2.2, 1.4]])
    d = O.dsample_clamp(f, pos)
    assert d[0, 0] == 0.0 and d[1, 1] == 0.0
    assert d[1, 0] != 0.0 and d[0, 1] != 0.0


def test_splat_is_adjoint_of_clamped_sampling():
    shape = (5, 6, 7)
    rng = np.random.default_rng(11)
    f = rng.normal(size=shape)
    w = rng.normal(size=shape)
    X = O.index_positions(shape)
    pos = X + rng.uniform(-1.5, 1.5, size=(3,) + shape)
    lhs = (O.sample_clamp(f, pos) * w).sum()
    rhs = (f * O.splat_clamp(w, pos, shape)).sum()
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_splat_equals_transpose_of_dense_sampling_matrix():
    # build W column by column from the sampler's definition on a 4^3 grid
    shape = (4, 4, 4)
    n = 64
    rng = np.random.default_rng(12)
    X = O.index_positions(shape)
    pos = X + rng.uniform(-1.2, 1.2, size=(3,) + shape)
    W = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        W[:, i] = O.sample_clamp(e.reshape(shape), pos).ravel()
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        np.testing.assert_allclose(O.splat_clamp(e.reshape(shape), pos, shape).ravel(), W[i],
                                   atol=1e-14)


@pytest.mark.parametrize("h", [1.0, 0.05])
def test_grad_matches_numpy_gradient(h):
    f = _rand_field((5, 6, 7), 13)
    g = O.grad_h(f, h)
    gz, gy, gx = np.gradient(f, h)
    np.testing.assert_allclose(g[0], gx, atol=1e-12)
    np.testing.assert_allclose(g[1], gy, atol=1e-12)
    np.testing.assert_allclose(g[2], gz, atol=1e-12)


def test_jacobian_of_affine_displacement_is_exact_everywhere():
    shape = (5, 6, 7)
    h = 0.5
    A = np.array([[0.1, -0.2, 0.05], [0.3, 0.02, -0.1], [-0.04, 0.15, 0.2]])
    X = O.index_positions(shape) * h          # physical positions
    u = np.einsum("ab,b...->a...", A, X) + np.array([0.3, -0.1, 0.2])[:, None, None, None]
    det = O.jacobian_det(u, h)
    np.testing.assert_allclose(det, np.linalg.det(np.eye(3) + A), atol=1e-12)


def test_periodic_laplacian_eigenvalue():
    P = (8, 10, 12)
    h = 0.7
    X = O.index_positions(P)
    k = (3, 2, 1)        # (kx, ky, kz)
    f = np.cos(2 * math.pi * (k[0] * X[0] / P[2] + k[1] * X[1] / P[1] + k[2] * X[2] / P[0]))
    lam = sum((2 - 2 * math.cos(2 * math.pi * k[c] / P[2 - c])) for c in range(3)) / h ** 2
    np.testing.assert_allclose(O.lap_periodic(f, h), -lam * f, atol=1e-12)


def test_smooth7_sizes():
    assert O.smooth7(32) == 32
    assert O.smooth7(264) == 270
    assert [O.smooth7(n) for n in (11, 13, 17, 19, 23, 29, 31)] == [12, 14, 18, 20, 24, 30, 32]
    g = O.level_grids((228, 160, 264), 3)
    assert [x["P"] for x in g] == [(60, 40, 70), (120, 80, 140), (240, 160, 280)]
    assert [x["h"] for x in g] == [4.0, 2.0, 1.0]
