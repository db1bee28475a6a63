"""Closed-form pins of the oracle's plain (V-) gradient and of the data term's
factors (CPU only).

The V-gradient of Beg et al. 2005, which the paper cites for its gradient
descent (Methods, Registration), is

    g_j = 2 v_j - K b_j,
    b_j(x) = (2/sigma^2) det(D phi_{j,1}(x)) sum_c w_c r_c(phi_{j,1}(x)) grad(J0c o phi_{j,0})(x),

with r_c = J0c o phi_10 - J1c.  Each pin below evaluates b_j for a flow whose
maps are known in closed form and compares it with the oracle's g through
b_j = L L (2 v_j - g_j): K is exactly (L^dagger L)^-1 for the periodic stencil
(pinned elsewhere), so applying the stencil operator twice undoes it without
any FFT.  The stencil here is written with np.roll, and shifts and gradients
come from np.roll and np.gradient, so nothing is taken from the oracle.

* constant integer translation: the maps are whole-voxel shifts, so the
  deformed template and the back-transported residual are np.roll shifts.
  This fixes the direction of the back-transport and the time index of the
  deformed template.
* affine velocity v(x) = A (x - c): inside the grid every map is affine,
  phi_{j,1} - c = (I + dt A)^(T-j) (x - c) and phi_{j,0} - c = (I - dt A)^j (x - c).
  With linear J0, J1 the whole b_j is a closed form, and det D phi_{j,1} =
  det(I + dt A)^(T-j).  This fixes which map the Jacobian is taken of, its
  power, and that it enters b at all.
* v = 0: b = (2/sigma^2) sum_c w_c (J0c - J1c) grad J0c.
* the data term of a Gaussian residual is the Riemann sum of its square,
  D -> sigma^-2 integral (J0 - J1)^2 = sigma^-2 pi^(3/2) s^3, which fixes the
  h^3 volume element and the 1/sigma^2 weight.

Every pin runs with sigma != 1 and h != 1.  `test_planted_mistakes_fail_a_pin`
plants plausible mistakes in a copy of the oracle's source and checks that
each one fails at least one pin.
"""

import importlib.util
import math
import os
import sys
import types

import numpy as np
import pytest

from oracle import lddmm as O

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "lddmm.py")


# ------------------------------------------------------------------ tools ----

def _lap(f, h):
    """Periodic 7-point Laplacian on a [nz, ny, nx] array (np.roll)."""
    out = -6.0 * f
    for ax in range(3):
        out = out + np.roll(f, 1, ax) + np.roll(f, -1, ax)
    return out / (h * h)


def _LL(w, alpha, gamma, h):
    """(gamma - alpha Lap)^2 w per component: undoes K = (L^dagger L)^-1."""
    def L(f):
        return gamma * f - alpha * _lap(f, h)
    return np.stack([L(L(w[c])) for c in range(3)])


def _body_force_from_gradient(v, g, alpha, gamma, h):
    """b_j recovered from g_j = 2 v_j - K b_j."""
    return np.stack([_LL(2.0 * v[j] - g[j], alpha, gamma, h) for j in range(v.shape[0])])


def _grad(f, h):
    """np.gradient as [d/dx, d/dy, d/dz] of a [nz, ny, nx] field."""
    gz, gy, gx = np.gradient(f, h)
    return np.stack([gx, gy, gz])


def _shift(f, s):
    """f(x - s) for an integer (x, y, z) shift s; f must vanish near the faces."""
    return np.roll(f, (int(s[2]), int(s[1]), int(s[0])), axis=(0, 1, 2))


def _blob(P, centre, s):
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64) for n in P), indexing="ij")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return np.exp(-r2 / (2.0 * s * s))


def _gradient_V(Om, J0, J1, v, prm):
    h = prm.spacing
    st = Om.energy_terms(v, J0, J1, prm, h)
    g, md = Om.gradient_V(v, st, prm, h)
    return g, md, st


# ------------------------------------------------------------------- pins ----

def pin_translation(Om):
    """Constant v = c with dt c a whole number of voxels per step (T = 2, c = 2).

    phi_{j,0}(x) = x - j dt c, phi_{j,1}(x) = x + (T - j) dt c, det = 1, so
    b_j = (2/sigma^2) sum_c w_c r_c(x + (T-j) dt c) grad J0c(x - j dt c)."""
    T, h, sigma, alpha, gamma = 2, 0.5, 0.5, 0.3, 1.0
    w = (1.0, 0.5)
    P = (26, 28, 30)
    cvox = np.array([2, -2, 2])                   # voxels per unit time, (x, y, z)
    J0 = [_blob(P, (14.0, 14.5, 12.5), 1.4), 0.7 * _blob(P, (16.0, 13.0, 13.5), 1.2)]
    J1 = [_blob(P, (15.5, 13.0, 13.0), 1.3), 0.4 * _blob(P, (13.5, 15.0, 12.0), 1.1)]
    # the supports must stay clear of the faces for np.roll to be a zero-filled shift
    for f in J0 + J1:
        assert max(np.abs(f[:3]).max(), np.abs(f[-3:]).max(), np.abs(f[:, :3]).max(),
                   np.abs(f[:, -3:]).max(), np.abs(f[:, :, :3]).max(),
                   np.abs(f[:, :, -3:]).max()) < 1e-11
    prm = Om.Params(T=T, alpha=alpha, gamma=gamma, sigma=sigma, weight=w, spacing=h)
    v = np.broadcast_to((h * cvox)[None, :, None, None, None].astype(np.float64),
                        (T, 3) + P).copy()
    g, md, st = _gradient_V(Om, J0, J1, v, prm)
    b = _body_force_from_gradient(v, g, alpha, gamma, h)
    dt = 1.0 / T
    r = [_shift(J0[c], T * dt * cvox) - J1[c] for c in range(2)]
    scale = 0.0
    for j in range(T):
        s_j = (j * dt * cvox).astype(int)             # phi_{j,0}(x) = x - s_j
        t_j = ((T - j) * dt * cvox).astype(int)       # phi_{j,1}(x) = x + t_j
        exp = np.zeros((3,) + P)
        for c in range(2):
            exp += w[c] * _shift(r[c], -t_j) * _grad(_shift(J0[c], s_j), h)
        exp *= 2.0 / sigma ** 2
        scale = max(scale, np.abs(exp).max())
        assert np.abs(b[j] - exp).max() < 1e-9 * np.abs(exp).max(), j
    assert scale > 0.1
    assert abs(md - 1.0) < 1e-12


def pin_affine(Om):
    """Affine v(x) = A (x - c), linear J0 and J1: b_j in closed form inside the grid."""
    T, h, sigma, alpha, gamma = 3, 0.5, 0.5, 0.2, 1.0
    P = (22, 24, 26)
    c = np.array([12.5, 11.5, 10.5])               # (x, y, z) index units
    A = np.array([[0.10, 0.04, -0.03],
                  [-0.05, 0.14, 0.02],
                  [0.03, -0.02, 0.08]])             # per unit time, index units
    a = np.array([0.3, -0.2, 0.25])
    bb = np.array([0.1, 0.35, -0.15])
    a0, b0 = 1.0, 0.6
    X = np.stack(np.meshgrid(*(np.arange(n, dtype=np.float64) for n in P),
                             indexing="ij")[::-1])  # (x, y, z) positions
    Xc = X - c[:, None, None, None]
    J0 = [a0 + np.einsum("d,d...->...", a, Xc)]
    J1 = [b0 + np.einsum("d,d...->...", bb, Xc)]
    v1 = h * np.einsum("de,e...->d...", A, Xc)       # physical velocity
    v = np.broadcast_to(v1, (T, 3) + P).copy()
    prm = Om.Params(T=T, alpha=alpha, gamma=gamma, sigma=sigma, weight=(1.0, 0.0), spacing=h)
    g, _, st = _gradient_V(Om, J0, J1, v, prm)
    b = _body_force_from_gradient(v, g, alpha, gamma, h)
    dt = 1.0 / T
    Mp = np.eye(3) + dt * A                            # one backward step
    Mm = np.eye(3) - dt * A                            # one forward step
    MmT = np.linalg.matrix_power(Mm, T)
    inner = (slice(7, P[0] - 7), slice(7, P[1] - 7), slice(7, P[2] - 7))
    for j in range(T):
        F1 = np.linalg.matrix_power(Mp, T - j)        # D phi_{j,1}
        F0 = np.linalg.matrix_power(Mm, j)            # D phi_{j,0}
        y = np.einsum("de,e...->d...", F1, Xc)        # phi_{j,1}(x) - c
        # r(y) = J0(phi_10(y)) - J1(y), phi_10(y) - c = (I - dt A)^T (y - c)
        r_at = a0 + np.einsum("d,d...->...", MmT.T @ a, y) - b0 - np.einsum("d,d...->...", bb, y)
        gJ = (F0.T @ a) / h                            # grad (J0 o phi_{j,0}), physical
        exp = (2.0 / sigma ** 2) * np.linalg.det(F1) * r_at[None] * gJ[:, None, None, None]
        got = b[j][(slice(None),) + inner]
        ref = exp[(slice(None),) + inner]
        assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max(), j


def pin_zero_velocity(Om):
    """v = 0: g = -K[(2/sigma^2) sum_c w_c (J0c - J1c) grad J0c]."""
    T, h, sigma, alpha, gamma = 3, 0.05, 0.5, 0.02, 1.0
    w = (1.0, 0.5)
    P = (12, 14, 16)
    rng = np.random.default_rng(3)
    J0 = [rng.uniform(0, 1, P), rng.uniform(0, 1, P)]
    J1 = [rng.uniform(0, 1, P), rng.uniform(0, 1, P)]
    prm = Om.Params(T=T, alpha=alpha, gamma=gamma, sigma=sigma, weight=w, spacing=h)
    v = np.zeros((T, 3) + P)
    g, md, _ = _gradient_V(Om, J0, J1, v, prm)
    b = _body_force_from_gradient(v, g, alpha, gamma, h)
    exp = sum(w[c] * (J0[c] - J1[c]) * _grad(J0[c], h) for c in range(2)) * (2.0 / sigma ** 2)
    for j in range(T):
        assert np.abs(b[j] - exp).max() < 1e-9 * np.abs(exp).max(), j
    assert md == 1.0


def pin_data_term_integral(Om):
    """D of a Gaussian residual at v = 0 is sigma^-2 times the integral of its square.

    J0 - J1 = exp(-|x - c|^2 / (2 s^2)) sampled at spacing h;
    its square integrates to pi^(3/2) s^3; at s = 5 voxels, 4.7 s from the faces,
    the Riemann sum and the cut tails differ from it by far less than 1e-9."""
    for h, sigma in ((0.05, 0.5), (0.2, 2.0)):
        P = (48, 48, 48)
        s = 5.0 * h
        J1 = np.full(P, 0.25)
        J0 = J1 + _blob(P, (23.5, 23.5, 23.5), 5.0)
        prm = Om.Params(T=2, sigma=sigma, weight=(1.0, 0.0), spacing=h)
        st = Om.energy_terms(np.zeros((2, 3) + P), [J0], [J1], prm, h)
        exact = math.pi ** 1.5 * s ** 3 / sigma ** 2
        assert abs(st["D"] - exact) < 1e-9 * exact, (h, sigma, st["D"], exact)
        assert st["R"] == 0.0


PINS = [pin_translation, pin_affine, pin_zero_velocity, pin_data_term_integral]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_oracle_passes_pin(pin):
    pin(O)


# ----------------------------------------------------- planted mistakes ----

# (name, text in oracle/lddmm.py, planted replacement).  Each must occur once.
MUTANTS = [
    ("det dropped from b", "b *= (2.0 / prm.sigma ** 2) * det", "b *= (2.0 / prm.sigma ** 2)"),
    ("template at t_{j+1}", 'grad_h(st["J0t"][c][j], h)', 'grad_h(st["J0t"][c][j + 1], h)'),
    ("residual pulled back the wrong way", 'X + u1[j] / h)', 'X - u1[j] / h)'),
    ("Jacobian of the forward map", "det = jacobian_det(u1[j], h)",
     'det = jacobian_det(st["u0"][j], h)'),
    ("data term over sigma", "D *= h ** 3 / prm.sigma ** 2", "D *= h ** 3 / prm.sigma"),
    ("data term without the volume element", "D *= h ** 3 / prm.sigma ** 2",
     "D *= h ** 2 / prm.sigma ** 2"),
    ("body force over sigma^2 without the 2", "b *= (2.0 / prm.sigma ** 2) * det",
     "b *= (1.0 / prm.sigma ** 2) * det"),
    ("residual sign", "r[c] = J0t[c][T] - J1[c]", "r[c] = J1[c] - J0t[c][T]"),
    ("gradient without the factor 2 on v", "g[j] = 2.0 * v[j] - apply_K", "g[j] = v[j] - apply_K"),
    ("template undeformed in b", 'grad_h(st["J0t"][c][j], h)', 'grad_h(st["J0t"][c][0], h)'),
]


def _load_mutant(old, new, tag):
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    name = f"_oracle_mutant_{tag}"
    mod = types.ModuleType(name)
    mod.__file__ = ORACLE_SRC
    sys.modules[name] = mod                  # dataclasses look the module up by name
    try:
        exec(compile(src.replace(old, new), ORACLE_SRC, "exec"), mod.__dict__)
    except Exception:
        del sys.modules[name]
        raise
    return mod


@pytest.mark.parametrize("k", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_planted_mistakes_fail_a_pin(k):
    name, old, new = MUTANTS[k]
    mod = _load_mutant(old, new, k)
    try:
        caught = []
        for pin in PINS:
            try:
                pin(mod)
            except AssertionError:
                caught.append(pin.__name__)
        assert caught, f"planted mistake '{name}' passes every pin"
    finally:
        del sys.modules[mod.__name__]
