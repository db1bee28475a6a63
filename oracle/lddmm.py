"""FP64 CPU oracle for masked LDDMM -- TEST INFRASTRUCTURE ONLY.

This is a plain, slow, deliberately unfused NumPy implementation of what the
GPU library computes.  It exists so the HIP path can be checked against an
independent reading of the paper.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product path never
does, and it shares no code, tables or helpers with the HIP library.

What it follows (Kutten et al., "Deformably Registering and Annotating Whole
CLARITY Brains to an Atlas via Masked LDDMM", SPIE 9896, 2016):

* Methods, Preprocessing: in the Mask-LDDMM pipeline the images are replaced
  by their masks during registration (channel weights (1, 0) below); the
  masked image M*I is the second channel.
* Methods, Registration: the objective
      E(v) = int_0^1 ||L v_t||^2 dt + sigma^-2 ||J0 o phi_10 - J1||^2,
  with L = (-alpha Lap + gamma) I_3, gamma = sigma = 1 by convention,
  minimised by gradient descent (the scheme of Beg et al. 2005, which the
  paper cites), with v discretised in time.
* Methods, Registration: the final maps phi_10 (pulls the template into
  target space) and phi_01.
* Methods, Postprocessing / the ITK section: labels are deformed with
  nearest-neighbour interpolation.

Readings where the paper is silent (each listed in the design doc):
* flow integrated semi-Lagrangian, first order, T intervals, dt = 1/T (or
  with fourth-order Runge-Kutta departure points, the paper's integrator);
* maps stored as displacements u = phi - id in physical units;
* displacements sampled with clamped coordinates, images with zero outside;
* derivatives by the np.gradient stencil (central inside, one-sided faces);
* K = (L^dagger L)^-1 with the periodic 7-point Laplacian, applied by DFT;
* Beg's V-gradient g_j = 2 v_j - K b_j for plain descent; the exact discrete
  reverse-mode gradient for the differentiable form;
* fixed step eps with an energy guard (halve on increase, at most 10 times).

Parity status: every function below is pinned by the CPU tests
(tests/test_oracle_*.py) against library routines, closed forms, invariants
or brute force, except the whole multi-iteration trajectory of `register`,
which the paper gives no printed values for (parity unpinned beyond the
invariants: monotone energy, resume equivalence, zero/constant fields).

Array conventions: scalar fields are float64 [nz, ny, nx] (x fastest);
vector fields are [3, nz, ny, nx] with component 0 = x, 1 = y, 2 = z;
time-varying velocity is [T, 3, nz, ny, nx].  Positions passed to the
samplers are in index units, component order (x, y, z).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# numpy axis of a [nz, ny, nx] array that corresponds to vector component c
AXIS = {0: 2, 1: 1, 2: 0}

STATUS_OK = 0
STATUS_EINVAL = -1
STATUS_ENONFINITE = -3
STATUS_WFOLD = 1
STATUS_WGUARD = 2

MAX_HALVINGS = 10


# ---------------------------------------------------------------------------
# Grids
# ---------------------------------------------------------------------------

def is_7smooth(n: int) -> bool:
    for p in (2, 3, 5, 7):
        while n % p == 0 and n > 1:
            n //= p
    return n == 1


def smooth7(n: int) -> int:
    """Smallest 7-smooth integer >= n (the FFT grid size along one axis)."""
    m = max(int(n), 2)
    while not is_7smooth(m):
        m += 1
    return m


def level_grids(N, n_levels):
    """Per-level user grids, computational (FFT) grids and spacings, coarsest first.

    N is (nz, ny, nx) of the finest user grid.  The coarsest computational grid
    is the smallest 7-smooth size >= ceil(N / 2^(L-1)) per axis; each finer
    level doubles it, so the levels nest exactly (pyramid of halving
    resolutions, as in the NeuroData multiresolution hierarchy, Introduction).
    Returns a list of dicts {N, P, h} with h = 2^level (finest 1), in units of
    the finest spacing.
    """
    out = []
    L = int(n_levels)
    f = 2 ** (L - 1)
    Pc = tuple(smooth7(-(-n // f)) for n in N)
    for lev in range(L - 1, -1, -1):
        s = 2 ** lev
        out.append({"N": tuple(-(-n // s) for n in N),
                    "P": tuple(p * (f // s) for p in Pc),
                    "h": float(s)})
    return out


def pad_to(f, P):
    """Zero-pad a [nz, ny, nx] field at the high-index end to shape P."""
    out = np.zeros(P, dtype=np.float64)
    nz, ny, nx = f.shape
    out[:nz, :ny, :nx] = f
    return out


def index_positions(shape):
    """Integer grid positions as float64, component order (x, y, z)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return np.stack([x, y, z])


# ---------------------------------------------------------------------------
# Trilinear sampling (ITK's linear interpolator, Introduction/ITK section)
# ---------------------------------------------------------------------------

def _corner_weights(frac, bit):
    return frac if bit else 1.0 - frac


def sample_zero(f, pos):
    """S_zero(f; y): trilinear interpolation of f at index positions y, zero outside.

    The interpolant is the trilinear extension of the samples f[i] with
    f[i] = 0 for every index outside the grid (cell = floor(y)).
    """
    nz, ny, nx = f.shape
    n = (nx, ny, nz)
    cell = [np.floor(pos[c]).astype(np.int64) for c in range(3)]
    frac = [pos[c] - cell[c] for c in range(3)]
    out = np.zeros(pos.shape[1:], dtype=np.float64)
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                b = (bx, by, bz)
                idx = [cell[c] + b[c] for c in range(3)]
                ok = np.ones(out.shape, dtype=bool)
                for c in range(3):
                    ok &= (idx[c] >= 0) & (idx[c] < n[c])
                w = (_corner_weights(frac[0], bx) * _corner_weights(frac[1], by)
                     * _corner_weights(frac[2], bz))
                val = f[np.clip(idx[2], 0, nz - 1), np.clip(idx[1], 0, ny - 1),
                        np.clip(idx[0], 0, nx - 1)]
                out += np.where(ok, w * val, 0.0)
    return out


def _clamped_cell(y, n):
    """Clamp y to [0, n-1]; cell i = min(floor(y), n-2); fraction y - i."""
    yc = np.clip(y, 0.0, n - 1.0)
    i = np.minimum(np.floor(yc).astype(np.int64), n - 2)
    return i, yc - i, (y < 0.0) | (y > n - 1.0)


def sample_clamp(f, pos):
    """S_clamp(f; y): trilinear interpolation with coordinates clamped to the grid."""
    nz, ny, nx = f.shape
    n = (nx, ny, nz)
    cells = [_clamped_cell(pos[c], n[c]) for c in range(3)]
    out = np.zeros(pos.shape[1:], dtype=np.float64)
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                b = (bx, by, bz)
                w = np.ones(out.shape)
                for c in range(3):
                    w = w * _corner_weights(cells[c][1], b[c])
                out += w * f[cells[2][0] + bz, cells[1][0] + by, cells[0][0] + bx]
    return out


def sample_clamp_vec(u, pos):
    return np.stack([sample_clamp(u[c], pos) for c in range(3)])


def dsample_clamp(f, pos):
    """d S_clamp(f; y) / d y_b for b = x, y, z (zero along clamped coordinates).

    On cell boundaries the derivative of the cell floor(y) (right derivative)
    is used; at y = n-1 the last cell [n-2, n-1].
    """
    nz, ny, nx = f.shape
    n = (nx, ny, nz)
    cells = [_clamped_cell(pos[c], n[c]) for c in range(3)]
    out = np.zeros((3,) + pos.shape[1:], dtype=np.float64)
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                b = (bx, by, bz)
                val = f[cells[2][0] + bz, cells[1][0] + by, cells[0][0] + bx]
                for d in range(3):
                    w = np.ones(val.shape)
                    for c in range(3):
                        if c == d:
                            w = w * (1.0 if b[c] else -1.0)
                        else:
                            w = w * _corner_weights(cells[c][1], b[c])
                    out[d] += np.where(cells[d][2], 0.0, w * val)
    return out


def dsample_zero(f, pos):
    """d S_zero(f; y) / d y_b for b = x, y, z (cell floor(y), right derivative)."""
    nz, ny, nx = f.shape
    n = (nx, ny, nz)
    cell = [np.floor(pos[c]).astype(np.int64) for c in range(3)]
    frac = [pos[c] - cell[c] for c in range(3)]
    out = np.zeros((3,) + pos.shape[1:], dtype=np.float64)
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                b = (bx, by, bz)
                idx = [cell[c] + b[c] for c in range(3)]
                ok = np.ones(pos.shape[1:], dtype=bool)
                for c in range(3):
                    ok &= (idx[c] >= 0) & (idx[c] < n[c])
                val = np.where(ok, f[np.clip(idx[2], 0, nz - 1), np.clip(idx[1], 0, ny - 1),
                                     np.clip(idx[0], 0, nx - 1)], 0.0)
                for d in range(3):
                    w = np.ones(val.shape)
                    for c in range(3):
                        if c == d:
                            w = w * (1.0 if b[c] else -1.0)
                        else:
                            w = w * _corner_weights(frac[c], b[c])
                    out[d] += w * val
    return out


def splat_clamp(w, pos, shape):
    """Transpose of S_clamp: scatter w(x) to the 8 corners of the clamped cell of y(x).

    Satisfies <S_clamp(f; y), w> = <f, splat_clamp(w, y)> for every f.
    """
    nz, ny, nx = shape
    n = (nx, ny, nz)
    cells = [_clamped_cell(pos[c], n[c]) for c in range(3)]
    out = np.zeros(shape, dtype=np.float64)
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                b = (bx, by, bz)
                wt = np.ones(w.shape)
                for c in range(3):
                    wt = wt * _corner_weights(cells[c][1], b[c])
                np.add.at(out, (cells[2][0] + bz, cells[1][0] + by, cells[0][0] + bx), wt * w)
    return out


def sample_nearest(f, pos):
    """Nearest-neighbour sample f[floor(y + 1/2)], zero outside (label transfer).

    The rounding is evaluated in FP64 here.  The library takes the same decision
    in FP32 (apply_nearest_f32 below), so the two differ only where a position
    lies within FP32 rounding of a half-integer."""
    nz, ny, nx = f.shape
    n = (nx, ny, nz)
    idx = [np.floor(pos[c] + 0.5).astype(np.int64) for c in range(3)]
    ok = np.ones(pos.shape[1:], dtype=bool)
    for c in range(3):
        ok &= (idx[c] >= 0) & (idx[c] < n[c])
    val = f[np.clip(idx[2], 0, nz - 1), np.clip(idx[1], 0, ny - 1), np.clip(idx[0], 0, nx - 1)]
    return np.where(ok, val, np.zeros((), dtype=f.dtype))


# ---------------------------------------------------------------------------
# Finite differences and the operator L (Methods, Registration)
# ---------------------------------------------------------------------------

def grad_h(f, h):
    """Gradient [d/dx, d/dy, d/dz] with spacing h: central inside, one-sided at faces."""
    out = np.zeros((3,) + f.shape, dtype=np.float64)
    for c in range(3):
        ax = AXIS[c]
        g = np.zeros_like(f, dtype=np.float64)
        n = f.shape[ax]
        sl = lambda a, b: tuple(slice(a, b) if k == ax else slice(None) for k in range(3))
        g[sl(1, n - 1)] = (f[sl(2, n)] - f[sl(0, n - 2)]) / (2.0 * h)
        g[sl(0, 1)] = (f[sl(1, 2)] - f[sl(0, 1)]) / h
        g[sl(n - 1, n)] = (f[sl(n - 1, n)] - f[sl(n - 2, n - 1)]) / h
        out[c] = g
    return out


def jacobian_det(u, h):
    """det(I + D u) for a displacement field u [3, ...] with spacing h."""
    J = np.zeros((3, 3) + u.shape[1:])
    for a in range(3):
        g = grad_h(u[a], h)
        for b in range(3):
            J[a, b] = g[b] + (1.0 if a == b else 0.0)
    return (J[0, 0] * (J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1])
            - J[0, 1] * (J[1, 0] * J[2, 2] - J[1, 2] * J[2, 0])
            + J[0, 2] * (J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0]))


def lap_periodic(f, h):
    """Periodic 7-point Laplacian with spacing h."""
    out = -6.0 * f
    for ax in range(3):
        out = out + np.roll(f, 1, axis=ax) + np.roll(f, -1, axis=ax)
    return out / (h * h)


def L_op(v, alpha, gamma, h):
    """L v = (-alpha Lap + gamma) v, applied per component (Methods, Registration)."""
    return np.stack([gamma * v[c] - alpha * lap_periodic(v[c], h) for c in range(3)])


def reg_energy(v, alpha, gamma, h):
    """R = int_0^1 ||L v_t||^2 dt ~ dt * sum_j h^3 sum_x |L v_j(x)|^2."""
    T = v.shape[0]
    dt = 1.0 / T
    tot = 0.0
    for j in range(T):
        Lv = L_op(v[j], alpha, gamma, h)
        tot += (Lv * Lv).sum()
    return dt * h ** 3 * tot


def laplacian_symbol(P, h):
    """lambda(k) = sum_d (2 - 2 cos(2 pi k_d / P_d)) / h^2 on the DFT grid of shape P."""
    nz, ny, nx = P
    lz = (2.0 - 2.0 * np.cos(2.0 * math.pi * np.arange(nz) / nz)) / (h * h)
    ly = (2.0 - 2.0 * np.cos(2.0 * math.pi * np.arange(ny) / ny)) / (h * h)
    lx = (2.0 - 2.0 * np.cos(2.0 * math.pi * np.arange(nx) / nx)) / (h * h)
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


def kernel_hat(P, h, alpha, gamma):
    """Fourier symbol of K = (L^dagger L)^-1 = (gamma + alpha lambda(k))^-2."""
    return 1.0 / (gamma + alpha * laplacian_symbol(P, h)) ** 2


def apply_K(b, alpha, gamma, h):
    """K b = IDFT(K_hat * DFT(b)) per component (periodic on the computational grid)."""
    Kh = kernel_hat(b.shape[1:], h, alpha, gamma)
    return np.stack([np.real(np.fft.ifftn(Kh * np.fft.fftn(b[c]))) for c in range(3)])


# ---------------------------------------------------------------------------
# Parameters and problem
# ---------------------------------------------------------------------------

@dataclass
class Params:
    """Registration constants (Methods, Registration): L = (-alpha Lap + gamma) I3,
    data weight 1/sigma^2, T time steps; gamma = sigma = 1 by convention."""

    alpha: float = 0.02
    gamma: float = 1.0
    sigma: float = 1.0
    T: int = 10
    n_levels: int = 1
    iters: tuple = (50,)
    step: float = 0.1
    guard: bool = True
    weight: tuple = (1.0, 0.0)      # (mask channel, masked-image channel)
    spacing: float = 1.0            # h at the finest level (physical units per voxel)
    integrator: str = "euler"       # departure points: "euler" or "rk4" (the paper's)


@dataclass
class Problem:
    """Template/target channels on the user grid (pre-aligned inputs J0, J1)."""

    M0: np.ndarray
    M1: np.ndarray
    MI0: np.ndarray = None
    MI1: np.ndarray = None

    def channels(self):
        J0 = [np.asarray(self.M0, np.float64)]
        J1 = [np.asarray(self.M1, np.float64)]
        if self.MI0 is not None:
            J0.append(np.asarray(self.MI0, np.float64))
            J1.append(np.asarray(self.MI1, np.float64))
        return J0, J1


# ---------------------------------------------------------------------------
# One level: forward sweep, energy, backward sweep, gradients
# ---------------------------------------------------------------------------

def step_velocity(vj, h, dt, sign, integrator):
    """Mean velocity over one step along the characteristic of the (time-constant
    within the step) field v_j through each grid point x, followed forward
    (sign = +1) or backward (sign = -1) in time for dt.  The departure / arrival
    point is y = x + sign dt vbar / h.

    euler: vbar = v_j(x).
    rk4  : the classical fourth-order Runge-Kutta steps of dy/ds = sign v_j(y)/h,
           with v_j sampled trilinearly (clamped coordinates) between grid points:
           k1 = v_j(x), k2 = v_j(x + sign dt/2 k1/h), k3 = v_j(x + sign dt/2 k2/h),
           k4 = v_j(x + sign dt k3/h), vbar = (k1 + 2 k2 + 2 k3 + k4) / 6.
    The paper integrates the flow with fourth-order Runge-Kutta (Methods,
    Registration); the first-order step is the semi-Lagrangian default here."""
    if integrator == "euler":
        return vj
    if integrator != "rk4":
        raise ValueError(integrator)
    X = index_positions(vj.shape[1:])
    k1 = vj
    k2 = sample_clamp_vec(vj, X + sign * 0.5 * dt * k1 / h)
    k3 = sample_clamp_vec(vj, X + sign * 0.5 * dt * k2 / h)
    k4 = sample_clamp_vec(vj, X + sign * dt * k3 / h)
    return (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0


def forward_sweep(v, J0, h, weighted, integrator="euler"):
    """Flow of the inverse maps and the deformed templates.

    u0[0] = 0;  u0[j+1](x) = -dt vbar_j(x) + S_clamp(u0[j]; x - dt vbar_j(x)/h)
    (semi-Lagrangian step of d/dt phi_t0 + D phi_t0 v_t = 0; vbar_j = v_j(x) for
    the first-order step, see step_velocity), and
    J0t[c][j](x) = S_zero(J0[c]; x + u0[j](x)/h) for weighted channels c.
    Returns (u0 list of T+1 fields, J0t dict c -> list of T+1 fields).
    """
    T = v.shape[0]
    dt = 1.0 / T
    shape = v.shape[2:]
    X = index_positions(shape)
    u = np.zeros((3,) + shape)
    u0 = [u]
    J0t = {c: [J0[c].copy()] for c in weighted}
    for j in range(T):
        vbar = step_velocity(v[j], h, dt, -1.0, integrator)
        y = X - dt * vbar / h
        u = -dt * vbar + sample_clamp_vec(u, y)
        u0.append(u)
        for c in weighted:
            J0t[c].append(sample_zero(J0[c], X + u / h))
    return u0, J0t


def backward_maps(v, h, integrator="euler"):
    """u1[T] = 0;  u1[j](x) = dt vbar_j(x) + S_clamp(u1[j+1]; x + dt vbar_j(x)/h)
    (phi_{t,1} - id; vbar_j as in step_velocity, followed forward in time)."""
    T = v.shape[0]
    dt = 1.0 / T
    shape = v.shape[2:]
    X = index_positions(shape)
    u = np.zeros((3,) + shape)
    u1 = [None] * (T + 1)
    u1[T] = u
    for j in range(T - 1, -1, -1):
        vbar = step_velocity(v[j], h, dt, 1.0, integrator)
        u = dt * vbar + sample_clamp_vec(u, X + dt * vbar / h)
        u1[j] = u
    return u1


def energy_terms(v, J0, J1, prm: Params, h):
    """E = R + D with D = (h^3/sigma^2) sum_c w_c sum_x (J0c o phi_10 - J1c)^2.

    Also returns the monitored in-mask image SSD h^3 sum (MI0 o phi_10 - MI1)^2
    when the image channel exists, and the forward state for the gradient.
    """
    weighted = [c for c in range(len(J0)) if prm.weight[c] > 0]
    if not np.all(np.isfinite(v)):
        nan = float("nan")
        return {"E": nan, "R": nan, "D": nan, "img_ssd": nan, "u0": None, "J0t": None,
                "r": None, "weighted": weighted}
    u0, J0t = forward_sweep(v, J0, h, weighted, prm.integrator)
    T = v.shape[0]
    X = index_positions(v.shape[2:])
    R = reg_energy(v, prm.alpha, prm.gamma, h)
    r = {}
    D = 0.0
    for c in weighted:
        r[c] = J0t[c][T] - J1[c]
        D += prm.weight[c] * (r[c] ** 2).sum()
    D *= h ** 3 / prm.sigma ** 2
    img = float("nan")
    if len(J0) > 1:
        JI = J0t[1][T] if 1 in weighted else sample_zero(J0[1], X + u0[T] / h)
        img = h ** 3 * ((JI - J1[1]) ** 2).sum()
    return {"E": R + D, "R": R, "D": D, "img_ssd": img,
            "u0": u0, "J0t": J0t, "r": r, "weighted": weighted}


def gradient_V(v, st, prm: Params, h):
    """Beg's V-gradient g_j = 2 v_j - K b_j (plain gradient descent).

    b_j = (2/sigma^2) det(D phi_{j,1}) sum_c w_c (r_c o phi_{j,1}) grad(J0c o phi_{j,0}),
    with r_c = J0c o phi_10 - J1c back-transported by the backward map u1[j].
    Returns (g [T,3,...], min over j, x of det).
    Pinned by closed forms of b_j: a whole-voxel translation, an affine
    velocity with linear images, and v = 0 (tests/test_oracle_gradient_pins.py).
    """
    T = v.shape[0]
    X = index_positions(v.shape[2:])
    u1 = backward_maps(v, h, prm.integrator)
    g = np.zeros_like(v)
    min_det = math.inf
    for j in range(T - 1, -1, -1):
        det = jacobian_det(u1[j], h)
        min_det = min(min_det, float(det.min()))
        b = np.zeros((3,) + v.shape[2:])
        for c in st["weighted"]:
            rw = sample_zero(st["r"][c], X + u1[j] / h)
            b += prm.weight[c] * rw * grad_h(st["J0t"][c][j], h)
        b *= (2.0 / prm.sigma ** 2) * det
        g[j] = 2.0 * v[j] - apply_K(b, prm.alpha, prm.gamma, h)
    return g, min_det


def gradient_L2(v, st, prm: Params, h, J0):
    """Exact gradient dE/dv of the discrete energy (reverse mode through the sweep).

    ubar_T = (2 h^3/sigma^2) sum_c w_c r_c (1/h) grad_y S_zero(J0c; y)|_{y = x + u0_T/h};
    for j = T-1..0, with y_j = x - dt v_j/h:
        vbar_j = -dt ubar_{j+1} - (dt/h) (d_y S_clamp(u0_j; y_j))^T ubar_{j+1}
        ubar_j = S_clamp^T ubar_{j+1}   (splat)
    dE/dv_j = vbar_j + 2 dt h^3 L(L v_j).
    """
    T = v.shape[0]
    dt = 1.0 / T
    shape = v.shape[2:]
    X = index_positions(shape)
    u0 = st["u0"]
    ub = np.zeros((3,) + shape)
    yT = X + u0[T] / h
    for c in st["weighted"]:
        ub += (2.0 * h ** 3 / prm.sigma ** 2) * prm.weight[c] * st["r"][c] \
            * dsample_zero(J0[c], yT) / h
    grad = np.zeros_like(v)
    for j in range(T - 1, -1, -1):
        y = X - dt * v[j] / h
        vb = -dt * ub
        for a in range(3):
            dS = dsample_clamp(u0[j][a], y)          # d S(u0_j[a]) / d y_b
            vb -= (dt / h) * dS * ub[a]
        ub = np.stack([splat_clamp(ub[a], y, shape) for a in range(3)])
        LLv = L_op(L_op(v[j], prm.alpha, prm.gamma, h), prm.alpha, prm.gamma, h)
        grad[j] = vb + 2.0 * dt * h ** 3 * LLv
    return grad


# ---------------------------------------------------------------------------
# Pyramid transfer
# ---------------------------------------------------------------------------

def downsample2(f):
    """2x block average of a [nz, ny, nx] field (even sizes)."""
    nz, ny, nx = f.shape
    return f.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))


def upsample2_clamp(f, Pf):
    """Cell-centred 2x trilinear upsample: fine i <-> coarse (i + 0.5)/2 - 0.5, clamped."""
    X = index_positions(Pf)
    return sample_clamp(f, (X + 0.5) / 2.0 - 0.5)


# ---------------------------------------------------------------------------
# Registration loop (gradient descent with energy guard)
# ---------------------------------------------------------------------------

TRACE_COLS = ("E", "R", "D", "step", "min_det", "img_ssd", "accepted", "E_best")


@dataclass
class Result:
    v: np.ndarray
    phi10: np.ndarray
    phi01: np.ndarray
    trace: list
    status: int
    levels: list = field(default_factory=list)


def _level_loop(v, J0, J1, prm: Params, h, iters, trace):
    """Gradient descent at one level; each iteration slot is one trial step.

    slot k: if the previous trial was accepted (or k is the first slot), compute
    g at the current v and try v - eps g; otherwise (previous trial rejected)
    try the midpoint of the current v and the rejected trial, which is
    v - eps g with the halved eps.  A trial is accepted when its energy does
    not exceed the current energy (always, without the guard); on rejection
    eps is halved, and after MAX_HALVINGS consecutive rejections the level stops.
    Row 0 of the level's trace is the starting energy.
    """
    st = energy_terms(v, J0, J1, prm, h)
    if not math.isfinite(st["E"]):
        trace.append([st["E"], st["R"], st["D"], prm.step, math.nan, st["img_ssd"], 1.0, st["E"]])
        return v, st, STATUS_ENONFINITE, math.nan
    trace.append([st["E"], st["R"], st["D"], prm.step, math.nan, st["img_ssd"], 1.0, st["E"]])
    eps = prm.step
    accepted_last = True
    halvings = 0
    stopped = False
    min_det_all = math.inf
    min_det = math.nan
    trial = None
    g = None
    for _ in range(iters):
        if stopped:
            trace.append([math.nan, math.nan, math.nan, eps, min_det, math.nan, 0.0, st["E"]])
            continue
        if accepted_last:
            g, min_det = gradient_V(v, st, prm, h)
            min_det_all = min(min_det_all, min_det)
            trial = v - eps * g
        else:
            trial = 0.5 * (v + trial)
        tst = energy_terms(trial, J0, J1, prm, h)
        ok = (not prm.guard) or (tst["E"] <= st["E"])
        used = eps
        if ok:
            v, st = trial, tst
            accepted_last = True
            halvings = 0
        else:
            accepted_last = False
            eps *= 0.5
            halvings += 1
            if halvings >= MAX_HALVINGS:
                stopped = True
        trace.append([tst["E"], tst["R"], tst["D"], used, min_det, tst["img_ssd"],
                      1.0 if ok else 0.0, st["E"]])
    status = STATUS_OK
    if not math.isfinite(st["E"]):
        status = STATUS_ENONFINITE
    elif stopped:
        status = STATUS_WGUARD
    return v, st, status, min_det_all


def register(problem: Problem, prm: Params, v_init=None):
    """Masked LDDMM registration (Methods, Registration), coarse-to-fine.

    Inputs are pre-aligned template/target channels on the user grid N.
    Status: ENONFINITE, else WGUARD if a level stopped on the guard, else WFOLD
    if the returned v folds (min over j < T and the finest computational grid
    of det(I + D u1_j) <= 0), else OK.
    v_init (optional) is [T, 3, *P_finest]; for several levels it is block-
    averaged down to the coarsest level.  Returns v on the finest computational
    grid, phi10 - id = u0_T and phi01 - id = u1_0 cropped to N, the per-slot
    trace (columns TRACE_COLS; one starting row per level) and a status.
    """
    J0u, J1u = problem.channels()
    N = J0u[0].shape
    T = prm.T
    grids = level_grids(N, prm.n_levels)
    Pf = grids[-1]["P"]
    # pad the finest level, then build coarser levels by block averaging
    J0f = [pad_to(f, Pf) for f in J0u]
    J1f = [pad_to(f, Pf) for f in J1u]
    pyr0 = [J0f]
    pyr1 = [J1f]
    for _ in range(prm.n_levels - 1):
        pyr0.append([downsample2(f) for f in pyr0[-1]])
        pyr1.append([downsample2(f) for f in pyr1[-1]])
    pyr0 = pyr0[::-1]
    pyr1 = pyr1[::-1]
    if v_init is None:
        v = np.zeros((T, 3) + grids[0]["P"])
    else:
        v = np.asarray(v_init, np.float64)
        for _ in range(prm.n_levels - 1):
            v = np.stack([np.stack([downsample2(v[j, c]) for c in range(3)]) for j in range(T)])
    trace = []
    status = STATUS_OK
    for li, g in enumerate(grids):
        if li > 0:
            v = np.stack([np.stack([upsample2_clamp(v[j, c], g["P"]) for c in range(3)])
                          for j in range(T)])
        iters = prm.iters[li] if li < len(prm.iters) else prm.iters[-1]
        v, st, s, _ = _level_loop(v, pyr0[li], pyr1[li], prm, prm.spacing * g["h"], iters,
                                  trace)
        if s == STATUS_ENONFINITE:
            status = s
            break
        if s == STATUS_WGUARD:
            status = STATUS_WGUARD
    nz, ny, nx = N
    if status == STATUS_ENONFINITE or v.shape[2:] != Pf:
        nan = np.full((3, nz, ny, nx), np.nan)
        return Result(v=v, phi10=nan, phi01=nan.copy(), trace=trace, status=STATUS_ENONFINITE,
                      levels=grids)
    h = prm.spacing * grids[-1]["h"]
    st = energy_terms(v, pyr0[-1], pyr1[-1], prm, h)
    u1 = backward_maps(v, h, prm.integrator)
    phi10 = st["u0"][T][:, :nz, :ny, :nx]
    phi01 = u1[0][:, :nz, :ny, :nx]
    # a fold of the returned result: det D phi_{t_j,1} <= 0 for some j < T, anywhere
    # on the finest computational grid, for the final v
    final_det = min(float(jacobian_det(u1[j], h).min()) for j in range(T))
    if status == STATUS_OK and final_det <= 0.0:
        status = STATUS_WFOLD
    return Result(v=v, phi10=phi10, phi01=phi01, trace=trace, status=status, levels=grids)


# ---------------------------------------------------------------------------
# Single-level entry points mirroring the library calls
# ---------------------------------------------------------------------------

def _single_level(problem: Problem):
    J0u, J1u = problem.channels()
    N = J0u[0].shape
    P = tuple(smooth7(n) for n in N)
    return [pad_to(f, P) for f in J0u], [pad_to(f, P) for f in J1u], P


def energy(problem: Problem, prm: Params, v):
    """(E, R, D) of velocity v [T, 3, *P] on the padded single-level grid."""
    h = prm.spacing
    J0, J1, P = _single_level(problem)
    st = energy_terms(np.asarray(v, np.float64), J0, J1, prm, h)
    return st


def gradient(problem: Problem, prm: Params, v, kind="V"):
    """Gradient of E at v: Beg's V-gradient (kind 'V') or exact dE/dv (kind 'L2')."""
    h = prm.spacing
    J0, J1, P = _single_level(problem)
    v = np.asarray(v, np.float64)
    st = energy_terms(v, J0, J1, prm, h)
    if kind == "V":
        g, md = gradient_V(v, st, prm, h)
        return g, st, md
    if prm.integrator != "euler":
        raise ValueError("the exact gradient is defined for the first-order step only")
    return gradient_L2(v, st, prm, h, J0), st, math.nan


def apply_warp(u, src, h=1.0, interp="linear"):
    """Deform src by the map x -> x + u(x)/h: src o phi (linear, zero outside) or labels (nearest)."""
    X = index_positions(src.shape)
    pos = X + np.asarray(u, np.float64) / h
    if interp == "linear":
        return sample_zero(np.asarray(src, np.float64), pos)
    return sample_nearest(np.asarray(src), pos)


def apply_nearest_f32(u, src, h=1.0):
    """Label transfer with the rounding decided in FP32, as the library decides it
    (reading: the paper names nearest-neighbour interpolation, Methods,
    Postprocessing, but no tie rule or precision): per axis the index is
    i + floor(u * (1/h) + 1/2), every operation in float32, with 1/h rounded to
    float32 once; zero outside the grid.  An integer decided by floating point:
    both sides take the decision in the kernel's precision."""
    src = np.asarray(src)
    u = np.asarray(u, np.float32)
    inv_h = np.float32(1.0 / h)
    nz, ny, nx = src.shape
    n = (nx, ny, nz)
    X = index_positions(src.shape).astype(np.int64)
    idx = []
    for c in range(3):
        d = u[c] * inv_h + np.float32(0.5)                 # float32 multiply and add
        idx.append(X[c] + np.floor(d).astype(np.int64))
    ok = np.ones(src.shape, dtype=bool)
    for c in range(3):
        ok &= (idx[c] >= 0) & (idx[c] < n[c])
    val = src[np.clip(idx[2], 0, nz - 1), np.clip(idx[1], 0, ny - 1), np.clip(idx[0], 0, nx - 1)]
    return np.where(ok, val, np.zeros((), dtype=src.dtype))
