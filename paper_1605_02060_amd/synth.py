"""Seeded synthetic inputs for masked LDDMM registration.

This module only draws random numbers and evaluates closed-form test images;
it holds none of the registration arithmetic (no flow, no interpolation of
fields, no smoothing operator of the method), so that the GPU library and the
CPU oracle can both be fed from it without sharing any of the method's code.

The paper registers CLARITY volumes to the Allen mouse atlas at 25 um
(Methods, Image Acquisition / Mask Generation).  Those volumes are not
available, so every workload here is synthetic:

* template I0: a sum of Gaussian blobs (small grids) or an "atlas-like" soft
  ellipsoid modulated by blobs (atlas-sized grid);
* target I1: the same closed-form template evaluated at x + d(x), where d is a
  random smooth displacement built from a few long-wavelength plane waves
  whose analytic Lipschitz bound is kept below 1, so x -> x + d(x) is a
  diffeomorphism;
* masks M = 1[I > tau] (Methods, Mask Generation: binary threshold), optionally
  followed by ball closing/opening for sparse targets;
* the masked image channel is M * I (Methods, Preprocessing: the masks are
  applied to the images).

Arrays are float32, shaped [nz, ny, nx] (x fastest in memory).  Vector fields
are [3, nz, ny, nx] with component 0 = x, 1 = y, 2 = z.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Pair",
    "blob_params",
    "eval_blobs",
    "plane_wave_displacement",
    "blob_pair",
    "atlas_pair",
    "random_velocity",
    "random_direction",
    "plane_wave_velocity",
    "batched_dims",
    "config_pair",
]


@dataclass
class Pair:
    """One template/target problem on the user grid (all float32)."""

    I0: np.ndarray
    I1: np.ndarray
    M0: np.ndarray
    M1: np.ndarray
    MI0: np.ndarray          # M0 * I0
    MI1: np.ndarray          # M1 * I1
    d: np.ndarray            # generating displacement [3, nz, ny, nx] (voxels)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.I0.shape


def _coords(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def blob_params(rng, n_blobs=8, sigma=(2.0, 5.0), amp=(0.3, 1.0),
                center_lo=(10.0, 10.0, 10.0), center_hi=(22.0, 22.0, 22.0)):
    """Draw Gaussian blob parameters: amplitudes, widths and (x, y, z) centres."""
    a = rng.uniform(amp[0], amp[1], n_blobs)
    s = rng.uniform(sigma[0], sigma[1], n_blobs)
    c = np.stack([rng.uniform(center_lo[k], center_hi[k], n_blobs) for k in range(3)], axis=1)
    return {"a": a, "s": s, "c": c}


def eval_blobs(p, x, y, z):
    """Closed-form sum of Gaussians at positions (x, y, z) (any broadcastable arrays)."""
    out = np.zeros(np.broadcast(x, y, z).shape, dtype=np.float64)
    for a, s, c in zip(p["a"], p["s"], p["c"]):
        r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
        out += a * np.exp(-r2 / (2.0 * s * s))
    return out


def plane_wave_params(rng, shape, n_waves=6, wavelength=None):
    """Draw the waves of plane_wave_displacement: list of (k [3] in cycles per voxel
    (x, y, z), phase, amplitude [3])."""
    nz, ny, nx = shape
    ext = float(max(nx, ny, nz))
    lo, hi = wavelength if wavelength is not None else (1.5 * ext, 3.0 * ext)
    waves = []
    for _ in range(n_waves):
        lam = rng.uniform(lo, hi)
        dirv = rng.normal(size=3)
        dirv /= np.linalg.norm(dirv)
        k = dirv / lam
        ph = rng.uniform(0.0, 2.0 * math.pi)
        A = rng.normal(size=3)
        waves.append((k, ph, A))
    return waves


def plane_wave_displacement(rng, shape, max_disp, n_waves=6, wavelength=None):
    """Random smooth displacement d(x) = sum_m A_m sin(2 pi k_m . x + p_m).

    Returns (d [3, nz, ny, nx] float64, lipschitz_bound).  Wavelengths default
    to [1.5, 3] x the largest extent; the field is rescaled so that
    max_x |d(x)| == max_disp.  The returned bound on |grad d| (Frobenius) is
    analytic: sum over waves of |A_m| * 2 pi |k_m|.
    """
    waves = plane_wave_params(rng, shape, n_waves, wavelength)
    x, y, z = _coords(shape)
    d = np.zeros((3,) + tuple(shape), dtype=np.float64)
    for k, ph, A in waves:
        wave = np.sin(2.0 * math.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        for comp in range(3):
            d[comp] += A[comp] * wave
    mag = np.sqrt((d * d).sum(axis=0)).max()
    scale = max_disp / mag if mag > 0 else 0.0
    d *= scale
    lip = float(sum(np.linalg.norm(A) * scale * 2.0 * math.pi * np.linalg.norm(k)
                    for k, ph, A in waves))
    return d, lip


def _ball_dilate(mask, r):
    from scipy.ndimage import distance_transform_edt
    return distance_transform_edt(~mask) <= r


def _ball_erode(mask, r):
    from scipy.ndimage import distance_transform_edt
    return distance_transform_edt(mask) > r


def blob_pair(shape, seed, max_disp=3.0, tau=0.1, n_blobs=8, sigma=(2.0, 5.0),
              amp=(0.3, 1.0), center_frac=(10.0 / 32.0, 22.0 / 32.0)):
    """Gaussian-blob template and its smoothly warped copy (small-grid workloads).

    Centres are uniform in [center_frac[0], center_frac[1]] x extent per axis
    (10..22 on a 32 grid).
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    ext = (nx, ny, nz)
    lo = tuple(center_frac[0] * e for e in ext)
    hi = tuple(center_frac[1] * e for e in ext)
    p = blob_params(rng, n_blobs, sigma, amp, lo, hi)
    x, y, z = _coords(shape)
    I0 = eval_blobs(p, x, y, z)
    d, lip = plane_wave_displacement(rng, shape, max_disp)
    I1 = eval_blobs(p, x + d[0], y + d[1], z + d[2])
    M0 = (I0 > tau)
    M1 = (I1 > tau)
    return _finish(I0, I1, M0, M1, d, {"seed": seed, "lipschitz": lip, "kind": "blobs"})


def blob_masks_device(shape, seed, device, max_disp=3.0, tau=0.1, n_blobs=8, sigma=(2.0, 5.0),
                      amp=(0.3, 1.0), center_frac=(10.0 / 32.0, 22.0 / 32.0)):
    """The masks (M0, M1) of blob_pair(shape, seed, ...), evaluated with torch in
    float64 on `device` (same draws, same formulas); float32 [nz, ny, nx]."""
    import torch
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    ext = (nx, ny, nz)
    lo = tuple(center_frac[0] * e for e in ext)
    hi = tuple(center_frac[1] * e for e in ext)
    p = blob_params(rng, n_blobs, sigma, amp, lo, hi)
    waves = plane_wave_params(rng, shape, 6, None)
    f64 = torch.float64
    z, y, x = torch.meshgrid(torch.arange(nz, dtype=f64, device=device),
                             torch.arange(ny, dtype=f64, device=device),
                             torch.arange(nx, dtype=f64, device=device), indexing="ij")

    def blobs(x, y, z):
        out = torch.zeros(x.shape, dtype=f64, device=device)
        for a, s, c in zip(p["a"], p["s"], p["c"]):
            r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
            out += a * torch.exp(-r2 / (2.0 * s * s))
        return out

    d = torch.zeros((3,) + tuple(shape), dtype=f64, device=device)
    for k, ph, A in waves:
        wave = torch.sin(2.0 * math.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        for comp in range(3):
            d[comp] += A[comp] * wave
    mag = float(torch.sqrt((d * d).sum(dim=0)).max())
    d *= max_disp / mag if mag > 0 else 0.0
    M0 = (blobs(x, y, z) > tau).to(torch.float32)
    M1 = (blobs(x + d[0], y + d[1], z + d[2]) > tau).to(torch.float32)
    return M0.contiguous(), M1.contiguous()


def warmstart_masks_device(seed, device):
    """Masks of the warm-start workload pair `seed` (the 96^3 blob recipe x3)."""
    return blob_masks_device((96, 96, 96), seed, device, max_disp=9.0, sigma=(6.0, 15.0))


def _finish(I0, I1, M0, M1, d, meta):
    f = np.float32
    I0 = I0.astype(f)
    I1 = I1.astype(f)
    M0 = M0.astype(f)
    M1 = M1.astype(f)
    return Pair(I0=I0, I1=I1, M0=M0, M1=M1, MI0=(M0 * I0).astype(f),
                MI1=(M1 * I1).astype(f), d=d.astype(f), meta=meta)


def _atlas_intensity(p_blobs, axes, centre, x, y, z, edge=2.0):
    """Soft ellipsoid (semi-axes `axes`, ~edge-voxel boundary) x (0.4 + 0.6 * blobs)."""
    rho = np.sqrt(((x - centre[0]) / axes[0]) ** 2 + ((y - centre[1]) / axes[1]) ** 2
                  + ((z - centre[2]) / axes[2]) ** 2)
    sd = (rho - 1.0) * min(axes)
    shell = 0.5 * (1.0 - np.tanh(sd / edge))
    b = eval_blobs(p_blobs, x, y, z)
    return shell * (0.4 + 0.6 * b / p_blobs["norm"])


def atlas_pair(shape=(228, 160, 264), seed=1, max_disp=12.0, tau=0.1,
               sparse=True, close_r=5.0, open_r=2.0):
    """Atlas-like template and a sparsely labelled warped target.

    The target intensity is I1 * S with S ~ Poisson(ln(10/9)) i.i.d., so that
    90% of voxels are zero and the rest are Poisson-count spots (the sparse
    labelling of CLARITY described in the Abstract and Challenges sections).
    The target mask thresholds the sparse image at tau, closes it with a ball
    of radius close_r and then opens it with radius open_r (voxels).
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    centre = (0.5 * (nx - 1), 0.5 * (ny - 1), 0.5 * (nz - 1))
    axes = (0.42 * nx, 0.42 * ny, 0.42 * nz)
    p = blob_params(rng, 24, (4.0, 12.0), (0.3, 1.0),
                    tuple(c - a for c, a in zip(centre, axes)),
                    tuple(c + a for c, a in zip(centre, axes)))
    x, y, z = _coords(shape)
    p["norm"] = 1.0
    braw = eval_blobs(p, x, y, z)
    p["norm"] = float(braw.max())
    del braw
    I0 = _atlas_intensity(p, axes, centre, x, y, z)
    d, lip = plane_wave_displacement(rng, shape, max_disp)
    I1 = _atlas_intensity(p, axes, centre, x + d[0], y + d[1], z + d[2])
    del x, y, z
    M0 = I0 > tau
    if sparse:
        S = rng.poisson(math.log(10.0 / 9.0), size=shape).astype(np.float64)
        I1s = I1 * S
        m = I1s > tau
        m = _ball_erode(_ball_dilate(m, close_r), close_r)
        m = _ball_dilate(_ball_erode(m, open_r), open_r)
        M1 = m
        I1 = I1s
    else:
        M1 = I1 > tau
    return _finish(I0, I1, M0, M1, d, {"seed": seed, "lipschitz": lip, "kind": "atlas",
                                       "sparse": sparse})


def random_velocity(shape, T, seed, vmax=2.0, sigma_s=8.0):
    """Random smooth time-varying velocity [T, 3, nz, ny, nx] (float32).

    Each (time step, component) is independent N(0,1) noise, Gaussian-filtered
    with periodic wrap (width sigma_s voxels); the field is scaled so that
    max_x |v_j(x)| == vmax for every time step j.
    """
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    v = np.zeros((T, 3) + tuple(shape), dtype=np.float64)
    for j in range(T):
        for c in range(3):
            v[j, c] = gaussian_filter(rng.normal(size=shape), sigma_s, mode="wrap")
        mag = np.sqrt((v[j] ** 2).sum(axis=0)).max()
        v[j] *= vmax / mag
    return v.astype(np.float32)


def plane_wave_velocity(grid, seed, vmax):
    """A smooth periodic field [3, nz, ny, nx] (float64) on a computational grid:
    per component four plane waves sin(2 pi k.x/P + p) with integer k in [1, 3]^3
    and random phase, scaled so that max_x |v_c(x)| == vmax for each component."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64) / n for n in grid), indexing="ij",
                          sparse=True)
    out = np.zeros((3,) + tuple(grid), dtype=np.float64)
    for c in range(3):
        for _ in range(4):
            k = rng.integers(1, 4, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            out[c] += np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        out[c] *= vmax / np.abs(out[c]).max()
    return out


def random_direction(shape, T, seed, vmax=1.0, sigma_s=8.0):
    """A random smooth perturbation direction, same recipe as random_velocity."""
    return random_velocity(shape, T, seed, vmax=vmax, sigma_s=sigma_s)


def batched_dims(seed=4, n=16, lo=64, hi=160):
    """Uneven grid sizes for the batched workload: rows (nx, ny, nz) in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(n, 3))


def batched_pair(k, dims=None):
    """Pair k of the batched workload: the 32^3 blob recipe scaled by
    s = min(dims)/32 (blob widths 2s-5s, max displacement 3s), seed 400 + k.
    Returned arrays are [nz][ny][nx]."""
    dims = batched_dims() if dims is None else dims
    nx, ny, nz = (int(d) for d in dims[k])
    s = min(nx, ny, nz) / 32.0
    return blob_pair((nz, ny, nx), 400 + k, max_disp=3.0 * s, sigma=(2.0 * s, 5.0 * s))


def config_pair(name, seed=None):
    """Named synthetic workloads.

    * "blobs32":   32^3, 8 blobs (sigma 2-5, amp U[0.3,1]), max disp 3, seed 0.
    * "atlas":     264 x 160 x 228 (x, y, z), sparse target, max disp 12, seed 1.
    * "blobs128":  128^3, blob recipe x4 (sigma 8-20), max disp 12, seed 2.
    * "blobs96":   96^3, blob recipe x3 (sigma 6-15), max disp 9, seed 10000.
    """
    if name == "blobs32":
        return blob_pair((32, 32, 32), 0 if seed is None else seed)
    if name == "atlas":
        return atlas_pair((228, 160, 264), 1 if seed is None else seed)
    if name == "blobs128":
        return blob_pair((128, 128, 128), 2 if seed is None else seed, max_disp=12.0,
                         sigma=(8.0, 20.0))
    if name == "blobs96":
        return blob_pair((96, 96, 96), 10000 if seed is None else seed, max_disp=9.0,
                         sigma=(6.0, 15.0))
    raise KeyError(name)
