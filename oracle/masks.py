"""CPU oracle of mask generation and the surface metrics -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU baseline of the benchmark may import
this module; the library never does.

Mask generation (Methods, Mask Generation): the template mask is the union of
the foreground labels; the target mask thresholds the image, opens the result
with a ball of 50 um radius (removing foreground grains) and closes it with a
ball of 125 um radius (filling holes).  Surface metrics (Methods, Evaluation):
the Hausdorff distance between the surfaces of the deformed template mask and
the target mask, and the median of all surface-to-surface distances from both
sides.  The readings taken:

* A ball of physical radius r on a grid of spacing h is the set of integer
  offsets o with (h o_x)^2 + (h o_y)^2 + (h o_z)^2 <= r^2 (an integer decision
  taken in FP64: |o|^2 <= (r/h)^2).
* Erosion keeps x when every x + o (o in the ball) is in the mask, dilation
  when some x + o is; voxels outside the grid count as background for both.
  Opening is erosion then dilation, closing dilation then erosion.
* The surface of a mask is the set of its voxels with at least one of the six
  face neighbours outside the mask (or outside the grid).
* Distances are Euclidean between voxel centres, in physical units:
  h sqrt(k) with k the integer squared index distance.  d_H is the larger of
  the two directed maxima; d_M is the median (numpy's: the mean of the two middle values for an even count) of
  the union of the distances from each surface voxel of one surface to the
  other surface, over both directions.  Either surface empty: both are NaN.

Pins (tests/test_oracle_masks.py): scipy.ndimage binary erosion / dilation /
opening / closing with the same ball and border, the algebra of openings and
closings (idempotent, anti-extensive / extensive, duality), brute-force
pairwise distances on small masks, scipy's exact Euclidean distance
transform, and closed forms for shifted cubes and identical masks.
"""

from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def ball_offsets(radius, h):
    """Integer offsets (dx, dy, dz) of the ball of physical radius `radius`."""
    q = float(radius) / float(h)
    rr = q * q
    m = int(np.floor(float(radius) / float(h))) + 1
    out = []
    for dz in range(-m, m + 1):
        for dy in range(-m, m + 1):
            for dx in range(-m, m + 1):
                if dx * dx + dy * dy + dz * dz <= rr:
                    out.append((dx, dy, dz))
    return out


def _shifted(A, o):
    """B(x) = A(x + o), background outside the grid."""
    B = np.zeros_like(A)
    dst, src = [], []
    for d, n in zip(o[::-1], A.shape):                    # (dz, nz), (dy, ny), (dx, nx)
        lo, hi = max(0, -d), min(n, n - d)                # x with 0 <= x + d < n
        if hi <= lo:
            return B                                      # shifted entirely off the grid
        dst.append(slice(lo, hi))
        src.append(slice(lo + d, hi + d))
    B[tuple(dst)] = A[tuple(src)]
    return B


def erode(A, radius, h):
    A = np.asarray(A) > 0
    out = np.ones_like(A)
    for o in ball_offsets(radius, h):
        out &= _shifted(A, o)
    return out


def dilate(A, radius, h):
    A = np.asarray(A) > 0
    out = np.zeros_like(A)
    for o in ball_offsets(radius, h):
        out |= _shifted(A, o)
    return out


def opening(A, radius, h):
    return dilate(erode(A, radius, h), radius, h)


def closing(A, radius, h):
    return erode(dilate(A, radius, h), radius, h)


def target_mask(I, tau, open_radius, close_radius, h):
    """M1 = close(open(1[I > tau]))."""
    return closing(opening(np.asarray(I) > tau, open_radius, h), close_radius, h)


def label_mask(L):
    """M0 = union of the foreground labels (label != 0)."""
    return np.asarray(L) != 0


def surface(A):
    """Mask voxels with a face neighbour outside the mask or the grid."""
    A = np.asarray(A) > 0
    inner = A.copy()
    for o in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        inner &= _shifted(A, o)
    return A & ~inner


def _index_points(S):
    z, y, x = np.nonzero(S)
    return np.stack([x, y, z], axis=1).astype(np.float64)


def directed_distances(Sa, Sb, h):
    """For every voxel of surface Sa, the distance to the nearest voxel of Sb:
    h sqrt(k), k the (integer) squared index distance, so the square root is of
    an exact integer."""
    d, _ = cKDTree(_index_points(Sb)).query(_index_points(Sa))
    return float(h) * d


def surface_distances(A, B, h):
    """(d_H, d_M, |S_A|, |S_B|) of the masks A and B."""
    Sa, Sb = surface(A), surface(B)
    na, nb = int(Sa.sum()), int(Sb.sum())
    if na == 0 or nb == 0:
        return float("nan"), float("nan"), na, nb
    dab = directed_distances(Sa, Sb, h)
    dba = directed_distances(Sb, Sa, h)
    alld = np.concatenate([dab, dba])
    return float(max(dab.max(), dba.max())), float(np.median(alld)), na, nb
