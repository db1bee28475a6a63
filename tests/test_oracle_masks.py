"""Pins of the mask-generation and surface-metric oracle (Methods, Mask
Generation; Evaluation): scipy.ndimage's binary morphology and exact distance
transform, the algebra of openings and closings, brute-force distances and
closed forms."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import masks as K


def _ball_structure(radius, h):
    offs = np.array(K.ball_offsets(radius, h))
    m = np.abs(offs).max()
    st = np.zeros((2 * m + 1,) * 3, dtype=bool)
    st[offs[:, 2] + m, offs[:, 1] + m, offs[:, 0] + m] = True
    return st


def _blobs(shape, seed, p=0.55, smooth=2.0):
    rng = np.random.default_rng(seed)
    return ndimage.gaussian_filter(rng.normal(size=shape), smooth) > np.quantile(
        ndimage.gaussian_filter(rng.normal(size=shape), smooth), p)


def test_ball_offsets():
    assert K.ball_offsets(0.5, 1.0) == [(0, 0, 0)]
    assert len(K.ball_offsets(1.0, 1.0)) == 7                        # the 6-neighbourhood
    assert len(K.ball_offsets(np.sqrt(2.0), 1.0)) == 19
    assert len(K.ball_offsets(2.0, 1.0)) == 33
    assert len(K.ball_offsets(0.125, 0.025)) == len(K.ball_offsets(5.0, 1.0)) == 515
    for o in K.ball_offsets(3.3, 1.1):
        assert sum(c * c for c in o) * 1.21 <= 3.3 ** 2 + 1e-12


@pytest.mark.parametrize("shape,radius,h", [((23, 26, 29), 1.0, 1.0), ((23, 26, 29), 2.5, 1.0),
                                            ((23, 26, 29), 0.125, 0.025),
                                            ((23, 26, 29), 0.05, 0.025),
                                            ((3, 4, 9), 4.0, 1.0), ((6, 5, 40), 9.0, 1.0)])
def test_morphology_matches_scipy(shape, radius, h):
    # the last two balls are longer than some axes of the grid
    A = _blobs(shape, 3, smooth=1.0)
    st = _ball_structure(radius, h)
    np.testing.assert_array_equal(K.erode(A, radius, h),
                                  ndimage.binary_erosion(A, st, border_value=0))
    np.testing.assert_array_equal(K.dilate(A, radius, h),
                                  ndimage.binary_dilation(A, st, border_value=0))
    np.testing.assert_array_equal(K.opening(A, radius, h),
                                  ndimage.binary_dilation(ndimage.binary_erosion(
                                      A, st, border_value=0), st, border_value=0))
    np.testing.assert_array_equal(K.closing(A, radius, h),
                                  ndimage.binary_erosion(ndimage.binary_dilation(
                                      A, st, border_value=0), st, border_value=0))


def test_opening_and_closing_algebra():
    A = _blobs((20, 21, 22), 4)
    r, h = 2.0, 1.0
    O, C = K.opening(A, r, h), K.closing(A, r, h)
    assert np.all(O <= A)                                             # anti-extensive
    np.testing.assert_array_equal(K.opening(O, r, h), O)              # idempotent
    # duality away from the border: erode(A) = not dilate(not A)
    core = (slice(3, -3),) * 3
    np.testing.assert_array_equal(K.erode(A, r, h)[core], ~K.dilate(~A, r, h)[core])
    # closing is extensive away from the border (outside the grid is background)
    inner = np.zeros_like(A)
    inner[3:-3, 3:-3, 3:-3] = True
    assert np.all((A & inner) <= C)
    np.testing.assert_array_equal(K.closing(C, r, h), C)


def test_target_mask_removes_grains_and_fills_holes():
    shape = (40, 40, 40)
    z, y, x = np.mgrid[:40, :40, :40]
    brain = (x - 20) ** 2 / 15 ** 2 + (y - 20) ** 2 / 13 ** 2 + (z - 20) ** 2 / 12 ** 2 <= 1
    I = np.where(brain, 1.0, 0.0)
    I[20, 20, 20] = 0.0                                   # a one-voxel hole
    I[2, 3, 4] = 1.0                                      # a foreground grain
    # a cluster of single-voxel grains 2 voxels apart: opening first removes
    # them; closing first would fuse them into a blob that survives the opening
    I[29:38:2, 29:38:2, 29:38:2] = 1.0
    I[28:40, 28:40, 28:40] *= ~brain[28:40, 28:40, 28:40]
    M = K.target_mask(I, 0.5, 0.05, 0.125, 0.025)         # paper's radii at 25 um
    assert M[20, 20, 20] and not M[2, 3, 4]
    assert not M[28:40, 28:40, 28:40].any()
    assert K.closing(I > 0.5, 0.125, 0.025)[33, 33, 33]   # the cluster closes into a blob
    assert abs(int(M.sum()) - int(brain.sum())) < 0.02 * brain.sum()


def test_label_mask_and_surface():
    L = np.zeros((5, 6, 7), np.int32)
    L[1:4, 1:5, 1:6] = 3
    L[2, 2, 2] = 7
    np.testing.assert_array_equal(K.label_mask(L), L != 0)
    S = K.surface(L != 0)
    assert S.sum() == 3 * 4 * 5 - 1 * 2 * 3                    # the box minus its interior
    full = np.ones((3, 4, 5), bool)
    assert K.surface(full).sum() == full.size - 1 * 2 * 3        # the grid's edge is a surface


def test_distances_match_brute_force_and_edt():
    A, B = _blobs((14, 15, 16), 5), _blobs((14, 15, 16), 6)
    h = 0.05
    Sa, Sb = K.surface(A), K.surface(B)
    pa = np.argwhere(Sa)[:, ::-1].astype(np.float64)
    pb = np.argwhere(Sb)[:, ::-1].astype(np.float64)
    brute = h * np.sqrt(((pa[:, None, :] - pb[None, :, :]) ** 2).sum(-1)).min(axis=1)
    np.testing.assert_allclose(K.directed_distances(Sa, Sb, h), brute, rtol=1e-15)
    edt = ndimage.distance_transform_edt(~Sb, sampling=h)
    np.testing.assert_allclose(K.directed_distances(Sa, Sb, h), edt[Sa], rtol=1e-12)
    dH, dM, na, nb = K.surface_distances(A, B, h)
    both = np.concatenate([brute, h * np.sqrt(((pb[:, None, :] - pa[None, :, :]) ** 2).sum(-1))
                           .min(axis=1)])
    assert dH == both.max() and dM == np.median(both) and (na, nb) == (len(pa), len(pb))


def test_closed_forms():
    # a cube against the same cube shifted by 3 voxels along x: every surface
    # voxel of the faces normal to x is 3 away, d_H = 3 h
    A = np.zeros((20, 20, 30), bool)
    A[5:15, 5:15, 5:15] = True
    B = np.roll(A, 3, axis=2)
    dH, dM, _, _ = K.surface_distances(A, B, 0.5)
    assert dH == 1.5
    # identical masks: all distances 0
    assert K.surface_distances(A, A, 0.5)[:2] == (0.0, 0.0)
    # empty surface
    dH, dM, na, nb = K.surface_distances(A, np.zeros_like(A), 1.0)
    assert np.isnan(dH) and np.isnan(dM) and nb == 0
