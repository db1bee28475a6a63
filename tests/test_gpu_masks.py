"""Mask generation and surface metrics on the GPU (Methods, Mask Generation;
Evaluation) against the oracle, through the C ABI.  Masks are integers, so the
comparison is bit for bit; the distances are spacing * sqrt(k) for exact integer
squared index distances k on both sides, so d_H and d_M are compared bit for
bit as well."""

import sys

import numpy as np
import pytest
import torch
from scipy import ndimage

from oracle import masks as K
from paper_1605_02060_amd import lddmm as L
from paper_1605_02060_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _blobs(shape, seed, p=0.55, smooth=2.0):
    rng = np.random.default_rng(seed)
    f = ndimage.gaussian_filter(rng.normal(size=shape), smooth)
    return f > np.quantile(f, p)


OPS = [(L.MORPH_ERODE, K.erode), (L.MORPH_DILATE, K.dilate), (L.MORPH_OPEN, K.opening),
       (L.MORPH_CLOSE, K.closing)]


@pytest.mark.parametrize("shape,radius,h", [((23, 26, 37), 1.0, 1.0), ((21, 19, 65), 2.5, 1.0),
                                            ((17, 30, 95), 0.125, 0.025),
                                            ((20, 24, 40), 12.0, 1.0), ((3, 4, 5), 2.0, 1.0)])
def test_morphology_matches_oracle(shape, radius, h):
    say(f"morphology {shape} r={radius} h={h}")
    A = _blobs(shape, 1)
    for op, ref in OPS:
        got = L.lddmm_morphology(t(A), op, radius, spacing=h).cpu().numpy()
        np.testing.assert_array_equal(got > 0, ref(A, radius, h), err_msg=str(op))


@pytest.mark.parametrize("shape", [(1, 1, 33), (1, 3, 1), (2, 1, 64), (5, 1, 1)])
def test_thin_grids(shape):
    # grids one voxel thick along one or two axes: every ball row but the centre
    # one leaves the grid
    say(f"morphology and surfaces on a thin grid {shape}")
    rng = np.random.default_rng(8)
    A = rng.random(shape) > 0.4
    B = rng.random(shape) > 0.5
    for op, ref in OPS:
        got = L.lddmm_morphology(t(A), op, 2.0).cpu().numpy()
        np.testing.assert_array_equal(got > 0, ref(A, 2.0, 1.0), err_msg=str(op))
    _check_distances(A, B, 1.0)


def test_morphology_largest_radius():
    say("morphology r = 31 voxels, 70 wide")
    A = _blobs((8, 9, 70), 2, p=0.3, smooth=1.0)
    for op, ref in OPS[:2]:
        got = L.lddmm_morphology(t(A), op, 31.0).cpu().numpy()
        np.testing.assert_array_equal(got > 0, ref(A, 31.0, 1.0))


def test_target_and_label_masks():
    say("target mask (threshold, open, close) and label mask")
    rng = np.random.default_rng(3)
    shape = (40, 44, 50)
    z, y, x = np.mgrid[:40, :44, :50]
    brain = (x - 25) ** 2 / 18 ** 2 + (y - 22) ** 2 / 15 ** 2 + (z - 20) ** 2 / 14 ** 2 <= 1
    I = (brain * rng.poisson(2.0, shape) + (rng.random(shape) > 0.995)).astype(np.float32)
    for ro, rc in ((0.05, 0.125), (0.0, 0.125), (0.05, 0.0)):
        got = L.lddmm_target_mask(t(I), 0.5, ro, rc, spacing=0.025).cpu().numpy()
        np.testing.assert_array_equal(got > 0, K.target_mask(I, 0.5, ro, rc, 0.025))
    lab = (rng.integers(0, 4, shape) * brain).astype(np.int32)
    np.testing.assert_array_equal(L.lddmm_label_mask(t(lab, torch.int32)).cpu().numpy() > 0,
                                  K.label_mask(lab))


def _check_distances(A, B, h):
    got = L.lddmm_surface_distance(t(A), t(B), spacing=h).cpu().numpy()
    dH, dM, na, nb = K.surface_distances(A, B, h)
    assert (got[2], got[3]) == (na, nb)
    if np.isnan(dH):
        assert np.isnan(got[0]) and np.isnan(got[1])
    else:
        assert got[0] == dH and got[1] == dM, (got, dH, dM)


@pytest.mark.parametrize("shape,h", [((23, 26, 37), 1.0), ((30, 17, 66), 0.05)])
def test_surface_distances_match_oracle(shape, h):
    say(f"surface distances {shape} h={h}")
    _check_distances(_blobs(shape, 4), _blobs(shape, 5), h)
    A = _blobs(shape, 6)
    _check_distances(A, ndimage.binary_erosion(A), h)


def test_surface_distance_special_cases():
    say("surface distances: shifted cube, identical, empty, single voxel")
    A = np.zeros((20, 20, 30), bool)
    A[5:15, 5:15, 5:15] = True
    _check_distances(A, np.roll(A, 3, axis=2), 0.5)
    got = L.lddmm_surface_distance(t(A), t(A), spacing=0.5).cpu().numpy()
    assert got[0] == 0.0 and got[1] == 0.0
    _check_distances(A, np.zeros_like(A), 1.0)
    one = np.zeros_like(A)
    one[10, 2, 27] = True
    _check_distances(A, one, 0.7)


def test_invalid_arguments():
    say("masks EINVAL")
    x = t(np.zeros((4, 5, 6), np.float32))
    for op, r in ((4, 1.0), (-1, 1.0), (L.MORPH_ERODE, -1.0), (L.MORPH_ERODE, 32.0),
                  (L.MORPH_ERODE, float("inf"))):
        with pytest.raises(L.LddmmError):
            L.lddmm_morphology(x, op, r)
    with pytest.raises(L.LddmmError):
        L.lddmm_morphology(x, L.MORPH_ERODE, 1.0, ws=torch.empty(8, dtype=torch.uint8,
                                                                 device=DEV))
    with pytest.raises(L.LddmmError):
        L.lddmm_target_mask(x, 0.5, 1.0, 40.0)


def test_atlas_size_masks_and_distances():
    # the atlas-like pair at 50 um: the sparse target's mask by the paper's
    # recipe (50 um opening, 125 um closing), and the surface distances between
    # it and the template mask, all 9.6 M voxels compared
    say("atlas size: target mask + surface distances, 228x160x264")
    p = synth.config_pair("atlas")
    h = 0.05
    # a dense image of the target's shape with foreground grains and holes (the
    # sparse Poisson target would not survive a one-voxel opening)
    rng = np.random.default_rng(7)
    I = p.I0 * (1.0 + 0.2 * rng.standard_normal(p.shape))
    I[rng.random(p.shape) > 0.999] = 1.0
    I[rng.random(p.shape) > 0.999] = 0.0
    I = I.astype(np.float32)
    M1g = L.lddmm_target_mask(t(I), 0.1, 0.05, 0.125, spacing=h)
    M1 = K.target_mask(I, 0.1, 0.05, 0.125, h)
    assert M1.sum() > 0.3 * (p.M0 > 0).sum()
    np.testing.assert_array_equal(M1g.cpu().numpy() > 0, M1)
    _check_distances(p.M0 > 0, M1, h)
