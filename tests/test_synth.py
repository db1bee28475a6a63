"""The seeded input generators: the torch evaluation of the blob masks draws the
same parameters and computes the same formulas as the NumPy one."""

import numpy as np
import torch

from paper_1605_02060_amd import synth


def test_device_masks_equal_numpy_masks():
    for shape, seed, disp in [((20, 24, 28), 5, 3.0), ((17, 13, 11), 9, 2.0)]:
        p = synth.blob_pair(shape, seed, max_disp=disp)
        M0, M1 = synth.blob_masks_device(shape, seed, "cpu", max_disp=disp)
        np.testing.assert_array_equal(M0.numpy(), p.M0)
        np.testing.assert_array_equal(M1.numpy(), p.M1)


def test_warmstart_masks_are_the_blobs96_recipe():
    p = synth.config_pair("blobs96", seed=10003)
    M0, M1 = synth.warmstart_masks_device(10003, "cpu")
    assert M0.dtype == torch.float32 and M0.shape == (96, 96, 96)
    np.testing.assert_array_equal(M0.numpy(), p.M0)
    np.testing.assert_array_equal(M1.numpy(), p.M1)


def test_batched_dims_and_pairs():
    dims = synth.batched_dims()
    assert dims.shape == (16, 3) and dims.min() >= 64 and dims.max() <= 160
    p = synth.batched_pair(15, dims)
    nx, ny, nz = dims[15]
    assert p.M0.shape == (nz, ny, nx)
    assert 0.02 < p.M0.mean() < 0.6 and 0.02 < p.M1.mean() < 0.6
