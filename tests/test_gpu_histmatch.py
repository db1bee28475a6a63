"""Image-LDDMM preprocessing on the GPU (Methods, Preprocessing): mask
application and histogram matching against the oracle, through the C ABI, and
an Image-LDDMM registration (data term on the masked, matched images only).

The bin counts are integers and compared bit for bit.  The bin of a value is an
integer decided in float32 on both sides; the quantile points and the map are
the same FP64 operations in the same order on both sides (no fused
multiply-adds in the library's histogram source), so the points and the
float32 output are compared bit for bit as well.
"""

import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import histmatch as H
from oracle import lddmm as O
from paper_1605_02060_amd import lddmm as L
from paper_1605_02060_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "histmatch_small.json")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def unaligned(a):
    """Device copy of a whose data pointer is 4 bytes past a 16-byte boundary."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    buf = torch.zeros(a.size + 1, dtype=torch.float32, device=DEV)
    v = buf[1:].view(a.shape)
    v.copy_(torch.as_tensor(a))
    assert v.data_ptr() % 16 == 4
    return v


def _check(src, ms, ref, mr, nb, npts, conv=t):
    out, pts, cnt = L.lddmm_histogram_match(conv(src), conv(ms), conv(ref), conv(mr), nb, npts)
    torch.cuda.synchronize()
    o, s, r, cs, cr = H.histogram_match(src, ms, ref, mr, nb, npts)
    np.testing.assert_array_equal(out.cpu().numpy(), o)
    if s is None:
        return
    np.testing.assert_array_equal(cnt.cpu().numpy(), np.stack([cs, cr]))
    np.testing.assert_array_equal(pts.cpu().numpy(), np.stack([s, r]))


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_hand_worked_examples(case):
    say(f"histmatch golden: {case['name']}")
    f = lambda k: np.array(case[k], np.float32).reshape(1, 1, -1)
    out, pts, cnt = L.lddmm_histogram_match(t(f("src")), t(f("src_mask")), t(f("ref")),
                                            t(f("ref_mask")), case["n_bins"], case["n_points"])
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy().ravel(), case["out"], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(pts.cpu().numpy(), [case["s"], case["r"]], rtol=1e-12, atol=1e-12)
    if "counts_src" in case:
        np.testing.assert_array_equal(cnt.cpu().numpy(), [case["counts_src"], case["counts_ref"]])


@pytest.mark.parametrize("nb,npts", [(32, 8), (1, 0), (7, 3), (1024, 62), (32, 0)])
@pytest.mark.parametrize("aligned", [True, False])
def test_matches_oracle_on_ragged_grids(nb, npts, aligned):
    say(f"histmatch ragged nb={nb} P={npts} aligned={aligned}")
    rng = np.random.default_rng(31 + nb + npts)
    src = rng.gamma(2.0, 1.5, (37, 41, 29)).astype(np.float32)
    ref = (rng.normal(4.0, 1.0, (33, 35, 47)) ** 2).astype(np.float32)
    ms = (rng.random(src.shape) > 0.35).astype(np.float32)
    mr = (rng.random(ref.shape) > 0.6).astype(np.float32)
    _check(src, ms, ref, mr, nb, npts, t if aligned else unaligned)


def test_matches_oracle_at_the_atlas_size():
    # the atlas grid (264 x 160 x 228) against a smaller target grid, soft-edged
    # ellipsoid masks; all 9.6 M outputs compared
    say("histmatch atlas size 228x160x264")
    rng = np.random.default_rng(40)
    shape_s, shape_r = (228, 160, 264), (200, 150, 240)
    def ball(shape, f):
        z, y, x = np.ogrid[:shape[0], :shape[1], :shape[2]]
        c = [(n - 1) / 2 for n in shape]
        rr = sum(((a - ci) / (f * ci)) ** 2 for a, ci in zip((z, y, x), c))
        return (rr < 1.0).astype(np.float32)
    src = rng.gamma(3.0, 0.2, shape_s).astype(np.float32)
    ref = rng.lognormal(0.0, 0.6, shape_r).astype(np.float32)
    _check(src, ball(shape_s, 0.85), ref, ball(shape_r, 0.8), 32, 8)


def test_degenerate_inputs_and_errors():
    say("histmatch degenerate / EINVAL")
    rng = np.random.default_rng(41)
    shape = (6, 7, 9)
    src = rng.random(shape).astype(np.float32)
    ref = rng.random(shape).astype(np.float32)
    ones, zeros = np.ones(shape, np.float32), np.zeros(shape, np.float32)
    _check(src, zeros, ref, ones, 32, 8)          # empty source mask: all zero
    _check(src, ones, ref, zeros, 32, 8)          # empty reference mask: all zero
    _check(np.full(shape, 2.5, np.float32), ones, ref, ones, 32, 8)   # constant source
    _check(src, ones, np.full(shape, -1.0, np.float32), ones, 32, 8)  # constant reference
    one = np.array([[[0.7]]], np.float32)
    _check(one, np.ones_like(one), src, ones, 32, 8)                 # a single voxel
    for nb, npts in ((0, 8), (1025, 8), (32, -1), (32, 63)):
        with pytest.raises(L.LddmmError):
            L.lddmm_histogram_match(t(src), t(ones), t(ref), t(ones), nb, npts)
    small = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(L.LddmmError):
        L.lddmm_histogram_match(t(src), t(ones), t(ref), t(ones), 32, 8, ws=small)


def test_mask_image():
    say("mask image")
    rng = np.random.default_rng(42)
    I = rng.normal(size=(11, 13, 17)).astype(np.float32)
    M = (rng.random(I.shape) > 0.5).astype(np.float32)
    out = L.lddmm_mask_image(t(I), t(M))
    np.testing.assert_array_equal(out.cpu().numpy(), np.where(M > 0, I, 0).astype(np.float32))


def test_image_lddmm_registration_matches_oracle():
    # Image-LDDMM: the template image is masked and histogram-matched to the
    # masked target image, and only the image channel enters the data term
    # (weights (0, 1)).  Each side preprocesses with its own implementation.
    say("image-LDDMM: histogram match + register w=(0,1), blobs32")
    p = synth.config_pair("blobs32")
    I0 = (np.sqrt(np.maximum(p.I0, 0.0)) * 3.0 + 0.2).astype(np.float32)   # a different contrast
    h = 0.05
    prm = O.Params(T=10, iters=(10,), step=0.05, spacing=h, weight=(0.0, 1.0))
    o0, *_ = H.histogram_match(I0, p.M0, p.I1, p.M1, 32, 8)
    o1 = np.where(p.M1 > 0, p.I1, 0).astype(np.float32)
    ref = O.register(O.Problem(p.M0, p.M1, o0, o1), prm)
    g0, _, _ = L.lddmm_histogram_match(t(I0), t(p.M0), t(p.I1), t(p.M1), 32, 8)
    g1 = L.lddmm_mask_image(t(p.I1), t(p.M1))
    np.testing.assert_array_equal(g0.cpu().numpy(), o0)
    lp = L.Params(alpha=prm.alpha, gamma=prm.gamma, sigma=prm.sigma, T=prm.T, n_levels=1,
                  iters=prm.iters, step=prm.step, guard=prm.guard, weight=prm.weight)
    res = L.lddmm_register(t(p.M0), t(p.M1), g0, g1, params=lp, spacing=h)
    torch.cuda.synchronize()
    tr, rt = res["trace"].cpu().numpy(), np.array(ref.trace)
    np.testing.assert_array_equal(tr[:, 6], rt[:, 6])
    fin = np.isfinite(rt[:, 0])
    assert np.all(np.abs(tr[fin, 0] - rt[fin, 0]) <= 1e-5 * np.abs(rt[fin, 0]))
    assert rt[-1, 2] < 0.8 * rt[0, 2]               # the image data term decreases
    assert np.abs(res["phi10"].cpu().numpy() - ref.phi10).max() / h < 1e-4
    assert np.abs(res["phi01"].cpu().numpy() - ref.phi01).max() / h < 1e-4
