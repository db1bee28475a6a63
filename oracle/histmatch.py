"""FP64 CPU oracle of the Image-LDDMM histogram matching -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU baseline of the benchmark may import
this module; the library never does.

The paper (Methods, Preprocessing) applies each brain mask to its image and
histogram-matches the masked template image to the masked target image: both
images get 32-bin histograms, the two are matched exactly at 8 quantile points
and by linear interpolation at every intensity between them.  It leaves the
details open; the readings taken here are:

* the histograms count the voxels inside each mask only (M > 0), so the zero
  background that masking creates does not enter them;
* n_bins equal-width bins span [lo, hi], the in-mask minimum and maximum; the
  bin of a value x is floor((x - lo) * (n_bins / (hi - lo))), clamped to the
  last bin, evaluated in single precision (it is an integer decision, so both
  implementations take it in the precision of the stored images);
  a constant image (hi == lo) puts every voxel in bin 0;
* the p-quantile of a histogram is the point where the cumulative
  distribution of its piecewise-uniform density (counts spread evenly over
  each bin) reaches p;
* the n_points match points sit at p = k / (n_points + 1), k = 1 .. n_points,
  and the two ends lo and hi are matched to each other as well, so the map
  covers the whole in-mask range;
* between neighbouring points the map is the straight line through them;
  a value at or above the last source point maps to the last target point;
* outside the source mask the output is 0 (the masked image); if either mask
  is empty the whole output is 0.

Pins (tests/test_oracle_histmatch.py): a hand-worked example
(tests/golden/histmatch_small.json), equal bin counts giving the straight
quantile line lo + p (hi - lo), agreement with numpy's sample quantiles to a
bin width on large uniform samples, and matching an affine copy a R + b
(a > 0, power-of-two a) of a reference back onto that reference.
"""

from __future__ import annotations

import numpy as np


def inside(M):
    """In-mask test: M > 0."""
    return np.asarray(M) > 0


def value_range(x):
    """(lo, hi) of the in-mask values x (float32)."""
    x = np.asarray(x, dtype=np.float32)
    return np.float32(x.min()), np.float32(x.max())


def bin_index(x, lo, hi, n_bins):
    """Bin of each value, decided in float32 as documented in the header."""
    x = np.asarray(x, dtype=np.float32)
    lo, hi = np.float32(lo), np.float32(hi)
    if hi > lo:
        scale = np.float32(n_bins) / np.float32(hi - lo)
    else:
        scale = np.float32(0.0)
    t = (x - lo) * scale                       # float32 subtraction, then product
    b = np.floor(t).astype(np.int64)
    return np.minimum(b, n_bins - 1)


def histogram(x, n_bins):
    """(counts[n_bins], lo, hi) of the in-mask values x."""
    lo, hi = value_range(x)
    counts = np.bincount(bin_index(x, lo, hi, n_bins), minlength=n_bins).astype(np.int64)
    return counts, lo, hi


def quantile(counts, lo, hi, p):
    """Point where the piecewise-uniform cumulative distribution of the histogram
    reaches p (0 < p < 1): the first bin b whose cumulative count reaches p n,
    entered by the fraction of its own count still needed."""
    n = int(np.sum(counts))
    width = (float(hi) - float(lo)) / len(counts)
    need = p * n
    before = 0
    for b, c in enumerate(counts):
        c = int(c)
        if c > 0 and before + c >= need:
            return float(lo) + (b + (need - before) / c) * width
        before += c
    return float(hi)


def match_points(counts, lo, hi, n_points):
    """[lo, q(1/(P+1)), ..., q(P/(P+1)), hi] for P = n_points."""
    pts = [float(lo)]
    for k in range(1, n_points + 1):
        pts.append(quantile(counts, lo, hi, k / (n_points + 1)))
    pts.append(float(hi))
    return np.array(pts)


def piecewise_linear(x, s, r):
    """Map x through the polyline (s_k, r_k): on [s_k, s_{k+1}) with k the last
    point not above x, r_k + (x - s_k) * slope_k, slope_k = (r_{k+1} - r_k) /
    (s_{k+1} - s_k); x >= s_last gives r_last.  Values below s_0 do not occur
    (s_0 is the in-mask minimum)."""
    x = np.asarray(x, dtype=np.float64)
    s, r = np.asarray(s, dtype=np.float64), np.asarray(r, dtype=np.float64)
    last = len(s) - 1
    k = np.searchsorted(s, x, side="right") - 1          # last point not above x
    k = np.clip(k, 0, last - 1)
    top = x >= s[last]
    kk = np.where(top, 0, k)
    # at the top end the polyline is not evaluated: avoid a 0/0 from equal points
    den = np.where(top, 1.0, s[kk + 1] - s[kk])
    slope = (r[kk + 1] - r[kk]) / den
    return np.where(top, r[last], r[kk] + (x - s[kk]) * slope)


def histogram_match(src, src_mask, ref, ref_mask, n_bins=32, n_points=8):
    """Masked source image with its in-mask intensities matched to those of the
    masked reference (Methods, Preprocessing).  Returns (out float32 array of
    src's shape, s, r, counts_src, counts_ref); s, r are the matched points
    (None when a mask is empty)."""
    src = np.asarray(src, dtype=np.float32)
    ref = np.asarray(ref, dtype=np.float32)
    ms, mr = inside(src_mask), inside(ref_mask)
    out = np.zeros(src.shape, dtype=np.float32)
    if not ms.any() or not mr.any():
        return out, None, None, None, None
    cs, los, his = histogram(src[ms], n_bins)
    cr, lor, hir = histogram(ref[mr], n_bins)
    s = match_points(cs, los, his, n_points)
    r = match_points(cr, lor, hir, n_points)
    out[ms] = piecewise_linear(src[ms], s, r).astype(np.float32)
    return out, s, r, cs, cr
