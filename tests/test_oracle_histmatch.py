"""Pins of the histogram-matching oracle (Methods, Preprocessing): hand-worked
examples, closed forms for equal bin counts, numpy's sample quantiles on large
uniform samples, and the exact inverse of an affine intensity change."""

import json
import os

import numpy as np
import pytest

from oracle import histmatch as H

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "histmatch_small.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_worked_examples(case):
    out, s, r, cs, cr = H.histogram_match(
        np.array(case["src"], np.float32), np.array(case["src_mask"], np.float32),
        np.array(case["ref"], np.float32), np.array(case["ref_mask"], np.float32),
        case["n_bins"], case["n_points"])
    if "counts_src" in case:
        np.testing.assert_array_equal(cs, case["counts_src"])
        np.testing.assert_array_equal(cr, case["counts_ref"])
    np.testing.assert_allclose(s, case["s"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r, case["r"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out, case["out"], rtol=1e-6, atol=1e-7)


def test_equal_counts_give_the_straight_quantile_line():
    # every bin holds m values (drawn inside the bin, away from its edges), the
    # minimum and maximum sit in the first and last bin: whatever the values,
    # the histogram's cumulative distribution is the straight line, so
    # q(p) = lo + p (hi - lo) at every match point
    rng = np.random.default_rng(5)
    nb, m, P = 32, 5, 8
    vals = [float(b) + rng.uniform(0.1, 0.9, m) for b in range(nb)]
    vals = np.concatenate(vals).astype(np.float32)
    vals[0], vals[-1] = 0.0, 32.0                       # lo in bin 0, hi clamped into bin 31
    counts, lo, hi = H.histogram(vals, nb)
    np.testing.assert_array_equal(counts, np.full(nb, m))
    pts = H.match_points(counts, lo, hi, P)
    want = lo + np.arange(P + 2) / (P + 1) * (hi - lo)
    np.testing.assert_allclose(pts, want, rtol=0, atol=1e-12)


def test_quantiles_agree_with_sample_quantiles():
    rng = np.random.default_rng(6)
    for dist in (rng.uniform(2.0, 7.0, 400_000), rng.normal(1.0, 0.5, 400_000)):
        x = dist.astype(np.float32)
        counts, lo, hi = H.histogram(x, 32)
        width = (float(hi) - float(lo)) / 32
        for k in range(1, 9):
            p = k / 9
            q = H.quantile(counts, lo, hi, p)
            # the histogram knows the values only to a bin; within a bin it
            # assumes them uniform, which is close for smooth densities
            assert abs(q - np.quantile(x.astype(np.float64), p)) < 0.25 * width


def test_affine_intensity_change_is_undone():
    # S = 2 R + 0.5 exactly in float32 (R on a 1/1024 grid): the bins of S are
    # those of R scaled, so every match point of S is 2 r_k + 0.5 and the
    # polyline is the inverse map; matching S to R returns R, and matching R to S
    # returns S (a swapped source and reference fails one of the two)
    rng = np.random.default_rng(7)
    shape = (9, 10, 11)
    R = (rng.integers(0, 4096, size=shape) / 1024.0).astype(np.float32)
    S = (2.0 * R + 0.5).astype(np.float32)
    ms = (rng.random(shape) > 0.2).astype(np.float32)
    ones = np.ones(shape, np.float32)
    out, s, r, cs, cr = H.histogram_match(S, ms, R, ms, 32, 8)
    np.testing.assert_array_equal(cs, cr)
    np.testing.assert_allclose(s, 2.0 * r + 0.5, rtol=1e-14)
    inside = ms > 0
    np.testing.assert_allclose(out[inside], R[inside], rtol=1e-6, atol=1e-6)
    assert np.all(out[~inside] == 0)
    back, *_ = H.histogram_match(R, ones, S, ones, 32, 8)
    np.testing.assert_allclose(back, S, rtol=1e-6, atol=1e-6)


def test_map_is_monotone_and_spans_the_reference_range():
    rng = np.random.default_rng(8)
    shape = (12, 13, 14)
    src = rng.gamma(2.0, 1.0, shape).astype(np.float32)
    ref = rng.normal(5.0, 2.0, shape).astype(np.float32)
    ms = (rng.random(shape) > 0.3).astype(np.float32)
    mr = (rng.random(shape) > 0.5).astype(np.float32)
    out, s, r, _, _ = H.histogram_match(src, ms, ref, mr)
    inside = ms > 0
    order = np.argsort(src[inside], kind="stable")
    assert np.all(np.diff(out[inside][order].astype(np.float64)) >= 0)
    assert out[inside].min() == np.float32(ref[mr > 0].min())
    assert out[inside].max() == np.float32(ref[mr > 0].max())
    assert np.all(out[~inside] == 0)
    assert np.all(np.diff(s) >= 0) and np.all(np.diff(r) >= 0)


def test_degenerate_cases():
    shape = (4, 5, 6)
    rng = np.random.default_rng(9)
    src = rng.random(shape).astype(np.float32)
    ref = rng.random(shape).astype(np.float32)
    ones, zeros = np.ones(shape, np.float32), np.zeros(shape, np.float32)
    for ms, mr in ((zeros, ones), (ones, zeros)):
        out, s, *_ = H.histogram_match(src, ms, ref, mr)
        assert s is None and np.all(out == 0)
    const = np.full(shape, 3.0, np.float32)
    out, s, r, cs, _ = H.histogram_match(const, ones, ref, ones)
    assert cs[0] == const.size and np.all(s == 3.0)
    assert np.all(out == np.float32(ref.max()))
