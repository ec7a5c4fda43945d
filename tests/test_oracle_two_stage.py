"""Pins for the oracle's two-stage filter (Sec. 5: a pooled first pass at a
third of the resolution, then a full-resolution pass on the restored map).

pool3 is checked against a pure-Python brute force on tiny ragged images,
against a numpy reshape mean where the image is a whole number of cells,
and against hand-derived rounding cases; restore_merge against np.repeat;
the two-stage mask against binary dilations (scipy) and, with both widths
infinite, the whole two-stage output against normalised box convolutions
(scipy), with r = 0 stages against the closed form.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import scenes as S


def brute_pool(d, b, rgb):
    h, w = d.shape
    h1, w1 = (h + 2) // 3, (w + 2) // 3
    d1 = np.zeros((h1, w1), np.float32)
    b1 = np.zeros((h1, w1), np.uint8)
    c1 = np.zeros((h1, w1, 3), np.uint8)
    for cy in range(h1):
        for cx in range(w1):
            vals, cols = [], []
            for y in range(3 * cy, min(3 * cy + 3, h)):
                for x in range(3 * cx, min(3 * cx + 3, w)):
                    cols.append([int(v) for v in rgb[y, x]])
                    if b[y, x]:
                        vals.append(float(d[y, x]))
            if vals:
                acc = 0.0
                for v in vals:
                    acc += v
                d1[cy, cx] = np.float32(acc / len(vals))
                b1[cy, cx] = 1
            n = len(cols)
            for ch in range(3):
                c1[cy, cx, ch] = (sum(c[ch] for c in cols) + n // 2) // n
    return d1, b1, c1


@pytest.mark.parametrize("h,w,dens", [(7, 8, 0.3), (9, 12, 0.1), (1, 1, 1.0),
                                      (2, 5, 0.5), (10, 4, 0.0)])
def test_pool3_brute_force(h, w, dens):
    d, b, rgb = S.tiny_random(np.random.default_rng(h * 31 + w), h, w, dens)
    got = oracle.pool3(d, b, rgb)
    ref = brute_pool(d, b, rgb)
    np.testing.assert_array_equal(got[1], ref[1])
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[2], ref[2])


def test_pool3_matches_reshape_mean():
    d, b, rgb = S.tiny_random(np.random.default_rng(3), 30, 45, 0.2)
    d1, b1, c1 = oracle.pool3(d, b, rgb)
    cells = lambda a: a.reshape(10, 3, 15, 3, *a.shape[2:]).swapaxes(1, 2) \
        .reshape(10, 15, 9, *a.shape[2:])
    bd = cells(b.astype(np.float64))
    dd = cells(d.astype(np.float64) * b)
    n = bd.sum(axis=2)
    np.testing.assert_array_equal(b1, (n > 0).astype(np.uint8))
    mean = np.divide(dd.sum(axis=2), n, out=np.zeros_like(n), where=n > 0)
    np.testing.assert_allclose(d1, mean.astype(np.float32), rtol=2e-7)
    csum = cells(rgb.astype(np.int64)).sum(axis=2)
    np.testing.assert_array_equal(c1, (csum + 4) // 9)


def test_pool3_rounding_cases():
    # one cell; colour sums 5 -> (5+4)//9 = 1, 4 -> 0, 13 -> 1, 14 -> 2
    d = np.zeros((3, 3), np.float32)
    b = np.zeros((3, 3), np.uint8)
    rgb = np.zeros((3, 3, 3), np.uint8)
    rgb[2, 2] = (5, 4, 13)
    rgb[0, 0, 2] = 1
    _, b1, c1 = oracle.pool3(d, b, rgb)
    assert b1[0, 0] == 0
    assert tuple(c1[0, 0]) == (1, 0, 2)
    # a partial 2x1 cell averages its two pixels only: (3 + 4 + 1) // 2 = 4
    rgb2 = np.array([[[3, 0, 0]], [[4, 0, 0]]], np.uint8)
    d2 = np.array([[1.0], [2.0]], np.float32)
    b2 = np.array([[1], [1]], np.uint8)
    dd, bb, cc = oracle.pool3(d2, b2, rgb2)
    assert dd[0, 0] == np.float32(1.5) and bb[0, 0] == 1
    assert cc[0, 0, 0] == 4


def test_restore_merge_is_nearest_with_originals_kept():
    rng = np.random.default_rng(4)
    h, w = 11, 14
    d, b, _ = S.tiny_random(rng, h, w, 0.2)
    o1 = rng.uniform(1, 20, size=((h + 2) // 3, (w + 2) // 3)).astype(np.float32)
    m1 = (rng.uniform(size=o1.shape) < 0.6).astype(np.uint8)
    d2, b2 = oracle.restore_merge(d, b, o1, m1)
    up = lambda a: np.repeat(np.repeat(a, 3, 0), 3, 1)[:h, :w]
    exp_b = ((b == 1) | (up(m1) == 1)).astype(np.uint8)
    exp_d = np.where(b == 1, d, np.where(up(m1) == 1, up(o1), 0)).astype(np.float32)
    np.testing.assert_array_equal(b2, exp_b)
    np.testing.assert_array_equal(d2, exp_d)


def test_two_stage_mask_is_a_chain_of_dilations():
    d, b, rgb = S.tiny_random(np.random.default_rng(5), 40, 50, 0.02)
    r1, r2 = 2, 1
    out, mask, st = oracle.densify_two_stage(d, b, rgb, r1, 2.0, 15.0, r2, 2.0,
                                             15.0, want_stages=True)
    dil = lambda a, r: ndimage.binary_dilation(a == 1, np.ones((2 * r + 1,) * 2))
    m1 = dil(st["valid1"], r1)
    np.testing.assert_array_equal(st["mask1"], m1.astype(np.uint8))
    up = np.repeat(np.repeat(m1, 3, 0), 3, 1)[:40, :50]
    b2 = (b == 1) | up
    np.testing.assert_array_equal(st["valid2"], b2.astype(np.uint8))
    np.testing.assert_array_equal(mask, dil(b2.astype(np.uint8), r2).astype(np.uint8))
    assert np.all(out[mask == 0] == 0)


def test_two_stage_box_filters_match_normalised_convolutions():
    """sigma_s = sigma_r = inf: each stage is the mean of the valid depths
    in its window, i.e. box(D*B) / box(B) with zero padding."""
    d, b, rgb = S.tiny_random(np.random.default_rng(6), 33, 41, 0.08)
    inf = float("inf")
    r1, r2 = 2, 1
    out, mask, st = oracle.densify_two_stage(d, b, rgb, r1, inf, inf, r2, inf,
                                             inf, want_stages=True)

    def box_mean(dd, bb, r):
        k = np.ones((2 * r + 1,) * 2)
        num = ndimage.correlate((dd * bb).astype(np.float64), k, mode="constant")
        den = ndimage.correlate(bb.astype(np.float64), k, mode="constant")
        return np.divide(num, den, out=np.zeros_like(num), where=den > 0), den > 0

    d1, b1, _ = oracle.pool3(d, b, rgb)
    o1, m1 = box_mean(d1, b1, r1)
    np.testing.assert_allclose(st["out1"], o1.astype(np.float32), rtol=1e-6)
    up = lambda a: np.repeat(np.repeat(a, 3, 0), 3, 1)[:33, :41]
    d2 = np.where(b == 1, d, np.where(up(m1), up(st["out1"]), 0))
    b2 = (b == 1) | up(m1)
    o2, m2 = box_mean(d2, b2, r2)
    np.testing.assert_array_equal(mask, m2.astype(np.uint8))
    np.testing.assert_allclose(out, o2, rtol=1e-12)


def test_two_stage_r0_is_restore_of_pooled_depth():
    d, b, rgb = S.tiny_random(np.random.default_rng(7), 20, 23, 0.1)
    out, mask, st = oracle.densify_two_stage(d, b, rgb, 0, 2.0, 10.0, 0, 2.0,
                                             10.0, want_stages=True)
    d1, b1, _ = oracle.pool3(d, b, rgb)
    up = lambda a: np.repeat(np.repeat(a, 3, 0), 3, 1)[:20, :23]
    exp = np.where(b == 1, d, np.where(up(b1) == 1, up(d1), 0))
    np.testing.assert_array_equal(mask, ((b == 1) | (up(b1) == 1)).astype(np.uint8))
    np.testing.assert_array_equal(out.astype(np.float32), exp.astype(np.float32))


def test_two_stage_constant_depth():
    d, b, rgb = S.tiny_random(np.random.default_rng(8), 36, 36, 0.05)
    d = np.where(b == 1, 7.25, 0).astype(np.float32)
    out, mask = oracle.densify_two_stage(d, b, rgb, 4, 2.0, 15.0, 2, 2.0, 15.0)
    np.testing.assert_allclose(out[mask == 1], 7.25, rtol=1e-13)
