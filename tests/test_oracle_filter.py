"""Pins for the oracle's joint bilateral filter (Eq. 1-4, Algorithm 1).

Each test ties the oracle to something other than itself:

* closed-form worked examples (tests/golden/worked_examples.json);
* Algorithm 1's scatter form (materialised weight volume, transpose
  convolution) against the Eq. 1 gather form;
* a pure-Python brute force on tiny inputs;
* sigma_r = inf reduces to a normalised convolution with a truncated
  Gaussian, computed with scipy.ndimage.correlate;
* the validity mask is the binary dilation of B (scipy maximum_filter);
* r = 0 is the identity; a constant 2^k depth is reproduced bit-exactly; a
  single sample fills its window exactly;
* convex hull, symmetries (transpose, flips, channel permutation, 2^k depth
  scaling) and the removal of the common factor exp(Emax).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

from synth.scenes import tiny_random

GOLDEN = os.path.join(os.path.dirname(__file__), "golden",
                      "worked_examples.json")


def _golden():
    with open(GOLDEN) as f:
        return {c["name"]: c for c in json.load(f)["cases"]}


def _sigma(case, key):
    if key in case:
        v = case[key]
        return math.inf if v == "inf" else float(v)
    sq = case[key + "_squared"]
    num, den = sq.split("/")
    return math.sqrt(float(num) / math.log(2.0))


def test_worked_two_equal_weights(orc):
    c = _golden()["two_equal_weights_midpoint"]
    out, mask = orc.densify(np.array(c["depth"], np.float32),
                            np.array(c["valid"], np.uint8),
                            np.array(c["rgb"], np.uint8), c["radius"],
                            c["sigma_s"], c["sigma_r"])
    assert out[0, 1] == 2.0
    np.testing.assert_array_equal(mask, np.array(c["expected"]["mask"]))


def test_worked_colour_weight_half(orc):
    c = _golden()["colour_weight_half"]
    sr = _sigma(c, "sigma_r")
    out, mask = orc.densify(np.array(c["depth"], np.float32),
                            np.array(c["valid"], np.uint8),
                            np.array(c["rgb"], np.uint8), c["radius"],
                            math.inf, sr)
    assert out[0, 1] == pytest.approx(5.0 / 3.0, rel=1e-15)


def test_worked_spatial_weight(orc):
    c = _golden()["spatial_weight_quarter"]
    ss = _sigma(c, "sigma_s")
    out, mask = orc.densify(np.array(c["depth"], np.float32),
                            np.array(c["valid"], np.uint8),
                            np.array(c["rgb"], np.uint8), c["radius"], ss,
                            math.inf)
    expect = (4 * 2 ** -0.5 + 2) / (2 ** -0.5 + 0.25)
    assert out[0, 0] == pytest.approx(expect, rel=1e-15)


CASES = [
    # (h, w, r, density, sigma_s, sigma_r, palette)
    (9, 11, 0, 0.3, 2.0, 12.0, None),
    (9, 11, 1, 0.3, 1.5, 12.0, 4),
    (12, 10, 2, 0.15, 2.0, 15.0, 3),
    (16, 16, 3, 0.1, 3.0, 40.0, None),
    (7, 13, 3, 0.5, 0.7, 20.0, 2),
]


def _inputs(seed, h, w, density, palette):
    return tiny_random(np.random.default_rng(seed), h, w, density,
                       n_colors=palette)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("seed", [0, 1])
def test_alg1_scatter_equals_eq1_gather(orc, case, seed):
    h, w, r, dens, ss, sr, pal = case
    d, b, rgb = _inputs(seed, h, w, dens, pal)
    g_out, g_mask = orc.densify(d, b, rgb, r, ss, sr)
    s_out, s_mask = orc.densify_alg1(d, b, rgb, r, ss, sr)
    np.testing.assert_array_equal(g_mask, s_mask)
    np.testing.assert_allclose(g_out, s_out, rtol=1e-13, atol=0)


def _brute_python(d, b, rgb, r, ss, sr):
    """Literal Eq. 1-4 with Python floats and math.exp, no rescaling."""
    h, w = d.shape
    out = np.zeros((h, w))
    mask = np.zeros((h, w), np.uint8)
    for y in range(h):
        for x in range(w):
            num = den = 0.0
            for yy in range(max(0, y - r), min(h, y + r + 1)):
                for xx in range(max(0, x - r), min(w, x + r + 1)):
                    if not b[yy, xx]:
                        continue
                    diff = [int(rgb[y, x, k]) - int(rgb[yy, xx, k])
                            for k in range(3)]
                    wc = math.exp(-sum(t * t for t in diff) / (2 * sr * sr))
                    wp = math.exp(-((xx - x) ** 2 + (yy - y) ** 2)
                                  / (2 * ss * ss))
                    num += float(d[yy, xx]) * wc * wp
                    den += wc * wp
            if den > 0:
                out[y, x] = num / den
                mask[y, x] = 1
    return out, mask


@pytest.mark.parametrize("case", CASES[:4])
def test_python_brute_force(orc, case):
    h, w, r, dens, ss, sr, pal = case
    d, b, rgb = _inputs(5, h, w, dens, pal)
    out, mask = orc.densify(d, b, rgb, r, ss, sr)
    bo, bm = _brute_python(d, b, rgb, r, ss, sr)
    np.testing.assert_array_equal(mask, bm)
    np.testing.assert_allclose(out, bo, rtol=1e-13, atol=0)


@pytest.mark.parametrize("r,ss", [(1, 1.0), (2, 1.5), (4, 2.5), (6, 3.0)])
def test_sigma_r_inf_is_normalised_convolution(orc, r, ss):
    d, b, rgb = _inputs(11, 24, 30, 0.12, None)
    out, mask = orc.densify(d, b, rgb, r, ss, math.inf)
    t = np.arange(-r, r + 1, dtype=np.float64)
    k1 = np.exp(-t * t / (2 * ss * ss))
    kern = np.outer(k1, k1)
    bd = b.astype(np.float64) * d.astype(np.float64)
    num = ndimage.correlate(bd, kern, mode="constant", cval=0.0)
    den = ndimage.correlate(b.astype(np.float64), kern, mode="constant",
                            cval=0.0)
    dil = ndimage.maximum_filter(b, size=2 * r + 1, mode="constant", cval=0)
    np.testing.assert_array_equal(mask, dil)
    sel = mask == 1
    np.testing.assert_allclose(out[sel], num[sel] / den[sel], rtol=1e-12)
    assert np.all(out[~sel] == 0.0)


@pytest.mark.parametrize("r", [0, 1, 2, 5])
def test_mask_is_binary_dilation(orc, r):
    for seed in range(3):
        d, b, rgb = _inputs(seed, 20, 17, 0.05 + 0.1 * seed, None)
        _, mask = orc.densify(d, b, rgb, r, 2.0, 10.0)
        dil = ndimage.maximum_filter(b, size=2 * r + 1, mode="constant",
                                     cval=0)
        np.testing.assert_array_equal(mask, dil)


def test_sigma_s_inf_is_box_range_filter(orc):
    """With sigma_s = inf every valid sample of the square window weighs
    exp(-c/(2 sr^2)); computed here with a sliding-window view."""
    d, b, rgb = _inputs(4, 10, 12, 0.3, 3)
    r, sr = 2, 25.0
    out, mask = orc.densify(d, b, rgb, r, math.inf, sr)
    h, w = d.shape
    pad = lambda a, v: np.pad(a, [(r, r), (r, r)] + [(0, 0)] * (a.ndim - 2),
                              constant_values=v)
    win = np.lib.stride_tricks.sliding_window_view
    rgbp = win(pad(rgb.astype(np.int64), 0), (2 * r + 1, 2 * r + 1),
               axis=(0, 1))              # h, w, 3, k, k
    bp = win(pad(b, 0), (2 * r + 1, 2 * r + 1))
    dp = win(pad(d.astype(np.float64), 0.0), (2 * r + 1, 2 * r + 1))
    c = ((rgbp - rgb.astype(np.int64)[:, :, :, None, None]) ** 2).sum(axis=2)
    wgt = np.exp(-c / (2 * sr * sr)) * bp
    num = (wgt * dp).sum(axis=(2, 3))
    den = wgt.sum(axis=(2, 3))
    sel = mask == 1
    np.testing.assert_allclose(out[sel], num[sel] / den[sel], rtol=1e-13)


def test_r0_is_identity_bit_exact(orc):
    d, b, rgb = _inputs(3, 33, 21, 0.4, None)
    out, mask = orc.densify(d, b, rgb, 0, 1.0, 1.0)
    np.testing.assert_array_equal(mask, b)
    np.testing.assert_array_equal(out, np.where(b == 1, d, 0).astype(np.float64))


@pytest.mark.parametrize("k", [-3, 0, 4])
def test_constant_power_of_two_depth_bit_exact(orc, k):
    d, b, rgb = _inputs(8, 25, 19, 0.2, 5)
    c = np.float32(2.0 ** k)
    d = np.where(b == 1, c, np.float32(0)).astype(np.float32)
    out, mask = orc.densify(d, b, rgb, 3, 2.0, 9.0)
    assert np.all(out[mask == 1] == float(c))


def test_constant_depth_within_ulps(orc):
    d, b, rgb = _inputs(9, 25, 19, 0.2, 5)
    d = np.where(b == 1, np.float32(7.3), np.float32(0)).astype(np.float32)
    out, mask = orc.densify(d, b, rgb, 3, 2.0, 9.0)
    np.testing.assert_allclose(out[mask == 1], float(np.float32(7.3)),
                               rtol=4e-16)


def test_single_sample_fills_window(orc):
    h, w, r = 15, 17, 4
    rng = np.random.default_rng(2)
    rgb = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    for (y, x) in [(7, 8), (0, 0), (14, 16), (2, 15)]:
        b = np.zeros((h, w), np.uint8)
        b[y, x] = 1
        d = np.zeros((h, w), np.float32)
        d[y, x] = np.float32(3.1415)
        out, mask = orc.densify(d, b, rgb, r, 1.3, 4.0)
        sq = np.zeros((h, w), np.uint8)
        sq[max(0, y - r):y + r + 1, max(0, x - r):x + r + 1] = 1
        np.testing.assert_array_equal(mask, sq)
        assert np.all(out[sq == 1] == float(np.float32(3.1415)))
        assert np.all(out[sq == 0] == 0.0)


def test_convex_hull(orc):
    d, b, rgb = _inputs(12, 30, 30, 0.08, 4)
    r = 3
    out, mask = orc.densify(d, b, rgb, r, 2.0, 12.0)
    big = np.float32(1e9)
    lo = ndimage.minimum_filter(np.where(b == 1, d, big), size=2 * r + 1,
                                mode="constant", cval=big)
    hi = ndimage.maximum_filter(np.where(b == 1, d, -big), size=2 * r + 1,
                                mode="constant", cval=-big)
    sel = mask == 1
    assert np.all(out[sel] >= lo[sel] * (1 - 1e-15))
    assert np.all(out[sel] <= hi[sel] * (1 + 1e-15))


def test_symmetries(orc):
    d, b, rgb = _inputs(13, 18, 23, 0.15, 3)
    r, ss, sr = 3, 2.0, 14.0
    out, mask = orc.densify(d, b, rgb, r, ss, sr)
    # transpose
    o2, m2 = orc.densify(d.T.copy(), b.T.copy(),
                         rgb.transpose(1, 0, 2).copy(), r, ss, sr)
    np.testing.assert_array_equal(m2, mask.T)
    np.testing.assert_allclose(o2, out.T, rtol=1e-14)
    # flips
    o3, _ = orc.densify(d[::-1].copy(), b[::-1].copy(), rgb[::-1].copy(),
                        r, ss, sr)
    np.testing.assert_allclose(o3, out[::-1], rtol=1e-14)
    o4, _ = orc.densify(d[:, ::-1].copy(), b[:, ::-1].copy(),
                        rgb[:, ::-1].copy(), r, ss, sr)
    np.testing.assert_allclose(o4, out[:, ::-1], rtol=1e-14)
    # channel permutation: the colour distance is unchanged, bit for bit
    o5, _ = orc.densify(d, b, rgb[:, :, [2, 0, 1]].copy(), r, ss, sr)
    np.testing.assert_array_equal(o5, out)
    # depth scaled by 2^5 scales the output by 2^5 exactly
    o6, _ = orc.densify((d * np.float32(32)).astype(np.float32), b, rgb, r,
                        ss, sr)
    np.testing.assert_array_equal(o6, out * 32.0)


def test_common_factor_removal_equals_literal_eq1(orc):
    for seed, (r, ss, sr) in enumerate([(2, 1.0, 12.0), (3, 2.0, 15.0),
                                        (5, 3.0, 12.0)]):
        d, b, rgb = _inputs(20 + seed, 20, 20, 0.2, 3)
        a, ma = orc.densify(d, b, rgb, r, ss, sr)
        p, mp = orc.densify_plain(d, b, rgb, r, ss, sr)
        np.testing.assert_array_equal(ma, mp)
        np.testing.assert_allclose(a, p, rtol=1e-13)


def test_underflowing_window_still_defined(orc):
    """All weights of pixel (0,1) are exp(-800) or smaller in the literal
    form (0/0 in double); two samples with identical colour and spatial
    distance must still average exactly."""
    rgb = np.zeros((1, 3, 3), np.uint8)
    rgb[0, 0] = (200, 0, 0)
    rgb[0, 2] = (200, 0, 0)
    rgb[0, 1] = (0, 0, 0)
    d = np.array([[2.0, 0.0, 6.0]], np.float32)
    b = np.array([[1, 0, 1]], np.uint8)
    lit, _ = orc.densify_plain(d, b, rgb, 1, 1.0, 1.0)
    assert math.isnan(lit[0, 1])
    out, mask = orc.densify(d, b, rgb, 1, 1.0, 1.0)
    assert mask[0, 1] == 1
    assert out[0, 1] == 4.0
