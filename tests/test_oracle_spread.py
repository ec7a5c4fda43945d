"""Pins for the oracle's per-pixel sensitivity to weight errors,
S(x) = sum_i w_i |D_i - out(x)| / sum_i w_i over the window of Eq. 1-4
(the weighted mean absolute deviation of the samples from the output).

A hand-derived case, a pure-Python brute force on tiny images, constant
depth (S = 0), and the property S exists for: a relative change of at most
e in every weight moves the output by at most e S / (1 - e).
"""
import math

import numpy as np
import pytest

from synth.scenes import tiny_random


def test_spread_worked_example(orc):
    """Pixel 1 of a 1x3 row (r = 1, sigma_s = inf): sample 0 (c = 0, D = 1)
    weighs 1, sample 2 (c = 100, D = 3) weighs 1/2 at sigma_r^2 = 50/ln 2:
    out = 5/3 and S = (|1 - 5/3| + |3 - 5/3| / 2) / (3/2) = 8/9."""
    rgb = np.array([[[50, 50, 50], [50, 50, 50], [60, 50, 50]]], np.uint8)
    d = np.array([[1.0, 0.0, 3.0]], np.float32)
    b = np.array([[1, 0, 1]], np.uint8)
    sr = math.sqrt(50.0 / math.log(2.0))
    out, mask = orc.densify(d, b, rgb, 1, math.inf, sr)
    sp = orc.densify_spread(d, b, rgb, 1, math.inf, sr, out)
    assert out[0, 1] == pytest.approx(5.0 / 3.0, rel=1e-14)
    assert sp[0, 1] == pytest.approx(8.0 / 9.0, rel=1e-13)


def _brute(d, b, rgb, r, ss, sr):
    h, w = d.shape
    out = np.zeros((h, w))
    sp = np.zeros((h, w))
    ws = {}
    for y in range(h):
        for x in range(w):
            taps = []
            for yy in range(max(0, y - r), min(h, y + r + 1)):
                for xx in range(max(0, x - r), min(w, x + r + 1)):
                    if b[yy, xx]:
                        c = float(((rgb[y, x].astype(int) - rgb[yy, xx].astype(int)) ** 2).sum())
                        s = float((yy - y) ** 2 + (xx - x) ** 2)
                        e = -c / (2 * sr * sr) - s / (2 * ss * ss)
                        taps.append((e, float(d[yy, xx])))
            if not taps:
                continue
            em = max(e for e, _ in taps)
            wt = [(math.exp(e - em), v) for e, v in taps]
            W = sum(a for a, _ in wt)
            o = sum(a * v for a, v in wt) / W
            out[y, x] = o
            sp[y, x] = sum(a * abs(v - o) for a, v in wt) / W
            ws[(y, x)] = wt
    return out, sp, ws


@pytest.mark.parametrize("seed,r,ss,sr", [(1, 1, 1.0, 10.0), (2, 2, 1.5, 20.0),
                                          (3, 3, 2.0, 6.0)])
def test_spread_brute_force(orc, seed, r, ss, sr):
    d, b, rgb = tiny_random(np.random.default_rng(seed), 9, 11, 0.3, n_colors=3)
    out, mask = orc.densify(d, b, rgb, r, ss, sr)
    sp = orc.densify_spread(d, b, rgb, r, ss, sr, out)
    bo, bs, _ = _brute(d, b, rgb, r, ss, sr)
    np.testing.assert_allclose(sp, bs, rtol=1e-12, atol=1e-14)
    assert np.all(sp[mask == 0] == 0)


def test_spread_constant_depth_is_zero(orc):
    d, b, rgb = tiny_random(np.random.default_rng(4), 8, 8, 0.4, n_colors=3)
    d = np.where(b == 1, 4.0, 0.0).astype(np.float32)
    out, mask = orc.densify(d, b, rgb, 2, 1.5, 12.0)
    sp = orc.densify_spread(d, b, rgb, 2, 1.5, 12.0, out)
    assert np.all(sp == 0.0)


def test_spread_bounds_weight_perturbations(orc):
    """Random relative weight errors of at most e move each output by at most
    e S / (1 - e) (checked on the brute-force weights)."""
    d, b, rgb = tiny_random(np.random.default_rng(5), 9, 9, 0.35, n_colors=4)
    r, ss, sr = 2, 1.5, 15.0
    out, mask = orc.densify(d, b, rgb, r, ss, sr)
    sp = orc.densify_spread(d, b, rgb, r, ss, sr, out)
    _, _, ws = _brute(d, b, rgb, r, ss, sr)
    rng = np.random.default_rng(6)
    e = 2.0 ** -11
    for (y, x), wt in ws.items():
        for _ in range(20):
            pert = [(a * (1 + e * rng.choice([-1.0, 1.0])), v) for a, v in wt]
            o2 = sum(a * v for a, v in pert) / sum(a for a, _ in pert)
            assert abs(o2 - out[y, x]) <= (e * sp[y, x] / (1 - e) * (1 + 1e-9)
                                           + 1e-13 * abs(out[y, x]))
