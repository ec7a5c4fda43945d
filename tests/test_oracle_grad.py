"""Pins for the oracle's gradient (Sec. 4: sigma_c, sigma_p trainable by
backpropagation), against central finite differences of the FP64 forward.

The loss is smooth, L = sum_x g(x) out(x) with a fixed random g, so the
finite differences converge to the analytic values; the held-out L1 loss of
the self-supervised fit is checked the same way away from its kinks.
"""
import math

import numpy as np
import pytest

from synth.scenes import tiny_random


def _loss(orc, d, b, rgb, r, ss, sr, g):
    out, mask = orc.densify(d, b, rgb, r, ss, sr)
    return float((g * np.where(mask == 1, out, 0.0)).sum())


CASES = [(2, 1.5, 12.0), (3, 2.0, 20.0), (1, 0.8, 6.0)]


@pytest.mark.parametrize("r,ss,sr", CASES)
def test_sigma_gradients_match_central_differences(orc, r, ss, sr):
    d, b, rgb = tiny_random(np.random.default_rng(r), 14, 15, 0.2, n_colors=3)
    g = np.random.default_rng(99).normal(size=d.shape)
    gd, gs, gr = orc.densify_grad(d, b, rgb, r, ss, sr, g)
    for which, analytic in (("s", gs), ("r", gr)):
        hs = []
        for h in (1e-3, 1e-4):
            if which == "s":
                fd = (_loss(orc, d, b, rgb, r, ss + h, sr, g)
                      - _loss(orc, d, b, rgb, r, ss - h, sr, g)) / (2 * h)
            else:
                fd = (_loss(orc, d, b, rgb, r, ss, sr + h, g)
                      - _loss(orc, d, b, rgb, r, ss, sr - h, g)) / (2 * h)
            hs.append(fd)
        # the two step sizes agree (converged), and both match the analytic
        assert analytic == pytest.approx(hs[1], rel=1e-6, abs=1e-9)
        assert analytic == pytest.approx(hs[0], rel=1e-5, abs=1e-8)


@pytest.mark.parametrize("r,ss,sr", CASES)
def test_depth_gradient_matches_differences(orc, r, ss, sr):
    d, b, rgb = tiny_random(np.random.default_rng(10 + r), 12, 13, 0.25,
                            n_colors=4)
    g = np.random.default_rng(7).normal(size=d.shape)
    gd, _, _ = orc.densify_grad(d, b, rgb, r, ss, sr, g)
    assert np.all(gd[b == 0] == 0.0)
    ys, xs = np.nonzero(b)
    for y, x in list(zip(ys, xs))[:12]:
        h = 1e-2
        dp = d.copy()
        dm = d.copy()
        dp[y, x] += np.float32(h)
        dm[y, x] -= np.float32(h)
        step = float(dp[y, x]) - float(dm[y, x])
        fd = (_loss(orc, dp, b, rgb, r, ss, sr, g)
              - _loss(orc, dm, b, rgb, r, ss, sr, g)) / step
        assert gd[y, x] == pytest.approx(fd, rel=1e-8, abs=1e-12)


def test_depth_gradient_columns_sum_to_g(orc):
    """Each output is an affine average of its samples: for one output pixel
    x, sum_j d out(x)/d D_j = 1, so with g = e_x the depth gradient sums to
    one (and is a probability vector)."""
    d, b, rgb = tiny_random(np.random.default_rng(4), 10, 10, 0.3, n_colors=3)
    out, mask = orc.densify(d, b, rgb, 2, 1.5, 10.0)
    for (y, x) in [(5, 5), (0, 9), (3, 0)]:
        if not mask[y, x]:
            continue
        g = np.zeros(d.shape)
        g[y, x] = 1.0
        gd, _, _ = orc.densify_grad(d, b, rgb, 2, 1.5, 10.0, g)
        assert gd.sum() == pytest.approx(1.0, rel=1e-14)
        assert np.all(gd >= 0)


def test_infinite_sigma_has_zero_gradient(orc):
    d, b, rgb = tiny_random(np.random.default_rng(5), 9, 9, 0.3)
    g = np.ones(d.shape)
    _, gs, gr = orc.densify_grad(d, b, rgb, 2, math.inf, math.inf, g)
    assert gs == 0.0 and gr == 0.0


def test_l1_holdout_gradient(orc):
    """Chain the L1 loss through the filter and compare with differences;
    targets sit away from the kink (|out - z| large compared to the step)."""
    rng = np.random.default_rng(12)
    d, b, rgb = tiny_random(rng, 12, 12, 0.25, n_colors=3)
    r, ss, sr = 2, 1.7, 14.0
    tv = (rng.uniform(size=d.shape) < 0.2).astype(np.uint8)
    out, mask = orc.densify(d, b, rgb, r, ss, sr)
    tz = np.where(tv == 1, out + rng.choice([-1.0, 1.0], d.shape) * 0.5,
                  0.0).astype(np.float32)
    loss, gouts = orc.l1_holdout_loss([out], [mask], [tz], [tv])
    _, gs, gr = orc.densify_grad(d, b, rgb, r, ss, sr, gouts[0])

    def L(ss_, sr_):
        o, m = orc.densify(d, b, rgb, r, ss_, sr_)
        return orc.l1_holdout_loss([o], [m], [tz], [tv])[0]

    h = 1e-4
    assert gs == pytest.approx((L(ss + h, sr) - L(ss - h, sr)) / (2 * h),
                               rel=1e-5)
    assert gr == pytest.approx((L(ss, sr + h) - L(ss, sr - h)) / (2 * h),
                               rel=1e-5)
