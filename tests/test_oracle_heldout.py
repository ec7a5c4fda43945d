"""Pins for the oracle's held-out L1 loss of the width fit (Sec. 4: the
filter widths are trainable by backpropagation; the held-out supervision is
the fit's reading: L1 with sign(0) = 0, targets on invalid output pixels
skipped, one mean over the contributing targets of all frames).

The expected values are worked out by hand (tests/golden/heldout_l1_cases.json);
plausible mistakes planted in a copy of the oracle's function (counting
targets on invalid pixels, averaging over every target, dropping the 1/n of
the gradient, sign(0) = 1, a reversed difference) each fail a case.
"""
import inspect
import json
import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "heldout_l1_cases.json")))["cases"]


def _frames(case):
    outs = [np.array(f["out"], np.float64) for f in case["frames"]]
    masks = [np.array(f["mask"], np.uint8) for f in case["frames"]]
    tgts = [np.array(f["target"], np.float32) for f in case["frames"]]
    tvs = [np.array(f["target_valid"], np.uint8) for f in case["frames"]]
    return outs, masks, tgts, tvs


def _check(fn, case):
    loss, grads = fn(*_frames(case))
    assert loss == pytest.approx(float(Fraction(case["loss"])), rel=1e-15, abs=0)
    assert len(grads) == len(case["frames"])
    for g, eg in zip(grads, case["grad"]):
        exp = np.array([[float(Fraction(v)) for v in row] for row in eg])
        np.testing.assert_allclose(g, exp, rtol=1e-15, atol=0)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_heldout_l1_golden(orc, case):
    _check(orc.l1_holdout_loss, case)


MUTANTS = [
    ("targets_on_invalid_pixels_count", "(tv == 1) & (m == 1)", "(tv == 1) | (m > 1)"),
    ("mean_over_every_target", "n = int(sum(int(u.sum()) for u in use))",
     "n = int(sum(int(t.sum()) for t in target_valid))"),
    ("gradient_without_one_over_n", "grads.append(np.sign(diff) / n)",
     "grads.append(np.sign(diff))"),
    ("sign_of_zero_is_one", "np.sign(diff) / n",
     "np.where(diff >= 0, 1.0, -1.0) / n"),
    ("reversed_difference", "o - t.astype(np.float64)", "t.astype(np.float64) - o"),
]


def _mutant(orc, old, new):
    src = inspect.getsource(orc.l1_holdout_loss)
    assert old in src, f"mutation site {old!r} not found"
    ns = {"np": np}
    exec(src.replace(old, new, 1), ns)
    return ns["l1_holdout_loss"]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_heldout_l1_mutant_fails_a_case(orc, name, old, new):
    fn = _mutant(orc, old, new)
    caught = 0
    for case in CASES:
        try:
            _check(fn, case)
        except AssertionError:
            caught += 1
    assert caught >= 1, f"mutant {name} passes every golden case"


def test_heldout_chain_matches_differences_of_the_loss(orc):
    """The upstream gradient of the golden loss, chained through the
    oracle's filter gradient, equals central differences of the loss in the
    widths (targets kept away from the L1 kinks)."""
    from synth.scenes import tiny_random
    rng = np.random.default_rng(21)
    frames = []
    for _ in range(2):
        d, b, rgb = tiny_random(rng, 11, 13, 0.3, n_colors=3)
        tv = (rng.uniform(size=d.shape) < 0.3).astype(np.uint8)
        frames.append((d, b, rgb, tv))
    r, ss, sr = 2, 1.6, 13.0
    outs = [orc.densify(d, b, c, r, ss, sr) for d, b, c, _ in frames]
    tz = [np.where(tv == 1, o + rng.choice([-0.7, 0.7], o.shape), 0.0).astype(np.float32)
          for (o, _), (_, _, _, tv) in zip(outs, frames)]

    def L(ss_, sr_):
        oo = [orc.densify(d, b, c, r, ss_, sr_) for d, b, c, _ in frames]
        return orc.l1_holdout_loss([o for o, _ in oo], [m for _, m in oo], tz,
                                   [f[3] for f in frames])[0]

    loss, g = orc.l1_holdout_loss([o for o, _ in outs], [m for _, m in outs], tz,
                                  [f[3] for f in frames])
    gs = gr = 0.0
    for (d, b, c, _), gf in zip(frames, g):
        _, a, bb = orc.densify_grad(d, b, c, r, ss, sr, gf)
        gs += a
        gr += bb
    h = 1e-4
    assert gs == pytest.approx((L(ss + h, sr) - L(ss - h, sr)) / (2 * h), rel=1e-5)
    assert gr == pytest.approx((L(ss, sr + h) - L(ss, sr - h)) / (2 * h), rel=1e-5)
    assert loss > 0
