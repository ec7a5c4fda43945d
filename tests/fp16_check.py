"""Acceptance of the FP16 range-weight form against the FP64 oracle.

Each range weight is 2^n times one FP16 result, v_exp_f16 of the colour
exponent's fraction f in [0, 1) rounded to FP16: at most one FP16 ulp of a
value in [1, 2] (2^-10 relative) from the exponential plus ln 2 * 2^-12
from rounding f. Since the output is a weighted mean, relative weight errors
of at most e move it by at most e S / (1 - e), where S is the oracle's
weighted mean absolute deviation of the window's depths from the output
(``oracle.densify_spread``); the FP32 sums and divide add at most the FP32
path's 1e-5 relative. Every valid pixel must lie within that bound; the
pixels above 1 mm are printed with their condition number kappa = S / out.
"""
import math

import numpy as np

import oracle

EPS_W = 2.0 ** -10 + math.log(2.0) * 2.0 ** -12


def fp16_report(out, mask, ref, rmask, d, b, rgb, r, ss, sr, label, p999_mm=None):
    """Check one FP16 result; returns max / p99.9 / mean in mm. With p999_mm,
    p99.9 of the absolute error must not exceed it."""
    np.testing.assert_array_equal(mask, rmask)
    sel = rmask == 1
    if not sel.any():
        return {"max_mm": 0.0, "p999_mm": 0.0, "mean_mm": 0.0, "n": 0}
    spread = oracle.densify_spread(d, b, rgb, r, ss, sr, ref)
    err = np.abs(out.astype(np.float64) - ref)
    bound = EPS_W * spread / (1.0 - EPS_W) + 1e-5 * np.abs(ref)
    mm = err[sel] * 1e3
    st = {"max_mm": float(mm.max()), "p999_mm": float(np.percentile(mm, 99.9)),
          "mean_mm": float(mm.mean()), "n": int(sel.sum()),
          "above_1mm": int((mm > 1.0).sum())}
    print(f"  fp16 {label}: max {st['max_mm']:.4f} mm p99.9 {st['p999_mm']:.4f} "
          f"mean {st['mean_mm']:.5f} over {st['n']} px, {st['above_1mm']} above 1 mm",
          flush=True)
    ys, xs = np.nonzero(sel & (err > 1e-3))
    order = np.argsort(-err[ys, xs])[:8]
    for k in order:
        y, x = ys[k], xs[k]
        print(f"    ({y},{x}) err {err[y, x] * 1e3:.3f} mm, out {ref[y, x]:.3f} m, "
              f"S {spread[y, x]:.3f} m, kappa {spread[y, x] / ref[y, x]:.3f}, "
              f"bound {bound[y, x] * 1e3:.3f} mm", flush=True)
    bad = sel & (err > bound)
    if bad.any():
        y, x = np.argwhere(bad)[0]
        raise AssertionError(
            f"{label}: {int(bad.sum())} pixels exceed the FP16 weight bound, e.g. "
            f"({y},{x}) err {err[y, x]:.3e} > {bound[y, x]:.3e} (S {spread[y, x]:.3e})")
    if p999_mm is not None:
        assert st["p999_mm"] <= p999_mm, (label, st)
    return st
