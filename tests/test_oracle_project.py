"""Pins for the oracle's projection and nearest-depth z-buffer (Sec. 2).

* hand-derived cases with exact binary arithmetic (tests/golden);
* a z-buffer brute force: points built to land on known pixels, winners
  chosen by numpy.lexsort over (pixel, float-Z bits, index);
* a fronto-parallel plane at Z = 2.5 that must give 2.5f everywhere it lands.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden",
                      "projection_cases.json")
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def _f32(s):
    return np.float32(float(s) if s in ("nan", "inf", "-inf")
                      else float.fromhex(s))


def _load_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def _pose(rows):
    return np.array([[float.fromhex(v) if isinstance(v, str) else float(v)
                      for v in row] for row in rows], dtype=np.float64)


@pytest.mark.parametrize("case", _load_cases(), ids=lambda c: c["name"])
def test_projection_golden(orc, case):
    pts = np.array([[_f32(v) for v in p] for p in case["points"]],
                   dtype=np.float32)
    w, h = case["width"], case["height"]
    keys, depth, valid, landed = orc.project(pts, _pose(case["pose"]),
                                             case["intrinsics"], w, h)
    exp_keys = np.full((h, w), EMPTY, dtype=np.uint64)
    exp_depth = np.zeros((h, w), np.float32)
    for e in case["expected"]:
        z = np.float32(float.fromhex(e["depth"]))
        bits = int(z.view(np.uint32))
        exp_keys[e["row"], e["col"]] = np.uint64((bits << 32) | e["index"])
        exp_depth[e["row"], e["col"]] = z
    assert landed == case["landed"]
    np.testing.assert_array_equal(keys, exp_keys)
    np.testing.assert_array_equal(depth.view(np.uint32),
                                  exp_depth.view(np.uint32))
    np.testing.assert_array_equal(valid, (exp_keys != EMPTY).astype(np.uint8))


def _points_on_known_pixels(rng, w, h, n, zvals):
    """Points with identity pose, f = 1, c = 0 that land on chosen pixels.

    X = (col + 0.5) Z with Z a power of two keeps X/Z = col + 0.5 exact, so
    the pixel of every point is known without evaluating the projection.
    """
    col = rng.integers(0, w, size=n)
    row = rng.integers(0, h, size=n)
    z = rng.choice(np.asarray(zvals, dtype=np.float64), size=n)
    pts = np.stack([(col + 0.5) * z, (row + 0.5) * z, z], axis=1)
    return pts.astype(np.float32), col, row, z.astype(np.float32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_zbuffer_matches_lexsort(orc, seed):
    rng = np.random.default_rng(seed)
    w, h, n = 7, 5, 400          # ~11 points per pixel: many collisions
    zvals = [0.25, 0.5, 1.0, 2.0, 4.0, 8.0]   # few values: many exact ties
    pts, col, row, z = _points_on_known_pixels(rng, w, h, n, zvals)
    keys, depth, valid, landed = orc.project(
        pts, np.hstack([np.eye(3), np.zeros((3, 1))]), (1.0, 1.0, 0.0, 0.0),
        w, h)
    assert landed == n
    pix = row * w + col
    zbits = z.view(np.uint32).astype(np.int64)
    order = np.lexsort((np.arange(n), zbits, pix))   # last key is primary
    first = np.ones(n, dtype=bool)
    first[1:] = pix[order][1:] != pix[order][:-1]
    win = order[first]
    exp = np.full(w * h, EMPTY, dtype=np.uint64)
    exp[pix[win]] = ((zbits[win].astype(np.uint64) << np.uint64(32))
                     | win.astype(np.uint64))
    np.testing.assert_array_equal(keys.ravel(), exp)
    exp_depth = np.zeros(w * h, np.float32)
    exp_depth[pix[win]] = z[win]
    np.testing.assert_array_equal(depth.ravel(), exp_depth)


def test_fronto_parallel_plane(orc):
    rng = np.random.default_rng(7)
    w, h = 64, 48
    fx = fy = 40.0
    n = 3000
    xy = rng.uniform(-1.5, 1.5, size=(n, 2))
    pts = np.concatenate([xy, np.full((n, 1), 2.5)], axis=1).astype(np.float32)
    keys, depth, valid, landed = orc.project(
        pts, np.hstack([np.eye(3), np.zeros((3, 1))]),
        (fx, fy, w / 2.0, h / 2.0), w, h)
    assert landed > 1000
    assert np.all(depth[valid == 1] == np.float32(2.5))
    assert np.all(depth[valid == 0] == 0.0)
    # every stored index is a real point index
    idx = (keys[valid == 1] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert np.all(idx < n)


def test_translation_moves_depth_exactly(orc):
    """Shifting the camera back by 1 along Z adds 1 to every Z (exact for
    power-of-two depths) and keeps pixels for points on the optical axis."""
    pts = np.array([[0, 0, 1], [0, 0, 2], [0, 0, 4]], np.float32)
    pose = np.hstack([np.eye(3), np.array([[0], [0], [1.0]])])
    keys, depth, valid, landed = orc.project(pts, pose, (4.0, 4.0, 4.0, 3.0),
                                             8, 6)
    assert landed == 3
    assert depth[3, 4] == np.float32(2.0)        # nearest (1 + 1)
    assert int(keys[3, 4]) & 0xFFFFFFFF == 0
