"""Pins for the oracle's occluded-point removal (Sec. 4.1) and for contour
removal with back-projection to a coloured cloud (Sec. 5, Sec. 2).

Occlusion: a pure-Python brute force on tiny images, scipy window sums on a
larger one, and closed forms (an isolated sample is kept, a far sample
inside a near patch is dropped, constant depth keeps everything).
Back-projection: closed form on a fronto-parallel plane, agreement with a
numpy transform for a random pose, the round trip through the oracle's own
projection (a different function), a step edge for the contour rule, and
row-major order of the output.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import scenes as S


def brute_occluded(d, b, k, tau):
    h, w = d.shape
    out = np.zeros((h, w), np.uint8)
    for y in range(h):
        for x in range(w):
            if not b[y, x]:
                continue
            vals = [float(d[yy, xx]) for yy in range(max(0, y - k), min(h, y + k + 1))
                    for xx in range(max(0, x - k), min(w, x + k + 1)) if b[yy, xx]]
            mean = sum(vals) / len(vals)
            out[y, x] = 0 if float(d[y, x]) - mean > tau * mean else 1
    return out


@pytest.mark.parametrize("h,w,dens,k", [(9, 11, 0.3, 1), (12, 7, 0.6, 2),
                                        (5, 5, 1.0, 3), (1, 9, 0.5, 2)])
def test_occluded_brute_force(h, w, dens, k):
    d, b, _ = S.tiny_random(np.random.default_rng(h * w + k), h, w, dens)
    np.testing.assert_array_equal(oracle.remove_occluded(d, b, k, 0.1),
                                  brute_occluded(d, b, k, 0.1))


def test_occluded_matches_window_sums():
    d, b, _ = S.tiny_random(np.random.default_rng(2), 80, 90, 0.1)
    k, tau = 3, 0.1
    ones = np.ones((2 * k + 1,) * 2)
    s = ndimage.correlate((d.astype(np.float64) * b), ones, mode="constant")
    n = ndimage.correlate(b.astype(np.float64), ones, mode="constant")
    mean = np.divide(s, n, out=np.zeros_like(s), where=n > 0)
    exp = ((b == 1) & ~(d - mean > tau * mean)).astype(np.uint8)
    np.testing.assert_array_equal(oracle.remove_occluded(d, b, k, tau), exp)


def test_occluded_closed_forms():
    h, w = 15, 15
    d = np.full((h, w), 5.0, np.float32)
    b = np.zeros((h, w), np.uint8)
    b[4:11, 4:11] = 1
    d[7, 7] = 20.0                      # a far sample inside a near patch
    b[0, 14], d[0, 14] = 1, 30.0        # an isolated sample
    out = oracle.remove_occluded(d, b, 3, 0.1)
    assert out[7, 7] == 0                # 20 - (48*5+20)/49 > 0.1 * mean
    assert out[0, 14] == 1               # mean of itself
    assert out[4:11, 4:11].sum() == 48   # every near sample kept
    flat = np.full((h, w), 3.5, np.float32)
    assert np.array_equal(oracle.remove_occluded(flat, b, 2, 0.0), b)


def _cam(w, h):
    c = S.Camera.pinhole(w, h)
    return c, np.array([c.fx, c.fy, c.cx, c.cy])


def test_backproject_plane_closed_form():
    h, w = 20, 30
    cam, K = _cam(w, h)
    z = np.float32(4.25)
    dense = np.full((h, w), z, np.float32)
    mask = np.ones((h, w), np.uint8)
    mask[::3, ::2] = 0
    rgb = np.random.default_rng(3).integers(0, 256, (h, w, 3), dtype=np.uint8)
    xyz, col = oracle.backproject(dense, mask, rgb, cam.pose, K, 0.05)
    ys, xs = np.nonzero(mask)            # row-major order
    exp = np.stack([(xs + 0.5 - K[2]) * float(z) / K[0],
                    (ys + 0.5 - K[3]) * float(z) / K[1],
                    np.full(xs.shape, float(z))], 1).astype(np.float32)
    assert len(xyz) == mask.sum()
    np.testing.assert_array_equal(xyz, exp)
    np.testing.assert_array_equal(col, rgb[ys, xs])


def test_backproject_random_pose_and_round_trip():
    rng = np.random.default_rng(4)
    h, w = 48, 64
    cam, K = _cam(w, h)
    R = S.random_rotation(rng)
    t = rng.uniform(-3, 3, 3)
    pose = np.hstack([R, t[:, None]])
    dense = rng.uniform(1, 20, (h, w)).astype(np.float32)
    mask = (rng.uniform(size=(h, w)) < 0.5).astype(np.uint8)
    rgb = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    xyz, col = oracle.backproject(dense, mask, rgb, pose, K, np.inf)
    ys, xs = np.nonzero(mask)
    z = dense[ys, xs].astype(np.float64)
    pc = np.stack([(xs + 0.5 - K[2]) * z / K[0], (ys + 0.5 - K[3]) * z / K[1], z], 1)
    np.testing.assert_allclose(xyz, ((pc - t) @ R).astype(np.float32), rtol=0,
                               atol=2e-6 * np.abs(pc).max())
    # projecting the cloud with the same pose lands every point in its pixel
    keys, d2, v2, landed = oracle.project(xyz, pose, K, w, h)
    assert landed == len(xyz)
    np.testing.assert_array_equal(v2, mask)
    np.testing.assert_allclose(d2[mask == 1], dense[mask == 1], rtol=1e-5)


def test_contour_step_edge():
    h, w = 10, 12
    cam, K = _cam(w, h)
    dense = np.where(np.arange(w)[None, :] < 6, 5.0, 10.0).astype(np.float32)
    dense = np.repeat(dense, h, 0)
    mask = np.ones((h, w), np.uint8)
    rgb = np.zeros((h, w, 3), np.uint8)
    xyz, _ = oracle.backproject(dense, mask, rgb, cam.pose, K, 0.05)
    assert len(xyz) == h * w - 2 * h    # both columns beside the step go
    xyz2, _ = oracle.backproject(dense, mask, rgb, cam.pose, K, 1.5)
    assert len(xyz2) == h * w           # a loose threshold keeps them
    # an invalid neighbour does not count as a jump
    m = mask.copy()
    m[:, 6] = 0
    xyz3, _ = oracle.backproject(dense, m, rgb, cam.pose, K, 0.05)
    assert len(xyz3) == m.sum()         # columns 5 and 7 face an invalid gap
