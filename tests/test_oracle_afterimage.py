"""Pins for the oracle's afterimage removal (Sec. 4.1): the motion mask
against scipy morphology, the motion-aware projection against the plain
projection in the limiting cases and against an independent per-point
pixel computation, and the effect on a scene with a moving object
(ghost points of older sweeps disappear)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import scenes as S


@pytest.mark.parametrize("k", [0, 1, 3])
def test_motion_mask_is_a_closing(k):
    rng = np.random.default_rng(k)
    a = rng.integers(0, 256, (40, 57, 3), dtype=np.uint8)
    b = a.copy()
    noise = rng.uniform(size=(40, 57)) < 0.15
    b[noise] = rng.integers(0, 256, (int(noise.sum()), 3), dtype=np.uint8)
    tau = 50.0
    raw = ((a.astype(np.int64) - b) ** 2).sum(-1) > tau * tau
    se = np.ones((2 * k + 1,) * 2, bool)
    dil = ndimage.binary_dilation(raw, se, border_value=0)
    closed = ndimage.binary_erosion(dil, se, border_value=1)
    np.testing.assert_array_equal(oracle.motion_mask(a, b, tau, k),
                                  closed.astype(np.uint8))


def test_motion_mask_limits():
    a = np.random.default_rng(1).integers(0, 256, (9, 11, 3), dtype=np.uint8)
    assert oracle.motion_mask(a, a, 0.0, 2).sum() == 0        # no change
    m = oracle.motion_mask(np.zeros_like(a), np.full_like(a, 200), 10.0, 2)
    assert m.sum() == m.size                                   # all changed
    # a single changed pixel survives a closing (closing is extensive)
    b = a.copy()
    b[4, 5] = 255 - b[4, 5]
    m = oracle.motion_mask(a, b, 1.0, 3)
    assert m[4, 5] == 1


def _scene():
    return S.moving_view(S.seeded(6, 4006))


def test_project_motion_limits():
    f, prev = _scene()
    c = f.camera
    args = (c.pose, c.intrinsics()[:4], c.width, c.height)
    keys, d, v, landed = oracle.project(f.points, *args)
    none = np.zeros((c.height, c.width), np.uint8)
    k2, d2, v2, l2 = oracle.project_motion(f.points, f.sweep_id, 2, none, *args)
    np.testing.assert_array_equal(k2, keys)
    assert l2 == landed
    # everything moving: only the latest sweep survives
    allm = np.ones_like(none)
    k3, d3, v3, _ = oracle.project_motion(f.points, f.sweep_id, 2, allm, *args)
    idx = np.nonzero(f.sweep_id == 2)[0]
    k4, d4, v4, _ = oracle.project(f.points[idx], *args)
    np.testing.assert_array_equal(v3, v4)
    np.testing.assert_array_equal(d3, d4)
    hit = v4 == 1
    np.testing.assert_array_equal((k3[hit] & 0xFFFFFFFF),
                                  idx[(k4[hit] & 0xFFFFFFFF).astype(np.int64)])


def test_project_motion_drops_exactly_older_points_in_the_mask():
    f, prev = _scene()
    c = f.camera
    motion = oracle.motion_mask(f.rgb, prev, 60.0, 2)
    # pixel of every point, computed independently in float64 numpy
    p = f.points.astype(np.float64)
    R, t = c.pose[:, :3], c.pose[:, 3]
    X = ((R[0, 0] * p[:, 0] + R[0, 1] * p[:, 1]) + R[0, 2] * p[:, 2]) + t[0]
    Y = ((R[1, 0] * p[:, 0] + R[1, 1] * p[:, 1]) + R[1, 2] * p[:, 2]) + t[1]
    Z = ((R[2, 0] * p[:, 0] + R[2, 1] * p[:, 1]) + R[2, 2] * p[:, 2]) + t[2]
    u = c.fx * (X / Z) + c.cx
    v = c.fy * (Y / Z) + c.cy
    ok = (Z > 0) & (u >= 0) & (u < c.width) & (v >= 0) & (v < c.height)
    col = np.floor(np.where(ok, u, 0)).astype(np.int64)
    row = np.floor(np.where(ok, v, 0)).astype(np.int64)
    drop = ok & (f.sweep_id != 2) & (motion[row, col] == 1)
    keep = ok & ~drop
    _, d1, v1, l1 = oracle.project_motion(f.points, f.sweep_id, 2, motion,
                                          c.pose, c.intrinsics()[:4], c.width,
                                          c.height)
    assert l1 == int(keep.sum())
    assert drop.sum() > 0


def test_afterimage_removal_reduces_ghost_depths():
    f, prev = _scene()
    c = f.camera
    args = (c.pose, c.intrinsics()[:4], c.width, c.height)
    _, d0, v0, _ = oracle.project(f.points, *args)
    motion = oracle.motion_mask(f.rgb, prev, 60.0, 2)
    _, d1, v1, _ = oracle.project_motion(f.points, f.sweep_id, 2, motion, *args)
    gt = f.gt_depth

    def ghosts(d, v):
        sel = (v == 1) & (gt > 0)
        return int((np.abs(d[sel] - gt[sel]) > 0.5).sum())
    # the latest sweep alone sets the floor (LiDAR-camera parallax at depth
    # edges and range noise); the older sweeps' ghosts are the excess, and
    # at least half of it must go (the sweep two steps back lies partly
    # outside a mask built from two consecutive frames)
    idx = np.nonzero(f.sweep_id == 2)[0]
    _, dl, vl, _ = oracle.project(f.points[idx], *args)
    g0, g1, floor = ghosts(d0, v0), ghosts(d1, v1), ghosts(dl, vl)
    assert g0 - floor > 1000, (g0, floor)
    assert g1 - floor < 0.5 * (g0 - floor), (g0, g1, floor)
