"""The seeded generator: determinism and workload shapes."""
import numpy as np
import pytest

from synth import scenes as S


def test_seeded_small_view_is_deterministic():
    a = S.small_view(S.seeded(1))
    b = S.small_view(S.seeded(1))
    np.testing.assert_array_equal(a.points, b.points)
    np.testing.assert_array_equal(a.rgb, b.rgb)
    c = S.small_view(S.seeded(1, seed=5))
    assert not np.array_equal(a.rgb, c.rgb)


def test_small_view_shape(orc):
    f = S.small_view(S.seeded(1))
    assert f.rgb.shape == (240, 320, 3) and f.rgb.dtype == np.uint8
    assert f.points.dtype == np.float32 and f.points.shape[1] == 3
    _, _, valid, landed = orc.project(f.points, f.camera.pose,
                                      f.camera.intrinsics(), 320, 240)
    assert 1500 < landed < 8000          # about 4k in-view hits
    assert (f.radius, f.sigma_s, f.sigma_r) == (5, 3.0, 12.0)


def test_widened_scan_reaches_count():
    rng = np.random.default_rng(3)
    f = S.small_view(rng, 640, 360, n_points=20000)
    assert len(f.points) == 20000


def test_holdout_split():
    m = S.holdout_split(np.random.default_rng(0), 1000, 0.1)
    assert m.sum() == 100


def test_log_uniform_range():
    rng = np.random.default_rng(0)
    v = [S.log_uniform_int(rng, 20000, 250000) for _ in range(200)]
    assert min(v) >= 20000 and max(v) <= 250000


def test_random_pose_is_rigid_and_invertible():
    rng = np.random.default_rng(4)
    f = S.small_view(rng, 64, 48, n_points=500)
    g = S.with_random_pose(f, rng)
    R, t = g.camera.pose[:, :3], g.camera.pose[:, 3]
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-12)
    assert np.linalg.det(R) == pytest.approx(1.0)
    back = g.points.astype(np.float64) @ R.T + t          # camera frame again
    np.testing.assert_allclose(back, f.points, atol=1e-4)


def test_serving_specs_and_arrivals():
    rng = np.random.default_rng(5)
    specs = S.serving_specs(rng, 64)
    assert all((w, h) in S.SERVING_SIZES for w, h, _, _ in specs)
    assert all(50000 <= n <= 400000 for _, _, n, _ in specs)
    arr = S.arrival_times(np.random.default_rng(6), 16, 20.0)
    ts = np.array([t for t, _ in arr])
    assert np.all(np.diff(ts) >= 0) and ts.max() < 20.0
    # 16 viewpoints at 30 Hz for 20 s: about 9600 frames (Poisson)
    assert abs(len(arr) - 9600) < 5 * np.sqrt(9600)
    per = np.bincount([v for _, v in arr], minlength=16)
    assert per.min() > 500
