"""The seeded generator: determinism and workload shapes."""
import numpy as np

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
