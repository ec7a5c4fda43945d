"""The oracle's pins must catch plausible mistakes.

Each case below plants one mistake in a copy of oracle.c (on the CPU, in a
temporary directory), builds it with the oracle's own flags, and runs the
pin suites against the mutant through ORACLE_LIB. A mutant that passes every
pin would mean the pins leave that part of the oracle unchecked.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PIN_SUITES = ["tests/test_oracle_project.py", "tests/test_oracle_filter.py",
              "tests/test_oracle_grad.py", "tests/test_oracle_two_stage.py",
              "tests/test_oracle_cloud.py", "tests/test_oracle_afterimage.py"]

# (name, text to replace, replacement, occurrences to replace or None = all)
MUTANTS = [
    ("spatial_sign", "- (s * ks)", "+ (s * ks)", None),
    ("drop_colour_term", "-(c * kr) - (s * ks)", "-(0.0 * kr) - (s * ks)", None),
    ("window_short_by_one", "for (int32_t b = -r; b <= r; ++b) {\n                const int32_t yy",
     "for (int32_t b = -r; b < r; ++b) {\n                const int32_t yy", 1),
    ("farthest_wins", "if (key < keys[pix]) keys[pix] = key;",
     "if (keys[pix] == EMPTY_KEY || key > keys[pix]) keys[pix] = key;", 1),
    ("focal_swapped", "const double u = fx * (X / Z) + cx;",
     "const double u = fy * (X / Z) + cx;", 1),
    ("principal_point_swapped", "const double v = fy * (Y / Z) + cy;",
     "const double v = fy * (Y / Z) + cx;", 1),
    ("depth_rounding_perturbed", "const float zf = (float)Z;",
     "const float zf = (float)(Z * (1.0 + 1e-7));", 1),
    ("grad_sigma_power", "1.0 / (sigma_r * sigma_r * sigma_r)",
     "1.0 / (sigma_r * sigma_r)", 1),
    ("grad_missing_centering", "ar += w * c * ((double)depth[q] - o);",
     "ar += w * c * ((double)depth[q]);", 1),
    ("grad_depth_unnormalised", "exp(-(c * kr) - (s * ks) - em) / den;",
     "exp(-(c * kr) - (s * ks) - em);", 1),
    ("invalid_samples_in_sum", "                        if (!valid[q]) continue;\n                        const double c = (double)color_dist2(rgb, p, q);\n                        const double s = (double)(a * a + b * b);\n                        const double e = -(c * kr) - (s * ks);\n                        const double w = exp(e - em);",
     "                        const double c = (double)color_dist2(rgb, p, q);\n                        const double s = (double)(a * a + b * b);\n                        const double e = -(c * kr) - (s * ks);\n                        const double w = exp(e - em);", 1),
    ("pool_divides_by_all_pixels", "(float)(sum / (double)n_valid)",
     "(float)(sum / (double)n_pix)", 1),
    ("pool_colour_truncates", "(csum[c] + n_pix / 2) / n_pix", "csum[c] / n_pix", 1),
    ("restore_cell_rounded", "(int64_t)(y / 3) * w1 + x / 3",
     "(int64_t)((y + 1) / 3) * w1 + x / 3", 1),
    ("occluded_absolute_threshold", "(double)depth[p] - mean > tau * mean",
     "(double)depth[p] - mean > tau", 1),
    ("contour_counts_invalid_neighbours", "        if (!m[q]) continue;\n        const double diff",
     "        const double diff", 1),
    ("backproject_pixel_corner", "const double Xc = ((double)x + 0.5 - cx) * Z / fx;",
     "const double Xc = ((double)x - cx) * Z / fx;", 1),
    ("backproject_pose_not_inverted", "double s = pose[0 + i] * a;\n                s = s + pose[4 + i] * b;\n                s = s + pose[8 + i] * c;",
     "double s = pose[4 * i] * a;\n                s = s + pose[4 * i + 1] * b;\n                s = s + pose[4 * i + 2] * c;", 1),
    ("motion_keeps_latest_only_outside", "if (sweep && sweep[i] != latest && motion[pix]) continue;",
     "if (sweep && sweep[i] != latest && !motion[pix]) continue;", 1),
    ("closing_erodes_at_border", "                    if (yy >= 0 && yy < h && xx >= 0 && xx < w &&\n                        !dil[(int64_t)yy * w + xx])",
     "                    if (yy < 0 || yy >= h || xx < 0 || xx >= w ||\n                        !dil[(int64_t)yy * w + xx])", 1),
    ("motion_threshold_not_squared", "raw[p] = (uint8_t)((double)c > tau * tau);",
     "raw[p] = (uint8_t)((double)c > tau);", 1),
    ("restore_prefers_first_pass", "            if (valid[p]) {\n                depth2[p] = depth[p];",
     "            if (valid[p] && !mask1[q]) {\n                depth2[p] = depth[p];", 1),
]


def _build_mutant(tmp_path, old, new, count):
    src = open(SRC).read()
    assert old in src, f"mutation anchor not found: {old!r}"
    mutated = src.replace(old, new) if count is None else src.replace(old, new, count)
    assert mutated != src
    c_path = tmp_path / "mutant.c"
    c_path.write_text(mutated)
    so = tmp_path / "libmutant.so"
    sys.path.insert(0, ROOT)
    import oracle
    subprocess.run(["gcc", *oracle.GCC_FLAGS, str(c_path), "-o", str(so),
                    "-lm"], check=True, capture_output=True)
    return so


@pytest.mark.parametrize("name,old,new,count", MUTANTS,
                         ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new, count):
    so = _build_mutant(tmp_path, old, new, count)
    env = dict(os.environ, ORACLE_LIB=str(so))
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q",
                          "-p", "no:cacheprovider", *PIN_SUITES],
                         cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=300)
    assert res.returncode != 0, (
        f"mutant {name} passed every pin:\n{res.stdout[-2000:]}")
