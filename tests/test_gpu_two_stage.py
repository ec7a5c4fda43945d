"""GPU checks of the two-stage filter (Sec. 5) and of the dense kernel.

* jbfd_pool3 and jbfd_restore_merge equal the oracle bit for bit (their
  arithmetic is integer, or the same double sums in the same order);
* the dense kernel (JBFD_DENSE) against the FP64 oracle: mask bit-exact,
  depth within 1e-5 relative, at every radius 0..4, densities from sparse to
  full, infinite widths and tiny widths (the exact pass), ragged sizes; and
  against the sparse kernel on the same inputs;
* the whole two-stage filter on a Full-HD scene against the oracle's
  composition (first-pass output kept as float32 in both): masks bit-exact
  at both stages, depth within 1e-5 relative.
"""
import math

import numpy as np
import pytest

import oracle
from synth import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("h,w,dens", [(7, 8, 0.3), (90, 121, 0.07),
                                      (360, 640, 0.5), (1, 1, 1.0), (2, 5, 0.0),
                                      # 534 cells a row: three workgroups,
                                      # the last one partly outside
                                      (31, 1600, 0.3)])
def test_pool3_bit_exact(tdev, h, w, dens):
    torch, dev = tdev
    from paper_2601_01210_amd import pool3
    d, b, rgb = S.tiny_random(np.random.default_rng(h + w), h, w, dens)
    got = pool3(_dev(torch, dev, d), _dev(torch, dev, b), _dev(torch, dev, rgb))
    torch.cuda.synchronize()
    ref = oracle.pool3(d, b, rgb)
    for g, r in zip(got, ref):
        np.testing.assert_array_equal(g.cpu().numpy(), r)


def test_restore_merge_bit_exact(tdev):
    torch, dev = tdev
    from paper_2601_01210_amd import restore_merge
    rng = np.random.default_rng(12)
    h, w = 101, 130
    d, b, _ = S.tiny_random(rng, h, w, 0.1)
    o1 = rng.uniform(1, 20, size=((h + 2) // 3, (w + 2) // 3)).astype(np.float32)
    m1 = (rng.uniform(size=o1.shape) < 0.7).astype(np.uint8)
    d2, b2 = restore_merge(*[_dev(torch, dev, a) for a in (d, b, o1, m1)])
    torch.cuda.synchronize()
    rd, rb = oracle.restore_merge(d, b, o1, m1)
    np.testing.assert_array_equal(b2.cpu().numpy(), rb)
    np.testing.assert_array_equal(d2.cpu().numpy(), rd)


DENSE_CASES = [
    # h, w, r, density, sigma_s, sigma_r
    (33, 47, 0, 0.5, 1.0, 10.0),
    (40, 53, 1, 1.0, 1.0, 12.0),
    (64, 64, 2, 0.95, 2.0, 15.0),
    (71, 90, 3, 0.3, 2.0, 15.0),
    (129, 257, 4, 0.5, 2.0, 15.0),
    (50, 66, 4, 0.05, 2.0, 15.0),
    (45, 61, 2, 0.8, math.inf, 10.0),
    (45, 61, 2, 0.8, 2.0, math.inf),
    (50, 66, 3, 0.9, 0.25, 0.25),       # tiny widths: exact pass
    (1, 37, 2, 0.5, 1.0, 12.0),
    (17, 1, 4, 0.5, 1.0, 12.0),
    # below 2048 tiles of 16x32 the 8x8-tile kernel runs
    (1000, 600, 4, 0.5, 2.0, 15.0),
    (800, 700, 1, 0.9, 1.0, 12.0),
    # at least 2048 16x32 tiles: the kernel with two pixel rows per thread,
    # ragged in both directions (an odd last row leaves its thread's second
    # pixel outside the image)
    (1101, 1000, 4, 0.5, 2.0, 15.0),
    (1090, 1030, 2, 0.9, 1.0, 12.0),
    (1057, 1040, 0, 0.9, 1.0, 12.0),
    (1090, 1030, 3, 0.9, 0.25, 0.25),   # tiny widths: exact pass
]


@pytest.mark.parametrize("case", DENSE_CASES,
                         ids=[f"{c[0]}x{c[1]}r{c[2]}d{c[3]}" for c in DENSE_CASES])
def test_dense_kernel_matches_oracle(tdev, case):
    torch, dev = tdev
    from paper_2601_01210_amd import densify
    h, w, r, dens, ss, sr = case
    d, b, rgb = S.tiny_random(np.random.default_rng(h * 7 + r), h, w, dens,
                              n_colors=6)
    td, tb, tc = _dev(torch, dev, d), _dev(torch, dev, b), _dev(torch, dev, rgb)
    out, mask = densify(td, tb, tc, r, ss, sr, dense=True)
    sp, spm = densify(td, tb, tc, r, ss, sr, ws=None)
    torch.cuda.synchronize()
    ref, rmask = oracle.densify(d, b, rgb, r, ss, sr)
    out, mask = out.cpu().numpy(), mask.cpu().numpy()
    np.testing.assert_array_equal(mask, rmask)
    np.testing.assert_array_equal(spm.cpu().numpy(), rmask)
    sel = mask == 1
    if sel.any():
        rel = np.abs(out[sel] - ref[sel]) / np.abs(ref[sel])
        assert rel.max() <= 1e-5, rel.max()
        sp = sp.cpu().numpy()
        assert (np.abs(out[sel] - sp[sel]) / np.abs(sp[sel])).max() <= 2e-6
    assert np.all(out[~sel] == 0)


def test_two_stage_fullhd_matches_oracle(tdev):
    torch, dev = tdev
    from paper_2601_01210_amd import densify_two_stage, project
    f = S.fullhd_view(S.seeded(2))
    cam = f.camera
    _, d, b, _ = oracle.project(f.points, cam.pose, cam.intrinsics(),
                                cam.width, cam.height)
    params = (4, 2.0, 15.0, 2, 2.0, 15.0)
    ref, rmask, st = oracle.densify_two_stage(d, b, f.rgb, *params,
                                              want_stages=True)
    zb, td, tb = project(_dev(torch, dev, f.points), cam.pose, cam.intrinsics(),
                         cam.width, cam.height)
    out, mask = densify_two_stage(td, tb, _dev(torch, dev, f.rgb), *params)
    torch.cuda.synchronize()
    out, mask = out.cpu().numpy(), mask.cpu().numpy()
    np.testing.assert_array_equal(mask, rmask)
    sel = mask == 1
    rel = np.abs(out[sel] - ref[sel]) / np.abs(ref[sel])
    print(f"  two-stage Full-HD: valid {sel.mean():.4f} of pixels (input "
          f"{b.mean():.4f}, after pass 1 {st['valid2'].mean():.4f}), max rel "
          f"{rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-5
    assert np.all(out[~sel] == 0)


def test_two_stage_small_and_ragged(tdev):
    """Ragged sizes (partial pooling cells) and the sparse kernel for a
    first-pass radius above the dense kernel's limit."""
    torch, dev = tdev
    from paper_2601_01210_amd import densify_two_stage
    for (h, w, p) in [(100, 131, (4, 2.0, 15.0, 2, 2.0, 15.0)),
                      (29, 31, (6, 2.0, 12.0, 1, 1.0, 12.0)),
                      (5, 4, (1, 1.0, 10.0, 0, 1.0, 10.0)),
                      # second radius above the dense kernel's limit: the
                      # restored image is stored and the sparse kernel reads it
                      (61, 70, (3, 2.0, 15.0, 6, 2.0, 15.0))]:
        d, b, rgb = S.tiny_random(np.random.default_rng(h), h, w, 0.05, n_colors=5)
        ref, rmask = oracle.densify_two_stage(d, b, rgb, *p)
        out, mask = densify_two_stage(_dev(torch, dev, d), _dev(torch, dev, b),
                                      _dev(torch, dev, rgb), *p)
        torch.cuda.synchronize()
        out, mask = out.cpu().numpy(), mask.cpu().numpy()
        np.testing.assert_array_equal(mask, rmask)
        sel = mask == 1
        if sel.any():
            assert (np.abs(out[sel] - ref[sel]) / np.abs(ref[sel])).max() <= 1e-5


@pytest.mark.parametrize("h,w,r2", [(1090, 1030, 2), (100, 131, 3), (61, 70, 6)],
                         ids=["1090x1030r2", "100x131r3", "61x70r6"])
def test_two_stage_equals_its_steps(tdev, h, w, r2):
    """The two-stage call (whose dense second pass restores its input while
    staging tiles) gives bit for bit what the separate steps give: pooling,
    first pass, the stored restore, second pass."""
    torch, dev = tdev
    from paper_2601_01210_amd import densify, densify_two_stage, pool3, restore_merge
    d, b, rgb = S.tiny_random(np.random.default_rng(h * w), h, w, 0.06, n_colors=6)
    td, tb, tc = _dev(torch, dev, d), _dev(torch, dev, b), _dev(torch, dev, rgb)
    p = (4, 2.0, 15.0, r2, 2.0, 15.0)
    out, mask = densify_two_stage(td, tb, tc, *p)
    d1, b1, c1 = pool3(td, tb, tc)
    o1, m1 = densify(d1, b1, c1, p[0], p[1], p[2], dense=True)
    d2, b2 = restore_merge(td, tb, o1, m1)
    if r2 <= 4:
        o2, m2 = densify(d2, b2, tc, r2, p[4], p[5], dense=True)
    else:
        o2, m2 = densify(d2, b2, tc, r2, p[4], p[5], ws=None)
    torch.cuda.synchronize()
    print(f"two-stage steps {h}x{w} r2={r2}: valid {float(mask.float().mean()):.3f}",
          flush=True)
    assert torch.equal(mask, m2)
    assert torch.equal(out.view(torch.int32), o2.view(torch.int32))
