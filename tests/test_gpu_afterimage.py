"""GPU checks of afterimage removal (Sec. 4.1) against the oracle.

* jbfd_motion_mask equals the oracle's closed mask bit for bit (integer
  distances against tau^2 in double on both sides), over closing sizes
  0..16, ragged and degenerate image shapes, and a Full-HD frame pair;
* jbfd_project_motion equals the oracle's motion-aware projection bit for
  bit (keys, depth, mask) on a moving-object scene, with the oracle's mask
  and with the GPU's own mask;
* the composition mask -> projection -> filter against the oracle's.
"""
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


def _pair(rng, h, w, frac):
    a = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    b = a.copy()
    ch = rng.uniform(size=(h, w)) < frac
    b[ch] = rng.integers(0, 256, (int(ch.sum()), 3), dtype=np.uint8)
    return a, b


# h, w, closing size k, tau, fraction of changed pixels; the workgroup
# tile is 64 - 4k wide for k <= 8 and 128 - 4k wide above, 32 rows tall
MASK_CASES = [(40, 57, 0, 50.0, 0.12), (40, 57, 1, 50.0, 0.12),
              (64, 90, 2, 60.0, 0.12), (33, 31, 5, 40.0, 0.02),
              (100, 140, 8, 40.0, 0.002), (100, 150, 9, 40.0, 0.002),
              (70, 70, 16, 30.0, 0.12), (130, 300, 16, 30.0, 0.001),
              (1, 1, 3, 10.0, 0.5), (1, 77, 2, 10.0, 0.12),
              (55, 1, 2, 10.0, 0.12), (20, 20, 2, 0.0, 0.12)]


@pytest.mark.parametrize("h,w,k,tau,frac", MASK_CASES,
                         ids=[f"{c[0]}x{c[1]}k{c[2]}" for c in MASK_CASES])
def test_motion_mask_bit_exact(tdev, h, w, k, tau, frac):
    torch, dev = tdev
    from paper_2601_01210_amd import motion_mask
    a, b = _pair(np.random.default_rng(h * 31 + k), h, w, frac)
    got = motion_mask(_dev(torch, dev, a), _dev(torch, dev, b), tau, k)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.motion_mask(a, b, tau, k))


def test_motion_mask_fullhd(tdev):
    torch, dev = tdev
    from paper_2601_01210_amd import motion_mask
    a, b = _pair(np.random.default_rng(5), 1080, 1920, 0.01)
    # a moving block as well as scattered changes
    b[300:500, 700:1000] = 255 - b[300:500, 700:1000]
    got = motion_mask(_dev(torch, dev, a), _dev(torch, dev, b), 60.0, 2)
    torch.cuda.synchronize()
    ref = oracle.motion_mask(a, b, 60.0, 2)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    print(f"  Full-HD motion mask: {ref.mean():.4f} of pixels moving", flush=True)


def _scene():
    return S.moving_view(S.seeded(6, 4006))


@pytest.mark.parametrize("latest", [2, 0])
def test_project_motion_bit_exact(tdev, latest):
    torch, dev = tdev
    from paper_2601_01210_amd import motion_mask, project_motion
    f, prev = _scene()
    c = f.camera
    args = (c.pose, c.intrinsics()[:4], c.width, c.height)
    ref_mask = oracle.motion_mask(f.rgb, prev, 60.0, 2)
    gmask = motion_mask(_dev(torch, dev, f.rgb), _dev(torch, dev, prev), 60.0, 2)
    pts, sw = _dev(torch, dev, f.points), _dev(torch, dev, f.sweep_id)
    for m in (_dev(torch, dev, ref_mask), gmask):
        zb, d, v = project_motion(pts, sw, latest, m, *args)
        torch.cuda.synchronize()
        keys, rd, rv, _ = oracle.project_motion(f.points, f.sweep_id, latest,
                                                ref_mask, *args)
        np.testing.assert_array_equal(zb.cpu().numpy().view(np.uint64), keys)
        np.testing.assert_array_equal(d.cpu().numpy(), rd)
        np.testing.assert_array_equal(v.cpu().numpy(), rv)


def test_project_motion_empty_cloud(tdev):
    torch, dev = tdev
    from paper_2601_01210_amd import project_motion
    m = torch.ones((6, 8), dtype=torch.uint8, device=dev)
    pts = torch.empty((0, 3), dtype=torch.float32, device=dev)
    sw = torch.empty((0,), dtype=torch.int8, device=dev)
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    zb, d, v = project_motion(pts, sw, 0, m, pose, (4.0, 4.0, 4.0, 3.0), 8, 6)
    torch.cuda.synchronize()
    assert int(v.sum()) == 0 and float(d.abs().sum()) == 0.0


def test_afterimage_pipeline_matches_oracle(tdev):
    torch, dev = tdev
    from paper_2601_01210_amd import densify, motion_mask, project_motion
    f, prev = _scene()
    c = f.camera
    args = (c.pose, c.intrinsics()[:4], c.width, c.height)
    gmask = motion_mask(_dev(torch, dev, f.rgb), _dev(torch, dev, prev), 60.0, 2)
    _, d, v = project_motion(_dev(torch, dev, f.points), _dev(torch, dev, f.sweep_id),
                             2, gmask, *args)
    out, mask = densify(d, v, _dev(torch, dev, f.rgb), f.radius, f.sigma_s,
                        f.sigma_r)
    torch.cuda.synchronize()
    rm = oracle.motion_mask(f.rgb, prev, 60.0, 2)
    _, rd, rv, _ = oracle.project_motion(f.points, f.sweep_id, 2, rm, *args)
    ref, rmask = oracle.densify(rd, rv, f.rgb, f.radius, f.sigma_s, f.sigma_r)
    out, mask = out.cpu().numpy(), mask.cpu().numpy()
    np.testing.assert_array_equal(mask, rmask)
    sel = mask == 1
    assert (np.abs(out[sel] - ref[sel]) / np.abs(ref[sel])).max() <= 1e-5
