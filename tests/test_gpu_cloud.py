"""GPU checks of occluded-point removal and of contour removal with
back-projection: both are integer decisions taken in double with the
oracle's operation order, so masks, point counts, point order, coordinates
and colours must equal the FP64 oracle bit for bit."""
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


@pytest.mark.parametrize("h,w,dens,k,tau", [(9, 11, 0.3, 1, 0.1),
                                            (70, 90, 0.1, 3, 0.1),
                                            (33, 17, 0.6, 8, 0.05),
                                            (1, 40, 0.5, 2, 0.2),
                                            (40, 40, 1.0, 0, 0.1),
                                            (100, 150, 0.2, 8, 0.05),
                                            (17, 130, 0.3, 5, 0.1),
                                            (50, 1, 0.7, 3, 0.1)])
def test_remove_occluded_bit_exact(tdev, h, w, dens, k, tau):
    torch, dev = tdev
    from paper_2601_01210_amd import remove_occluded
    d, b, _ = S.tiny_random(np.random.default_rng(h * k + w), h, w, dens)
    got = remove_occluded(_dev(torch, dev, d), _dev(torch, dev, b), k, tau)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(),
                                  oracle.remove_occluded(d, b, k, np.float32(tau)))


def test_remove_occluded_on_a_scene(tdev):
    torch, dev = tdev
    from paper_2601_01210_amd import remove_occluded
    f = S.fullhd_view(S.seeded(2))
    c = f.camera
    _, d, b, _ = oracle.project(f.points, c.pose, c.intrinsics(), c.width, c.height)
    got = remove_occluded(_dev(torch, dev, d), _dev(torch, dev, b), 3, 0.1)
    torch.cuda.synchronize()
    ref = oracle.remove_occluded(d, b, 3, np.float32(0.1))
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    print(f"  occluded samples dropped: {int(b.sum() - ref.sum())} of {int(b.sum())}",
          flush=True)


@pytest.mark.parametrize("tau", [0.03, float("inf")])
def test_backproject_bit_exact(tdev, tau):
    torch, dev = tdev
    from paper_2601_01210_amd import backproject, densify, project
    f = S.serving_view((640, 360, 20000, 77))        # a random world pose
    c = f.camera
    zb, td, tb = project(_dev(torch, dev, f.points), c.pose, c.intrinsics(),
                         c.width, c.height)
    rgb = _dev(torch, dev, f.rgb)
    out, mask = densify(td, tb, rgb, 5, 3.0, 12.0)
    xyz, col, cnt = backproject(out, mask, rgb, c.pose, c.intrinsics()[:4], tau)
    torch.cuda.synchronize()
    n = int(cnt.item())
    rx, rc = oracle.backproject(out.cpu().numpy(), mask.cpu().numpy(), f.rgb,
                                c.pose, c.intrinsics()[:4], np.float32(tau))
    assert n == len(rx)
    np.testing.assert_array_equal(xyz[:n].cpu().numpy(), rx)
    np.testing.assert_array_equal(col[:n].cpu().numpy(), rc)
    print(f"  tau={tau}: {n} points of {int(mask.sum())} valid pixels", flush=True)


def test_backproject_ragged_and_empty(tdev):
    torch, dev = tdev
    from paper_2601_01210_amd import backproject
    rng = np.random.default_rng(9)
    # chunks of 1024 pixels straddle rows; widths below four put several
    # rows into one thread's four pixels
    for h, w, dens in [(37, 29, 0.5), (5, 3, 1.0), (8, 8, 0.0), (1, 3000, 0.6),
                       (3000, 1, 0.6), (700, 2, 0.8), (61, 67, 0.9), (2, 2, 1.0)]:
        yy, xx = np.mgrid[0:h, 0:w]
        # a smooth ramp (kept by the contour rule) with random jumps
        dense = (5.0 + 0.01 * xx + 0.02 * yy).astype(np.float32)
        jump = rng.uniform(size=(h, w)) < 0.05
        dense[jump] += rng.uniform(1, 5, int(jump.sum())).astype(np.float32)
        mask = (rng.uniform(size=(h, w)) < dens).astype(np.uint8)
        dense[mask == 0] = 0
        rgb = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
        cam = S.Camera.pinhole(w, h)
        K = (cam.fx, cam.fy, cam.cx, cam.cy)
        xyz, col, cnt = backproject(*[_dev(torch, dev, a) for a in (dense, mask, rgb)],
                                    cam.pose, K, 0.1)
        torch.cuda.synchronize()
        rx, rc = oracle.backproject(dense, mask, rgb, cam.pose, K, np.float32(0.1))
        n = int(cnt.item())
        assert n == len(rx)
        np.testing.assert_array_equal(xyz[:n].cpu().numpy(), rx)
        np.testing.assert_array_equal(col[:n].cpu().numpy(), rc)
