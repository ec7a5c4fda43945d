"""GPU checks of the sample-list builder (jbfd_densify_prepare) against the
list layout built on the host from its definition.

The lists are the filter's gather index: strip s (8 columns) lists, sorted by
row and then column, every valid sample in its halo columns
[8s - r, 8s + 8 + r); a record is {(r,g) f16x2, (b,0) f16x2, depth,
-|rgb|^2/2, table word 4 ((x - (8s - r)) + ts y)} and rowoff[s][y] is the
index of the first record of row y in strip s (rowoff[s][H] ends the strip).
Records are bit-exact data moves, so the comparison is exact. The workspace
offsets below restate the library's layout (rowoff, bandcnt and grpcnt
blocks and room for the largest spatial table, each 256-byte aligned, then
the records).
"""
import numpy as np
import pytest

from synth import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _align(x):
    return (x + 255) & ~255


def _layout(h, w):
    n_strips = (w + 7) // 8
    n_groups = (n_strips + 7) // 8
    n_bands = (h + 31) // 32
    off = _align(n_strips * (h + 1) * 4)          # after rowoff
    off = _align(off + n_strips * n_bands * 4)    # after bandcnt
    off = _align(off + n_groups * n_bands * 4)    # after grpcnt
    off = _align(off + (2 * 32 + 15) * _table_stride(32) * 4)   # after the table
    return n_strips, off


def _table_stride(r):
    return ((2 * r + 15 + 7) // 16) * 16 + 8


def _expected(depth, valid, rgb, r):
    h, w = valid.shape
    n_strips = (w + 7) // 8
    ts = _table_stride(r)
    rowoff = np.zeros((n_strips, h + 1), np.int64)
    recs = []
    c = rgb.astype(np.float32)
    nq2h = (-0.5 * (c[..., 0] ** 2 + c[..., 1] ** 2 + c[..., 2] ** 2)).astype(np.float32)
    f16 = rgb.astype(np.float16).view(np.uint16).astype(np.uint32)
    n = 0
    for s in range(n_strips):
        x0, x1 = max(8 * s - r, 0), min(8 * s + 8 + r, w)
        for y in range(h):
            rowoff[s, y] = n
            xs = x0 + np.nonzero(valid[y, x0:x1])[0]
            for x in xs:
                recs.append((f16[y, x, 0] | (f16[y, x, 1] << 16),
                             f16[y, x, 2],
                             depth[y, x:x + 1].view(np.uint32)[0],
                             nq2h[y, x:x + 1].view(np.uint32)[0],
                             4 * ((x - (8 * s - r)) + ts * y)))
            n += len(xs)
        rowoff[s, h] = n
    return rowoff, np.array(recs, np.uint32).reshape(-1, 5)


CASES = [
    # h, w, r, density
    (1, 1, 0, 1.0),
    (17, 23, 2, 0.3),
    (40, 130, 5, 0.1),
    (70, 9, 15, 0.2),         # narrower than one group, halo past both edges
    (100, 150, 15, 0.07),
    (33, 520, 7, 0.5),        # nine groups: the group prefix spans batches
    (129, 257, 32, 0.05),
    (50, 60, 4, 0.0),         # nothing valid
    (3, 32767, 32, 0.05),     # widest image: 4096 strips, 512 groups
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}r{c[2]}" for c in CASES])
def test_lists_match_layout(torch_dev, case):
    torch, dev = torch_dev
    from paper_2601_01210_amd import densify_prepare, densify_workspace
    h, w, r, dens = case
    d, b, rgb = S.tiny_random(np.random.default_rng(hash(case) & 0xFFFF), h, w,
                              dens, n_colors=6)
    n_valid = int(b.sum())
    print(f"lists {h}x{w} r={r} valid={n_valid}", flush=True)
    ws = densify_workspace(h, w, r, max(n_valid, 1), device=dev)
    ws.fill_(0xAB)
    densify_prepare(torch.from_numpy(d).to(dev), torch.from_numpy(b).to(dev),
                    torch.from_numpy(rgb).to(dev), r, ws)
    torch.cuda.synchronize()
    raw = ws.cpu().numpy()
    n_strips, rec_off = _layout(h, w)
    rowoff = raw[: n_strips * (h + 1) * 4].view(np.int32).reshape(n_strips, h + 1)
    e_rowoff, e_recs = _expected(d, b, rgb, r)
    np.testing.assert_array_equal(rowoff, e_rowoff)
    n = len(e_recs)
    recs = raw[rec_off: rec_off + n * 20].view(np.uint32).reshape(n, 5)
    np.testing.assert_array_equal(recs, e_recs)


def test_lists_fullhd_frame(torch_dev):
    """The Full-HD single-view workload at r = 15 (30 groups x 34 bands)."""
    torch, dev = torch_dev
    import oracle
    from paper_2601_01210_amd import densify_prepare, densify_workspace
    f = S.fullhd_view(S.seeded(2, 1002))
    cam = f.camera
    h, w, r = cam.height, cam.width, f.radius
    _, depth, valid, _ = oracle.project(f.points, cam.pose, cam.intrinsics(), w, h)
    depth = np.asarray(depth, np.float32).reshape(h, w)
    valid = np.asarray(valid, np.uint8).reshape(h, w)
    rgb = np.asarray(f.rgb, np.uint8).reshape(h, w, 3)
    ws = densify_workspace(h, w, r, int(valid.sum()), device=dev)
    densify_prepare(torch.from_numpy(depth).to(dev), torch.from_numpy(valid).to(dev),
                    torch.from_numpy(rgb).to(dev), r, ws)
    torch.cuda.synchronize()
    raw = ws.cpu().numpy()
    n_strips, rec_off = _layout(h, w)
    rowoff = raw[: n_strips * (h + 1) * 4].view(np.int32).reshape(n_strips, h + 1)
    # row offsets: per strip, the running count of halo samples row by row
    cnt = np.zeros((n_strips, h), np.int64)
    for s in range(n_strips):
        x0, x1 = max(8 * s - r, 0), min(8 * s + 8 + r, w)
        cnt[s] = valid[:, x0:x1].sum(axis=1)
    ends = np.cumsum(cnt.sum(axis=1))
    starts = np.concatenate([[0], ends[:-1]])
    e_rowoff = starts[:, None] + np.concatenate(
        [np.zeros((n_strips, 1), np.int64), np.cumsum(cnt, axis=1)], axis=1)
    np.testing.assert_array_equal(rowoff, e_rowoff)
    # records of a few strips in full
    ts = _table_stride(r)
    f16 = rgb.astype(np.float16).view(np.uint16).astype(np.uint32)
    for s in (0, 1, 117, n_strips - 1):
        x0, x1 = max(8 * s - r, 0), min(8 * s + 8 + r, w)
        ys, xs = np.nonzero(valid[:, x0:x1])
        xs = xs + x0
        a, z = int(rowoff[s, 0]), int(rowoff[s, h])
        recs = raw[rec_off + a * 20: rec_off + z * 20].view(np.uint32).reshape(-1, 5)
        np.testing.assert_array_equal(recs[:, 0], f16[ys, xs, 0] | (f16[ys, xs, 1] << 16))
        np.testing.assert_array_equal(recs[:, 1], f16[ys, xs, 2])
        np.testing.assert_array_equal(recs[:, 2], depth[ys, xs].view(np.uint32))
        np.testing.assert_array_equal(
            recs[:, 4], (4 * ((xs - (8 * s - r)) + ts * ys)).astype(np.uint32))
