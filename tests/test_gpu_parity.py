"""GPU parity against the FP64 oracle, through the C ABI.

* projection: z-buffer keys (depth bits | point index), sparse depth and
  mask bit-exact, on hand-built edge cases, adversarial pixel-edge points
  and the seeded scenes;
* filter (FP32): mask bit-exact; every valid pixel within 1e-5 relative of
  the oracle; depth 0 where the mask is 0; on ragged sizes that span
  several tiles, radius 0..32, empty and fully dense inputs, extreme sigmas,
  and full-size small and Full-HD frames.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from synth import scenes as S

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _gpu_project(torch, dev, pts, pose, intr, w, h):
    from paper_2601_01210_amd import project
    p = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).to(dev)
    zbuf, depth, valid = project(p, pose, intr, w, h)
    torch.cuda.synchronize()
    return (zbuf.cpu().numpy().view(np.uint64), depth.cpu().numpy(),
            valid.cpu().numpy())


def _check_projection(torch, dev, pts, pose, intr, w, h):
    keys, depth, valid, _ = oracle.project(pts, pose, intr, w, h)
    gk, gd, gv = _gpu_project(torch, dev, pts, pose, intr, w, h)
    np.testing.assert_array_equal(gk, keys)
    np.testing.assert_array_equal(gd.view(np.uint32), depth.view(np.uint32))
    np.testing.assert_array_equal(gv, valid)
    return keys


def test_project_golden_cases(torch_dev):
    torch, dev = torch_dev
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "projection_cases.json")
    for case in json.load(open(path))["cases"]:
        pts = np.array([[np.float32(float(v) if v in ("nan", "inf") else
                                    float.fromhex(v)) for v in p]
                        for p in case["points"]], np.float32)
        pose = np.array([[float.fromhex(v) if isinstance(v, str) else float(v)
                          for v in row] for row in case["pose"]])
        print("golden case", case["name"], flush=True)
        _check_projection(torch, dev, pts, pose, case["intrinsics"],
                          case["width"], case["height"])


def test_project_pixel_edges(torch_dev):
    """Points whose u, v sit exactly on, or one float32 step either side of,
    pixel edges; depths from a few values so that exact ties occur."""
    torch, dev = torch_dev
    rng = np.random.default_rng(0)
    w, h = 97, 61
    n = 20000
    col = rng.integers(-1, w + 1, size=n).astype(np.float64)
    row = rng.integers(-1, h + 1, size=n).astype(np.float64)
    z = rng.choice([0.5, 1.0, 2.0, 3.0, 7.25], size=n)
    x = np.float32((col - w / 2.0) * z / 40.0)
    y = np.float32((row - h / 2.0) * z / 40.0)
    nudge = rng.integers(-1, 2, size=(n, 2))
    x = np.nextafter(x, np.float32(np.inf) * nudge[:, 0]).astype(np.float32)
    y = np.nextafter(y, np.float32(np.inf) * nudge[:, 1]).astype(np.float32)
    pts = np.stack([x, y, z.astype(np.float32)], axis=1)
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    _check_projection(torch, dev, pts, pose, (40.0, 40.0, w / 2.0, h / 2.0),
                      w, h)


def test_project_rotated_pose_random(torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(1)
    a = 0.3
    rot = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0],
                    [-math.sin(a), 0, math.cos(a)]])
    pose = np.hstack([rot, np.array([[0.1], [-0.2], [0.5]])])
    pts = rng.normal(0, 3, size=(50000, 3)).astype(np.float32)
    pts[:, 2] = np.abs(pts[:, 2]) + 0.5
    pts[::97] = np.nan
    pts[1::89, 2] = -1.0
    _check_projection(torch, dev, pts, pose, (300.0, 280.0, 320.0, 240.0),
                      640, 480)


def test_project_empty_and_keys_only(torch_dev):
    torch, dev = torch_dev
    from paper_2601_01210_amd import project
    pts = torch.zeros((0, 3), dtype=torch.float32, device=dev)
    zbuf, d, v = project(pts, np.hstack([np.eye(3), np.zeros((3, 1))]),
                         (4.0, 4.0, 4.0, 3.0), 8, 6)
    torch.cuda.synchronize()
    assert np.all(zbuf.cpu().numpy().view(np.uint64) == np.uint64(2 ** 64 - 1))
    assert np.all(d.cpu().numpy() == 0) and np.all(v.cpu().numpy() == 0)
    pts = torch.tensor([[0.0, 0.0, 2.0]], device=dev)
    zbuf, d, v = project(pts, np.hstack([np.eye(3), np.zeros((3, 1))]),
                         (4.0, 4.0, 4.0, 3.0), 8, 6, want_sparse=False)
    torch.cuda.synchronize()
    assert d is None and v is None
    k = zbuf.cpu().numpy().view(np.uint64)
    assert k[3, 4] == (np.float32(2.0).view(np.uint32).astype(np.uint64) << 32)


@pytest.mark.parametrize("w,h", [(1920, 1080), (97, 61), (1, 1), (3, 7)])
def test_project_recycled_frame_loop(torch_dev, w, h):
    """jbfd_project_recycled over a loop of frames that reuses one key
    buffer: each frame's depth and mask equal the oracle's bit for bit
    (no key of an earlier frame survives), and the buffer holds only empty
    keys after every frame. Odd sizes take the decode's per-pixel path."""
    torch, dev = torch_dev
    from paper_2601_01210_amd import project, zbuf_clear
    rng = np.random.default_rng(w * 7 + h)
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    intr = (0.6 * w + 1.0, 0.6 * w + 1.0, w / 2.0, h / 2.0)
    zbuf = torch.empty((h, w), dtype=torch.int64, device=dev)
    zbuf_clear(zbuf)
    empty = np.uint64(2 ** 64 - 1)
    for frame, n in enumerate([5000, 17, 0, 40000, 3]):
        pts = rng.normal(0, 1.0, size=(n, 3)).astype(np.float32)
        pts[:, 2] = np.abs(pts[:, 2]) * 4 + 0.5
        print(f"recycled frame {frame} {w}x{h} n={n}", flush=True)
        _, depth, valid, _ = oracle.project(pts, pose, intr, w, h)
        p = torch.from_numpy(pts).to(dev)
        _, gd, gv = project(p, pose, intr, w, h, zbuf=zbuf, recycle=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(gd.cpu().numpy().view(np.uint32),
                                      depth.view(np.uint32))
        np.testing.assert_array_equal(gv.cpu().numpy(), valid)
        assert np.all(zbuf.cpu().numpy().view(np.uint64) == empty)


FUSED_CASES = [
    # w, h, r, precision
    (1920, 1080, 15, "FP32"),
    (97, 61, 5, "FP32"),
    (130, 3, 32, "FP32"),
    (9, 70, 15, "FP16_RANGE"),     # narrower than a group: halo past both edges
    (200, 150, 0, "FP32"),
]


@pytest.mark.parametrize("case", FUSED_CASES, ids=[f"{c[0]}x{c[1]}r{c[2]}{c[3]}" for c in FUSED_CASES])
def test_project_densify_equals_separate_calls(torch_dev, case):
    """jbfd_project_densify over a frame loop equals jbfd_project_recycled +
    jbfd_densify_prepare + jbfd_densify with the same workspace, bit for bit
    (sparse and dense outputs), and leaves the key buffer empty; with a
    workspace too small for the lists' tables it equals the streaming
    filter."""
    torch, dev = torch_dev
    from paper_2601_01210_amd import (Precision, densify, densify_prepare,
                                      densify_workspace, project, project_densify,
                                      zbuf_clear)
    w, h, r, pname = case
    prec = Precision[pname]
    rng = np.random.default_rng(w + 13 * h + r)
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    intr = (0.7 * w + 1.0, 0.7 * w + 1.0, w / 2.0, h / 2.0)
    rgb = torch.from_numpy(rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)).to(dev)
    za = zbuf_clear(torch.empty((h, w), dtype=torch.int64, device=dev))
    zb = zbuf_clear(torch.empty((h, w), dtype=torch.int64, device=dev))
    empty = np.uint64(2 ** 64 - 1)
    for frame, n in enumerate([int(0.08 * w * h) + 5, 0, int(0.02 * w * h) + 1]):
        pts = rng.normal(0, 1.0, size=(n, 3)).astype(np.float32)
        pts[:, 2] = np.abs(pts[:, 2]) * 4 + 0.5
        p = torch.from_numpy(pts).to(dev)
        print(f"fused {w}x{h} r={r} {pname} frame {frame} n={n}", flush=True)
        for ws_kind in ("lists", "small"):
            nmax = max(n, 1)
            ws = densify_workspace(h, w, r, nmax, device=dev)
            if ws_kind == "small":
                ws = torch.empty(256, dtype=torch.uint8, device=dev)
            d1, v1, o1, m1 = project_densify(p, pose, intr, w, h, rgb, r, 3.0, 12.0,
                                             za, ws, prec)
            ws2 = torch.empty_like(ws)
            _, d2, v2 = project(p, pose, intr, w, h, zbuf=zb, recycle=True)
            if ws_kind == "lists":
                densify_prepare(d2, v2, rgb, r, ws2)
                o2, m2 = densify(d2, v2, rgb, r, 3.0, 12.0, prec, ws=ws2,
                                 lists_ready=True)
            else:
                o2, m2 = densify(d2, v2, rgb, r, 3.0, 12.0, prec, ws=None)
            torch.cuda.synchronize()
            assert torch.equal(d1.view(torch.int32), d2.view(torch.int32))
            assert torch.equal(v1, v2)
            assert torch.equal(m1, m2)
            assert torch.equal(o1.view(torch.int32), o2.view(torch.int32)), ws_kind
            assert np.all(za.cpu().numpy().view(np.uint64) == empty)
            assert np.all(zb.cpu().numpy().view(np.uint64) == empty)


def test_project_densify_graph_replays(torch_dev):
    """jbfd_project_densify captured in a HIP graph: every replay, with eager
    work of the same kind and synchronisations between the replays, gives
    the eager call's results bit for bit and leaves the key buffer empty
    (the key buffer is cleared by kernel stores, so replays need no memset
    node)."""
    torch, dev = torch_dev
    from paper_2601_01210_amd import densify_workspace, project_densify, zbuf_clear
    w, h, r = 640, 360, 15
    rng = np.random.default_rng(77)
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    intr = (0.7 * w, 0.7 * w, w / 2.0, h / 2.0)
    rgb = torch.from_numpy(rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)).to(dev)
    pts = rng.normal(0, 1.0, size=(20000, 3)).astype(np.float32)
    pts[:, 2] = np.abs(pts[:, 2]) * 4 + 0.5
    p = torch.from_numpy(pts).to(dev)
    other = torch.from_numpy(pts[::-1].copy() * np.float32(1.1)).to(dev)
    ws = densify_workspace(h, w, r, 20000, device=dev)
    ws_e = torch.empty_like(ws)
    ze = zbuf_clear(torch.empty((h, w), dtype=torch.int64, device=dev))
    ref = [t.clone() for t in project_densify(p, pose, intr, w, h, rgb, r, 3.0, 12.0,
                                              ze, ws_e)]
    zg = zbuf_clear(torch.empty((h, w), dtype=torch.int64, device=dev))
    outs = (torch.empty((h, w), dtype=torch.float32, device=dev),
            torch.empty((h, w), dtype=torch.uint8, device=dev),
            torch.empty((h, w), dtype=torch.float32, device=dev),
            torch.empty((h, w), dtype=torch.uint8, device=dev))

    def call():
        return project_densify(p, pose, intr, w, h, rgb, r, 3.0, 12.0, zg, ws,
                               depth=outs[0], valid=outs[1], out=outs[2], mask=outs[3])

    call()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
        call()
    torch.cuda.synchronize()
    empty = np.uint64(2 ** 64 - 1)
    for rep in range(4):
        print(f"graph replay {rep}", flush=True)
        for t in outs:
            t.fill_(7)
        # eager work between replays: another frame through the same kernels
        project_densify(other, pose, intr, w, h, rgb, r, 3.0, 12.0, ze, ws_e)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a.view(torch.uint8), b.view(torch.uint8)), rep
        assert np.all(zg.cpu().numpy().view(np.uint64) == empty)


def test_project_largest_sides(torch_dev):
    """Images of the largest side (32767) in either direction, with points
    spread over the whole width or height: keys bit-exact."""
    torch, dev = torch_dev
    rng = np.random.default_rng(4)
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    for w, h in [(32767, 3), (3, 32767)]:
        n = 60000
        z = rng.uniform(1.0, 10.0, n)
        u = rng.uniform(-2, w + 2, n)
        v = rng.uniform(-2, h + 2, n)
        f = 50.0
        pts = np.stack([(u - w / 2.0) * z / f, (v - h / 2.0) * z / f, z],
                       axis=1).astype(np.float32)
        print(f"projection {w}x{h}", flush=True)
        _check_projection(torch, dev, pts, pose, (f, f, w / 2.0, h / 2.0), w, h)


def test_project_scenes(torch_dev):
    torch, dev = torch_dev
    for name, f in [("small", S.small_view(S.seeded(1))),
                    ("fullhd", S.fullhd_view(S.seeded(2)))]:
        print("projection scene", name, len(f.points), flush=True)
        cam = f.camera
        _check_projection(torch, dev, f.points, cam.pose, cam.intrinsics(),
                          cam.width, cam.height)


# ---------------------------------------------------------------------------
# filter
# ---------------------------------------------------------------------------


def _gpu_densify(torch, dev, d, b, rgb, r, ss, sr, prec=0, ws="auto",
                 max_samples=None):
    from paper_2601_01210_amd import densify
    td = torch.from_numpy(np.ascontiguousarray(d, np.float32)).to(dev)
    tb = torch.from_numpy(np.ascontiguousarray(b, np.uint8)).to(dev)
    tc = torch.from_numpy(np.ascontiguousarray(rgb, np.uint8)).to(dev)
    if max_samples is None:
        max_samples = int(b.sum())
    out, mask = densify(td, tb, tc, r, ss, sr, precision=prec, ws=ws,
                        max_samples=max_samples)
    torch.cuda.synchronize()
    return out.cpu().numpy(), mask.cpu().numpy()


def check_filter(torch, dev, d, b, rgb, r, ss, sr, tol=REL_TOL, ws="auto",
                 max_samples=None):
    ref, rmask = oracle.densify(d, b, rgb, r, ss, sr)
    out, mask = _gpu_densify(torch, dev, d, b, rgb, r, ss, sr, ws=ws,
                             max_samples=max_samples)
    np.testing.assert_array_equal(mask, rmask)
    sel = mask == 1
    assert np.all(out[~sel] == 0.0)
    err = np.abs(out[sel].astype(np.float64) - ref[sel])
    rel = err / np.abs(ref[sel])
    worst = float(rel.max()) if rel.size else 0.0
    print(f"  r={r} ss={ss} sr={sr} shape={d.shape} valid={int(sel.sum())} "
          f"max_rel={worst:.3e}", flush=True)
    assert worst <= tol
    return out, mask, worst


FILTER_CASES = [
    # h, w, r, density, sigma_s, sigma_r, palette
    (1, 1, 0, 1.0, 1.0, 1.0, None),
    (1, 37, 3, 0.3, 2.0, 12.0, 3),
    (37, 1, 3, 0.3, 2.0, 12.0, 3),
    (17, 23, 2, 0.2, 1.5, 12.0, None),
    (40, 53, 5, 0.07, 3.0, 12.0, 4),
    (64, 64, 15, 0.07, 6.0, 15.0, 5),
    (71, 90, 32, 0.05, 8.0, 20.0, 4),
    (100, 130, 7, 1.0, 3.0, 12.0, 6),        # every pixel valid
    (33, 47, 4, 0.0, 2.0, 12.0, None),        # nothing valid
    (45, 61, 6, 0.1, math.inf, 10.0, 3),      # pure range filter
    (45, 61, 6, 0.1, 2.0, math.inf, 3),       # pure spatial (normalised conv)
    (45, 61, 6, 0.1, math.inf, math.inf, 3),  # box average
    (50, 66, 5, 0.08, 0.25, 0.25, 8),         # smallest sigmas: heavy rescale
    (50, 66, 9, 0.03, 3.0, 2.0, 8),           # far colours: underflow-prone
    (129, 257, 16, 0.06, 5.0, 14.0, 7),       # radius at the template edge
    (129, 257, 17, 0.06, 5.0, 14.0, 7),       # first radius of the big table
    (3, 32767, 32, 0.05, 8.0, 20.0, 5),       # widest image, largest radius
    (32767, 2, 32, 0.05, 8.0, 20.0, 5),       # tallest image
]


@pytest.mark.parametrize("path", ["lists", "stream"])
@pytest.mark.parametrize("case", FILTER_CASES,
                         ids=[f"{c[0]}x{c[1]}r{c[2]}" for c in FILTER_CASES])
def test_filter_random(torch_dev, case, path):
    """Both filter paths: per-strip sample lists (workspace sized by the
    exact sample count) and direct streaming of the inputs (no workspace)."""
    torch, dev = torch_dev
    h, w, r, dens, ss, sr, pal = case
    d, b, rgb = S.tiny_random(np.random.default_rng(hash(case) & 0xFFFF), h, w,
                              dens, n_colors=pal)
    check_filter(torch, dev, d, b, rgb, r, ss, sr,
                 ws="auto" if path == "lists" else None)


@pytest.mark.parametrize("frac", [0.0, 0.05, 0.33, 0.9])
def test_filter_list_overflow_falls_back(torch_dev, frac):
    """A workspace sized for fewer samples than the image holds: blocks
    whose list range does not fit stream their halo instead (strips early in
    the list fit, later ones do not), with the same results."""
    torch, dev = torch_dev
    d, b, rgb = S.tiny_random(np.random.default_rng(9), 90, 120, 0.2,
                              n_colors=4)
    check_filter(torch, dev, d, b, rgb, 6, 3.0, 12.0, ws="auto",
                 max_samples=int(int(b.sum()) * frac))


def _patchy(rng, h, w, density, patch):
    """tiny_random plus a fully valid square patch (y0, x0, edge)."""
    d, b, rgb = S.tiny_random(rng, h, w, density, n_colors=5)
    y0, x0, e = patch
    b[y0:y0 + e, x0:x0 + e] = 1
    d = np.where(b == 1, np.where(d > 0, d, np.float32(7.5)), np.float32(0.0))
    return d.astype(np.float32), b, rgb


STAGE_CASES = [
    # h, w, r, density, patch (y0, x0, edge) or None: what the halo staging
    # of the list-free filter meets
    (70, 90, 5, 0.30, None),            # tiles staged (about 200 samples each)
    (70, 90, 5, 0.45, None),            # most tiles over the tile capacity
    (70, 90, 5, 0.02, (20, 20, 12)),    # one block's halo over its capacity
    (70, 90, 2, 0.60, None),            # small halo, dense
    (90, 120, 15, 0.05, None),          # nine rounds per tile
    (100, 100, 32, 0.02, None),         # 25 rounds per tile
    (19, 300, 5, 0.20, (0, 250, 19)),   # partial tiles at the bottom edge
]


@pytest.mark.parametrize("case", STAGE_CASES,
                         ids=[f"{c[0]}x{c[1]}r{c[2]}d{c[3]}" for c in STAGE_CASES])
def test_filter_halo_staging(torch_dev, case):
    """Without sample lists each workgroup stages its tile's halo once and
    hands every wave its block's samples; past the capacities (256 samples
    per tile halo, 128 per block halo) a wave streams its own halo. Every
    case matches the oracle and the list path."""
    torch, dev = torch_dev
    h, w, r, dens, patch = case
    rng = np.random.default_rng(h * 1000 + w + r)
    if patch is None:
        d, b, rgb = S.tiny_random(rng, h, w, dens, n_colors=5)
    else:
        d, b, rgb = _patchy(rng, h, w, dens, patch)
    out, mask, _ = check_filter(torch, dev, d, b, rgb, r, 3.0, 12.0, ws=None)
    lo, lm = _gpu_densify(torch, dev, d, b, rgb, r, 3.0, 12.0)
    np.testing.assert_array_equal(mask, lm)
    sel = mask == 1
    if sel.any():
        rel = np.abs(out[sel].astype(np.float64) - lo[sel]) / lo[sel]
        assert rel.max() <= 2e-6


@pytest.mark.parametrize("case", [(60, 90, 5, 0.08, 3.0, 12.0, 5),
                                  (70, 100, 15, 0.05, 6.0, 15.0, 6),
                                  (50, 66, 5, 0.08, 0.25, 0.25, 8)],
                         ids=["r5", "r15", "tiny-sigmas"])
def test_filter_direct_and_clamped_forms(torch_dev, case):
    """FP32 without aux forms each exponent exactly with one fma and lets
    weights underflow (lanes whose sum ends below 2^-16, zero included, take
    the exact pass); with aux it keeps the clamped weights the backward
    replays. Both match the oracle and each other (mask bit for bit), on the
    list and the stream path."""
    torch, dev = torch_dev
    from paper_2601_01210_amd import densify
    h, w, r, dens, ss, sr, pal = case
    d, b, rgb = S.tiny_random(np.random.default_rng(h * w + r), h, w, dens, n_colors=pal)
    ref, rmask = oracle.densify(d, b, rgb, r, ss, sr)
    td = torch.from_numpy(d).to(dev)
    tb = torch.from_numpy(b).to(dev)
    tc = torch.from_numpy(rgb).to(dev)
    sel = rmask == 1
    for ws in ("auto", None):
        o1, m1 = densify(td, tb, tc, r, ss, sr, ws=ws, max_samples=int(b.sum()))
        o2, m2, _ = densify(td, tb, tc, r, ss, sr, want_aux=True, ws=ws,
                            max_samples=int(b.sum()))
        torch.cuda.synchronize()
        for o, m in ((o1, m1), (o2, m2)):
            o, m = o.cpu().numpy(), m.cpu().numpy()
            np.testing.assert_array_equal(m, rmask)
            if sel.any():
                rel = np.abs(o[sel].astype(np.float64) - ref[sel]) / ref[sel]
                assert rel.max() <= REL_TOL
        a, c = o1.cpu().numpy(), o2.cpu().numpy()
        if sel.any():
            assert (np.abs(a[sel].astype(np.float64) - c[sel]) / c[sel]).max() <= 2e-6


def test_filter_paths_agree(torch_dev):
    torch, dev = torch_dev
    f = S.small_view(S.seeded(1))
    cam = f.camera
    _, depth, valid, _ = oracle.project(f.points, cam.pose, cam.intrinsics(),
                                        cam.width, cam.height)
    a, ma = _gpu_densify(torch, dev, depth, valid, f.rgb, 5, 3.0, 12.0)
    b, mb = _gpu_densify(torch, dev, depth, valid, f.rgb, 5, 3.0, 12.0, ws=None)
    np.testing.assert_array_equal(ma, mb)
    sel = ma == 1
    rel = np.abs(a[sel].astype(np.float64) - b[sel]) / b[sel]
    assert rel.max() <= 2e-6


def test_filter_ignores_depth_where_invalid(torch_dev):
    torch, dev = torch_dev
    d, b, rgb = S.tiny_random(np.random.default_rng(3), 40, 40, 0.1,
                              n_colors=3)
    out1, m1 = _gpu_densify(torch, dev, d, b, rgb, 4, 2.0, 12.0)
    junk = np.where(b == 1, d, np.float32(1e30)).astype(np.float32)
    out2, m2 = _gpu_densify(torch, dev, junk, b, rgb, 4, 2.0, 12.0)
    np.testing.assert_array_equal(out1, out2)
    np.testing.assert_array_equal(m1, m2)


def test_filter_constant_power_of_two_depth(torch_dev):
    """Same weights in numerator and denominator: a constant 2^k depth comes
    back exactly (scaling by 2^k commutes with rounding)."""
    torch, dev = torch_dev
    d, b, rgb = S.tiny_random(np.random.default_rng(4), 70, 90, 0.1,
                              n_colors=4)
    d = np.where(b == 1, np.float32(4.0), np.float32(0)).astype(np.float32)
    out, mask = _gpu_densify(torch, dev, d, b, rgb, 6, 3.0, 12.0)
    assert np.all(out[mask == 1] == 4.0)


def test_filter_deterministic(torch_dev):
    torch, dev = torch_dev
    f = S.small_view(S.seeded(1))
    cam = f.camera
    _, depth, valid, _ = oracle.project(f.points, cam.pose, cam.intrinsics(),
                                        cam.width, cam.height)
    a = _gpu_densify(torch, dev, depth, valid, f.rgb, 5, 3.0, 12.0)
    b = _gpu_densify(torch, dev, depth, valid, f.rgb, 5, 3.0, 12.0)
    np.testing.assert_array_equal(a[0].view(np.uint32), b[0].view(np.uint32))


@pytest.mark.parametrize("cfg", ["small", "fullhd"])
def test_pipeline_scene(torch_dev, cfg):
    """project -> densify on the GPU vs the oracle on the whole frame."""
    torch, dev = torch_dev
    from paper_2601_01210_amd import densify, project
    f = S.small_view(S.seeded(1)) if cfg == "small" else \
        S.fullhd_view(S.seeded(2))
    cam = f.camera
    print("pipeline", cfg, cam.width, cam.height, len(f.points), flush=True)
    _, depth, valid, _ = oracle.project(f.points, cam.pose, cam.intrinsics(),
                                        cam.width, cam.height)
    ref, rmask = oracle.densify(depth, valid, f.rgb, f.radius, f.sigma_s,
                                f.sigma_r)
    pts = torch.from_numpy(f.points).to(dev)
    zbuf, gd, gv = project(pts, cam.pose, cam.intrinsics(), cam.width,
                           cam.height)
    rgb = torch.from_numpy(f.rgb).to(dev)
    out, mask = densify(gd, gv, rgb, f.radius, f.sigma_s, f.sigma_r,
                        max_samples=len(f.points))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    mask = mask.cpu().numpy()
    np.testing.assert_array_equal(mask, rmask)
    sel = mask == 1
    rel = np.abs(out[sel] - ref[sel]) / ref[sel]
    print(f"  valid={int(sel.sum())} max_rel={rel.max():.3e} "
          f"mean_rel={rel.mean():.3e}", flush=True)
    assert rel.max() <= REL_TOL
    assert np.all(out[~sel] == 0)


def test_single_view_step_graph_replays(torch_dev):
    """project + densify_prepare + densify captured once in a HIP graph and
    replayed with new points and colours copied into the same buffers:
    every replay equals the eager calls on the same inputs."""
    torch, dev = torch_dev
    from paper_2601_01210_amd import (densify, densify_prepare,
                                      densify_workspace, project)
    frames = [S.small_view(np.random.default_rng(70 + k), 320, 240,
                           n_points=6000) for k in range(3)]
    cam = frames[0].camera
    W, H, r = cam.width, cam.height, 5
    pts = torch.empty((6000, 3), dtype=torch.float32, device=dev)
    rgb = torch.empty((H, W, 3), dtype=torch.uint8, device=dev)
    zb = torch.empty((H, W), dtype=torch.int64, device=dev)
    d = torch.empty((H, W), dtype=torch.float32, device=dev)
    v = torch.empty((H, W), dtype=torch.uint8, device=dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    m = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ws = densify_workspace(H, W, r, 6000, dev)

    def step():
        project(pts, cam.pose, cam.intrinsics(), W, H, zbuf=zb, depth=d,
                valid=v)
        densify_prepare(d, v, rgb, r, ws)
        densify(d, v, rgb, r, 3.0, 12.0, out=out, mask=m, ws=ws,
                lists_ready=True)

    pts.copy_(torch.from_numpy(frames[0].points))
    rgb.copy_(torch.from_numpy(frames[0].rgb))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for k in (1, 2, 0, 1):
        f = frames[k]
        pts.copy_(torch.from_numpy(f.points))
        rgb.copy_(torch.from_numpy(f.rgb))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (out.clone(), m.clone(), zb.clone())
        step()
        torch.cuda.synchronize()
        assert torch.equal(got[2], zb)
        assert torch.equal(got[1], m)
        assert torch.equal(got[0].view(torch.int32), out.view(torch.int32))
