"""GPU checks of the batched path (jbfd_batch_prepare / jbfd_batch_run).

One batch of uneven views (mixed 1280x720 / 1920x1080, 20k-250k points,
log-uniform, the small-view scene generator, r=5, sigma_s=3, sigma_r=12)
runs as one persistent launch (and, compared bit for bit, as the staged
launch sequence). Each view's sparse depth and mask (the z-buffer's result)
must equal the oracle's bit for bit, with the key buffer left empty; the
dense mask must equal the oracle's; FP32 depth must agree with the FP64
oracle to 1e-5 relative and be bit-identical to the single-view
jbfd_densify (same tile body, same arithmetic). The FP16 range-weight form runs on the same batch,
side by side: its mask must equal the oracle's, every valid pixel must lie
within the per-pixel bound of FP16 weights (fp16_check), and max / p99.9 /
mean in mm are printed per view with every pixel above 1 mm named with its
condition number.

The batch is also captured into a HIP graph and replayed with the
descriptor table rewritten between replays (new poses, point counts and
views): every replay must equal the eager run on the same inputs.
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


@pytest.fixture(scope="module")
def frames():
    return S.batch_views(S.seeded(3))


@pytest.fixture(scope="module")
def refs(frames):
    out = []
    for f in frames:
        cam = f.camera
        z, d, b, _ = oracle.project(f.points, cam.pose, cam.intrinsics(),
                                    cam.width, cam.height)
        ref, m = oracle.densify(d, b, f.rgb, f.radius, f.sigma_s, f.sigma_r)
        out.append((z, d, b, ref, m))
    return out


def _dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _views(torch, dev, frames, **over):
    from paper_2601_01210_amd import BatchView
    vs = []
    for f in frames:
        cam = f.camera
        kw = dict(radius=f.radius, sigma_s=f.sigma_s, sigma_r=f.sigma_r)
        kw.update(over)
        vs.append(BatchView(_dev(torch, dev, f.points), cam.pose,
                            cam.intrinsics(), cam.width, cam.height,
                            _dev(torch, dev, f.rgb), **kw).allocate())
    return vs


def _run(torch, views, precision, lists=False, staged=False, max_radius=None):
    from paper_2601_01210_amd import batch_run, batch_upload
    table, host = batch_upload(views)
    r = max(v.radius for v in views) if max_radius is None else max_radius
    batch_run(table, r, precision, lists=lists, staged=staged)
    torch.cuda.synchronize()
    return table, host


def _same_outputs(torch, a, b, what):
    assert torch.equal(a.zbuf, b.zbuf), what
    assert torch.equal(a.sparse_depth.view(torch.int32),
                       b.sparse_depth.view(torch.int32)), what
    assert torch.equal(a.sparse_valid, b.sparse_valid), what
    assert torch.equal(a.dense_depth.view(torch.int32),
                       b.dense_depth.view(torch.int32)), what
    assert torch.equal(a.dense_valid, b.dense_valid), what


def _zkeys(t):
    return t.cpu().numpy().view(np.uint64)


def test_batch_fp32_matches_oracle_and_single_views(tdev, frames, refs):
    torch, dev = tdev
    from paper_2601_01210_amd import Precision, densify, project
    views = _views(torch, dev, frames)
    print(f"  batch: {[(v.width, v.height, v.points.shape[0]) for v in views]}",
          flush=True)
    _run(torch, views, Precision.FP32)
    for k, (v, (z, d, b, ref, m)) in enumerate(zip(views, refs)):
        # the run leaves its key buffer empty (the decode writes the empty
        # key back); the z-buffer's result is the sparse depth and mask
        assert np.all(_zkeys(v.zbuf) == np.uint64(2 ** 64 - 1))
        np.testing.assert_array_equal(v.sparse_valid.cpu().numpy(), b)
        np.testing.assert_array_equal(v.sparse_depth.cpu().numpy(),
                                      d.astype(np.float32))
        out, mask = v.dense_depth.cpu().numpy(), v.dense_valid.cpu().numpy()
        np.testing.assert_array_equal(mask, m)
        sel = m == 1
        rel = np.abs(out[sel] - ref[sel]) / np.abs(ref[sel])
        assert rel.max() <= 1e-5, (k, rel.max())
        assert np.all(out[~sel] == 0)
        # single-view calls on the same inputs (streaming the halo, as the
        # batch views without list workspaces) give identical bits
        zs, ds, bs = project(v.points, v.pose, v.intrinsics, v.width, v.height)
        so, sm = densify(ds, bs, v.rgb, v.radius, v.sigma_s, v.sigma_r, ws=None)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_zkeys(zs), z)
        np.testing.assert_array_equal(so.cpu().numpy().view(np.uint32),
                                      out.view(np.uint32))
        np.testing.assert_array_equal(sm.cpu().numpy(), mask)
        print(f"  view {k}: {v.width}x{v.height} n={v.points.shape[0]} "
              f"valid={int(b.sum())} max_rel={rel.max():.2e}", flush=True)


def test_batch_fp16_side_by_side(tdev, frames, refs):
    torch, dev = tdev
    from paper_2601_01210_amd import Precision
    v32 = _views(torch, dev, frames)
    v16 = _views(torch, dev, frames)
    _run(torch, v32, Precision.FP32)
    _run(torch, v16, Precision.FP16_RANGE)
    from fp16_check import fp16_report
    for k, (a, c, (z, d, b, ref, m)) in enumerate(zip(v32, v16, refs)):
        f = frames[k]
        sel = m == 1
        e32 = np.abs(a.dense_depth.cpu().numpy()[sel] - ref[sel]) * 1e3
        print(f"  view {k}: fp32 max {e32.max():.4f} mm", flush=True)
        fp16_report(c.dense_depth.cpu().numpy(), c.dense_valid.cpu().numpy(), ref,
                    m, d, b, f.rgb, f.radius, f.sigma_s, f.sigma_r, f"view {k}")


def test_batch_mixed_filters_and_degenerate_views(tdev):
    """Views of one batch may differ in radius and widths (up to r=15 and
    sigma = +inf), and may be empty (no points) or smaller than a tile."""
    torch, dev = tdev
    from paper_2601_01210_amd import BatchView, Precision, densify, project
    rng = np.random.default_rng(31)
    f1 = S.small_view(rng, 320, 240)
    f2 = S.small_view(rng, 200, 150, n_points=9000)
    f3 = S.small_view(rng, 7, 5, n_points=300)
    specs = [(f1, 15, 6.0, 15.0), (f2, 3, float("inf"), 20.0),
             (f1, 0, 3.0, 12.0), (f3, 5, 3.0, float("inf")), (f2, 5, 3.0, 12.0)]
    views = []
    for f, r, ss, sr in specs:
        cam = f.camera
        views.append(BatchView(_dev(torch, dev, f.points), cam.pose,
                               cam.intrinsics(), cam.width, cam.height,
                               _dev(torch, dev, f.rgb), r, ss, sr).allocate())
    views[-1].n_points = 0                         # an empty view
    _run(torch, views, Precision.FP32)
    for k, ((f, r, ss, sr), v) in enumerate(zip(specs, views)):
        pts = v.points[: v.points.shape[0] if v.n_points is None else v.n_points]
        zs, ds, bs = project(pts.contiguous(), v.pose, v.intrinsics, v.width,
                             v.height)
        so, sm = densify(ds, bs, v.rgb, r, ss, sr, ws=None)
        torch.cuda.synchronize()
        assert torch.equal(ds.view(torch.int32), v.sparse_depth.view(torch.int32)), k
        assert torch.equal(bs, v.sparse_valid), k
        assert bool((v.zbuf == -1).all()), k
        assert torch.equal(so.view(torch.int32), v.dense_depth.view(torch.int32)), k
        assert torch.equal(sm, v.dense_valid), k
        _, d, b, _ = oracle.project(f.points[: len(pts)], f.camera.pose,
                                    f.camera.intrinsics(), v.width, v.height)
        ref, m = oracle.densify(d, b, f.rgb, r, ss, sr)
        np.testing.assert_array_equal(v.dense_valid.cpu().numpy(), m)
        out = v.dense_depth.cpu().numpy()
        np.testing.assert_allclose(out[m == 1], ref[m == 1], rtol=1e-5)
    assert int(views[-1].dense_valid.sum()) == 0
    assert int(views[-1].sparse_valid.sum()) == 0


def test_batch_lists_streaming_and_overflow_agree(tdev, frames):
    """With JBFD_BATCH_LISTS the batch builds each view's sample lists in
    its list workspace and the filter walks them; without a workspace the
    filter streams the halo,
    and with a workspace too small for every record the blocks whose lists
    do not fit stream. The masks agree bit for bit; the depths too, except
    at lanes that take the exact pass (tiny weight sums), whose running
    shift groups the samples differently when streaming: there they agree
    to rounding."""
    torch, dev = tdev
    from paper_2601_01210_amd import Precision, densify_ws_bytes
    sub = frames[:4]
    with_lists = _views(torch, dev, sub, lists=True)
    streaming = _views(torch, dev, sub)
    small = _views(torch, dev, sub)
    for v in small:
        # room for a tenth of the valid pixels' records
        n = densify_ws_bytes(v.height, v.width, v.radius, max(v.points.shape[0] // 10, 1))
        v.list_ws = torch.empty(n, dtype=torch.uint8, device=dev)
    for vs in (with_lists, streaming, small):
        _run(torch, vs, Precision.FP32, lists=True)
    from paper_2601_01210_amd import densify
    for a, b, c in zip(with_lists, streaming, small):
        assert a.list_ws is not None and b.list_ws is None
        # with lists, the batch equals single-view calls with lists
        so, sm = densify(a.sparse_depth, a.sparse_valid, a.rgb, a.radius, a.sigma_s,
                         a.sigma_r)
        torch.cuda.synchronize()
        assert torch.equal(so.view(torch.int32), a.dense_depth.view(torch.int32))
        assert torch.equal(sm, a.dense_valid)
        for x in (b, c):
            assert torch.equal(a.dense_valid, x.dense_valid)
            da, dx = a.dense_depth.cpu().numpy(), x.dense_depth.cpu().numpy()
            sel = a.dense_valid.cpu().numpy() == 1
            rel = np.abs(da[sel] - dx[sel]) / np.abs(da[sel])
            assert rel.max() <= 1e-6, rel.max()
            assert (da != dx).mean() <= 1e-4, (da != dx).mean()
    # without the flag, views that carry a list workspace stream too
    flagless = _views(torch, dev, sub, lists=True)
    _run(torch, flagless, Precision.FP32)
    for b, x in zip(streaming, flagless):
        assert torch.equal(b.dense_depth.view(torch.int32),
                           x.dense_depth.view(torch.int32))
        assert torch.equal(b.dense_valid, x.dense_valid)


def test_batch_graph_replays_match_eager(tdev, frames):
    """Capture one batch run, then replay it with the table rewritten
    between replays; each replay equals an eager run on the same table."""
    torch, dev = tdev
    from paper_2601_01210_amd import Precision, batch_run, batch_upload
    views = _views(torch, dev, frames[:4])
    eager = _views(torch, dev, frames[:4])
    max_r = 5
    table, host = batch_upload(views)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch_run(table, max_r, Precision.FP16_RANGE)     # warm-up
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        batch_run(table, max_r, Precision.FP16_RANGE)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    etable = None
    for rep in range(4):
        # new inputs: rotate the frames' poses slightly and cut point counts
        for v, e in zip(views, eager):
            ang = rng.uniform(-0.02, 0.02)
            c, s_ = np.cos(ang), np.sin(ang)
            pose = np.asarray(v.pose, np.float64).reshape(3, 4).copy()
            pose[:, :3] = pose[:, :3] @ np.array([[c, 0, s_], [0, 1, 0],
                                                   [-s_, 0, c]])
            n = int(rng.integers(0, v.points.shape[0] + 1))
            v.pose = e.pose = pose
            v.n_points = e.n_points = n
        torch.cuda.synchronize()
        table, host = batch_upload(views, table, host)
        g.replay()
        torch.cuda.synchronize()
        etable, _ = batch_upload(eager, etable)
        batch_run(etable, max_r, Precision.FP16_RANGE)
        torch.cuda.synchronize()
        for k, (v, e) in enumerate(zip(views, eager)):
            assert torch.equal(v.zbuf, e.zbuf), (rep, k)
            assert torch.equal(v.dense_depth.view(torch.int32),
                               e.dense_depth.view(torch.int32)), (rep, k)
            assert torch.equal(v.dense_valid, e.dense_valid), (rep, k)
        print(f"  replay {rep}: n={[v.n_points for v in views]} ok", flush=True)


@pytest.mark.parametrize("prec_name", ["FP32", "FP16_RANGE"])
def test_batch_one_launch_equals_staged(tdev, frames, prec_name):
    """The one persistent launch (work queue over every view's clear,
    projection, decode and filter items) and the staged launch sequence
    give the same bits: keys, sparse depth and mask, dense depth and mask."""
    torch, dev = tdev
    from paper_2601_01210_amd import Precision, batch_check
    prec = getattr(Precision, prec_name)
    one = _views(torch, dev, frames)
    staged = _views(torch, dev, frames)
    t1, _ = _run(torch, one, prec)
    t2, _ = _run(torch, staged, prec, staged=True)
    batch_check(t1)
    batch_check(t2)
    for k, (a, b) in enumerate(zip(one, staged)):
        _same_outputs(torch, a, b, (prec_name, k))


def test_batch_one_launch_reruns_on_an_unchanged_table(tdev, frames):
    """The last workgroup of a one-launch run resets the queue, so the same
    table runs again without being rewritten and gives the same outputs."""
    torch, dev = tdev
    from paper_2601_01210_amd import Precision, batch_check, batch_run
    views = _views(torch, dev, frames[:3])
    table, _ = _run(torch, views, Precision.FP32)
    first = [(v.dense_depth.clone(), v.dense_valid.clone(), v.zbuf.clone())
             for v in views]
    for v in views:                      # outputs are rewritten, not kept
        v.dense_depth.fill_(7.0)
        v.dense_valid.fill_(9)
    for _ in range(2):
        batch_run(table, 5, Precision.FP32)
        torch.cuda.synchronize()
        for (d, m, z), v in zip(first, views):
            assert torch.equal(d.view(torch.int32), v.dense_depth.view(torch.int32))
            assert torch.equal(m, v.dense_valid)
            assert torch.equal(z, v.zbuf)
    # the header's run words (workgroups exited, error) are zero again; the
    # queues were reset too, or the reruns above would have done nothing
    words = table[:48].cpu().numpy().view(np.uint32)
    assert list(words[9:11]) == [0, 0]
    batch_check(table)


@pytest.mark.parametrize("staged", [False, True], ids=["one_launch", "staged"])
def test_batch_radius_above_launch_bound_is_refused(tdev, staged):
    """A view whose radius exceeds the run's max_radius (here r = 20 in a
    run bounded by 16, whose LDS table holds windows up to r = 16) gets zero
    depth and mask instead of a table overrun, the other views are
    unaffected, and jbfd_batch_check reports JBFD_EINVAL; a run with an
    adequate bound on a fresh table is clean."""
    torch, dev = tdev
    from paper_2601_01210_amd import Precision, batch_check, densify, project
    from paper_2601_01210_amd.binding import JBFD_EINVAL, JbfdError
    rng = np.random.default_rng(41)
    f = S.small_view(rng, 320, 240)
    g = S.small_view(rng, 160, 120, n_points=5000)
    views = _views(torch, dev, [f, g])
    views[0].radius, views[0].sigma_s = 20, 6.0
    table, _ = _run(torch, views, Precision.FP32, staged=staged, max_radius=16)
    assert int(views[0].dense_valid.sum()) == 0
    assert int(views[0].dense_depth.abs().sum()) == 0
    zs, ds, bs = project(views[1].points, views[1].pose, views[1].intrinsics,
                         views[1].width, views[1].height)
    so, sm = densify(ds, bs, views[1].rgb, views[1].radius, views[1].sigma_s,
                     views[1].sigma_r, ws=None)
    torch.cuda.synchronize()
    assert torch.equal(so.view(torch.int32), views[1].dense_depth.view(torch.int32))
    assert torch.equal(sm, views[1].dense_valid)
    with pytest.raises(JbfdError) as e:
        batch_check(table)
    assert e.value.status == JBFD_EINVAL
    ok_table, _ = _run(torch, views, Precision.FP32, staged=staged, max_radius=32)
    batch_check(ok_table)
    assert int(views[0].dense_valid.sum()) > 0
