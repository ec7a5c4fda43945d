"""C-ABI contract checks that need no GPU.

The library must load, export every function include/jbfd.h declares, and
reject bad arguments on the host before touching the device (so these
calls are safe without a GPU: validation precedes any HIP call).
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jbfd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jbfd_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2601_01210_amd import binding
    return binding.lib()


def test_header_declares_entry_points():
    names = _declared()
    for n in ["jbfd_project", "jbfd_densify", "jbfd_densify_backward",
              "jbfd_status_string", "jbfd_last_error", "jbfd_abi_version"]:
        assert n in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings(L):
    from paper_2601_01210_amd import binding
    assert L.jbfd_abi_version() == 5
    for code in range(5):
        assert L.jbfd_status_string(code)
    assert L.jbfd_status_string(99) == b"unknown status"


def _K(w=8, h=6):
    from paper_2601_01210_amd.binding import Intrinsics
    return Intrinsics(4.0, 4.0, 4.0, 3.0, w, h)


def test_project_rejects_bad_arguments(L):
    from paper_2601_01210_amd.binding import JBFD_EINVAL
    pose = (C.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    K = _K()
    assert L.jbfd_project(fake, 10, pose, C.byref(K), None, None, None,
                          None) == JBFD_EINVAL
    assert b"zbuf" in L.jbfd_last_error()
    assert L.jbfd_project(fake, -1, pose, C.byref(K), fake, None, None,
                          None) == JBFD_EINVAL
    assert L.jbfd_project(fake, 1 << 32, pose, C.byref(K), fake, None, None,
                          None) == JBFD_EINVAL
    assert L.jbfd_project(None, 5, pose, C.byref(K), fake, None, None,
                          None) == JBFD_EINVAL
    bad = _K(0, 6)
    assert L.jbfd_project(fake, 1, pose, C.byref(bad), fake, None, None,
                          None) == JBFD_EINVAL
    nanpose = (C.c_double * 12)(1, 0, 0, float("nan"), 0, 1, 0, 0, 0, 0, 1, 0)
    assert L.jbfd_project(fake, 1, nanpose, C.byref(K), fake, None, None,
                          None) == JBFD_EINVAL
    assert b"pose" in L.jbfd_last_error()


def test_recycled_projection_rejects_bad_arguments(L):
    from paper_2601_01210_amd import binding
    from paper_2601_01210_amd.binding import JBFD_EINVAL
    binding.lib()   # argument types
    pose = (C.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    K = _K()
    # the sparse outputs are required: the decode is what clears the keys
    assert L.jbfd_project_recycled(fake, 10, pose, C.byref(K), fake, None, fake,
                                   None) == JBFD_EINVAL
    assert b"sparse" in L.jbfd_last_error()
    assert L.jbfd_project_recycled(fake, 10, pose, C.byref(K), fake, fake, None,
                                   None) == JBFD_EINVAL
    # and the checks of jbfd_project, under the entry point's own name
    assert L.jbfd_project_recycled(fake, -1, pose, C.byref(K), fake, fake, fake,
                                   None) == JBFD_EINVAL
    assert b"jbfd_project_recycled" in L.jbfd_last_error()
    assert L.jbfd_project_recycled(fake, 1, pose, C.byref(K), None, fake, fake,
                                   None) == JBFD_EINVAL
    assert L.jbfd_zbuf_clear(None, 6, 8, None) == JBFD_EINVAL
    # the fused projection + filter: the checks of both calls
    pd = L.jbfd_project_densify
    pd.restype = C.c_int
    args = lambda **o: [o.get("pts", fake), o.get("n", 10), pose, C.byref(o.get("K", K)),
                        o.get("rgb", fake), o.get("r", 5), o.get("ss", C.c_float(3.0)),
                        o.get("sr", C.c_float(12.0)), o.get("prec", 0),
                        o.get("zbuf", fake), o.get("d", fake), o.get("v", fake),
                        o.get("out", fake), o.get("m", fake), o.get("ws", None),
                        C.c_size_t(0), None]
    for bad, msg in ((dict(zbuf=None), b"zbuf"), (dict(rgb=None), b"null buffer"),
                     (dict(d=None), b"null buffer"), (dict(m=None), b"null buffer"),
                     (dict(r=33), b"radius"), (dict(prec=7), b"precision"),
                     (dict(n=-1), b"n = -1"), (dict(K=_K(0, 6)), b"image size"),
                     (dict(ss=C.c_float(0.0)), b"sigma_s"),
                     (dict(ws=C.c_void_p(0x1010)), b"aligned")):
        assert pd(*args(**bad)) == JBFD_EINVAL, bad
        assert msg in L.jbfd_last_error(), (bad, L.jbfd_last_error())
    assert L.jbfd_zbuf_clear(fake, 0, 8, None) == JBFD_EINVAL
    assert L.jbfd_zbuf_clear(fake, 6, -1, None) == JBFD_EINVAL


@pytest.mark.parametrize("radius,ss,sr", [(-1, 3.0, 12.0), (33, 3.0, 12.0),
                                          (5, 0.1, 12.0), (5, 3.0, 0.0),
                                          (5, float("nan"), 12.0),
                                          (5, 3.0, -float("inf"))])
def test_densify_rejects_bad_filter(L, radius, ss, sr):
    from paper_2601_01210_amd.binding import JBFD_EINVAL
    f = C.c_void_p(0x1000)
    st = L.jbfd_densify(f, f, f, 10, 10, radius, C.c_float(ss), C.c_float(sr),
                        0, f, f, None, None, 0, 0, None)
    assert st == JBFD_EINVAL


def test_densify_rejects_sizes_and_nulls(L):
    from paper_2601_01210_amd.binding import JBFD_EINVAL
    f = C.c_void_p(0x1000)
    args = (C.c_float(1), C.c_float(1))
    assert L.jbfd_densify(f, f, f, 0, 10, 2, *args, 0, f, f, None, None, 0, 0,
                          None) == JBFD_EINVAL
    assert L.jbfd_densify(f, f, f, 10, 32768, 2, *args, 0, f, f, None, None,
                          0, 0, None) == JBFD_EINVAL
    assert L.jbfd_densify(None, f, f, 10, 10, 2, *args, 0, f, f, None, None,
                          0, 0, None) == JBFD_EINVAL
    assert L.jbfd_densify(f, f, f, 10, 10, 2, *args, 7, f, f, None, None, 0, 0,
                          None) == JBFD_EINVAL
    # aux is an FP32-only output
    assert L.jbfd_densify(f, f, f, 10, 10, 2, *args, 1, f, f, f, None, 0, 0,
                          None) == JBFD_EINVAL
    # the workspace must be 256-byte aligned
    assert L.jbfd_densify(f, f, f, 10, 10, 2, *args, 0, f, f, None,
                          C.c_void_p(0x1010), 4096, 0, None) == JBFD_EINVAL
    assert b"aligned" in L.jbfd_last_error()
    assert L.jbfd_densify(f, f, f, 10, 10, 2, *args, 0, f, f, None, None, 0,
                          8, None) == JBFD_EINVAL
    assert L.jbfd_densify_prepare(f, f, f, 10, 10, 2, None, 0,
                                  None) == JBFD_EINVAL


def test_densify_ws_bytes(L):
    a = L.jbfd_densify_ws_bytes(1080, 1920, 15, 0)
    b = L.jbfd_densify_ws_bytes(1080, 1920, 15, 1000)
    assert a > 0 and b - a == 1000 * 5 * 20   # 5 strips per column at r=15
    assert L.jbfd_densify_ws_bytes(1080, 1920, 5, 1000) - \
        L.jbfd_densify_ws_bytes(1080, 1920, 5, 0) == 1000 * 3 * 20
    assert L.jbfd_densify_ws_bytes(0, 10, 5, 10) == 0
    assert L.jbfd_densify_ws_bytes(10, 10, 33, 10) == 0


def test_backward_workspace_checks(L):
    from paper_2601_01210_amd.binding import JBFD_EINVAL, JBFD_ENOSPC
    f = C.c_void_p(0x1000)
    need = L.jbfd_densify_backward_ws_bytes(100, 100)
    assert need > 0
    assert L.jbfd_densify_backward_ws_bytes(0, 100) == 0
    # the same side limit as every other workspace query
    assert L.jbfd_densify_backward_ws_bytes(32768, 100) == 0
    assert L.jbfd_densify_backward_ws_bytes(100, 32768) == 0
    assert L.jbfd_densify_backward_ws_bytes(32767, 1) > 0
    st = L.jbfd_densify_backward(f, f, f, 100, 100, 3, C.c_float(2),
                                 C.c_float(10), f, f, f, f, f, f, need - 1,
                                 None)
    assert st == JBFD_ENOSPC
    st = L.jbfd_densify_backward(f, f, f, 100, 100, 3, C.c_float(2),
                                 C.c_float(10), f, None, f, f, f, f, need,
                                 None)
    assert st == JBFD_EINVAL


def _views(n, w=40, h=30, radius=5, n_points=100):
    from paper_2601_01210_amd.binding import Intrinsics, View
    out = []
    for k in range(n):
        v = View()
        base = 0x10000 * (k + 1)
        v.points, v.n_points = base + 0x100, n_points
        v.cam_from_world = (C.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
        v.K = Intrinsics(20.0, 20.0, w / 2, h / 2, w + k, h + 2 * k)
        v.rgb, v.radius, v.sigma_s, v.sigma_r = base + 0x200, radius, 3.0, 12.0
        v.zbuf, v.sparse_depth, v.sparse_valid = base + 0x300, base + 0x400, \
            base + 0x500
        v.dense_depth, v.dense_valid = base + 0x600, base + 0x700
        out.append(v)
    return out


def test_batch_prepare_serialises_table(L):
    """The table is a 16-byte header {n_views, total_tiles, pad} then one
    entry per view; tiles are 16x16 and numbered view after view."""
    import numpy as np
    from paper_2601_01210_amd import binding
    views = _views(3)
    n = binding.batch_table_bytes(3)
    assert n > 16 and binding.batch_table_bytes(0) == 0
    host = np.zeros(n, np.uint8)
    binding.batch_prepare_raw(views, host)
    hdr = host[:16].view(np.int32)
    tiles = [((40 + k + 15) // 16) * ((30 + 2 * k + 15) // 16) for k in range(3)]
    assert hdr[0] == 3 and hdr[1] == sum(tiles)
    # 1024-element chunks of pixels and of points, per view
    assert hdr[2] == sum(-(-(40 + k) * (30 + 2 * k) // 1024) for k in range(3))
    assert hdr[3] == 3 * -(-100 // 1024)
    # table too small
    with pytest.raises(binding.JbfdError) as e:
        binding.batch_prepare_raw(views, np.zeros(n - 8, np.uint8))
    assert e.value.status == binding.JBFD_ENOSPC


@pytest.mark.parametrize("field,value,msg", [
    ("rgb", 0, b"null"), ("dense_valid", 0, b"null"), ("n_points", -1, b"n_points"),
    ("radius", 40, b"radius"), ("sigma_s", 0.0, b"sigma"),
    ("sigma_r", float("nan"), b"sigma")])
def test_batch_prepare_rejects_bad_views(L, field, value, msg):
    import numpy as np
    from paper_2601_01210_amd import binding
    views = _views(2)
    setattr(views[1], field, value)
    host = np.zeros(binding.batch_table_bytes(2), np.uint8)
    with pytest.raises(binding.JbfdError) as e:
        binding.batch_prepare_raw(views, host)
    assert e.value.status == binding.JBFD_EINVAL
    assert b"view 1" in L.jbfd_last_error() and msg in L.jbfd_last_error()


def test_batch_prepare_rejects_bad_pose_and_size(L):
    import numpy as np
    from paper_2601_01210_amd import binding
    host = np.zeros(binding.batch_table_bytes(1), np.uint8)
    v = _views(1)
    v[0].cam_from_world[7] = float("inf")
    with pytest.raises(binding.JbfdError):
        binding.batch_prepare_raw(v, host)
    v = _views(1, w=40000)
    with pytest.raises(binding.JbfdError):
        binding.batch_prepare_raw(v, host)
    v = _views(1, n_points=0)
    v[0].points = 0                      # no points: a null pointer is fine
    binding.batch_prepare_raw(v, host)


def test_batch_run_rejects_bad_arguments(L):
    from paper_2601_01210_amd.binding import JBFD_EINVAL
    fake = C.c_void_p(0x1000)
    assert L.jbfd_batch_run(None, 5, 0, 0, None) == JBFD_EINVAL
    assert L.jbfd_batch_run(C.c_void_p(0x1004), 5, 0, 0, None) == JBFD_EINVAL
    assert L.jbfd_batch_run(fake, 33, 0, 0, None) == JBFD_EINVAL
    assert L.jbfd_batch_run(fake, -1, 0, 0, None) == JBFD_EINVAL
    assert L.jbfd_batch_run(fake, 5, 7, 0, None) == JBFD_EINVAL
    assert L.jbfd_batch_run(fake, 5, 0, 4, None) == JBFD_EINVAL    # unknown flag
    assert L.jbfd_batch_check(None, None) == JBFD_EINVAL
    assert L.jbfd_batch_check(C.c_void_p(0x1004), None) == JBFD_EINVAL


def test_two_stage_and_dense_reject_bad_arguments(L):
    from paper_2601_01210_amd.binding import (JBFD_EINVAL, JBFD_ENOSPC,
                                              JBFD_EUNSUPPORTED, TwoStage)
    fake = C.c_void_p(0x1000)
    ws = C.c_void_p(0x10000)
    assert L.jbfd_pool3(None, fake, fake, 8, 8, fake, fake, fake, None) == JBFD_EINVAL
    assert L.jbfd_pool3(fake, fake, fake, 0, 8, fake, fake, fake, None) == JBFD_EINVAL
    assert L.jbfd_restore_merge(fake, fake, fake, None, 8, 8, fake, fake,
                                None) == JBFD_EINVAL
    n = L.jbfd_two_stage_ws_bytes(1080, 1920)
    assert n >= 1080 * 1920 * 5 + 360 * 640 * 13
    assert L.jbfd_two_stage_ws_bytes(0, 5) == 0
    p = TwoStage(4, 2.0, 15.0, 2, 2.0, 15.0)
    args = lambda ws_, nb, pp: (fake, fake, fake, 1080, 1920, pp, fake, fake,
                                ws_, nb, None)
    assert L.jbfd_densify_two_stage(*args(ws, n - 1, C.byref(p))) == JBFD_ENOSPC
    assert L.jbfd_densify_two_stage(*args(C.c_void_p(0x10010), n,
                                          C.byref(p))) == JBFD_EINVAL
    assert L.jbfd_densify_two_stage(*args(ws, n, None)) == JBFD_EINVAL
    bad = TwoStage(4, 2.0, 15.0, 40, 2.0, 15.0)
    assert L.jbfd_densify_two_stage(*args(ws, n, C.byref(bad))) == JBFD_EINVAL
    bad = TwoStage(4, 0.1, 15.0, 2, 2.0, 15.0)
    assert L.jbfd_densify_two_stage(*args(ws, n, C.byref(bad))) == JBFD_EINVAL
    # dense kernel: radius <= 4, FP32, no aux
    dargs = lambda r, prec, aux: (fake, fake, fake, 8, 8, r, 2.0, 10.0, prec,
                                  fake, fake, aux, None, 0, 2, None)
    assert L.jbfd_densify(*dargs(5, 0, None)) == JBFD_EUNSUPPORTED
    assert L.jbfd_densify(*dargs(2, 1, None)) == JBFD_EUNSUPPORTED
    assert L.jbfd_densify(*dargs(2, 0, fake)) == JBFD_EUNSUPPORTED
    assert L.jbfd_densify(*dargs(2, 0, None)[:-2], 4, None) == JBFD_EINVAL


def test_occlusion_and_backproject_reject_bad_arguments(L):
    from paper_2601_01210_amd.binding import JBFD_EINVAL, JBFD_ENOSPC
    fake, other = C.c_void_p(0x1000), C.c_void_p(0x2000)
    assert L.jbfd_remove_occluded(fake, fake, 8, 8, 2, 0.1, fake, None) == JBFD_EINVAL
    assert L.jbfd_remove_occluded(fake, fake, 8, 8, 9, 0.1, other, None) == JBFD_EINVAL
    assert L.jbfd_remove_occluded(fake, fake, 8, 8, 2, -0.1, other, None) == JBFD_EINVAL
    assert L.jbfd_remove_occluded(fake, fake, 8, 8, 2, float("inf"), other,
                                  None) == JBFD_EINVAL
    pose = (C.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    K = _K(8, 6)
    ws = C.c_void_p(0x10000)
    n = L.jbfd_backproject_ws_bytes(6, 8)
    assert n >= 4
    call = lambda k, tau, w_, nb: L.jbfd_backproject(fake, fake, fake, 6, 8, pose,
                                                     C.byref(k), tau, fake, fake,
                                                     fake, w_, nb, None)
    assert call(K, 0.05, ws, n - 1 if n > 256 else 0) in (JBFD_ENOSPC, JBFD_EINVAL)
    assert call(K, float("nan"), ws, n) == JBFD_EINVAL
    assert call(_K(9, 6), 0.05, ws, n) == JBFD_EINVAL       # size mismatch
    zero = _K(8, 6)
    zero.fx = 0.0
    assert call(zero, 0.05, ws, n) == JBFD_EINVAL
    assert call(K, 0.05, C.c_void_p(0x10004), n) == JBFD_EINVAL
    # images above 2^26 pixels are refused (the write pass's chunk prefix
    # grows with the square of the image size)
    assert L.jbfd_backproject_ws_bytes(8192, 8192) > 0
    assert L.jbfd_backproject_ws_bytes(8193, 8193) == 0
    big = _K(8193, 8193)
    assert L.jbfd_backproject(fake, fake, fake, 8193, 8193, pose, C.byref(big), 0.05,
                              fake, fake, fake, ws, 1 << 40, None) == JBFD_EINVAL
    assert b"limit" in L.jbfd_last_error()


def test_afterimage_entry_points_reject_bad_arguments(L):
    from paper_2601_01210_amd.binding import JBFD_EINVAL
    fake = C.c_void_p(0x1000)
    mm = lambda tau, k, out: L.jbfd_motion_mask(fake, fake, 6, 8, tau, k, out,
                                                None)
    assert mm(30.0, -1, fake) == JBFD_EINVAL
    assert mm(30.0, 17, fake) == JBFD_EINVAL
    assert mm(-1.0, 2, fake) == JBFD_EINVAL
    assert mm(float("nan"), 2, fake) == JBFD_EINVAL
    assert mm(float("inf"), 2, fake) == JBFD_EINVAL
    assert mm(30.0, 2, None) == JBFD_EINVAL
    assert L.jbfd_motion_mask(fake, fake, 0, 8, 30.0, 2, fake, None) == JBFD_EINVAL
    pose = (C.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    K = _K()
    pm = lambda pts, n_, sw, mo: L.jbfd_project_motion(pts, n_, sw, 0, mo, pose,
                                                       C.byref(K), fake, None,
                                                       None, None)
    assert pm(fake, 10, fake, None) == JBFD_EINVAL          # no motion mask
    assert pm(fake, 10, None, fake) == JBFD_EINVAL          # no sweep ids
    assert pm(fake, -1, fake, fake) == JBFD_EINVAL
    assert pm(fake, 1 << 32, fake, fake) == JBFD_EINVAL
    bad = (C.c_double * 12)(1, 0, 0, 0, 0, float("nan"), 0, 0, 0, 0, 1, 0)
    assert L.jbfd_project_motion(fake, 10, fake, 0, fake, bad, C.byref(K), fake,
                                 None, None, None) == JBFD_EINVAL


def test_batch_prepare_checks_list_workspaces(L):
    """A view's list workspace must be 256-byte aligned and hold at least
    the list tables (host-side checks; nothing runs on a device)."""
    from paper_2601_01210_amd.binding import (JBFD_EINVAL, JBFD_ENOSPC, JBFD_OK,
                                              Intrinsics, View)
    import numpy as np
    fake = 0x100000
    v = View()
    v.points, v.n_points = fake, 10
    v.cam_from_world = (C.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    v.K = Intrinsics(4.0, 4.0, 4.0, 3.0, 64, 48)
    v.rgb = v.zbuf = v.sparse_depth = v.sparse_valid = fake
    v.dense_depth = v.dense_valid = fake
    v.radius, v.sigma_s, v.sigma_r = 5, 3.0, 12.0
    nb = L.jbfd_batch_table_bytes(1)
    host = np.zeros(nb, np.uint8)
    tables = L.jbfd_densify_ws_bytes(48, 64, 5, 0)
    prep = lambda: L.jbfd_batch_prepare(C.byref(v), 1, host.ctypes.data, nb)
    v.list_ws, v.list_ws_bytes = None, 0
    assert prep() == JBFD_OK                            # no lists: streams
    v.list_ws, v.list_ws_bytes = fake, tables
    assert prep() == JBFD_OK
    v.list_ws_bytes = tables - 1
    assert prep() == JBFD_ENOSPC
    v.list_ws, v.list_ws_bytes = fake + 4, tables
    assert prep() == JBFD_EINVAL


def test_noalloc_rejects_lists_beyond_its_array(L):
    """jbfd_project_densify_noalloc refuses, before any HIP call, a request
    whose sample lists may exceed its fixed array (4K image, 2M points,
    r = 32), and states the sizes; bad arguments are EINVAL as usual."""
    from paper_2601_01210_amd.binding import (JBFD_EINVAL, JBFD_ENOSPC,
                                              NOALLOC_WS_BYTES, Intrinsics)
    pose = (C.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    K = Intrinsics(1000.0, 1000.0, 1920.0, 1080.0, 3840, 2160)
    args = (fake, 2_000_000, pose, C.byref(K), fake, 32, 6.0, 15.0, 0, fake, fake,
            fake, fake, fake, None)
    assert L.jbfd_densify_ws_bytes(2160, 3840, 32, 2_000_000) > NOALLOC_WS_BYTES
    assert L.jbfd_project_densify_noalloc(*args) == JBFD_ENOSPC
    msg = L.jbfd_last_error().decode()
    assert "3840 x 2160" in msg and str(NOALLOC_WS_BYTES) in msg
    bad = list(args)
    bad[5] = 33                                   # radius above the maximum
    assert L.jbfd_project_densify_noalloc(*bad) == JBFD_EINVAL
    bad = list(args)
    bad[9] = None                                 # null key buffer
    assert L.jbfd_project_densify_noalloc(*bad) == JBFD_EINVAL
