"""ctypes binding of libjbfd.so (argument marshalling only).

Each function takes and returns torch tensors on the current HIP device and
enqueues work on torch's current stream; it validates shapes and dtypes so
that the C library receives exactly the layouts include/jbfd.h documents.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import enum
import math
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# JBFD_LIB names another build of the library (e.g. one whose host code is
# compiled with sanitizers); by default the in-tree libjbfd.so
_LIB_PATH = os.environ.get("JBFD_LIB") or os.path.join(_HERE, "libjbfd.so")

JBFD_OK, JBFD_EINVAL, JBFD_EUNSUPPORTED, JBFD_EHIP, JBFD_ENOSPC = range(5)


class Precision(enum.IntEnum):
    FP32 = 0
    FP16_RANGE = 1


class JbfdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"jbfd status {status}: {message}")
        self.status = status


class Intrinsics(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("width", C.c_int32),
                ("height", C.c_int32)]


class TwoStage(C.Structure):
    """Mirror of jbfd_two_stage (include/jbfd.h)."""
    _fields_ = [("radius1", C.c_int32), ("sigma_s1", C.c_float),
                ("sigma_r1", C.c_float), ("radius2", C.c_int32),
                ("sigma_s2", C.c_float), ("sigma_r2", C.c_float)]


class View(C.Structure):
    """Mirror of jbfd_view (include/jbfd.h)."""
    _fields_ = [("points", C.c_void_p), ("n_points", C.c_int64),
                ("cam_from_world", C.c_double * 12), ("K", Intrinsics),
                ("rgb", C.c_void_p), ("radius", C.c_int32),
                ("sigma_s", C.c_float), ("sigma_r", C.c_float),
                ("zbuf", C.c_void_p), ("sparse_depth", C.c_void_p),
                ("sparse_valid", C.c_void_p), ("dense_depth", C.c_void_p),
                ("dense_valid", C.c_void_p), ("list_ws", C.c_void_p),
                ("list_ws_bytes", C.c_size_t)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libjbfd.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it with "
                "`python -m paper_2601_01210_amd.build` (hipcc, gfx950)")
        L = C.CDLL(_LIB_PATH)
        vp, i32, i64, f32, sz = (C.c_void_p, C.c_int32, C.c_int64, C.c_float,
                                 C.c_size_t)
        L.jbfd_abi_version.restype = C.c_int
        L.jbfd_status_string.restype = C.c_char_p
        L.jbfd_status_string.argtypes = [C.c_int]
        L.jbfd_last_error.restype = C.c_char_p
        L.jbfd_project.restype = C.c_int
        L.jbfd_project.argtypes = [vp, i64, C.POINTER(C.c_double),
                                   C.POINTER(Intrinsics), vp, vp, vp, vp]
        L.jbfd_project_recycled.restype = C.c_int
        L.jbfd_project_recycled.argtypes = L.jbfd_project.argtypes
        L.jbfd_zbuf_clear.restype = C.c_int
        L.jbfd_zbuf_clear.argtypes = [vp, i32, i32, vp]
        L.jbfd_project_densify.restype = C.c_int
        L.jbfd_project_densify.argtypes = [vp, i64, C.POINTER(C.c_double),
                                           C.POINTER(Intrinsics), vp, i32, f32, f32,
                                           C.c_int, vp, vp, vp, vp, vp, vp, sz, vp]
        L.jbfd_project_densify_noalloc.restype = C.c_int
        L.jbfd_project_densify_noalloc.argtypes = [
            vp, i64, C.POINTER(C.c_double), C.POINTER(Intrinsics), vp, i32, f32, f32,
            C.c_int, vp, vp, vp, vp, vp, vp]
        L.jbfd_densify.restype = C.c_int
        L.jbfd_densify.argtypes = [vp, vp, vp, i32, i32, i32, f32, f32,
                                   C.c_int, vp, vp, vp, vp, sz, C.c_uint32,
                                   vp]
        L.jbfd_densify_prepare.restype = C.c_int
        L.jbfd_densify_prepare.argtypes = [vp, vp, vp, i32, i32, i32, vp, sz,
                                           vp]
        L.jbfd_densify_ws_bytes.restype = sz
        L.jbfd_densify_ws_bytes.argtypes = [i32, i32, i32, i64]
        L.jbfd_densify_backward.restype = C.c_int
        L.jbfd_densify_backward.argtypes = [vp, vp, vp, i32, i32, i32, f32,
                                            f32, vp, vp, vp, vp, vp, vp, sz,
                                            vp]
        L.jbfd_densify_backward_ws_bytes.restype = sz
        L.jbfd_densify_backward_ws_bytes.argtypes = [i32, i32]
        L.jbfd_pool3.restype = C.c_int
        L.jbfd_pool3.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp]
        L.jbfd_restore_merge.restype = C.c_int
        L.jbfd_restore_merge.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, vp]
        L.jbfd_two_stage_ws_bytes.restype = sz
        L.jbfd_two_stage_ws_bytes.argtypes = [i32, i32]
        L.jbfd_densify_two_stage.restype = C.c_int
        L.jbfd_densify_two_stage.argtypes = [vp, vp, vp, i32, i32,
                                             C.POINTER(TwoStage), vp, vp, vp,
                                             sz, vp]
        L.jbfd_remove_occluded.restype = C.c_int
        L.jbfd_remove_occluded.argtypes = [vp, vp, i32, i32, i32, f32, vp, vp]
        L.jbfd_backproject_ws_bytes.restype = sz
        L.jbfd_backproject_ws_bytes.argtypes = [i32, i32]
        L.jbfd_backproject.restype = C.c_int
        L.jbfd_backproject.argtypes = [vp, vp, vp, i32, i32,
                                       C.POINTER(C.c_double),
                                       C.POINTER(Intrinsics), f32, vp, vp, vp,
                                       vp, sz, vp]
        L.jbfd_motion_mask.restype = C.c_int
        L.jbfd_motion_mask.argtypes = [vp, vp, i32, i32, f32, i32, vp, vp]
        L.jbfd_project_motion.restype = C.c_int
        L.jbfd_project_motion.argtypes = [vp, i64, vp, C.c_int8, vp,
                                          C.POINTER(C.c_double),
                                          C.POINTER(Intrinsics), vp, vp, vp,
                                          vp]
        L.jbfd_batch_table_bytes.restype = sz
        L.jbfd_batch_table_bytes.argtypes = [i32]
        L.jbfd_batch_prepare.restype = C.c_int
        L.jbfd_batch_prepare.argtypes = [C.POINTER(View), i32, vp, sz]
        L.jbfd_batch_run.restype = C.c_int
        L.jbfd_batch_run.argtypes = [vp, i32, C.c_int, C.c_uint32, vp]
        L.jbfd_batch_check.restype = C.c_int
        L.jbfd_batch_check.argtypes = [vp, vp]
        _lib = L
    return _lib


def abi_version() -> int:
    return lib().jbfd_abi_version()


def _check(status: int):
    if status != JBFD_OK:
        msg = lib().jbfd_last_error().decode()
        raise JbfdError(status, msg)


def _torch():
    import torch
    return torch


def _stream(device=None):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _need(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got "
                         f"{tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _pose_array(pose) -> C.Array:
    a = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(12))
    return (C.c_double * 12)(*a.tolist())


def project(points, pose, intrinsics: Sequence[float], width: int,
            height: int, zbuf=None, depth=None, valid=None,
            want_sparse: bool = True, recycle: bool = False):
    """Nearest-depth projection (jbfd_project).

    points      (N,3) float32 device tensor, world xyz in merged order
    pose        3x4 camera-from-world [R|t] (host array-like)
    intrinsics  (fx, fy, cx, cy)
    recycle     use jbfd_project_recycled: ``zbuf`` (required) holds only
                empty keys (see :func:`zbuf_clear`) and is left so; the
                winning keys are not returned
    Returns (zbuf uint64-as-int64 (H,W), depth float32 (H,W), valid uint8
    (H,W)); depth/valid are None when ``want_sparse`` is False.
    """
    torch = _torch()
    _need(points, torch.float32, None, "points")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must have shape (N, 3)")
    dev = points.device
    if zbuf is None:
        if recycle:
            raise ValueError("recycle needs a key buffer cleared by zbuf_clear")
        zbuf = torch.empty((height, width), dtype=torch.int64, device=dev)
    _need(zbuf, torch.int64, (height, width), "zbuf")
    if want_sparse:
        if depth is None:
            depth = torch.empty((height, width), dtype=torch.float32, device=dev)
        if valid is None:
            valid = torch.empty((height, width), dtype=torch.uint8, device=dev)
        _need(depth, torch.float32, (height, width), "depth")
        _need(valid, torch.uint8, (height, width), "valid")
    K = Intrinsics(float(intrinsics[0]), float(intrinsics[1]),
                   float(intrinsics[2]), float(intrinsics[3]), int(width),
                   int(height))
    if recycle:
        if not want_sparse:
            raise ValueError("recycle needs the sparse depth and mask")
        fn = lib().jbfd_project_recycled
    else:
        fn = lib().jbfd_project
    _check(fn(_ptr(points), int(points.shape[0]), _pose_array(pose), C.byref(K),
              _ptr(zbuf), _ptr(depth), _ptr(valid), _stream(dev)))
    return zbuf, depth, valid


def project_densify(points, pose, intrinsics: Sequence[float], width: int,
                    height: int, rgb, radius: int, sigma_s: float, sigma_r: float,
                    zbuf, ws, precision: Precision = Precision.FP32, depth=None,
                    valid=None, out=None, mask=None):
    """Projection and filter in one call (jbfd_project_densify): the decode
    of the key image is fused into the list build. ``zbuf`` holds only empty
    keys (see :func:`zbuf_clear`) and is left so; ``ws`` is a list workspace
    (:func:`densify_workspace`). Returns (depth, valid, out, mask)."""
    torch = _torch()
    _need(points, torch.float32, None, "points")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must have shape (N, 3)")
    dev = points.device
    h, w = int(height), int(width)
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    _need(zbuf, torch.int64, (h, w), "zbuf")
    _need(ws, torch.uint8, None, "ws")
    if depth is None:
        depth = torch.empty((h, w), dtype=torch.float32, device=dev)
    if valid is None:
        valid = torch.empty((h, w), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty((h, w), dtype=torch.float32, device=dev)
    if mask is None:
        mask = torch.empty((h, w), dtype=torch.uint8, device=dev)
    for t, dt, nm in ((depth, torch.float32, "depth"), (valid, torch.uint8, "valid"),
                      (out, torch.float32, "out"), (mask, torch.uint8, "mask")):
        _need(t, dt, (h, w), nm)
    K = Intrinsics(float(intrinsics[0]), float(intrinsics[1]),
                   float(intrinsics[2]), float(intrinsics[3]), w, h)
    _check(lib().jbfd_project_densify(
        _ptr(points), int(points.shape[0]), _pose_array(pose), C.byref(K), _ptr(rgb),
        int(radius), float(sigma_s), float(sigma_r), int(precision), _ptr(zbuf),
        _ptr(depth), _ptr(valid), _ptr(out), _ptr(mask), _ptr(ws), ws.numel(),
        _stream(dev)))
    return depth, valid, out, mask


NOALLOC_WS_BYTES = 32 << 20   # JBFD_NOALLOC_WS_BYTES


def project_densify_noalloc(points, pose, intrinsics: Sequence[float], width: int,
                            height: int, rgb, radius: int, sigma_s: float,
                            sigma_r: float, zbuf,
                            precision: Precision = Precision.FP32, depth=None,
                            valid=None, out=None, mask=None):
    """:func:`project_densify` without a workspace
    (jbfd_project_densify_noalloc): the sample lists live in the library's
    fixed per-GPU array. Raises JbfdError (JBFD_ENOSPC) when the lists of
    this size may not fit it. Returns (depth, valid, out, mask)."""
    torch = _torch()
    _need(points, torch.float32, None, "points")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must have shape (N, 3)")
    dev = points.device
    h, w = int(height), int(width)
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    _need(zbuf, torch.int64, (h, w), "zbuf")
    if depth is None:
        depth = torch.empty((h, w), dtype=torch.float32, device=dev)
    if valid is None:
        valid = torch.empty((h, w), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty((h, w), dtype=torch.float32, device=dev)
    if mask is None:
        mask = torch.empty((h, w), dtype=torch.uint8, device=dev)
    for t, dt, nm in ((depth, torch.float32, "depth"), (valid, torch.uint8, "valid"),
                      (out, torch.float32, "out"), (mask, torch.uint8, "mask")):
        _need(t, dt, (h, w), nm)
    K = Intrinsics(float(intrinsics[0]), float(intrinsics[1]),
                   float(intrinsics[2]), float(intrinsics[3]), w, h)
    _check(lib().jbfd_project_densify_noalloc(
        _ptr(points), int(points.shape[0]), _pose_array(pose), C.byref(K), _ptr(rgb),
        int(radius), float(sigma_s), float(sigma_r), int(precision), _ptr(zbuf),
        _ptr(depth), _ptr(valid), _ptr(out), _ptr(mask), _stream(dev)))
    return depth, valid, out, mask


def zbuf_clear(zbuf):
    """Fill a (H,W) int64 device key buffer with empty keys (jbfd_zbuf_clear)."""
    torch = _torch()
    _need(zbuf, torch.int64, None, "zbuf")
    if zbuf.dim() != 2:
        raise ValueError("zbuf must have shape (H, W)")
    h, w = zbuf.shape
    _check(lib().jbfd_zbuf_clear(_ptr(zbuf), h, w, _stream(zbuf.device)))
    return zbuf


def densify_ws_bytes(h: int, w: int, radius: int, max_samples: int) -> int:
    return int(lib().jbfd_densify_ws_bytes(h, w, radius, max_samples))


def densify_workspace(h: int, w: int, radius: int, max_samples: int,
                      device=None):
    """Device workspace for jbfd_densify's sample lists (uint8 tensor)."""
    torch = _torch()
    n = densify_ws_bytes(h, w, radius, max_samples)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


JBFD_LISTS_READY, JBFD_DENSE = 1, 2


def densify(depth, valid, rgb, radius: int, sigma_s: float, sigma_r: float,
            precision: Precision = Precision.FP32, out=None, mask=None,
            aux=None, want_aux: bool = False, ws="auto",
            max_samples: Optional[int] = None, lists_ready: bool = False,
            dense: bool = False):
    """Joint bilateral filter (jbfd_densify).

    depth (H,W) float32, valid (H,W) uint8, rgb (H,W,3) uint8, all on the
    device. ``ws`` is a workspace tensor from :func:`densify_workspace`,
    ``None`` (filter streams the inputs directly) or "auto" (allocate one
    sized for ``max_samples`` valid samples, default H*W/4).
    ``dense`` selects the kernel for inputs where most pixels hold a
    sample (radius <= 4, FP32, no aux; the workspace is not used).
    Returns (dense depth float32, mask uint8[, aux float32 (H,W,2)]).
    """
    torch = _torch()
    _need(depth, torch.float32, None, "depth")
    if depth.dim() != 2:
        raise ValueError("depth must be (H, W)")
    h, w = depth.shape
    _need(valid, torch.uint8, (h, w), "valid")
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    dev = depth.device
    if out is None:
        out = torch.empty((h, w), dtype=torch.float32, device=dev)
    if mask is None:
        mask = torch.empty((h, w), dtype=torch.uint8, device=dev)
    _need(out, torch.float32, (h, w), "out")
    _need(mask, torch.uint8, (h, w), "mask")
    if want_aux and aux is None:
        aux = torch.empty((h, w, 2), dtype=torch.float32, device=dev)
    if aux is not None:
        _need(aux, torch.float32, (h, w, 2), "aux")
    if dense:
        ws = None
    if isinstance(ws, str):
        if ws != "auto":
            raise ValueError("ws must be a tensor, None or 'auto'")
        ms = max_samples if max_samples is not None else (h * w) // 4
        ws = densify_workspace(h, w, radius, ms, dev)
    if ws is not None:
        _need(ws, torch.uint8, None, "ws")
    _check(lib().jbfd_densify(_ptr(depth), _ptr(valid), _ptr(rgb), h, w,
                              int(radius), float(sigma_s), float(sigma_r),
                              int(precision), _ptr(out), _ptr(mask),
                              _ptr(aux), _ptr(ws),
                              ws.numel() if ws is not None else 0,
                              (JBFD_LISTS_READY if lists_ready else 0) |
                              (JBFD_DENSE if dense else 0), _stream(dev)))
    if aux is not None:
        return out, mask, aux
    return out, mask


def densify_prepare(depth, valid, rgb, radius: int, ws):
    """Build the per-strip sample lists of jbfd_densify in ``ws``."""
    torch = _torch()
    h, w = depth.shape
    _need(depth, torch.float32, (h, w), "depth")
    _need(valid, torch.uint8, (h, w), "valid")
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    _need(ws, torch.uint8, None, "ws")
    _check(lib().jbfd_densify_prepare(_ptr(depth), _ptr(valid), _ptr(rgb), h,
                                      w, int(radius), _ptr(ws), ws.numel(),
                                      _stream(depth.device)))
    return ws


def densify_backward(depth, valid, rgb, radius: int, sigma_s: float,
                     sigma_r: float, out, aux, grad_out, grad_depth=None,
                     grad_sigmas=None, ws=None):
    """Gradient through the filter (jbfd_densify_backward).

    Returns (grad_depth float32 (H,W), grad_sigmas float64 (2,) device tensor
    holding dL/dsigma_s, dL/dsigma_r).
    """
    torch = _torch()
    h, w = depth.shape
    _need(depth, torch.float32, (h, w), "depth")
    _need(valid, torch.uint8, (h, w), "valid")
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    _need(out, torch.float32, (h, w), "out")
    _need(aux, torch.float32, (h, w, 2), "aux")
    _need(grad_out, torch.float32, (h, w), "grad_out")
    dev = depth.device
    if grad_depth is None:
        grad_depth = torch.empty((h, w), dtype=torch.float32, device=dev)
    if grad_sigmas is None:
        grad_sigmas = torch.empty(2, dtype=torch.float64, device=dev)
    nbytes = int(lib().jbfd_densify_backward_ws_bytes(h, w))
    if ws is None:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    _check(lib().jbfd_densify_backward(
        _ptr(depth), _ptr(valid), _ptr(rgb), h, w, int(radius),
        float(sigma_s), float(sigma_r), _ptr(out), _ptr(aux), _ptr(grad_out),
        _ptr(grad_depth), _ptr(grad_sigmas), _ptr(ws), ws.numel(),
        _stream(dev)))
    return grad_depth, grad_sigmas


# ---------------------------------------------------------------------------
# batches of views (jbfd_batch_prepare / jbfd_batch_run)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class BatchView:
    """One view of a batch: inputs plus the device buffers the batch writes.

    points (N,3) float32 and rgb (H,W,3) uint8 are device tensors; pose is a
    3x4 camera-from-world matrix and intrinsics (fx, fy, cx, cy), both host.
    ``n_points`` may be smaller than ``points.shape[0]`` (a slot buffer
    sized for the largest frame).
    """
    points: object
    pose: object
    intrinsics: Tuple[float, float, float, float]
    width: int
    height: int
    rgb: object
    radius: int
    sigma_s: float
    sigma_r: float
    zbuf: object = None
    sparse_depth: object = None
    sparse_valid: object = None
    dense_depth: object = None
    dense_valid: object = None
    n_points: Optional[int] = None
    list_ws: object = None
    lists: bool = False
    list_radius: Optional[int] = None

    def allocate(self, device=None):
        """Allocate any output buffer that is still None, and (``lists``) a
        sample-list workspace sized for every point of the buffer at
        ``list_radius`` (default: the view's radius); with a larger radius
        the blocks whose lists do not fit stream their halo instead.

        Without lists the batch filter streams each block's halo. At small
        radii that is the faster choice for a batch (building the lists of
        eight 720p/1080p views costs more than the walk saves at r = 5); at
        large radii the list walk is much cheaper than streaming.

        A new key buffer is cleared to empty keys (jbfd_zbuf_clear), as a
        batch run requires on entry; every batch run leaves it so."""
        torch = _torch()
        dev = device if device is not None else self.points.device
        hw = (self.height, self.width)
        if self.lists and self.list_ws is None:
            r = self.radius if self.list_radius is None else self.list_radius
            self.list_ws = densify_workspace(self.height, self.width, int(r),
                                             max(int(self.points.shape[0]), 1), dev)
        if self.zbuf is None:
            self.zbuf = zbuf_clear(torch.empty(hw, dtype=torch.int64, device=dev))
        if self.sparse_depth is None:
            self.sparse_depth = torch.empty(hw, dtype=torch.float32, device=dev)
        if self.sparse_valid is None:
            self.sparse_valid = torch.empty(hw, dtype=torch.uint8, device=dev)
        if self.dense_depth is None:
            self.dense_depth = torch.empty(hw, dtype=torch.float32, device=dev)
        if self.dense_valid is None:
            self.dense_valid = torch.empty(hw, dtype=torch.uint8, device=dev)
        return self

    def descriptor(self) -> View:
        torch = _torch()
        h, w = self.height, self.width
        _need(self.points, torch.float32, None, "points")
        if self.points.dim() != 2 or self.points.shape[1] != 3:
            raise ValueError("points must have shape (N, 3)")
        n = self.points.shape[0] if self.n_points is None else int(self.n_points)
        if not 0 <= n <= self.points.shape[0]:
            raise ValueError("n_points exceeds the points buffer")
        _need(self.rgb, torch.uint8, (h, w, 3), "rgb")
        _need(self.zbuf, torch.int64, (h, w), "zbuf")
        _need(self.sparse_depth, torch.float32, (h, w), "sparse_depth")
        _need(self.sparse_valid, torch.uint8, (h, w), "sparse_valid")
        _need(self.dense_depth, torch.float32, (h, w), "dense_depth")
        _need(self.dense_valid, torch.uint8, (h, w), "dense_valid")
        k = self.intrinsics
        v = View()
        v.points = self.points.data_ptr()
        v.n_points = n
        v.cam_from_world = _pose_array(self.pose)
        v.K = Intrinsics(float(k[0]), float(k[1]), float(k[2]), float(k[3]),
                         int(w), int(h))
        v.rgb = self.rgb.data_ptr()
        v.radius = int(self.radius)
        v.sigma_s = float(self.sigma_s)
        v.sigma_r = float(self.sigma_r)
        v.zbuf = self.zbuf.data_ptr()
        v.sparse_depth = self.sparse_depth.data_ptr()
        v.sparse_valid = self.sparse_valid.data_ptr()
        v.dense_depth = self.dense_depth.data_ptr()
        v.dense_valid = self.dense_valid.data_ptr()
        if self.list_ws is not None:
            _need(self.list_ws, torch.uint8, None, "list_ws")
            v.list_ws = self.list_ws.data_ptr()
            v.list_ws_bytes = self.list_ws.numel()
        return v


def batch_table_bytes(n_views: int) -> int:
    return int(lib().jbfd_batch_table_bytes(int(n_views)))


def batch_prepare_raw(views: Sequence[View], host) -> None:
    """jbfd_batch_prepare on plain descriptors into host memory ``host``
    (a writable buffer: numpy uint8 array or CPU torch uint8 tensor)."""
    arr = (View * len(views))(*views)
    if hasattr(host, "data_ptr"):
        ptr, nbytes = host.data_ptr(), host.numel()
    else:
        ptr, nbytes = host.ctypes.data, host.nbytes
    _check(lib().jbfd_batch_prepare(arr, len(views), C.c_void_p(ptr), nbytes))


def batch_upload(views: Sequence[BatchView], table=None, host=None):
    """Serialise ``views`` and copy the table to the device on the current
    stream. ``table`` (device uint8) and ``host`` (pinned CPU uint8) are
    reused when given; the host buffer must not be rewritten until the copy
    has run (synchronise the stream or alternate two host buffers).
    Returns (table, host)."""
    torch = _torch()
    n = batch_table_bytes(len(views))
    dev = views[0].points.device
    if host is None:
        host = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    if table is None:
        table = torch.empty(n, dtype=torch.uint8, device=dev)
    if host.numel() < n or table.numel() < n:
        raise ValueError(f"batch table needs {n} bytes")
    batch_prepare_raw([v.descriptor() for v in views], host)
    table[:n].copy_(host[:n], non_blocking=True)
    return table, host


JBFD_BATCH_LISTS, JBFD_BATCH_STAGED = 1, 2


def batch_run(table, max_radius: int, precision: Precision = Precision.FP32,
              lists: bool = False, staged: bool = False):
    """Enqueue jbfd_batch_run on the current stream (graph-capturable): one
    persistent launch by default. ``staged``: the same work as a sequence of
    launches (JBFD_BATCH_STAGED); ``lists``: a launch sequence that builds
    and walks the sample lists of the views that carry a list workspace
    (JBFD_BATCH_LISTS); otherwise every view streams."""
    torch = _torch()
    _need(table, torch.uint8, None, "table")
    flags = (JBFD_BATCH_LISTS if lists else 0) | (JBFD_BATCH_STAGED if staged else 0)
    _check(lib().jbfd_batch_run(_ptr(table), int(max_radius), int(precision), flags,
                                _stream(table.device)))


def batch_check(table):
    """Synchronise the current stream and raise JbfdError if a run on this
    table since its preparation met a view whose radius exceeded the run's
    max_radius (JBFD_EINVAL) or gave up a wait (JBFD_EHIP)."""
    torch = _torch()
    _need(table, torch.uint8, None, "table")
    _check(lib().jbfd_batch_check(_ptr(table), _stream(table.device)))


# ---------------------------------------------------------------------------
# two-stage filtering (jbfd_pool3, jbfd_restore_merge, jbfd_densify_two_stage)
# ---------------------------------------------------------------------------

def pool3(depth, valid, rgb):
    """3x3 pooling: (depth1 float32, valid1 uint8, rgb1 uint8) at
    ((H+2)//3, (W+2)//3)."""
    torch = _torch()
    h, w = depth.shape
    _need(depth, torch.float32, (h, w), "depth")
    _need(valid, torch.uint8, (h, w), "valid")
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    h1, w1 = (h + 2) // 3, (w + 2) // 3
    dev = depth.device
    d1 = torch.empty((h1, w1), dtype=torch.float32, device=dev)
    b1 = torch.empty((h1, w1), dtype=torch.uint8, device=dev)
    c1 = torch.empty((h1, w1, 3), dtype=torch.uint8, device=dev)
    _check(lib().jbfd_pool3(_ptr(depth), _ptr(valid), _ptr(rgb), h, w, _ptr(d1),
                            _ptr(b1), _ptr(c1), _stream(dev)))
    return d1, b1, c1


def restore_merge(depth, valid, out1, mask1):
    """Second-pass input: the original depth where valid, else the first
    pass's output of the pixel's 3x3 cell where that is valid."""
    torch = _torch()
    h, w = depth.shape
    h1, w1 = (h + 2) // 3, (w + 2) // 3
    _need(depth, torch.float32, (h, w), "depth")
    _need(valid, torch.uint8, (h, w), "valid")
    _need(out1, torch.float32, (h1, w1), "out1")
    _need(mask1, torch.uint8, (h1, w1), "mask1")
    dev = depth.device
    d2 = torch.empty((h, w), dtype=torch.float32, device=dev)
    b2 = torch.empty((h, w), dtype=torch.uint8, device=dev)
    _check(lib().jbfd_restore_merge(_ptr(depth), _ptr(valid), _ptr(out1),
                                    _ptr(mask1), h, w, _ptr(d2), _ptr(b2),
                                    _stream(dev)))
    return d2, b2


def two_stage_ws_bytes(h: int, w: int) -> int:
    return int(lib().jbfd_two_stage_ws_bytes(h, w))


def densify_two_stage(depth, valid, rgb, radius1: int, sigma_s1: float,
                      sigma_r1: float, radius2: int, sigma_s2: float,
                      sigma_r2: float, out=None, mask=None, ws=None):
    """Two-stage filter (jbfd_densify_two_stage): returns (dense depth,
    mask); ``ws`` (device uint8, two_stage_ws_bytes) is allocated if None."""
    torch = _torch()
    h, w = depth.shape
    _need(depth, torch.float32, (h, w), "depth")
    _need(valid, torch.uint8, (h, w), "valid")
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    dev = depth.device
    if out is None:
        out = torch.empty((h, w), dtype=torch.float32, device=dev)
    if mask is None:
        mask = torch.empty((h, w), dtype=torch.uint8, device=dev)
    if ws is None:
        ws = torch.empty(max(two_stage_ws_bytes(h, w), 256), dtype=torch.uint8,
                         device=dev)
    _need(ws, torch.uint8, None, "ws")
    p = TwoStage(int(radius1), float(sigma_s1), float(sigma_r1), int(radius2),
                 float(sigma_s2), float(sigma_r2))
    _check(lib().jbfd_densify_two_stage(_ptr(depth), _ptr(valid), _ptr(rgb), h, w,
                                        C.byref(p), _ptr(out), _ptr(mask),
                                        _ptr(ws), ws.numel(), _stream(dev)))
    return out, mask


# ---------------------------------------------------------------------------
# occluded-point removal, contour removal and back-projection
# ---------------------------------------------------------------------------

def remove_occluded(depth, valid, k: int, tau: float, out=None):
    """jbfd_remove_occluded: the valid mask with occluded samples dropped."""
    torch = _torch()
    h, w = depth.shape
    _need(depth, torch.float32, (h, w), "depth")
    _need(valid, torch.uint8, (h, w), "valid")
    if out is None:
        out = torch.empty((h, w), dtype=torch.uint8, device=depth.device)
    _need(out, torch.uint8, (h, w), "out")
    _check(lib().jbfd_remove_occluded(_ptr(depth), _ptr(valid), h, w, int(k),
                                      float(tau), _ptr(out),
                                      _stream(depth.device)))
    return out


def backproject_ws_bytes(h: int, w: int) -> int:
    return int(lib().jbfd_backproject_ws_bytes(h, w))


def backproject(dense, mask, rgb, pose, intrinsics, tau: float = float("inf"),
                xyz=None, rgb_out=None, count=None, ws=None):
    """jbfd_backproject: returns (xyz float32 (H*W,3), rgb uint8 (H*W,3),
    count int64 (1,)), all on the device; the first count rows are the
    points in row-major pixel order (read count to slice on the host)."""
    torch = _torch()
    h, w = dense.shape
    _need(dense, torch.float32, (h, w), "dense")
    _need(mask, torch.uint8, (h, w), "mask")
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    dev = dense.device
    if xyz is None:
        xyz = torch.empty((h * w, 3), dtype=torch.float32, device=dev)
    if rgb_out is None:
        rgb_out = torch.empty((h * w, 3), dtype=torch.uint8, device=dev)
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device=dev)
    if ws is None:
        ws = torch.empty(max(backproject_ws_bytes(h, w), 256), dtype=torch.uint8,
                         device=dev)
    _need(xyz, torch.float32, (h * w, 3), "xyz")
    _need(rgb_out, torch.uint8, (h * w, 3), "rgb_out")
    _need(count, torch.int64, (1,), "count")
    _need(ws, torch.uint8, None, "ws")
    K = Intrinsics(float(intrinsics[0]), float(intrinsics[1]),
                   float(intrinsics[2]), float(intrinsics[3]), int(w), int(h))
    _check(lib().jbfd_backproject(_ptr(dense), _ptr(mask), _ptr(rgb), h, w,
                                  _pose_array(pose), C.byref(K), float(tau),
                                  _ptr(xyz), _ptr(rgb_out), _ptr(count),
                                  _ptr(ws), ws.numel(), _stream(dev)))
    return xyz, rgb_out, count


# ---------------------------------------------------------------------------
# afterimage removal
# ---------------------------------------------------------------------------

def motion_mask(rgb, rgb_prev, tau: float, k: int, out=None):
    """jbfd_motion_mask: closed mask of pixels whose colour changed by more
    than tau between two (H,W,3) uint8 frames."""
    torch = _torch()
    h, w = rgb.shape[:2]
    _need(rgb, torch.uint8, (h, w, 3), "rgb")
    _need(rgb_prev, torch.uint8, (h, w, 3), "rgb_prev")
    dev = rgb.device
    if out is None:
        out = torch.empty((h, w), dtype=torch.uint8, device=dev)
    _need(out, torch.uint8, (h, w), "out")
    _check(lib().jbfd_motion_mask(_ptr(rgb), _ptr(rgb_prev), h, w, float(tau),
                                  int(k), _ptr(out), _stream(dev)))
    return out


def project_motion(points, sweep, latest: int, motion, pose,
                   intrinsics: Sequence[float], width: int, height: int,
                   zbuf=None, depth=None, valid=None, want_sparse: bool = True):
    """jbfd_project_motion: project() with points of sweeps other than
    ``latest`` dropped where ``motion`` (H,W uint8) is set. ``sweep`` is an
    (N,) int8 device tensor."""
    torch = _torch()
    _need(points, torch.float32, None, "points")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must have shape (N, 3)")
    n = int(points.shape[0])
    _need(sweep, torch.int8, (n,), "sweep")
    _need(motion, torch.uint8, (height, width), "motion")
    dev = points.device
    if zbuf is None:
        zbuf = torch.empty((height, width), dtype=torch.int64, device=dev)
    _need(zbuf, torch.int64, (height, width), "zbuf")
    if want_sparse:
        if depth is None:
            depth = torch.empty((height, width), dtype=torch.float32, device=dev)
        if valid is None:
            valid = torch.empty((height, width), dtype=torch.uint8, device=dev)
        _need(depth, torch.float32, (height, width), "depth")
        _need(valid, torch.uint8, (height, width), "valid")
    K = Intrinsics(float(intrinsics[0]), float(intrinsics[1]),
                   float(intrinsics[2]), float(intrinsics[3]), int(width),
                   int(height))
    _check(lib().jbfd_project_motion(_ptr(points), n, _ptr(sweep), int(latest),
                                     _ptr(motion), _pose_array(pose), C.byref(K),
                                     _ptr(zbuf), _ptr(depth), _ptr(valid),
                                     _stream(dev)))
    return zbuf, depth, valid
