"""FP64 CPU oracle (test infrastructure, not the product).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package. It wraps ``oracle.c`` (plain C, double precision,
no FMA contraction) through ctypes on numpy arrays, and shares nothing with
the GPU library or its Python binding.

Functions (the C file documents the formulas and the passages they follow):

* :func:`project`         Sec. 2 projection + nearest-depth z-buffer
* :func:`densify`         Eq. 1-4 gather (common factor exp(Emax) removed)
* :func:`densify_plain`   Eq. 1-4 literally (no rescaling)
* :func:`densify_alg1`    Algorithm 1 steps 1-5 (materialised weights)
* :func:`densify_spread`  per-pixel sensitivity of Eq. 1-4 to weight errors
* :func:`densify_grad`    gradient w.r.t. depths, sigma_s, sigma_r
* :func:`l1_holdout_loss` the self-supervised held-out L1 loss and its
                          upstream gradient
* :func:`pool3`, :func:`restore_merge`, :func:`densify_two_stage`
                          Sec. 5 two-stage filtering (pooled first pass,
                          full-resolution second pass)
* :func:`remove_occluded` Sec. 4.1 occluded-point removal
* :func:`backproject`     Sec. 5 contour removal + Sec. 2 coloured cloud
* :func:`motion_mask`, :func:`project_motion`
                          Sec. 4.1 afterimage removal
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
             "-shared", "-fPIC", "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", _LIB)
        if path == _LIB and not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(path)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        L.oracle_project.restype = C.c_int64
        L.oracle_project.argtypes = [f32p, C.c_int64, f64p, f64p, C.c_int32,
                                     C.c_int32, u64p, f32p, u8p]
        L.oracle_densify.restype = C.c_int64
        L.oracle_densify.argtypes = [f32p, u8p, u8p, C.c_int32, C.c_int32,
                                     C.c_int32, C.c_double, C.c_double, f64p,
                                     u8p, vp, vp, vp]
        L.oracle_densify_plain.restype = None
        L.oracle_densify_plain.argtypes = [f32p, u8p, u8p, C.c_int32,
                                           C.c_int32, C.c_int32, C.c_double,
                                           C.c_double, f64p, u8p]
        L.oracle_densify_alg1.restype = C.c_int
        L.oracle_densify_alg1.argtypes = [f32p, u8p, u8p, C.c_int32,
                                          C.c_int32, C.c_int32, C.c_double,
                                          C.c_double, f64p, u8p]
        L.oracle_densify_grad.restype = None
        L.oracle_densify_grad.argtypes = [f32p, u8p, u8p, C.c_int32,
                                          C.c_int32, C.c_int32, C.c_double,
                                          C.c_double, f64p, f64p,
                                          C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
        L.oracle_densify_spread.restype = None
        L.oracle_densify_spread.argtypes = [f32p, u8p, u8p, C.c_int32,
                                            C.c_int32, C.c_int32, C.c_double,
                                            C.c_double, f64p, f64p]
        L.oracle_pool3.restype = None
        L.oracle_pool3.argtypes = [f32p, u8p, u8p, C.c_int32, C.c_int32,
                                   f32p, u8p, u8p]
        L.oracle_restore_merge.restype = None
        L.oracle_restore_merge.argtypes = [f32p, u8p, f32p, u8p, C.c_int32,
                                           C.c_int32, f32p, u8p]
        L.oracle_remove_occluded.restype = None
        L.oracle_remove_occluded.argtypes = [f32p, u8p, C.c_int32, C.c_int32,
                                             C.c_int32, C.c_double, u8p]
        L.oracle_backproject.restype = C.c_int64
        L.oracle_backproject.argtypes = [f32p, u8p, u8p, C.c_int32, C.c_int32,
                                         f64p, f64p, C.c_double, f32p, u8p]
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
        L.oracle_motion_mask.restype = None
        L.oracle_motion_mask.argtypes = [u8p, u8p, C.c_int32, C.c_int32,
                                         C.c_double, C.c_int32, u8p]
        L.oracle_project_motion.restype = C.c_int64
        L.oracle_project_motion.argtypes = [f32p, C.c_int64, i8p, C.c_int8,
                                            u8p, f64p, f64p, C.c_int32,
                                            C.c_int32, u64p, f32p, u8p]
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def project(points, pose, intrinsics, width: int, height: int):
    """Returns (keys uint64 HxW, depth float32 HxW, valid uint8 HxW, landed).

    ``intrinsics`` is (fx, fy, cx, cy); ``pose`` is camera-from-world 3x4.
    """
    pts = _c(points, np.float32).reshape(-1, 3)
    pose = _c(pose, np.float64).reshape(12)
    intr = _c(intrinsics[:4], np.float64)
    keys = np.empty((height, width), np.uint64)
    depth = np.empty((height, width), np.float32)
    valid = np.empty((height, width), np.uint8)
    landed = lib().oracle_project(pts, pts.shape[0], pose, intr, width,
                                  height, keys, depth, valid)
    return keys, depth, valid, int(landed)


def densify(depth, valid, rgb, radius: int, sigma_s: float, sigma_r: float,
            want_stats: bool = False):
    """Eq. 1-4 in double. Returns (out float64 HxW, mask uint8 HxW) and, with
    ``want_stats``, a dict with per-pixel count, weight sum, Emax and the
    number of (pixel, sample) pairs."""
    d = _c(depth, np.float32)
    h, w = d.shape
    b = _c(valid, np.uint8)
    c = _c(rgb, np.uint8).reshape(h, w, 3)
    out = np.empty((h, w), np.float64)
    mask = np.empty((h, w), np.uint8)
    if want_stats:
        cnt = np.empty((h, w), np.int32)
        ws = np.empty((h, w), np.float64)
        em = np.empty((h, w), np.float64)
        pairs = lib().oracle_densify(d, b, c, h, w, radius, sigma_s, sigma_r,
                                     out, mask, cnt.ctypes.data,
                                     ws.ctypes.data, em.ctypes.data)
        return out, mask, dict(count=cnt, wsum=ws, emax=em, pairs=int(pairs))
    lib().oracle_densify(d, b, c, h, w, radius, sigma_s, sigma_r, out, mask,
                         None, None, None)
    return out, mask


def densify_plain(depth, valid, rgb, radius, sigma_s, sigma_r):
    d = _c(depth, np.float32)
    h, w = d.shape
    out = np.empty((h, w), np.float64)
    mask = np.empty((h, w), np.uint8)
    lib().oracle_densify_plain(d, _c(valid, np.uint8),
                               _c(rgb, np.uint8).reshape(h, w, 3), h, w,
                               radius, sigma_s, sigma_r, out, mask)
    return out, mask


def densify_alg1(depth, valid, rgb, radius, sigma_s, sigma_r):
    d = _c(depth, np.float32)
    h, w = d.shape
    if h * w * (2 * radius + 1) ** 2 > 50_000_000:
        raise ValueError("Algorithm 1 oracle materialises H*W*(2r+1)^2 "
                         "weights; input too large")
    out = np.empty((h, w), np.float64)
    mask = np.empty((h, w), np.uint8)
    rc = lib().oracle_densify_alg1(d, _c(valid, np.uint8),
                                   _c(rgb, np.uint8).reshape(h, w, 3), h, w,
                                   radius, sigma_s, sigma_r, out, mask)
    if rc != 0:
        raise MemoryError("oracle_densify_alg1: allocation failed")
    return out, mask


def densify_spread(depth, valid, rgb, radius, sigma_s, sigma_r, out):
    """Per pixel sum w_i |D_i - out| / sum w_i over the window (the weighted
    mean absolute deviation of the samples from ``out``, the oracle's own
    output): a relative error of at most e in every weight moves the output
    by at most e S / (1 - e). 0 where the window holds no sample."""
    d = _c(depth, np.float32)
    h, w = d.shape
    sp = np.empty((h, w), np.float64)
    lib().oracle_densify_spread(d, _c(valid, np.uint8),
                                _c(rgb, np.uint8).reshape(h, w, 3), h, w,
                                radius, sigma_s, sigma_r, _c(out, np.float64), sp)
    return sp


def densify_grad(depth, valid, rgb, radius, sigma_s, sigma_r, g):
    """Returns (grad_depth float64 HxW, grad_sigma_s, grad_sigma_r)."""
    d = _c(depth, np.float32)
    h, w = d.shape
    gd = np.empty((h, w), np.float64)
    gs = C.c_double()
    gr = C.c_double()
    lib().oracle_densify_grad(d, _c(valid, np.uint8),
                              _c(rgb, np.uint8).reshape(h, w, 3), h, w,
                              radius, sigma_s, sigma_r, _c(g, np.float64), gd,
                              C.byref(gs), C.byref(gr))
    return gd, gs.value, gr.value


def l1_holdout_loss(outs, masks, targets, target_valid):
    """Mean absolute error over held-out targets whose output pixel is valid.

    ``outs``/``masks`` are per-frame dense outputs, ``targets`` the held-out
    depths rasterised through their own z-buffer and ``target_valid`` their
    presence masks. Returns (loss, list of dL/d out per frame); sign(0) = 0.
    """
    use = [(tv == 1) & (m == 1) for tv, m in zip(target_valid, masks)]
    n = int(sum(int(u.sum()) for u in use))
    if n == 0:
        return 0.0, [np.zeros_like(o) for o in outs]
    loss = 0.0
    grads = []
    for o, t, u in zip(outs, targets, use):
        diff = np.where(u, o - t.astype(np.float64), 0.0)
        loss += float(np.abs(diff).sum())
        grads.append(np.sign(diff) / n)
    return loss / n, grads


def pool3(depth, valid, rgb):
    """3x3 pooling (readings in oracle.c): (depth1 float32, valid1 uint8,
    rgb1 uint8) at ((H+2)//3, (W+2)//3)."""
    d = _c(depth, np.float32)
    h, w = d.shape
    h1, w1 = (h + 2) // 3, (w + 2) // 3
    d1 = np.empty((h1, w1), np.float32)
    b1 = np.empty((h1, w1), np.uint8)
    c1 = np.empty((h1, w1, 3), np.uint8)
    lib().oracle_pool3(d, _c(valid, np.uint8), _c(rgb, np.uint8).reshape(h, w, 3),
                       h, w, d1, b1, c1)
    return d1, b1, c1


def restore_merge(depth, valid, out1, mask1):
    """Second-pass input: original depth where valid, else the first pass's
    output of the pixel's cell where that is valid."""
    d = _c(depth, np.float32)
    h, w = d.shape
    d2 = np.empty((h, w), np.float32)
    b2 = np.empty((h, w), np.uint8)
    lib().oracle_restore_merge(d, _c(valid, np.uint8), _c(out1, np.float32),
                               _c(mask1, np.uint8), h, w, d2, b2)
    return d2, b2


def densify_two_stage(depth, valid, rgb, r1, sigma_s1, sigma_r1, r2, sigma_s2,
                      sigma_r2, want_stages: bool = False):
    """Sec. 5 two-stage filter: pool3 -> densify (r1) -> restore_merge ->
    densify (r2). The first pass's output is kept as float32 between the
    stages (the precision of the stored depth map). Returns (out float64,
    mask) and, with ``want_stages``, a dict of the intermediates."""
    d1, b1, c1 = pool3(depth, valid, rgb)
    o1, m1 = densify(d1, b1, c1, r1, sigma_s1, sigma_r1)
    o1 = o1.astype(np.float32)
    d2, b2 = restore_merge(depth, valid, o1, m1)
    out, mask = densify(d2, b2, rgb, r2, sigma_s2, sigma_r2)
    if want_stages:
        return out, mask, dict(depth1=d1, valid1=b1, rgb1=c1, out1=o1,
                               mask1=m1, depth2=d2, valid2=b2)
    return out, mask


def remove_occluded(depth, valid, k: int, tau: float):
    """Valid mask with occluded samples dropped (readings in oracle.c)."""
    d = _c(depth, np.float32)
    h, w = d.shape
    out = np.empty((h, w), np.uint8)
    lib().oracle_remove_occluded(d, _c(valid, np.uint8), h, w, int(k),
                                 float(tau), out)
    return out


def backproject(dense, mask, rgb, pose, intrinsics, tau: float):
    """Coloured world points of the kept output pixels, row-major:
    (xyz float32 (n,3), rgb uint8 (n,3))."""
    d = _c(dense, np.float32)
    h, w = d.shape
    xyz = np.empty((h * w, 3), np.float32)
    col = np.empty((h * w, 3), np.uint8)
    n = lib().oracle_backproject(d, _c(mask, np.uint8),
                                 _c(rgb, np.uint8).reshape(h, w, 3), h, w,
                                 _c(pose, np.float64).reshape(12),
                                 _c(intrinsics[:4], np.float64), float(tau),
                                 xyz, col)
    return xyz[:n].copy(), col[:n].copy()


def motion_mask(rgb, rgb_prev, tau: float, k: int):
    """Closed motion mask between two RGB frames (readings in oracle.c)."""
    a = _c(rgb, np.uint8)
    h, w = a.shape[:2]
    out = np.empty((h, w), np.uint8)
    lib().oracle_motion_mask(a.reshape(h, w, 3), _c(rgb_prev, np.uint8).reshape(h, w, 3),
                             h, w, float(tau), int(k), out)
    return out


def project_motion(points, sweep, latest: int, motion, pose, intrinsics,
                   width: int, height: int):
    """project() with points of older sweeps dropped inside the motion
    mask. Returns (keys, depth, valid, landed)."""
    pts = _c(points, np.float32).reshape(-1, 3)
    keys = np.empty((height, width), np.uint64)
    depth = np.empty((height, width), np.float32)
    valid = np.empty((height, width), np.uint8)
    landed = lib().oracle_project_motion(pts, pts.shape[0], _c(sweep, np.int8),
                                         int(latest), _c(motion, np.uint8),
                                         _c(pose, np.float64).reshape(12),
                                         _c(intrinsics[:4], np.float64), width,
                                         height, keys, depth, valid)
    return keys, depth, valid, int(landed)
