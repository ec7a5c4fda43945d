"""Seeded synthetic scenes shaped like the paper's capture (Sec. 2 and Sec. 5).

The paper's data (one RGB camera at 1920x1080 and three interleaved LiDAR
sweeps per viewpoint, about 1e5 merged points per frame) is not public, so
every input here is generated from a seed:

* a static scene of axis-aligned boxes and planes, each with a base colour,
  optional two-shade checker/stripe texture, and an optional back wall;
* an RGB frame and a ground-truth Z map rendered by casting one ray through
  each pixel centre of a pinhole camera (world frame == camera frame,
  +Z forward, +Y down);
* LiDAR sweeps cast from their own origins, first hit per ray, with
  Gaussian range noise along the ray; points are emitted as float32 world
  coordinates in sweep order (the merge of Sec. 4.1 is this concatenation).

This module only *creates* inputs. It contains none of the densification
method's arithmetic (no projection into the image, no z-buffer, no filter),
so both the oracle and the GPU path can consume its output without sharing
any of the computation under test.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# --------------------------------------------------------------------------
# data classes
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    # camera-from-world rigid transform, row-major 3x4 [R|t], float64
    pose: np.ndarray = dataclasses.field(
        default_factory=lambda: np.hstack([np.eye(3), np.zeros((3, 1))]))

    @staticmethod
    def pinhole(width: int, height: int, hfov_deg: float = 60.0) -> "Camera":
        f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
        return Camera(width, height, f, f, width / 2.0, height / 2.0)

    def intrinsics(self):
        return (self.fx, self.fy, self.cx, self.cy, self.width, self.height)


@dataclasses.dataclass
class Scene:
    lo: np.ndarray          # (K,3) box minimum corners, world frame
    hi: np.ndarray          # (K,3) box maximum corners
    color: np.ndarray       # (K,3) base colour, 0..255
    color2: np.ndarray      # (K,3) second texture shade, 0..255
    tex_kind: np.ndarray    # (K,) 0 = flat, 1 = checker, 2 = stripe
    tex_period: np.ndarray  # (K,) texture period in metres
    background: np.ndarray  # (3,) colour of rays that hit nothing


@dataclasses.dataclass
class Frame:
    """One viewpoint's input: merged points, RGB, camera, and diagnostics."""
    points: np.ndarray          # (N,3) float32 world xyz, merged sweep order
    rgb: np.ndarray             # (H,W,3) uint8, interleaved
    camera: Camera
    gt_depth: np.ndarray        # (H,W) float32 ray-cast Z (0 where no hit)
    sweep_id: np.ndarray        # (N,) int8 which sweep each point came from
    radius: int = 5
    sigma_s: float = 3.0
    sigma_r: float = 12.0

    @property
    def height(self) -> int:
        return self.camera.height

    @property
    def width(self) -> int:
        return self.camera.width


# --------------------------------------------------------------------------
# scene construction
# --------------------------------------------------------------------------


def make_scene(rng: np.random.Generator, cam: Camera, n_objects: int,
               back_wall: Optional[float], textured: bool,
               depth_range=(1.0, 20.0), planes_fraction: float = 0.0) -> Scene:
    """Random axis-aligned boxes (and thin planes) placed inside the frustum.

    Each object's centre depth is uniform in ``depth_range``; its centre is
    placed at a uniformly random image position at that depth, so every
    object is at least partly visible. Half extents scale with depth so that
    far objects still cover a useful part of the frame.
    """
    lo, hi = [], []
    tan_x = (cam.width / 2.0) / cam.fx
    tan_y = (cam.height / 2.0) / cam.fy
    for k in range(n_objects):
        z = rng.uniform(*depth_range)
        u = rng.uniform(-1.0, 1.0)
        v = rng.uniform(-1.0, 1.0)
        c = np.array([u * tan_x * z, v * tan_y * z, z])
        half = rng.uniform(0.3, 0.9, size=3) * z * tan_x
        half[2] = rng.uniform(0.05, 0.25) * z * 0.3
        if rng.uniform() < planes_fraction:
            # a thin plane facing the camera or a floor/side slab
            axis = rng.integers(0, 3)
            half[axis] = 0.01
        # never let a box contain the camera or reach behind it
        half[2] = min(half[2], 0.5 * (z - 0.2))
        lo.append(c - half)
        hi.append(c + half)
    if back_wall is not None:
        big = back_wall * 4.0
        lo.append(np.array([-big, -big, back_wall]))
        hi.append(np.array([big, big, back_wall + 0.5]))
    lo = np.array(lo, dtype=np.float64).reshape(-1, 3)
    hi = np.array(hi, dtype=np.float64).reshape(-1, 3)
    k = lo.shape[0]
    color = rng.integers(0, 256, size=(k, 3)).astype(np.float64)
    shade = rng.integers(-60, 61, size=(k, 3)).astype(np.float64)
    color2 = np.clip(color + shade, 0, 255)
    if textured:
        tex_kind = rng.integers(0, 3, size=k)
    else:
        tex_kind = np.zeros(k, dtype=np.int64)
    tex_period = rng.uniform(0.05, 0.5, size=k)
    background = rng.integers(0, 256, size=3).astype(np.float64)
    return Scene(lo, hi, color, color2, tex_kind, tex_period, background)


# --------------------------------------------------------------------------
# ray casting (slab method), chunked to bound memory
# --------------------------------------------------------------------------


def raycast(scene: Scene, origins: np.ndarray, dirs: np.ndarray,
            chunk: int = 1 << 16):
    """First hit of each ray against the scene's boxes.

    Returns ``t`` (ray parameter, inf on miss), ``obj`` (-1 on miss) and the
    entering ``axis`` (0,1,2) of the hit face.
    """
    dirs = np.asarray(dirs, dtype=np.float64)
    n = dirs.shape[0]
    origins = np.broadcast_to(np.asarray(origins, dtype=np.float64), (n, 3))
    t_out = np.full(n, np.inf)
    obj_out = np.full(n, -1, dtype=np.int64)
    axis_out = np.zeros(n, dtype=np.int64)
    lo = scene.lo[None, :, :]
    hi = scene.hi[None, :, :]
    for s in range(0, n, chunk):
        o = origins[s:s + chunk, None, :]
        d = dirs[s:s + chunk, None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / d
            t1 = (lo - o) * inv
            t2 = (hi - o) * inv
        tmin = np.minimum(t1, t2)
        tmax = np.maximum(t1, t2)
        # a zero direction component inside the slab gives nan; treat as open
        tmin = np.where(np.isnan(tmin), -np.inf, tmin)
        tmax = np.where(np.isnan(tmax), np.inf, tmax)
        tnear = tmin.max(axis=2)
        tfar = tmax.min(axis=2)
        hit = (tfar >= tnear) & (tnear > 1e-6)
        tn = np.where(hit, tnear, np.inf)
        best = tn.argmin(axis=1)
        rows = np.arange(best.shape[0])
        tb = tn[rows, best]
        ok = np.isfinite(tb)
        t_out[s:s + chunk] = tb
        obj_out[s:s + chunk] = np.where(ok, best, -1)
        axis_out[s:s + chunk] = tmin[rows, best].argmax(axis=1)
    return t_out, obj_out, axis_out


def _shade(scene: Scene, obj, axis, pts):
    """Base colour, or the two-shade texture evaluated on the hit face."""
    col = np.tile(scene.background, (obj.shape[0], 1))
    hit = obj >= 0
    if not np.any(hit):
        return col
    o = obj[hit]
    p = pts[hit]
    a = axis[hit]
    # the two in-face coordinates of the hit point
    u = np.where(a == 0, p[:, 1], p[:, 0])
    v = np.where(a == 2, p[:, 1], p[:, 2])
    per = scene.tex_period[o]
    iu = np.floor(u / per).astype(np.int64)
    iv = np.floor(v / per).astype(np.int64)
    kind = scene.tex_kind[o]
    alt = np.where(kind == 1, (iu + iv) & 1, np.where(kind == 2, iu & 1, 0))
    c = np.where(alt[:, None] == 1, scene.color2[o], scene.color[o])
    col[hit] = c
    return col


def _slab(lo, hi, o, d):
    """Ray/box slab test for one box: entering t (inf on miss) and axis."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t1 = (lo[None, :] - o) * inv
        t2 = (hi[None, :] - o) * inv
    tmin = np.minimum(t1, t2)
    tmax = np.maximum(t1, t2)
    tmin = np.where(np.isnan(tmin), -np.inf, tmin)
    tmax = np.where(np.isnan(tmax), np.inf, tmax)
    tnear = tmin.max(axis=1)
    tfar = tmax.min(axis=1)
    hit = (tfar >= tnear) & (tnear > 1e-6)
    return np.where(hit, tnear, np.inf), tmin.argmax(axis=1)


def render(scene: Scene, cam: Camera, rng: np.random.Generator,
           noise_sigma: float = 8.0):
    """RGB (uint8, HxWx3) and ground-truth Z (float32) through pixel centres.

    The camera sits at the world origin looking along +Z. Each box is only
    tested against the rays inside its screen-space bounding rectangle (the
    rectangle spanned by the directions to its corners), which keeps
    full-HD and 4K renders fast.
    """
    assert np.allclose(cam.pose, np.hstack([np.eye(3), np.zeros((3, 1))]))
    h, w = cam.height, cam.width
    n = h * w
    xs = (np.arange(w, dtype=np.float64) + 0.5 - cam.cx) / cam.fx
    ys = (np.arange(h, dtype=np.float64) + 0.5 - cam.cy) / cam.fy
    t_best = np.full(n, np.inf)
    obj = np.full(n, -1, dtype=np.int64)
    axis = np.zeros(n, dtype=np.int64)
    origin = np.zeros(3)
    for k in range(scene.lo.shape[0]):
        lo, hi = scene.lo[k], scene.hi[k]
        if lo[2] > 1e-3:
            cx = np.array([lo[0], hi[0]])[:, None] / np.array([lo[2], hi[2]])
            cy = np.array([lo[1], hi[1]])[:, None] / np.array([lo[2], hi[2]])
            c0 = np.searchsorted(xs, cx.min(), side="left") - 1
            c1 = np.searchsorted(xs, cx.max(), side="right") + 1
            r0 = np.searchsorted(ys, cy.min(), side="left") - 1
            r1 = np.searchsorted(ys, cy.max(), side="right") + 1
            c0, c1 = max(c0, 0), min(c1, w)
            r0, r1 = max(r0, 0), min(r1, h)
        else:
            c0, c1, r0, r1 = 0, w, 0, h
        if c1 <= c0 or r1 <= r0:
            continue
        rr, cc = np.meshgrid(np.arange(r0, r1), np.arange(c0, c1),
                             indexing="ij")
        idx = (rr * w + cc).ravel()
        d = np.stack([xs[cc.ravel()], ys[rr.ravel()],
                      np.ones(idx.shape[0])], axis=1)
        t, ax = _slab(lo, hi, origin[None, :], d)
        better = t < t_best[idx]
        sel = idx[better]
        t_best[sel] = t[better]
        obj[sel] = k
        axis[sel] = ax[better]
    d_all = np.stack([np.tile(xs, h), np.repeat(ys, w), np.ones(n)], axis=1)
    pts = t_best[:, None] * d_all
    pts[obj < 0] = 0.0
    col = _shade(scene, obj, axis, pts)
    col = col + rng.normal(0.0, noise_sigma, size=col.shape)
    rgb = np.clip(np.rint(col), 0, 255).astype(np.uint8).reshape(h, w, 3)
    gt = np.where(obj >= 0, t_best, 0.0).astype(np.float32).reshape(h, w)
    return rgb, gt


def lidar_sweep(scene: Scene, rng: np.random.Generator, origin: np.ndarray,
                n_beams: int, elev_deg: float, n_az: int,
                az_range_deg=(-180.0, 180.0), az_phase: float = 0.0,
                range_noise: float = 0.01):
    """One spinning-LiDAR sweep: beams x azimuth steps, first hit per ray.

    The sensor spins about the camera's vertical (Y) axis; azimuth 0 looks
    along +Z. ``az_phase`` is a fraction of one azimuth step, used to
    stagger sweeps. Returns float32 world points of the rays that hit.
    """
    elev = np.radians(np.linspace(-elev_deg, elev_deg, n_beams))
    a0, a1 = np.radians(az_range_deg[0]), np.radians(az_range_deg[1])
    step = (a1 - a0) / n_az
    az = a0 + (np.arange(n_az) + az_phase) * step
    el, azm = np.meshgrid(elev, az, indexing="ij")
    d = np.stack([np.cos(el) * np.sin(azm), -np.sin(el),
                  np.cos(el) * np.cos(azm)], axis=-1).reshape(-1, 3)
    t, obj, _ = raycast(scene, origin, d)
    hit = obj >= 0
    t = t[hit] + rng.normal(0.0, range_noise, size=int(hit.sum()))
    pts = origin[None, :] + t[:, None] * d[hit]
    return pts.astype(np.float32)


def _random_offset(rng: np.random.Generator, radius: float, exact: bool):
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    if not exact:
        v *= radius * rng.uniform() ** (1.0 / 3.0)
    else:
        v *= radius
    return v


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

FILTER_SMALL = dict(radius=5, sigma_s=3.0, sigma_r=12.0)
FILTER_FULLHD = dict(radius=15, sigma_s=6.0, sigma_r=15.0)


def small_view(rng: np.random.Generator, width=320, height=240,
               n_points: Optional[int] = None, n_beams=16, n_az=1800,
               elev_deg=15.0, noise_rng: Optional[np.random.Generator] = None) -> Frame:
    """6 axis-aligned boxes at depths U(1,20) m, no back wall, base colour +
    N(0,8) pixel noise, one 16-beam 360-degree sweep from 0.3 m away.

    With ``n_points`` set the sweep is confined to the camera's field of view
    and densified until about that many points hit (the widened scan used by
    the batched workload); the merged cloud is then cut to ``n_points``.
    With ``noise_rng`` the pixel and range noise come from it and everything
    else from ``rng``: frames with the same ``rng`` seed and different noise
    generators are one static scene seen with fresh noise.
    """
    noise = rng if noise_rng is None else noise_rng
    cam = Camera.pinhole(width, height)
    scene = make_scene(rng, cam, 6, back_wall=None, textured=False)
    rgb, gt = render(scene, cam, noise)
    origin = _random_offset(rng, 0.3, exact=True)
    if n_points is None:
        pts = lidar_sweep(scene, noise, origin, n_beams, elev_deg, n_az)
    else:
        cover = max(float((gt > 0).mean()), 0.02)
        rays = int(n_points / cover * 1.15) + 64
        hfov = math.degrees(math.atan((width / 2.0) / cam.fx)) * 1.05
        vfov = math.degrees(math.atan((height / 2.0) / cam.fy)) * 1.05
        beams = max(8, int(round(math.sqrt(rays * vfov / hfov))))
        az = max(16, int(math.ceil(rays / beams)))
        pts = lidar_sweep(scene, noise, origin, beams, vfov, az,
                          az_range_deg=(-hfov, hfov))
        pts = pts[:n_points]
    frame = Frame(pts, rgb, cam, gt, np.zeros(len(pts), np.int8),
                  **FILTER_SMALL)
    return frame


def fullhd_view(rng: np.random.Generator, width=1920, height=1080,
                n_objects=40, n_sweeps=3, n_beams=32, n_az=2048,
                elev_deg=22.5) -> Frame:
    """40 textured boxes/planes at 1-20 m plus a back wall at 20 m, three
    staggered 32-beam sweeps from origins within 0.5 m of the camera.

    The sweeps cover the camera's horizontal field of view plus 5 percent
    and are offset by a third of an azimuth step each, so the merged cloud
    holds about 1.5e5 in-image points (about 7 percent of the pixels).
    """
    cam = Camera.pinhole(width, height)
    scene = make_scene(rng, cam, n_objects, back_wall=20.0, textured=True,
                       planes_fraction=0.3)
    rgb, gt = render(scene, cam, rng)
    hfov = math.degrees(math.atan((width / 2.0) / cam.fx)) * 1.05
    sweeps, ids = [], []
    for s in range(n_sweeps):
        origin = _random_offset(rng, 0.5, exact=False)
        pts = lidar_sweep(scene, rng, origin, n_beams, elev_deg, n_az,
                          az_range_deg=(-hfov, hfov), az_phase=s / n_sweeps)
        sweeps.append(pts)
        ids.append(np.full(len(pts), s, np.int8))
    pts = np.concatenate(sweeps, axis=0)
    return Frame(pts, rgb, cam, gt, np.concatenate(ids), **FILTER_FULLHD)


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_views(rng: np.random.Generator, n_views=8,
                sizes=((1280, 720), (1920, 1080)),
                n_range=(20000, 250000)) -> List[Frame]:
    """Uneven viewpoints for one batched launch: resolution drawn from
    ``sizes``, point count log-uniform in ``n_range``, small-view scenes
    (6 boxes) with the scan widened to reach the count."""
    frames = []
    for _ in range(n_views):
        w, h = sizes[rng.integers(0, len(sizes))]
        n = log_uniform_int(rng, *n_range)
        frames.append(small_view(rng, w, h, n_points=n))
    return frames


def seeded(config_id: int, seed: Optional[int] = None):
    """Root generator for a workload: seed defaults to 1000 + id."""
    return np.random.default_rng(
        np.random.SeedSequence(1000 + config_id if seed is None else seed))


def spawn(rng_seed: int, n: int) -> List[np.random.Generator]:
    return [np.random.default_rng(s)
            for s in np.random.SeedSequence(rng_seed).spawn(n)]


def tiny_random(rng: np.random.Generator, h: int, w: int, density: float,
                depth_range=(1.0, 20.0), n_colors: Optional[int] = None):
    """Random sparse depth image, mask and RGB for small parity cases.

    With ``n_colors`` the RGB is drawn from a small palette (plus noise),
    which gives windows that mix similar and very different colours.
    """
    valid = (rng.uniform(size=(h, w)) < density).astype(np.uint8)
    depth = rng.uniform(*depth_range, size=(h, w)).astype(np.float32)
    depth = np.where(valid == 1, depth, np.float32(0.0)).astype(np.float32)
    if n_colors is None:
        rgb = rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)
    else:
        pal = rng.integers(0, 256, size=(n_colors, 3))
        idx = rng.integers(0, n_colors, size=(h, w))
        col = pal[idx] + rng.normal(0, 8, size=(h, w, 3))
        rgb = np.clip(np.rint(col), 0, 255).astype(np.uint8)
    return depth, valid, rgb


def holdout_split(rng: np.random.Generator, n: int, fraction: float = 0.1):
    """Boolean mask of held-out points (the self-supervised fit's targets)."""
    k = int(round(n * fraction))
    idx = rng.permutation(n)[:k]
    m = np.zeros(n, dtype=bool)
    m[idx] = True
    return m


# --------------------------------------------------------------------------
# serving workload: many viewpoints, each with its own world frame, and
# frames arriving on jittered 30 fps clocks
# --------------------------------------------------------------------------

SERVING_SIZES = ((1280, 720), (1920, 1080), (3840, 2160))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation matrix (QR of a Gaussian matrix)."""
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def with_random_pose(frame: Frame, rng: np.random.Generator,
                     max_offset: float = 10.0) -> Frame:
    """The same frame expressed in a random world frame: the camera gets the
    pose [R|t] (camera from world) and the points become R^T (p - t),
    rounded to float32."""
    R = random_rotation(rng)
    t = rng.uniform(-max_offset, max_offset, size=3)
    pw = (frame.points.astype(np.float64) - t) @ R      # rows: R^T (p - t)
    cam = dataclasses.replace(frame.camera, pose=np.hstack([R, t[:, None]]))
    return dataclasses.replace(frame, points=pw.astype(np.float32),
                               camera=cam)


def serving_specs(rng: np.random.Generator, n_views: int = 16,
                  sizes=SERVING_SIZES, n_range=(50000, 400000)):
    """Per viewpoint (width, height, n_points, seed): resolution drawn from
    ``sizes``, point count log-uniform in ``n_range``."""
    specs = []
    for _ in range(n_views):
        w, h = sizes[int(rng.integers(0, len(sizes)))]
        n = log_uniform_int(rng, *n_range)
        specs.append((int(w), int(h), int(n), int(rng.integers(0, 2 ** 63))))
    return specs


def serving_view(spec) -> Frame:
    """One serving viewpoint from its spec: a small-view scene (6 boxes,
    scan widened to reach the point count) in its own random world frame."""
    w, h, n, seed = spec
    rng = np.random.default_rng(seed)
    return with_random_pose(small_view(rng, w, h, n_points=n), rng)


def serving_frame(spec, k: int) -> Frame:
    """Frame k of a serving viewpoint: the viewpoint's static scene, camera
    and world pose (from the spec's seed) with pixel and LiDAR range noise
    drawn afresh (the k-th generator spawned from the seed)."""
    w, h, n, seed = spec
    rng = np.random.default_rng(seed)
    noise = np.random.default_rng(np.random.SeedSequence(seed).spawn(k + 1)[k])
    return with_random_pose(small_view(rng, w, h, n_points=n, noise_rng=noise), rng)


def arrival_times(rng: np.random.Generator, n_views: int, duration_s: float,
                  rate_hz: float = 30.0):
    """Sorted (time, viewpoint) pairs: each viewpoint starts at a random
    phase and then emits frames with exponential gaps of mean 1/rate_hz."""
    out = []
    for v in range(n_views):
        t = rng.uniform(0.0, 1.0 / rate_hz)
        while t < duration_s:
            out.append((float(t), v))
            t += rng.exponential(1.0 / rate_hz)
    out.sort()
    return out


# --------------------------------------------------------------------------
# a moving object: afterimages in merged sweeps
# --------------------------------------------------------------------------

def _shift_object(scene: Scene, obj: int, dx: float) -> Scene:
    lo, hi = scene.lo.copy(), scene.hi.copy()
    lo[obj, 0] += dx
    hi[obj, 0] += dx
    return dataclasses.replace(scene, lo=lo, hi=hi)


def moving_view(rng: np.random.Generator, width=640, height=360,
                n_objects=12, n_sweeps=3, n_beams=32, n_az=1024,
                elev_deg=22.5, step_fraction=0.35):
    """A textured scene whose nearest object moves sideways. The current
    RGB frame and the last sweep see it at its current place; sweep s sees
    it (n_sweeps - 1 - s) steps back; the previous RGB frame sees it one
    step back. One step is ``step_fraction`` of the object's width. Returns
    (frame at the current time with per-point sweep ids, previous RGB)."""
    cam = Camera.pinhole(width, height)
    scene = make_scene(rng, cam, n_objects, back_wall=20.0, textured=True)
    obj = int(np.argmin(0.5 * (scene.lo[:, 2] + scene.hi[:, 2])))
    step = step_fraction * float(scene.hi[obj, 0] - scene.lo[obj, 0])
    rgb, gt = render(scene, cam, rng)
    rgb_prev, _ = render(_shift_object(scene, obj, -step), cam, rng)
    hfov = math.degrees(math.atan((width / 2.0) / cam.fx)) * 1.05
    sweeps, ids = [], []
    for s in range(n_sweeps):
        seen = _shift_object(scene, obj, -step * (n_sweeps - 1 - s))
        origin = _random_offset(rng, 0.3, exact=False)
        pts = lidar_sweep(seen, rng, origin, n_beams, elev_deg, n_az,
                          az_range_deg=(-hfov, hfov), az_phase=s / n_sweeps)
        sweeps.append(pts)
        ids.append(np.full(len(pts), s, np.int8))
    frame = Frame(np.concatenate(sweeps, axis=0), rgb, cam, gt,
                  np.concatenate(ids), **FILTER_SMALL)
    return frame, rgb_prev
