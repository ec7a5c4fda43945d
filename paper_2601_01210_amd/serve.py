"""Serving loop: continuous batching of densification requests on one GPU.

Frames arrive from many viewpoints at their own clocks (mixed resolutions
and point counts). The paper runs each viewpoint on its own PC with no
exchange between them (Sec. 2); here all viewpoints share one GPU and the
loop keeps it busy:

* **Slots** hold one frame's device buffers (points, RGB, z-buffer, sparse
  and dense depth, masks) plus pinned host buffers for the results. A slot
  is keyed by (width, height, max points) and reused by later frames of
  that shape, so buffers stay resident on the device.
* **Admission** is FIFO under an HBM budget: the head request takes a free
  slot of its shape, or a new one if the bytes of all slots stay within
  the budget (free slots of other shapes are released to make room). A
  request that does not fit waits at the head, so a large frame is never
  starved by smaller ones behind it.
* **Continuous batching**: every admitted request joins the next batch,
  which is launched as soon as fewer than ``max_inflight`` batches are on
  the device. Requests that arrive while a batch runs are admitted as slots
  free up and go out with the next one.
* **Executor** (GPU): per batch, host-to-device copies on a copy stream,
  then one replay of a HIP graph of the batch kernels (jbfd_batch_run) on
  the compute stream behind a rewritten descriptor table, then device-to-
  host copies on a third stream. Copies of one batch overlap the kernels
  of the neighbouring ones. All streams have the default priority.

Latency is measured from a request's scheduled arrival to the moment its
depth and mask are in pinned host memory (the completion is observed by
polling the batch's last event). ``run_plain`` is the per-frame baseline on
the same arrivals: copy in, project, densify, copy out and synchronise,
one frame at a time on one stream.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import binding

FHD_PIXELS = 1920 * 1080


@dataclasses.dataclass
class Viewpoint:
    """Static description of one viewpoint (camera and filter)."""
    vid: int
    width: int
    height: int
    intrinsics: Tuple[float, float, float, float]
    pose: object                      # 3x4 camera-from-world
    radius: int
    sigma_s: float
    sigma_r: float
    max_points: int

    @property
    def key(self) -> Tuple[int, int, int]:
        return (self.width, self.height, self.max_points)


@dataclasses.dataclass
class Request:
    """One frame of one viewpoint. ``points``/``rgb`` are host buffers
    (pinned CPU tensors on the GPU executor)."""
    vp: Viewpoint
    seq: int
    t_arrival: float                  # seconds after the run starts
    points: object = None
    rgb: object = None
    n_points: int = 0
    t_admit: float = -1.0
    t_launch: float = -1.0
    t_done: float = -1.0
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class AdmissionError(RuntimeError):
    pass


class SlotPool:
    """Slots under an HBM byte budget (see module docstring)."""

    def __init__(self, budget_bytes: int, size_of: Callable[[tuple], int],
                 alloc: Callable[[tuple], object], free: Callable[[object], None]):
        self.budget = int(budget_bytes)
        self.size_of, self.alloc, self.free_fn = size_of, alloc, free
        self.free: Dict[tuple, List[object]] = {}
        self.used = 0            # bytes of every live slot (busy or free)
        self.busy = 0
        self.peak = 0
        self.allocations = 0

    def fits_ever(self, key) -> bool:
        return self.size_of(key) <= self.budget

    def acquire(self, key):
        """A slot for ``key`` or None when the budget is exhausted."""
        lst = self.free.get(key)
        if lst:
            self.busy += 1
            return lst.pop()
        need = self.size_of(key)
        if need > self.budget:
            raise AdmissionError(f"a {key} slot needs {need} bytes, budget "
                                 f"is {self.budget}")
        if self.used + need > self.budget:
            # release idle slots of other shapes, largest first
            idle = sorted(((self.size_of(k), k) for k, v in self.free.items()
                           for _ in v), reverse=True)
            for size, k in idle:
                if self.used + need <= self.budget:
                    break
                self.free_fn(self.free[k].pop())
                self.used -= size
        if self.used + need > self.budget:
            return None
        slot = self.alloc(key)
        self.allocations += 1
        self.used += need
        self.peak = max(self.peak, self.used)
        self.busy += 1
        return slot

    def release(self, key, slot) -> None:
        self.busy -= 1
        self.free.setdefault(key, []).append(slot)

    def close(self) -> None:
        for k, v in self.free.items():
            for s in v:
                self.free_fn(s)
                self.used -= self.size_of(k)
        self.free.clear()


@dataclasses.dataclass
class Stats:
    n: int
    frames_per_s: float
    fhd_frames_per_s: float
    p50_ms: float
    p99_ms: float
    max_ms: float
    mean_batch: float
    failed: int

    def as_dict(self):
        return dataclasses.asdict(self)


def summarize(requests: Sequence[Request], warmup_s: float,
              batches: Sequence[int] = ()) -> Stats:
    """Throughput and latency over requests that arrived after ``warmup_s``.
    Throughput counts frames completed in [warmup_s, last completion]."""
    done = [r for r in requests if r.t_arrival >= warmup_s and r.error is None
            and r.t_done >= 0]
    failed = sum(1 for r in requests if r.error is not None)
    if not done:
        return Stats(0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, failed)
    lat = np.array([r.latency for r in done]) * 1e3
    span = max(r.t_done for r in done) - warmup_s
    px = sum(r.vp.width * r.vp.height for r in done)
    return Stats(len(done), len(done) / span, px / FHD_PIXELS / span,
                 float(np.percentile(lat, 50)), float(np.percentile(lat, 99)),
                 float(lat.max()),
                 float(np.mean(batches)) if len(batches) else 0.0, failed)


class Server:
    """Admission, batching and completion over an executor.

    The executor provides slot_bytes(key), alloc_slot(key), free_slot(slot),
    launch(batch: list of (Request, slot)) -> handle, done(handle) -> bool
    and finish(handle) (results of the batch are in host memory).
    """

    def __init__(self, executor, budget_bytes: int, max_batch: int = 16,
                 max_inflight: int = 2,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 on_done: Optional[Callable[[Request, object], None]] = None):
        if max_batch < 1 or max_inflight < 1:
            raise ValueError("max_batch and max_inflight must be >= 1")
        self.ex = executor
        self.pool = SlotPool(budget_bytes, executor.slot_bytes,
                             executor.alloc_slot, executor.free_slot)
        self.max_batch, self.max_inflight = max_batch, max_inflight
        self.clock, self.sleep = clock, sleep
        self.on_done = on_done
        self.queue: Deque[Request] = deque()
        self.admitted: List[Tuple[Request, object]] = []
        self.inflight: Deque[Tuple[object, List[Tuple[Request, object]]]] = deque()
        self.batch_sizes: List[int] = []
        self.max_seen_inflight = 0

    def prefill(self, keys: Sequence[tuple], per_key: int) -> None:
        """Allocate up to ``per_key`` idle slots of each shape ahead of
        time (within the budget), so the first frames do not pay for it."""
        got = []
        for key in keys:
            for _ in range(per_key):
                if not self.pool.fits_ever(key):
                    break
                s = self.pool.acquire(key)
                if s is None:
                    break
                got.append((key, s))
        for key, s in got:
            self.pool.release(key, s)

    # -- one scheduling round -------------------------------------------
    def _complete(self, now: float) -> bool:
        progressed = False
        while self.inflight and self.ex.done(self.inflight[0][0]):
            handle, batch = self.inflight.popleft()
            t = self.clock() - self._t0
            self.ex.finish(handle)
            for req, slot in batch:
                req.t_done = t
                if self.on_done is not None:
                    self.on_done(req, slot)
                self.pool.release(req.vp.key, slot)
            progressed = True
        return progressed

    def _admit(self, now: float) -> bool:
        progressed = False
        while self.queue and len(self.admitted) < self.max_batch:
            req = self.queue[0]
            if not self.pool.fits_ever(req.vp.key):
                self.queue.popleft()
                req.error = "larger than the HBM budget"
                progressed = True
                continue
            slot = self.pool.acquire(req.vp.key)
            if slot is None:
                break                      # head waits: no starvation
            self.queue.popleft()
            req.t_admit = now
            self.admitted.append((req, slot))
            progressed = True
        return progressed

    def _launch(self, now: float) -> bool:
        if not self.admitted or len(self.inflight) >= self.max_inflight:
            return False
        batch, self.admitted = self.admitted, []
        for req, _ in batch:
            req.t_launch = now
        try:
            handle = self.ex.launch(batch)
        except Exception as e:             # the batch fails, the loop goes on
            for req, slot in batch:
                req.error = f"launch failed: {e}"
                self.pool.release(req.vp.key, slot)
            return True
        self.inflight.append((handle, batch))
        self.batch_sizes.append(len(batch))
        self.max_seen_inflight = max(self.max_seen_inflight, len(self.inflight))
        return True

    def run(self, requests: Sequence[Request], poll_s: float = 50e-6
            ) -> List[Request]:
        """Serve ``requests`` (sorted by t_arrival) on the executor, with
        arrivals released on the clock. Returns the requests."""
        order = sorted(requests, key=lambda r: r.t_arrival)
        self._t0 = self.clock()
        i = 0
        while i < len(order) or self.queue or self.admitted or self.inflight:
            now = self.clock() - self._t0
            while i < len(order) and order[i].t_arrival <= now:
                self.queue.append(order[i])
                i += 1
            progressed = self._complete(now)
            progressed |= self._admit(now)
            progressed |= self._launch(now)
            if not progressed:
                nxt = order[i].t_arrival - now if i < len(order) else poll_s
                self.sleep(max(0.0, min(poll_s, nxt)))
        return order


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GpuSlot:
    view: "binding.BatchView"
    out_host: object
    mask_host: object
    nbytes: int


class GpuExecutor:
    """Batches of slots through jbfd_batch_run (graph replay, see module
    docstring). Every view in a batch uses ``precision``; the graph is
    captured once per (radius bound, precision) at first use."""

    def __init__(self, device=None, precision=binding.Precision.FP16_RANGE,
                 max_batch: int = 16, max_inflight: int = 2,
                 use_graphs: bool = True, timing: bool = False):
        import torch
        self.torch = torch
        self.dev = torch.device(device if device is not None else "cuda:0")
        self.prec = precision
        self.max_batch = max_batch
        self.h2d = torch.cuda.Stream(self.dev)
        self.comp = torch.cuda.Stream(self.dev)
        self.d2h = torch.cuda.Stream(self.dev)
        nb = binding.batch_table_bytes(max_batch)
        self.table = torch.empty(nb, dtype=torch.uint8, device=self.dev)
        self.host_tables = [torch.empty(nb, dtype=torch.uint8, pin_memory=True)
                            for _ in range(max_inflight + 1)]
        # event after the last copy out of each host table: a table is
        # rewritten only once its previous copy has run
        self.host_events: List[Optional[object]] = [None] * len(self.host_tables)
        self.n_launch = 0
        self.use_graphs = use_graphs
        self.graphs: Dict[Tuple[int, int], object] = {}
        # optional: HIP events around each batch's kernels on the compute
        # stream; kernel_ms collects their durations at finish()
        self.timing = timing
        self.kernel_ms: List[float] = []

    # slots ---------------------------------------------------------------
    @staticmethod
    def slot_bytes(key) -> int:
        w, h, n = key
        hw = w * h
        # points, rgb, z-buffer, sparse depth + mask, dense depth + mask
        return 12 * n + 3 * hw + 8 * hw + 5 * hw + 5 * hw

    def alloc_slot(self, key) -> GpuSlot:
        torch = self.torch
        w, h, n = key
        pts = torch.empty((n, 3), dtype=torch.float32, device=self.dev)
        rgb = torch.empty((h, w, 3), dtype=torch.uint8, device=self.dev)
        v = binding.BatchView(pts, np.eye(3, 4), (1.0, 1.0, 0.0, 0.0), w, h,
                              rgb, 0, 1.0, 1.0).allocate(self.dev)
        out_host = torch.empty((h, w), dtype=torch.float32, pin_memory=True)
        mask_host = torch.empty((h, w), dtype=torch.uint8, pin_memory=True)
        return GpuSlot(v, out_host, mask_host, self.slot_bytes(key))

    def free_slot(self, slot: GpuSlot) -> None:
        slot.view = None            # the caching allocator keeps the memory

    # graphs ----------------------------------------------------------------
    def _graph(self, max_radius: int):
        torch = self.torch
        bucket = 16 if max_radius <= 16 else 32
        k = (bucket, int(self.prec))
        if k in self.graphs:
            return self.graphs[k]
        # a valid table (one tiny empty view) for the eager warm-up run
        dummy = binding.BatchView(
            torch.zeros((1, 3), dtype=torch.float32, device=self.dev),
            np.eye(3, 4), (1.0, 1.0, 0.5, 0.5), 2, 2,
            torch.zeros((2, 2, 3), dtype=torch.uint8, device=self.dev),
            0, 1.0, 1.0).allocate(self.dev)
        dummy.n_points = 0
        with torch.cuda.stream(self.comp):
            binding.batch_upload([dummy], self.table)
            binding.batch_run(self.table, bucket, self.prec)
        self.comp.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.comp,
                              capture_error_mode="thread_local"):
            binding.batch_run(self.table, bucket, self.prec)
        self.comp.synchronize()
        self.graphs[k] = (g, dummy)
        return self.graphs[k]

    def prewarm(self, max_radius: int) -> None:
        if self.use_graphs:
            self._graph(max_radius)

    # batches ---------------------------------------------------------------
    def launch(self, batch):
        torch = self.torch
        if len(batch) > self.max_batch:
            raise ValueError("batch larger than the descriptor table")
        max_r = max(req.vp.radius for req, _ in batch)
        graph = self._graph(max_r)[0] if self.use_graphs else None
        views = []
        ev_in = torch.cuda.Event()
        with torch.cuda.stream(self.h2d):
            for req, slot in batch:
                v, vp = slot.view, req.vp
                n = int(req.n_points)
                if n > v.points.shape[0]:
                    raise ValueError("frame has more points than its slot")
                if n:
                    v.points[:n].copy_(req.points[:n], non_blocking=True)
                v.rgb.copy_(req.rgb, non_blocking=True)
                v.n_points = n
                v.pose, v.intrinsics = vp.pose, vp.intrinsics
                v.radius, v.sigma_s, v.sigma_r = vp.radius, vp.sigma_s, vp.sigma_r
                views.append(v)
            ev_in.record(self.h2d)
        k = self.n_launch % len(self.host_tables)
        host = self.host_tables[k]
        if self.host_events[k] is not None:
            self.host_events[k].synchronize()
        self.n_launch += 1
        ev_c = torch.cuda.Event(enable_timing=self.timing)
        ev_k = torch.cuda.Event(enable_timing=True) if self.timing else None
        with torch.cuda.stream(self.comp):
            self.comp.wait_event(ev_in)
            binding.batch_upload(views, self.table, host)
            if ev_k is not None:
                ev_k.record(self.comp)
            if graph is not None:
                graph.replay()
            else:
                binding.batch_run(self.table, max_r, self.prec)
            ev_c.record(self.comp)
        self.host_events[k] = ev_c
        ev_out = torch.cuda.Event()
        with torch.cuda.stream(self.d2h):
            self.d2h.wait_event(ev_c)
            for req, slot in batch:
                slot.out_host.copy_(slot.view.dense_depth, non_blocking=True)
                slot.mask_host.copy_(slot.view.dense_valid, non_blocking=True)
            ev_out.record(self.d2h)
        return (ev_out, ev_k, ev_c)

    def done(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle) -> None:
        handle[0].synchronize()
        if handle[1] is not None:
            self.kernel_ms.append(handle[1].elapsed_time(handle[2]))


class PlainRunner:
    """Per-frame baseline: each request in arrival order, alone on one
    stream: copy in, jbfd_project, jbfd_densify, copy out, synchronise.
    Buffers (one set per frame shape, resident on the device) are kept
    between runs."""

    def __init__(self, precision, device=None, lists: bool = True):
        import torch
        self.torch = torch
        self.prec = precision
        self.dev = torch.device(device if device is not None else "cuda:0")
        self.stream = torch.cuda.Stream(self.dev)
        self.lists = lists
        self.bufs: Dict[tuple, dict] = {}

    def _buffers(self, vp: Viewpoint) -> dict:
        torch, dev = self.torch, self.dev
        k = (vp.key, vp.radius)
        if k not in self.bufs:
            w, h, n = vp.key
            self.bufs[k] = dict(
                pts=torch.empty((n, 3), dtype=torch.float32, device=dev),
                rgb=torch.empty((h, w, 3), dtype=torch.uint8, device=dev),
                zbuf=torch.empty((h, w), dtype=torch.int64, device=dev),
                d=torch.empty((h, w), dtype=torch.float32, device=dev),
                v=torch.empty((h, w), dtype=torch.uint8, device=dev),
                out=torch.empty((h, w), dtype=torch.float32, device=dev),
                mask=torch.empty((h, w), dtype=torch.uint8, device=dev),
                ws=(binding.densify_workspace(h, w, vp.radius, n, dev)
                    if self.lists else None),
                out_h=torch.empty((h, w), dtype=torch.float32, pin_memory=True),
                mask_h=torch.empty((h, w), dtype=torch.uint8, pin_memory=True))
        return self.bufs[k]

    def run(self, requests: Sequence[Request], clock=time.perf_counter,
            sleep=time.sleep,
            on_done: Optional[Callable[[Request, object, object], None]] = None
            ) -> List[Request]:
        torch, s = self.torch, self.stream
        order = sorted(requests, key=lambda r: r.t_arrival)
        for req in order:                     # buffers before the clock starts
            self._buffers(req.vp)
        torch.cuda.synchronize(self.dev)
        t0 = clock()
        for req in order:
            while clock() - t0 < req.t_arrival:
                sleep(max(0.0, min(50e-6, req.t_arrival - (clock() - t0))))
            b, vp, n = self._buffers(req.vp), req.vp, int(req.n_points)
            with torch.cuda.stream(s):
                if n:
                    b["pts"][:n].copy_(req.points[:n], non_blocking=True)
                b["rgb"].copy_(req.rgb, non_blocking=True)
                binding.project(b["pts"][:n], vp.pose, vp.intrinsics, vp.width,
                                vp.height, b["zbuf"], b["d"], b["v"])
                binding.densify(b["d"], b["v"], b["rgb"], vp.radius,
                                vp.sigma_s, vp.sigma_r, self.prec, b["out"],
                                b["mask"], ws=b["ws"], max_samples=n)
                b["out_h"].copy_(b["out"], non_blocking=True)
                b["mask_h"].copy_(b["mask"], non_blocking=True)
            s.synchronize()
            req.t_done = clock() - t0
            if on_done is not None:
                on_done(req, b["out_h"], b["mask_h"])
        return order


def run_plain(requests: Sequence[Request], precision, device=None,
              clock=time.perf_counter, sleep=time.sleep,
              on_done: Optional[Callable[[Request, object, object], None]] = None,
              lists: bool = True) -> List[Request]:
    """One-off PlainRunner run over ``requests``."""
    return PlainRunner(precision, device, lists).run(requests, clock, sleep,
                                                     on_done)
