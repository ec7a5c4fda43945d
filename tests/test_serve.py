"""Host logic of the serving loop, on a fake executor and a fake clock.

The executor models one device: a batch starts when the previous one has
finished (or at launch) and takes a fixed time plus a per-pixel time.
"""
import numpy as np
import pytest

from paper_2601_01210_amd import serve as SV


class Clock:
    def __init__(self):
        self.now = 0.0

    def __call__(self):
        return self.now

    def sleep(self, dt):
        self.now += max(dt, 1e-6)


class FakeExec:
    def __init__(self, clock, fixed=2e-4, per_px=1e-10, fail_on=()):
        self.clock, self.fixed, self.per_px = clock, fixed, per_px
        self.end = 0.0
        self.fail_on = set(fail_on)
        self.n_launch = 0
        self.live = 0
        self.max_batch_seen = 0

    @staticmethod
    def slot_bytes(key):
        w, h, n = key
        return w * h + n

    def alloc_slot(self, key):
        self.live += 1
        return {"key": key}

    def free_slot(self, slot):
        self.live -= 1

    def launch(self, batch):
        k = self.n_launch
        self.n_launch += 1
        if k in self.fail_on:
            raise RuntimeError("injected failure")
        self.max_batch_seen = max(self.max_batch_seen, len(batch))
        start = max(self.clock(), self.end)
        px = sum(r.vp.width * r.vp.height for r, _ in batch)
        self.end = start + self.fixed + self.per_px * px
        return self.end

    def done(self, h):
        return self.clock() >= h

    def finish(self, h):
        assert self.clock() >= h


def vp(vid, w, h, n=1000):
    return SV.Viewpoint(vid, w, h, (1.0, 1.0, 0.0, 0.0), None, 5, 3.0, 12.0, n)


def requests(arrivals, vps):
    seq = {}
    out = []
    for t, v in arrivals:
        seq[v] = seq.get(v, 0) + 1
        out.append(SV.Request(vps[v], seq[v], t, n_points=vps[v].max_points))
    return out


def make(budget, clock, **kw):
    ex = FakeExec(clock, **{k: kw.pop(k) for k in list(kw) if k in
                            ("fixed", "per_px", "fail_on")})
    srv = SV.Server(ex, budget, clock=clock, sleep=clock.sleep, **kw)
    return ex, srv


def test_every_request_served_in_order_of_events():
    clock = Clock()
    vps = [vp(0, 1280, 720), vp(1, 1920, 1080), vp(2, 3840, 2160)]
    from synth import scenes as S
    arr = S.arrival_times(np.random.default_rng(1), 3, 1.0)
    reqs = requests(arr, vps)
    ex, srv = make(10 ** 9, clock, max_batch=4, max_inflight=2)
    srv.run(reqs)
    for r in reqs:
        assert r.error is None
        assert r.t_arrival <= r.t_admit <= r.t_launch <= r.t_done
    assert max(srv.batch_sizes) <= 4 and ex.max_batch_seen <= 4
    assert srv.max_seen_inflight <= 2
    assert srv.pool.busy == 0
    # slots are reused: a handful per shape, not one per frame
    assert srv.pool.allocations <= 3 * 4 * 2 < len(reqs)


def test_latency_of_a_lone_request_is_its_service_time():
    clock = Clock()
    v = vp(0, 1920, 1080)
    r = SV.Request(v, 1, 0.25, n_points=1000)
    ex, srv = make(10 ** 9, clock, fixed=1e-3, per_px=0.0)
    srv.run([r], poll_s=1e-5)
    assert r.t_launch == pytest.approx(0.25, abs=2e-5)
    assert r.latency == pytest.approx(1e-3, abs=3e-5)


def test_budget_is_never_exceeded_and_head_is_not_starved():
    """Budget for one 4K slot or a few small ones; a 4K frame arriving
    amid a stream of small frames is admitted in FIFO order."""
    clock = Clock()
    big, small = vp(0, 3840, 2160), vp(1, 320, 240)
    need_big = FakeExec.slot_bytes(big.key)
    arr = [(i * 1e-4, 1) for i in range(200)]
    arr.insert(50, (50e-4 + 1e-6, 0))
    reqs = requests(arr, [big, small])
    ex, srv = make(need_big + 2 * FakeExec.slot_bytes(small.key), clock,
                   max_batch=8, max_inflight=2, per_px=1e-9)
    peak = []
    orig = srv.pool.acquire

    def acquire(key):
        s = orig(key)
        peak.append(srv.pool.used)
        return s
    srv.pool.acquire = acquire
    srv.run(reqs)
    assert all(r.error is None for r in reqs)
    assert max(peak) <= srv.pool.budget
    admits = [r.t_admit for r in sorted(reqs, key=lambda r: r.t_arrival)]
    assert admits == sorted(admits)              # FIFO admission
    # the big frame forced idle small slots out to make room
    assert ex.live * FakeExec.slot_bytes(small.key) <= srv.pool.budget


def test_request_larger_than_budget_is_rejected_and_others_go_on():
    clock = Clock()
    vps = [vp(0, 3840, 2160), vp(1, 320, 240)]
    reqs = requests([(0.0, 1), (0.001, 0), (0.002, 1)], vps)
    ex, srv = make(FakeExec.slot_bytes(vps[1].key) * 2, clock)
    srv.run(reqs)
    assert reqs[1].error and "budget" in reqs[1].error
    assert reqs[0].error is None and reqs[2].error is None
    assert reqs[0].t_done > 0 and reqs[2].t_done > 0


def test_launch_failure_fails_that_batch_only():
    clock = Clock()
    vps = [vp(0, 640, 480)]
    reqs = requests([(i * 0.01, 0) for i in range(6)], vps)
    ex, srv = make(10 ** 9, clock, max_batch=1, fail_on=(1,))
    srv.run(reqs)
    failed = [r for r in reqs if r.error]
    assert len(failed) == 1 and "injected" in failed[0].error
    assert all(r.t_done > 0 for r in reqs if not r.error)
    assert srv.pool.busy == 0
    st = SV.summarize(reqs, 0.0, srv.batch_sizes)
    assert st.failed == 1 and st.n == 5


def test_continuous_batching_groups_arrivals_during_a_busy_device():
    """While one long batch runs, later arrivals pile up and leave together
    in the next batch (not one launch per frame)."""
    clock = Clock()
    vps = [vp(v, 1920, 1080) for v in range(8)]
    arr = [(0.0, 0)] + [(1e-3 + 1e-5 * v, v) for v in range(1, 8)]
    reqs = requests(arr, vps)
    ex, srv = make(10 ** 9, clock, fixed=5e-3, per_px=0.0, max_batch=16,
                   max_inflight=1)
    srv.run(reqs)
    assert srv.batch_sizes == [1, 7]


def test_summary_statistics():
    v = vp(0, 1920, 1080)
    reqs = []
    for i in range(100):
        r = SV.Request(v, i, 1.0 + i * 0.01, n_points=1)
        r.t_done = r.t_arrival + (i + 1) * 1e-3
        reqs.append(r)
    warm = SV.Request(v, -1, 0.5, n_points=1)
    warm.t_done = 0.6
    st = SV.summarize(reqs + [warm], 1.0, [1, 2, 3])
    assert st.n == 100
    assert st.p50_ms == pytest.approx(50.5)
    assert st.p99_ms == pytest.approx(np.percentile(np.arange(1, 101), 99))
    span = reqs[-1].t_done - 1.0
    assert st.frames_per_s == pytest.approx(100 / span)
    assert st.fhd_frames_per_s == pytest.approx(100 / span)
    assert st.mean_batch == pytest.approx(2.0)


def test_pool_evicts_idle_slots_of_other_shapes():
    freed = []
    pool = SV.SlotPool(100, lambda k: k[0], lambda k: {"k": k}, freed.append)
    a = pool.acquire((60, 0, 0))
    pool.release((60, 0, 0), a)
    b = pool.acquire((50, 0, 0))          # needs the idle 60-byte slot freed
    assert b is not None and freed == [a] and pool.used == 50
    c = pool.acquire((60, 0, 0))          # 50 busy + 60 > 100: must wait
    assert c is None
    with pytest.raises(SV.AdmissionError):
        pool.acquire((101, 0, 0))
