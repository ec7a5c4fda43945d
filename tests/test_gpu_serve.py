"""GPU checks of the serving loop: every result is the same alone and in
the mix.

Six viewpoints of mixed small shapes, each alternating between two frames,
arrive in a burst and then on jittered clocks under an HBM budget that
holds only a few slots, so requests wait for slots, form batches of
several views, and overlap on the device. Each served result is compared
bit for bit with the same frame served alone (a batch of one through the
same executor), and against the FP64 oracle: mask bit-exact, FP32 depth
within 1e-5 relative, FP16 range weights within the arithmetic bound. The
per-frame baseline (run_plain) is checked against the oracle too.
"""
import numpy as np
import pytest

import oracle
from synth import scenes as S

pytestmark = pytest.mark.gpu

SIZES = ((160, 120), (320, 240), (640, 360))


@pytest.fixture(scope="module")
def tdev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def workload(tdev):
    torch, dev = tdev
    from paper_2601_01210_amd import serve as SV
    rng = S.seeded(4, 4242)
    specs = S.serving_specs(rng, 6, sizes=SIZES, n_range=(3000, 20000))
    vps, frames = [], []
    for vid, (w, h, n, seed) in enumerate(specs):
        fr = [S.serving_view((w, h, n, seed)), S.serving_view((w, h, n, seed + 1))]
        cam = fr[0].camera
        # both frames of a viewpoint share its shape; each keeps its pose
        vps.append([SV.Viewpoint(vid, w, h, cam.intrinsics()[:4], f.camera.pose,
                                 f.radius, f.sigma_s, f.sigma_r, n) for f in fr])
        frames.append(fr)
    refs = {}
    for vid, fr in enumerate(frames):
        for k, f in enumerate(fr):
            c = f.camera
            _, d, b, _ = oracle.project(f.points, c.pose, c.intrinsics(),
                                        c.width, c.height)
            refs[(vid, k)] = (d, b) + tuple(oracle.densify(
                d, b, f.rgb, f.radius, f.sigma_s, f.sigma_r))
    pinned = {(vid, k): (torch.from_numpy(f.points).pin_memory(),
                         torch.from_numpy(f.rgb).pin_memory())
              for vid, fr in enumerate(frames) for k, f in enumerate(fr)}
    arr = [(0.0, i % 6) for i in range(24)]                  # a burst
    arr += [(0.02 + t, v) for t, v in S.arrival_times(rng, 6, 0.3, 60.0)]
    return vps, frames, refs, pinned, sorted(arr)


def _requests(SV, vps, pinned, arr):
    seq = {}
    out = []
    for t, v in arr:
        k = seq.get(v, 0)
        seq[v] = k + 1
        p, c = pinned[(v, k % 2)]
        r = SV.Request(vps[v][k % 2], k, t, p, c, p.shape[0])
        r.frame = (v, k % 2)
        out.append(r)
    return out


def _serve(SV, prec, dev, reqs, budget, max_batch=8):
    ex = SV.GpuExecutor(dev, precision=prec, max_batch=max_batch)
    ex.prewarm(5)
    res = {}

    def on_done(req, slot):
        res[id(req)] = (slot.out_host.numpy().copy(),
                        slot.mask_host.numpy().copy())
    srv = SV.Server(ex, budget, max_batch=max_batch, max_inflight=2,
                    on_done=on_done)
    srv.run(reqs)
    return srv, res


@pytest.mark.parametrize("prec_name", ["FP32", "FP16_RANGE"])
def test_served_equals_alone_and_oracle(tdev, workload, prec_name):
    torch, dev = tdev
    from paper_2601_01210_amd import Precision
    from paper_2601_01210_amd import serve as SV
    prec = Precision[prec_name]
    vps, frames, refs, pinned, arr = workload
    big = max(SV.GpuExecutor.slot_bytes(v[0].key) for v in vps)
    reqs = _requests(SV, vps, pinned, arr)
    srv, res = _serve(SV, prec, dev, reqs, budget=3 * big)
    st = SV.summarize(reqs, 0.0, srv.batch_sizes)
    print(f"  {prec_name}: {len(reqs)} requests, batches {len(srv.batch_sizes)}"
          f" (max {max(srv.batch_sizes)}), slots {srv.pool.allocations}, "
          f"peak {srv.pool.peak} of {srv.pool.budget} B, p50 {st.p50_ms:.2f} "
          f"p99 {st.p99_ms:.2f} ms", flush=True)
    assert all(r.error is None for r in reqs)
    assert max(srv.batch_sizes) > 1 and srv.pool.peak <= srv.pool.budget
    # alone: each distinct frame as a batch of one
    alone = {}
    for key in refs:
        v, k = key
        r = [x for x in reqs if x.frame == key][0]
        solo = SV.Request(r.vp, 0, 0.0, r.points, r.rgb, r.n_points)
        _, rs = _serve(SV, prec, dev, [solo], budget=big, max_batch=1)
        alone[key] = rs[id(solo)]
    for r in reqs:
        out, mask = res[id(r)]
        a_out, a_mask = alone[r.frame]
        np.testing.assert_array_equal(out.view(np.uint32), a_out.view(np.uint32))
        np.testing.assert_array_equal(mask, a_mask)
    for key, (d, b, ref, m) in refs.items():
        out, mask = alone[key]
        np.testing.assert_array_equal(mask, m)
        sel = m == 1
        if prec == Precision.FP32:
            np.testing.assert_allclose(out[sel], ref[sel], rtol=1e-5)
        else:
            from fp16_check import fp16_report
            v, _ = key
            fr = frames[key[0]][key[1]]
            fp16_report(out, mask, ref, m, d, b, fr.rgb, fr.radius, fr.sigma_s,
                        fr.sigma_r, f"viewpoint {v}")


def test_plain_baseline_matches_oracle(tdev, workload):
    torch, dev = tdev
    from paper_2601_01210_amd import Precision
    from paper_2601_01210_amd import serve as SV
    vps, frames, refs, pinned, arr = workload
    reqs = _requests(SV, vps, pinned, arr[:30])
    got = {}

    def on_done(req, out_h, mask_h):
        got[id(req)] = (out_h.numpy().copy(), mask_h.numpy().copy())
    SV.run_plain(reqs, Precision.FP32, dev, on_done=on_done)
    for r in reqs:
        d, b, ref, m = refs[r.frame]
        out, mask = got[id(r)]
        np.testing.assert_array_equal(mask, m)
        np.testing.assert_allclose(out[m == 1], ref[m == 1], rtol=1e-5)
        assert r.t_done >= r.t_arrival
