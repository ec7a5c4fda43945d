"""The self-supervised width fit, end to end against the FP64 oracle
(Sec. 4: the filter widths are trainable by backpropagation).

Two Full-HD frames of the small-scene generator (six boxes, one 16-beam
sweep), 10% of each frame's points held out before projection and
rasterised through their own z-buffer as targets, r = 5, starting widths
sigma_s = 2, sigma_r = 40: the fit's starting point. On the GPU the loss
is formed exactly as ``fit_sigmas`` forms it (``Densify`` through
torch.autograd, one mean over the contributing targets of both frames) and
differentiated by autograd into the hand-written backward; the oracle
chains ``l1_holdout_loss`` into ``densify_grad`` per frame.

Bars: held-out target rasters bit-exact; loss within 1e-5 relative (each
output within 1e-5 of the oracle); both width gradients within 2e-4
relative (the FP32 backward's stated tolerance against the FP64 gradient),
where a target lying within the FP32 output tolerance of its output takes
the GPU's sign of the L1 slope (both signs are correct readings there);
and the autograd gradient equal to the binding's backward called with the
same upstream gradient.
"""
import numpy as np
import pytest

import oracle
from synth import scenes as S

pytestmark = pytest.mark.gpu

R, SS0, SR0 = 5, 2.0, 40.0


@pytest.fixture(scope="module")
def chain():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_01210_amd import autograd as AG
    from paper_2601_01210_amd import binding
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5005)
    gpu_frames, orc_frames = [], []
    for _ in range(2):
        f = S.small_view(rng, 1920, 1080)
        cam = f.camera
        held = S.holdout_split(rng, len(f.points), 0.1)
        pin, pout = f.points[~held], f.points[held]
        _, od, ov, _ = oracle.project(pin, cam.pose, cam.intrinsics(), cam.width,
                                      cam.height)
        _, otd, otv, _ = oracle.project(pout, cam.pose, cam.intrinsics(),
                                        cam.width, cam.height)
        _, gd, gv = binding.project(torch.from_numpy(np.ascontiguousarray(pin)).to(dev),
                                    cam.pose, cam.intrinsics(), cam.width, cam.height)
        gtd, gtv = AG.heldout_targets(
            torch.from_numpy(np.ascontiguousarray(pout)).to(dev), cam.pose,
            cam.intrinsics(), cam.width, cam.height)
        gpu_frames.append(AG.FitFrame(gd, gv, torch.from_numpy(f.rgb).to(dev), gtd, gtv))
        orc_frames.append((od, ov, f.rgb, otd, otv))
    torch.cuda.synchronize()
    return torch, dev, AG, binding, gpu_frames, orc_frames


# Targets within this relative distance of their output sit inside the FP32
# output tolerance (1e-5): there either sign of the L1 slope is a correct
# reading of the same loss, so the oracle takes the GPU's.
KINK = 2e-5


def _oracle_chain(orc_frames, ss, sr, gpu_outs=None):
    outs, masks = [], []
    for d, v, rgb, _, _ in orc_frames:
        o, m = oracle.densify(d, v, rgb, R, ss, sr)
        outs.append(o)
        masks.append(m)
    loss, g = oracle.l1_holdout_loss(outs, masks, [f[3] for f in orc_frames],
                                     [f[4] for f in orc_frames])
    n = sum(int(((f[4] == 1) & (m == 1)).sum()) for f, m in zip(orc_frames, masks))
    kinks = 0
    if gpu_outs is not None:
        for k, (f, o, m) in enumerate(zip(orc_frames, outs, masks)):
            t = f[3].astype(np.float64)
            near = (f[4] == 1) & (m == 1) & (np.abs(o - t) <= KINK * t)
            kinks += int(near.sum())
            g[k] = np.where(near, np.sign(gpu_outs[k].astype(np.float64) - t) / n, g[k])
    gs = gr = 0.0
    for (d, v, rgb, _, _), gf in zip(orc_frames, g):
        _, a, b = oracle.densify_grad(d, v, rgb, R, ss, sr, gf)
        gs += a
        gr += b
    return loss, gs, gr, outs, masks, n, kinks


def _gpu_outs(binding, frames, ss, sr):
    outs = []
    for f in frames:
        o, _ = binding.densify(f.depth, f.valid, f.rgb, R, ss, sr, ws=None)
        outs.append(o.cpu().numpy())
    return outs


def _gpu_chain(torch, AG, frames, ss, sr):
    params = torch.tensor([ss, sr], dtype=torch.float64, device=frames[0].depth.device,
                          requires_grad=True)
    losses, count, outs = [], 0, []
    for f in frames:
        out, mask = AG.Densify.apply(f.depth, f.valid, f.rgb, R, params[0], params[1])
        use = (f.target_valid == 1) & (mask == 1)
        diff = torch.where(use, out - f.target, torch.zeros_like(out))
        losses.append(diff.abs().sum())
        count += int(use.sum())
        outs.append((out.detach(), mask))
    loss = torch.stack(losses).sum() / max(count, 1)
    loss.backward()
    torch.cuda.synchronize()
    g = params.grad.detach().cpu().numpy()
    return float(loss), float(g[0]), float(g[1]), outs, count


@pytest.mark.parametrize("ss,sr", [(SS0, SR0), (3.0, 12.0)])
def test_fit_chain_matches_oracle(chain, ss, sr):
    torch, dev, AG, binding, gpu_frames, orc_frames = chain
    for gf, of in zip(gpu_frames, orc_frames):
        np.testing.assert_array_equal(gf.target.cpu().numpy(), of[3])
        np.testing.assert_array_equal(gf.target_valid.cpu().numpy(), of[4])
        np.testing.assert_array_equal(gf.valid.cpu().numpy(), of[1])
    gloss, ggs, ggr, gouts, gn = _gpu_chain(torch, AG, gpu_frames, ss, sr)
    oloss, ogs, ogr, oouts, omasks, on, kinks = _oracle_chain(
        orc_frames, ss, sr, [o.cpu().numpy() for o, _ in gouts])
    print(f"  sigma=({ss},{sr}) targets {gn} ({kinks} at a kink): loss gpu "
          f"{gloss:.7f} oracle {oloss:.7f}; dL/dss gpu {ggs:.6e} oracle {ogs:.6e}; "
          f"dL/dsr gpu {ggr:.6e} oracle {ogr:.6e}", flush=True)
    assert gn == on and gn > 20
    assert gloss == pytest.approx(oloss, rel=1e-5)
    assert ggs == pytest.approx(ogs, rel=2e-4)
    assert ggr == pytest.approx(ogr, rel=2e-4)


def test_autograd_equals_binding_backward(chain):
    """The gradient autograd delivers is the binding's backward applied to
    the upstream gradient sign(out - target) / n at the contributing pixels."""
    torch, dev, AG, binding, gpu_frames, _ = chain
    _, ggs, ggr, gouts, n = _gpu_chain(torch, AG, gpu_frames, SS0, SR0)
    tot = np.zeros(2)
    for f, (out, mask) in zip(gpu_frames, gouts):
        o2, m2, aux = binding.densify(f.depth, f.valid, f.rgb, R, SS0, SR0,
                                      want_aux=True, ws=None)
        assert torch.equal(o2, out) and torch.equal(m2, mask)
        use = (f.target_valid == 1) & (mask == 1)
        g = torch.where(use, torch.sign(out - f.target), torch.zeros_like(out))
        g = (g * (1.0 / max(n, 1))).float().contiguous()
        _, gsig = binding.densify_backward(f.depth, f.valid, f.rgb, R, SS0, SR0, o2,
                                           aux, g)
        tot += gsig.cpu().numpy()
    torch.cuda.synchronize()
    assert ggs == pytest.approx(tot[0], rel=1e-12, abs=0)
    assert ggr == pytest.approx(tot[1], rel=1e-12, abs=0)


def test_fit_steps_follow_adam_on_the_oracle_gradient(chain):
    """Three Adam steps of fit_sigmas against the same three steps taken on
    the oracle's loss and gradient (FP64): the widths agree to 1e-4 relative
    after each step."""
    torch, dev, AG, binding, gpu_frames, orc_frames = chain
    lr, b1, b2, eps = 0.05, 0.9, 0.999, 1e-8
    _, _, hist = AG.fit_sigmas(gpu_frames, R, SS0, SR0, steps=3, lr=lr)
    p = np.array([SS0, SR0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 4):
        loss, gs, gr, _, _, _, _ = _oracle_chain(
            orc_frames, p[0], p[1], _gpu_outs(binding, gpu_frames, p[0], p[1]))
        assert hist[t - 1]["loss"] == pytest.approx(loss, rel=1e-5)
        g = np.array([gs, gr])
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p = np.maximum(p - lr * mh / (np.sqrt(vh) + eps), AG.MIN_SIGMA)
        assert hist[t - 1]["sigma_s"] == pytest.approx(p[0], rel=1e-4)
        assert hist[t - 1]["sigma_r"] == pytest.approx(p[1], rel=1e-4)


def test_fit_resumes_from_its_checkpoint(chain, tmp_path):
    """Four steps in one go equal two steps, a checkpoint, and two more steps
    resumed from it (widths, moments and history)."""
    torch, dev, AG, binding, gpu_frames, _ = chain
    ck = str(tmp_path / "fit.json")
    s1, r1, h1 = AG.fit_sigmas(gpu_frames, R, SS0, SR0, steps=4)
    AG.fit_sigmas(gpu_frames, R, SS0, SR0, steps=2, checkpoint=ck)
    st = AG.load_state(ck)
    assert st["step"] == 2 and st["adam"]["step"] == 2 and len(st["history"]) == 2
    s2, r2, h2 = AG.fit_sigmas(gpu_frames, R, SS0, SR0, steps=4, checkpoint=ck,
                               resume=True)
    assert (s2, r2) == (s1, r1)
    assert [h["sigma_s"] for h in h2] == [h["sigma_s"] for h in h1]
    assert [h["loss"] for h in h2] == [h["loss"] for h in h1]
    assert AG.load_state(ck)["step"] == 4
