"""Differentiable densification and a self-supervised fit of the filter widths.

Sec. 4 notes that the filter is built from network-style layers so its
Gaussian widths can be trained by backpropagation when dense ground truth
exists. Here the gradient comes from the hand-written HIP backward
(jbfd_densify_backward) and the supervision from held-out LiDAR points, so
no dense ground truth is needed:

* ``Densify``   torch.autograd.Function over jbfd_densify / _backward; the
  gradients flow to the sparse depths and to sigma_s, sigma_r;
* ``heldout_targets``  projects the held-out points through their own
  z-buffer (one target per pixel, the nearest);
* ``l1_loss``   mean |out - target| over target pixels whose output is valid;
* ``fit_sigmas``  Adam on (sigma_s, sigma_r) with the widths clamped to
  at least 0.25.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from typing import List, Optional, Sequence

from . import binding

MIN_SIGMA = 0.25


def _torch():
    import torch
    return torch


class Densify:
    """``Densify.apply(depth, valid, rgb, radius, sigma_s, sigma_r)`` returns
    (dense depth, mask); sigma_s and sigma_r are 0-d float tensors."""

    _fn = None

    @classmethod
    def apply(cls, depth, valid, rgb, radius, sigma_s, sigma_r):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(depth, valid, rgb, radius, sigma_s, sigma_r)


def _make_function():
    torch = _torch()

    class _Densify(torch.autograd.Function):
        @staticmethod
        def forward(ctx, depth, valid, rgb, radius, sigma_s, sigma_r):
            ss, sr = float(sigma_s), float(sigma_r)
            out, mask, aux = binding.densify(depth, valid, rgb, radius, ss, sr,
                                             want_aux=True, ws=None)
            ctx.save_for_backward(depth, valid, rgb, out, aux)
            ctx.radius, ctx.ss, ctx.sr = radius, ss, sr
            ctx.sdtype = (sigma_s.dtype, sigma_r.dtype)
            ctx.mark_non_differentiable(mask)
            return out, mask

        @staticmethod
        def backward(ctx, g_out, g_mask):
            depth, valid, rgb, out, aux = ctx.saved_tensors
            gd, gsig = binding.densify_backward(
                depth, valid, rgb, ctx.radius, ctx.ss, ctx.sr, out, aux,
                g_out.contiguous().float())
            g_ss = gsig[0].to(ctx.sdtype[0])
            g_sr = gsig[1].to(ctx.sdtype[1])
            return gd, None, None, None, g_ss, g_sr

    return _Densify


def heldout_targets(points, pose, intrinsics, width, height):
    """Nearest held-out point per pixel: (depth float32 (H,W), valid uint8)."""
    _, depth, valid = binding.project(points, pose, intrinsics, width, height)
    return depth, valid


def l1_loss(out, mask, target, target_valid):
    """Mean |out - target| over pixels with a target and a valid output."""
    torch = _torch()
    use = (target_valid == 1) & (mask == 1)
    n = use.sum()
    diff = torch.where(use, out - target, torch.zeros_like(out))
    return diff.abs().sum() / n.clamp(min=1), int(n)


@dataclasses.dataclass
class FitFrame:
    depth: object          # (H,W) float32 sparse input depth (device)
    valid: object          # (H,W) uint8
    rgb: object            # (H,W,3) uint8
    target: object         # (H,W) float32 held-out depth
    target_valid: object   # (H,W) uint8


def fit_sigmas(frames: Sequence[FitFrame], radius: int, sigma_s0: float,
               sigma_r0: float, steps: int = 200, lr: float = 0.05,
               betas=(0.9, 0.999), eps: float = 1e-8,
               log: Optional[list] = None, checkpoint: Optional[str] = None,
               resume: bool = False):
    """Adam on (sigma_s, sigma_r) minimising the held-out L1 loss summed over
    the frames' contributing targets. Returns (sigma_s, sigma_r, history).

    ``checkpoint``: a JSON file rewritten (atomically) after every step with
    the widths, Adam's moments and step count, and the history; with
    ``resume`` the fit continues from that file when it exists, so an
    interrupted fit of ``steps`` steps ends where an uninterrupted one would.
    """
    torch = _torch()
    dev = frames[0].depth.device
    params = torch.tensor([sigma_s0, sigma_r0], dtype=torch.float64,
                          device=dev, requires_grad=True)
    opt = torch.optim.Adam([params], lr=lr, betas=betas, eps=eps)
    history: List[dict] = []
    start = 0
    if resume and checkpoint and os.path.exists(checkpoint):
        st = load_state(checkpoint)
        with torch.no_grad():
            params.copy_(torch.tensor([st["sigma_s"], st["sigma_r"]],
                                      dtype=torch.float64))
        adam = st["adam"]
        if adam["step"] > 0:
            opt.state[params] = {
                "step": torch.tensor(float(adam["step"])),
                "exp_avg": torch.tensor(adam["exp_avg"], dtype=torch.float64,
                                        device=dev),
                "exp_avg_sq": torch.tensor(adam["exp_avg_sq"],
                                           dtype=torch.float64, device=dev)}
        history = list(st["history"])
        start = int(st["step"])
    for step in range(start, steps):
        opt.zero_grad()
        count = 0
        losses = []
        for f in frames:
            out, mask = Densify.apply(f.depth, f.valid, f.rgb, radius,
                                      params[0], params[1])
            use = (f.target_valid == 1) & (mask == 1)
            diff = torch.where(use, out - f.target, torch.zeros_like(out))
            losses.append(diff.abs().sum())
            count += int(use.sum())
        loss = torch.stack(losses).sum() / max(count, 1)
        loss.backward()
        opt.step()
        with torch.no_grad():
            params.clamp_(min=MIN_SIGMA)
        p = params.detach().cpu().tolist()
        rec = {"step": step, "loss": float(loss.detach()), "sigma_s": p[0],
               "sigma_r": p[1], "targets": count}
        history.append(rec)
        if log is not None:
            log.append(rec)
        if checkpoint:
            save_state(checkpoint, p[0], p[1], history, opt.state[params],
                       step + 1)
    return float(params[0]), float(params[1]), history


def save_state(path: str, sigma_s: float, sigma_r: float, history,
               adam_state=None, step: Optional[int] = None) -> None:
    """Checkpoint of the fit: the widths, Adam's moments and step count, and
    the history, written to a temporary file and renamed over ``path``."""
    adam = {"step": 0, "exp_avg": [0.0, 0.0], "exp_avg_sq": [0.0, 0.0]}
    if adam_state:
        adam = {"step": int(float(adam_state["step"])),
                "exp_avg": adam_state["exp_avg"].detach().cpu().tolist(),
                "exp_avg_sq": adam_state["exp_avg_sq"].detach().cpu().tolist()}
    state = {"sigma_s": sigma_s, "sigma_r": sigma_r,
             "step": len(history) if step is None else step, "adam": adam,
             "history": history}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(state, f)
    os.replace(tmp, path)


def load_state(path: str) -> dict:
    with open(path) as f:
        return json.load(f)
