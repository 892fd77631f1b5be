"""Differentiable DAS and gradient-based sound-speed autofocus.

``das(e, c, plan)`` is a torch.autograd.Function around bf_das whose backward
calls the hand-written adjoint kernel (bf_das_adjoint): the gradient with
respect to the decoded data is the transpose of the beamforming map, and the
gradient with respect to the scalar sound speed c flows through the delays
only (ds/dc = -tof * fs / c).  ``sharpness(img)`` wraps bf_sharpness, the
negative normalised L4 norm -sum I^4 / (sum I^2)^2 per image.

``autofocus`` minimises the summed sharpness loss of a batch of frames over c
with the exact gradient.  Frames given as a list are beamformed one by one,
each under torch.utils.checkpoint, so its image is recomputed in backward
instead of being kept alive (the memory of a batch stays at one image).
Frames given as one stacked tensor (F, n_tx, n_ch, S) go through the
frame-stack entry points: the forward runs one launch per frame
(bf_das_frames), the LDS adjoint one launch per gradient over the whole stack
(bf_das_adjoint_frames), and the sharpness one launch for all F images.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint


class _DasFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, e, c, plan):
        img = plan.das(e, c=float(c))
        ctx.save_for_backward(e, c)
        ctx.plan = plan
        return img

    @staticmethod
    def backward(ctx, grad_img):
        e, c = ctx.saved_tensors
        want_e, want_c = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        ge, gc = ctx.plan.das_adjoint(e, grad_img, c=float(c), want_e=want_e, want_c=want_c)
        # a stack of frames gives one dL/dc term per frame; c is shared
        gc_out = (gc.to(device=c.device, dtype=c.dtype).sum().reshape(c.shape)
                  if want_c else None)
        return ge if want_e else None, gc_out, None


class _SharpnessFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, img, n_images):
        from . import sharpness as _sharp
        loss, g = _sharp(img.reshape(n_images, -1), grad=True)
        ctx.save_for_backward(g.reshape(img.shape))
        return loss.sum()

    @staticmethod
    def backward(ctx, grad_loss):
        (g,) = ctx.saved_tensors
        return g * grad_loss, None


def das(e, c, plan):
    """Differentiable DAS image of decoded data e at sound speed c (0-d
    tensor); e may be a stack of frames (F, n_tx, n_ch, S)."""
    return _DasFunction.apply(e, c, plan)


def sharpness(img, n_images: int = 1):
    """Differentiable -sum I^4 / (sum I^2)^2 of one image, or its sum over
    the n_images images stacked along the first axis of img."""
    return _SharpnessFunction.apply(img, n_images)


def _stacked(frames, plan):
    return torch.is_tensor(frames) and frames.dim() == len(plan.e_shape) + 1


def focus_loss(frames, c, plan, use_checkpoint: bool = True):
    """Sum over frames of the sharpness loss at sound speed c.  frames: a
    list of decoded frames, or one stacked (F, n_tx, n_ch, S) tensor."""
    if _stacked(frames, plan):
        nf = int(frames.shape[0])
        if use_checkpoint:
            return checkpoint(lambda ee, cc: sharpness(das(ee, cc, plan), nf), frames, c,
                              use_reentrant=False)
        return sharpness(das(frames, c, plan), nf)
    total = None
    for e in frames:
        if use_checkpoint:
            term = checkpoint(lambda ee, cc: sharpness(das(ee, cc, plan)), e, c, use_reentrant=False)
        else:
            term = sharpness(das(e, c, plan))
        total = term if total is None else total + term
    return total


def scan(frames, plan, cs):
    """Forward-only loss at each sound speed of `cs` (no gradients)."""
    out = []
    with torch.no_grad():
        for cv in cs:
            c = torch.tensor(float(cv), dtype=torch.float64)
            out.append(float(focus_loss(frames, c, plan, use_checkpoint=False)))
    return out


def autofocus(frames, plan, bounds=(1450.0, 1600.0), scan_step: float = 2.5, iters: int = 12):
    """Sound speed minimising the summed sharpness loss of `frames`.

    The loss of an RF (not envelope) image oscillates with c on the scale of
    a fraction of a wavelength of delay, so a gradient method alone stops at
    the nearest stationary point.  A forward scan at `scan_step` locates the
    best basin; secant iterations on dL/dc = 0 with the exact adjoint gradient
    (checkpointed frames) then refine inside +-scan_step of it.
    Returns (c, scan list of (c, loss), refinement list of (c, loss, dL/dc))."""
    import numpy as np
    cs = np.arange(bounds[0], bounds[1] + 1e-9, scan_step)
    losses = scan(frames, plan, cs)
    k = int(np.argmin(losses))
    lo, hi = float(cs[max(k - 1, 0)]), float(cs[min(k + 1, len(cs) - 1)])
    hist = []

    def grad_at(cv):
        c = torch.tensor(cv, dtype=torch.float64, requires_grad=True)
        loss = focus_loss(frames, c, plan)
        loss.backward()
        hist.append((cv, float(loss), float(c.grad)))
        return float(c.grad)

    a, b = lo, hi
    ga, gb = grad_at(a), grad_at(b)
    c_best = float(cs[k])
    if ga < 0 < gb:                 # a minimum is bracketed: safeguarded secant
        for _ in range(iters):
            cm = b - gb * (b - a) / (gb - ga)
            if not (a < cm < b):
                cm = 0.5 * (a + b)
            gm = grad_at(cm)
            if abs(gm) < 1e-12 or b - a < 1e-3:
                break
            if gm < 0:
                a, ga = cm, gm
            else:
                b, gb = cm, gm
        c_best = min(hist, key=lambda h: h[1])[0]
    return c_best, list(zip(cs.tolist(), losses)), hist
