"""Differentiable deskew and gradient-based calibration of the sheet angle.

``DeskewFunction`` wraps the library's forward kernel (float32 stack ->
deskewed volume) and its fused backward kernel, which returns the adjoint
(gradient with respect to the stack, the transpose resampling written as a
gather) and the gradient with respect to every image's offset.  The offsets
are a differentiable function of the sheet angle through Eq. 1,
``o[n] = n * z * cos(alpha) / p``, so torch carries the chain rule from the
per-image shear gradient to alpha.
"""
from __future__ import annotations

import math

import torch

from . import api


class DeskewFunction(torch.autograd.Function):
    """vol = D(stack; offsets) on a fixed frame (origin, width).  ``tune``:
    the forward's launch shape (None: library default; "auto": the shape
    the library's tuner picks for this frame, measured once)."""

    @staticmethod
    def forward(ctx, stack, offsets, origin, width, tune=None):
        out = api.deskew(stack, offsets=offsets.detach(), origin=int(origin), width=int(width),
                         psum=False, pmax=False, tune=tune)
        ctx.save_for_backward(stack, offsets)
        ctx.origin = int(origin)
        return out["vol"]

    @staticmethod
    def backward(ctx, grad_vol):
        stack, offsets = ctx.saved_tensors
        need_in, need_off = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_in or need_off):
            return None, None, None, None, None
        gi, go = api.backward(stack, grad_vol.contiguous(), offsets.detach().contiguous(),
                              ctx.origin, grad_in=need_in, grad_offsets=need_off)
        return gi, go, None, None, None


def deskew_volume(stack: torch.Tensor, offsets: torch.Tensor, origin: int,
                  width: int, tune=None) -> torch.Tensor:
    """Differentiable deskewed volume of a float32 CUDA stack (``tune`` as
    :class:`DeskewFunction`)."""
    return DeskewFunction.apply(stack, offsets, origin, width, tune)


def offsets_from_angle(angle_deg: torch.Tensor, n_planes: int, step_um: float,
                       pixel_um: float) -> torch.Tensor:
    """Eq. 1 per image: o[n] = n * (z cos(alpha)) / p, differentiable in alpha
    (degrees), FP64 on the angle's device."""
    alpha = angle_deg * (math.pi / 180.0)
    s = (step_um * torch.cos(alpha)) / pixel_um
    n = torch.arange(n_planes, dtype=torch.float64, device=angle_deg.device)
    return n * s


def minimise_angle(loss_and_grad, angle0_deg: float, iters: int = 300, lr: float = 0.05,
                   tol_deg: float = 1e-4):
    """1-D Adam on an angle (degrees) given ``loss_and_grad(angle) -> (L,
    dL/dangle)``.  The step halves whenever the gradient changes sign; the
    search stops once the step is below ``tol_deg``.  Returns (angle,
    history of (angle, loss))."""
    b1, b2, eps = 0.9, 0.999, 1e-30
    a = float(angle0_deg)
    m = v = 0.0
    prev = 0.0
    hist = []
    for t in range(1, iters + 1):
        loss, g = loss_and_grad(a)
        hist.append((a, float(loss)))
        if g == 0.0:
            break
        sign = math.copysign(1.0, g)
        if prev and sign != prev:
            lr *= 0.5
        prev = sign
        if lr < tol_deg:
            break
        m = b1 * m + (1.0 - b1) * g
        v = b2 * v + (1.0 - b2) * g * g
        mh = m / (1.0 - b1 ** t)
        vh = v / (1.0 - b2 ** t)
        a -= lr * mh / (math.sqrt(vh) + eps)
    return a, hist


def calibrate_stages(n_planes: int, first: int = 8):
    """Plane counts of the coarse-to-fine calibration: first, 2*first, ...,
    n_planes.  A shift error grows linearly with the plane index, so the
    first planes stay within a pixel of alignment for a wide range of
    angles; each doubling halves the angle range it can correct."""
    ks, k = [], max(2, min(first, n_planes))
    while k < n_planes:
        ks.append(k)
        k *= 2
    ks.append(n_planes)
    return ks


def calibrate_with(loss_and_grad_k, n_planes: int, angle0_deg: float, lr0: float = 0.5,
                   first: int = 8, tol_deg: float = 1e-4, iters: int = 200):
    """Coarse-to-fine angle calibration driven by ``loss_and_grad_k(angle,
    k) -> (L, dL/dangle)`` restricted to the first k planes.  Each stage runs
    ``minimise_angle`` from the previous estimate with a step that shrinks
    with k.  Returns (angle, history over all stages)."""
    a = float(angle0_deg)
    hist = []
    ks = calibrate_stages(n_planes, first)
    for i, k in enumerate(ks):
        lr = lr0 * ks[0] / k
        tol = tol_deg if i == len(ks) - 1 else lr / 64.0
        a, h = minimise_angle(lambda x: loss_and_grad_k(x, k), a, iters=iters, lr=lr,
                              tol_deg=tol)
        hist.extend(h)
    return a, hist


def calibrate_angle(stack: torch.Tensor, target: torch.Tensor, angle0_deg: float,
                    step_um: float, pixel_um: float, origin: int, width: int,
                    first: int = 8, lr0: float = 0.5, tol_deg: float = 1e-4):
    """Recover the sheet angle whose deskew of ``stack`` best matches
    ``target`` in least squares, by gradient descent through the adjoint:
    the loss gradient reaches alpha via the per-image shear gradient and
    Eq. 1.  Coarse to fine over the number of planes (``calibrate_with``).
    Returns (angle_deg, history)."""
    def loss_and_grad_k(a, k):
        angle = torch.tensor(a, dtype=torch.float64, device=stack.device, requires_grad=True)
        offs = offsets_from_angle(angle, k, step_um, pixel_um)
        vol = deskew_volume(stack[:k], offs, origin, width)
        loss = 0.5 * (vol.double() - target[:k].double()).pow(2).sum()
        loss.backward()
        return float(loss.detach()), float(angle.grad)

    return calibrate_with(loss_and_grad_k, stack.shape[0], angle0_deg, lr0=lr0, first=first,
                          tol_deg=tol_deg)
