"""torch.autograd binding of the renderer.

``render(params, cams, ...)`` returns the images of the views and records a
node whose backward calls the library's backward compositing, which
recomputes each pixel's transmittance front to back instead of storing any
per-(pixel, Gaussian) state.  Frozen Gaussians get a zero gradient and no
gradient work (Section 3.2.4).
"""
from __future__ import annotations

import torch

from .core import Context, camera_array


class _SlotRing:
    """Forward-state slots of a context, handed out round-robin."""

    def __init__(self, n):
        self.n = n
        self.i = 0

    def next(self):
        s = self.i
        self.i = (self.i + 1) % self.n
        return s


_rings: dict[int, _SlotRing] = {}


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params, frozen, gctx: Context, degree: int, cams, bg, slot: int):
        V = len(cams)
        H, W = cams[0].height, cams[0].width
        image = torch.empty((V, 3, H, W), dtype=torch.float32, device=params.device)
        gctx.render_forward(params, degree, cams, bg, image, slot)
        fctx.save_for_backward(params)
        fctx.frozen = frozen
        fctx.gctx, fctx.degree, fctx.cams, fctx.bg, fctx.slot = gctx, degree, cams, bg, slot
        return image

    @staticmethod
    def backward(fctx, dL_dimage):
        (params,) = fctx.saved_tensors
        grad = torch.zeros_like(params)
        fctx.gctx.render_backward(params, fctx.degree, fctx.cams, fctx.bg, fctx.slot,
                                  dL_dimage.contiguous(), fctx.frozen, grad)
        return grad, None, None, None, None, None, None


def render(params: torch.Tensor, cams, gctx: Context, degree: int, bg=(0.0, 0.0, 0.0),
           frozen: torch.Tensor | None = None, slot: int | None = None) -> torch.Tensor:
    """Differentiable render of ``cams`` (up to 8 views per call).

    params: [R, n] float32 device tensor (requires_grad for training).
    Returns [V, 3, H, W].  The forward state lives in a slot of ``gctx`` until
    the backward runs; slots are used round-robin, so at most ``n_slots``
    renders of one context may await their backward at a time.
    """
    if slot is None:
        ring = _rings.setdefault(id(gctx), _SlotRing(gctx.limits.n_slots))
        slot = ring.next()
    carr = camera_array(cams) if isinstance(cams, (list, tuple)) else cams
    return RenderFunction.apply(params, frozen, gctx, degree, carr, tuple(bg), slot)
