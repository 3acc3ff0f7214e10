"""One-time calibration of the initial freeze thresholds for a workload.

The paper picks eps_f_xyz and eps_f_rgb once, by watching how the gradient
magnitudes of each parameter group converge, and keeps them for every scene
(Section 4.1).  Gradient magnitudes depend on the loss normalisation, the
image size and the Gaussian density, so on a synthetic workload whose
scale differs from the paper's scenes the same observation is made here,
written as a rule: train without freezing up to the start of the freeze
window while tracking the gradient-norm moving averages, and choose eps0 so
that the threshold at the window start equals the q-quantile of the positive
averages of the Gaussians seen so far.  q is the rule's single parameter.
"""
from __future__ import annotations

import numpy as np
import torch

from .schedule import FreezeSchedule
from .train import FLT_MAX, Trainer


def ema_snapshot(tr: Trainer) -> np.ndarray:
    """[4, n] gradient-norm EMAs (xyz, rgb, opacity, scale); FLT_MAX = never seen."""
    torch.cuda.synchronize()
    return tr.ema.cpu().numpy()


def thresholds_from_quantile(ema: np.ndarray, sched: FreezeSchedule, q: float):
    """eps0 per group such that eps(window start) is the q-quantile of the
    positive averages.  Gaussians whose average is zero (no gradient reached
    them, e.g. fully occluded ones) are left out of the quantile: any
    positive threshold freezes them."""
    f = sched.factor(sched.warmup, sched.window_close())
    out = []
    for k in (0, 1):
        e = ema[k]
        pos = e[(e < FLT_MAX) & (e > 0)]
        out.append(float(np.quantile(pos, q)) / f if pos.size else 0.0)
    return tuple(out)
