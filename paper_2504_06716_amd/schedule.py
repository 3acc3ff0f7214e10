"""Host-side GSta schedule: freeze thresholds, freeze-map lifecycle, early
stop and the plateau learning-rate scheduler (Algorithm 1 and the "GSta
Details" of Section 4.1).  Pure Python scalars; the per-Gaussian work runs
in libgsta."""
from __future__ import annotations

import math
from dataclasses import dataclass

NONE, UPDATE, RESET = 0, 1, 2


@dataclass
class FreezeSchedule:
    """Freeze-map lifecycle (Section 4.1, "GSta Details").

    * no freezing before ``warmup``;
    * inside the window [warmup, min(window_end, stop_iter)] the map is
      updated every ``every`` iterations and accumulates (sticky);
    * at every multiple of ``reset_every`` inside the window the map is
      reset and no re-freezing happens for ``wait`` iterations;
    * when the window closes (early stop or window end) the map is reset
      and every Gaussian is trained again (finetune).
    Thresholds follow eq. 5 read as eps0 * clamp(lam1 + lam2 * k'/K, lam1,
    lam2) with k' = min(k, k_stop) (``linear``: eps0 * (lam1 + (lam2 - lam1)
    * k'/K)).  ``rule`` replaces the thresholds by one of the ablation's naive
    rules (Section 4.3): "mingrad" freezes the ``fraction`` of Gaussians with
    the lowest positional gradient average, "random" a random ``fraction``;
    the lifecycle stays the same."""

    total_iters: int
    warmup: int = 3000
    every: int = 250
    reset_every: int = 2000
    wait: int = 500
    window_end: int = 10000
    eps_xyz0: float = 3e-5
    eps_rgb0: float = 1e-4
    lam1: float = 0.5
    lam2: float = 1.5
    linear: bool = False
    rule: str = "gradient"           # "gradient" (eqs. 4-6), or the ablation's "mingrad" / "random"
    fraction: float = 0.25           # share the ablation rules freeze at each update
    seed: int = 5                    # Philox key of the "random" rule
    accumulate: bool = True          # ablation rules: OR into the map (else replace it at each update)
    fraction_at: dict | None = None  # ablation rules: per-update fraction {iteration: fraction}

    def rule_fraction(self, k: int) -> float:
        if self.fraction_at is not None and k in self.fraction_at:
            return self.fraction_at[k]
        return self.fraction

    def factor(self, k: int, k_stop: int | None = None) -> float:
        kk = k if k_stop is None else min(k, k_stop)
        K = self.total_iters
        if self.linear:
            return self.lam1 + (self.lam2 - self.lam1) * kk / K
        return min(max(self.lam1 + self.lam2 * kk / K, self.lam1), self.lam2)

    def thresholds(self, k: int, k_stop: int | None = None):
        f = self.factor(k, k_stop)
        return self.eps_xyz0 * f, self.eps_rgb0 * f

    def window_close(self, stop_iter: int | None = None) -> int:
        return self.window_end if stop_iter is None else min(self.window_end, stop_iter)

    def action(self, k: int, stop_iter: int | None = None) -> int:
        """What happens to the freeze map before iteration k."""
        end = self.window_close(stop_iter)
        if k == end:
            return RESET                                 # finetune: everyone trains again
        if k < self.warmup or k > end:
            return NONE
        if k > self.warmup and k % self.reset_every == 0:
            return RESET
        if k % self.every != 0:
            return NONE
        last_reset = (k // self.reset_every) * self.reset_every
        if last_reset > self.warmup and k - last_reset < self.wait:
            return NONE
        return UPDATE


def training_end(total_iters: int, window_end: int, stop_iter: int | None, finetune_iters: int) -> int:
    """Iterations of a whole training (Algorithm 1): when the freezing
    window closes (early stop or window_end) before total_iters, K_f =
    finetune_iters more iterations train every Gaussian and training ends
    there, also past total_iters; otherwise it ends at total_iters."""
    close = window_end if stop_iter is None else min(window_end, stop_iter)
    return total_iters if close >= total_iters else close + finetune_iters


@dataclass
class DensifySchedule:
    """Adaptive densification (Section 4.1): densify and prune every
    ``every`` iterations from ``start`` while k < min(``stop``, early stop);
    opacity reset every ``reset_every`` iterations in [reset_every, min(stop,
    early stop)].  Thresholds eps_den_xyz = 2e-4 and eps_den_rgb = 1e-6 are
    scaled by the same eq. 5 factor as the freezing thresholds; the colour
    criterion is drawn on a fraction ``rgb_prob`` of the densify steps.  The
    clone / split sizes and the prune opacity are 3DGS conventions."""

    total_iters: int
    start: int = 500
    stop: int = 10000
    every: int = 100
    reset_every: int = 3000
    eps_xyz0: float = 2e-4
    eps_rgb0: float = 1e-6
    rgb_prob: float = 0.2
    lam1: float = 0.5
    lam2: float = 1.5
    percent_dense: float = 0.01          # clone iff largest scale <= percent_dense * extent
    min_opacity: float = 0.005           # prune below
    split_div: float = 1.6               # children's scales = parent's / split_div
    reset_opacity: float = 0.01          # opacity cap of the reset
    seed: int = 4

    def end(self, stop_iter: int | None = None) -> int:
        return self.stop if stop_iter is None else min(self.stop, stop_iter)

    def densify_now(self, k: int, stop_iter: int | None = None) -> bool:
        return self.start <= k < self.end(stop_iter) and k % self.every == 0 and k > 0

    def reset_now(self, k: int, stop_iter: int | None = None) -> bool:
        return self.reset_every <= k <= self.end(stop_iter) and k % self.reset_every == 0

    def thresholds(self, k: int, k_stop: int | None = None):
        kk = k if k_stop is None else min(k, k_stop)
        f = min(max(self.lam1 + self.lam2 * kk / self.total_iters, self.lam1), self.lam2)
        return self.eps_xyz0 * f, self.eps_rgb0 * f

    def split_log_scale(self, extent: float) -> float:
        return math.log(self.percent_dense * extent)

    def prune_logit(self) -> float:
        return math.log(self.min_opacity / (1.0 - self.min_opacity))

    def reset_logit(self) -> float:
        return math.log(self.reset_opacity / (1.0 - self.reset_opacity))


def scene_extent(campos) -> float:
    """1.1 x the largest distance of a camera centre from their mean."""
    import numpy as np
    c = np.asarray(campos, np.float64)
    return 1.1 * float(np.linalg.norm(c - c.mean(0), axis=1).max())


def early_stop(psnrs, eps: float = 0.2) -> bool:
    """Eq. 7 with patience 1: the last two PSNR gains are both below eps."""
    if len(psnrs) < 3:
        return False
    return (psnrs[-1] - psnrs[-2] < eps) and (psnrs[-2] - psnrs[-3] < eps)


class PlateauLR:
    """Section 3.2.3: scale the position learning rate by ``factor`` after
    more than ``patience`` evaluations in a row whose PSNR does not exceed
    the best so far by more than ``eps`` (dB)."""

    def __init__(self, factor: float = 0.75, patience: int = 1, eps: float = 1.0):
        self.factor, self.patience, self.eps = factor, patience, eps
        self.scale = 1.0
        self.best = None
        self.bad = 0

    def step(self, psnr: float) -> float:
        if self.best is None or psnr > self.best + self.eps:
            self.best = psnr
            self.bad = 0
        else:
            self.bad += 1
        if self.bad > self.patience:
            self.scale *= self.factor
            self.bad = 0
        return self.scale


@dataclass
class LearningRates:
    """Per parameter group; the position LR decays exponentially from
    ``pos_init`` to ``pos_final`` (times the scene extent) over ``decay_iters``
    and is further scaled by the plateau scheduler.  Opacity uses 0.025
    (Section 4.1)."""

    extent: float = 3.3
    pos_init: float = 1.6e-4
    pos_final: float = 1.6e-6
    decay_iters: int = 30000
    scale: float = 5e-3
    rotation: float = 1e-3
    opacity: float = 0.025
    f_dc: float = 2.5e-3
    f_rest: float = 2.5e-3 / 20.0

    def position(self, k: int) -> float:
        t = min(max(k / max(self.decay_iters, 1), 0.0), 1.0)
        return self.extent * math.exp((1 - t) * math.log(self.pos_init) + t * math.log(self.pos_final))

    def rows(self, k: int, degree: int, pos_scale: float = 1.0):
        R = 11 + 3 * (degree + 1) ** 2
        lr = [0.0] * R
        lr[0:3] = [self.position(k) * pos_scale] * 3
        lr[3:6] = [self.scale] * 3
        lr[6:10] = [self.rotation] * 4
        lr[10] = self.opacity
        lr[11:14] = [self.f_dc] * 3
        for r in range(14, R):
            lr[r] = self.f_rest
        return lr
